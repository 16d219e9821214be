// ch.hip -- fused Cahn-Hilliard steps (Section 5.1) with the state kept in
// registers: the right-hand-side policy of the fused stepper (stepper.h).
#include "long_core.h"
#include "stepper.h"

namespace bb {
namespace {

// ---------------------------------------------------------------- Cahn-Hilliard
// `steps` steps of C <- A^{-1} (C + alpha d2(C^3 - C)), periodic, state in registers.
__device__ __forceinline__ double ch_nl(double c) { return fma(c * c, c, -c); }

// Right-hand side of one step on this lane's chunk, in place:
// f_t = c_t + alpha (N_{t-1} - 2 N_t + N_{t+1}), N = c^3 - c, with the
// neighbour rows cl (above the chunk) and cr (below it) and the periodic wrap
// terms of rows 0 and n-1 (r0 = c_0, rn1 = c_{n-1} of the system).
// nrow = n - (first row of the chunk); with FULL the chunks tile n and row
// n-1 is the last row of the last chunk (last_chunk).
template <int C, bool FULL>
__device__ __forceinline__ void ch_rhs(double (&c)[C], double cl, double cr, double r0, double rn1,
                                       double alpha, int j, bool last_chunk, int nrow)
{
    const double wrap_first = alpha * ch_nl(rn1);   // row 0 sees row n-1 on its left
    const double wrap_last = alpha * ch_nl(r0);     // row n-1 sees row 0 on its right
    double nprev = ch_nl(cl), ncur = ch_nl(c[0]);
    rows_up<C>([&](int t) {
        const double nnext = ch_nl(t + 1 < C ? c[t + 1] : cr);
        double f = fma(alpha, fma(-2.0, ncur, nprev) + nnext, c[t]);
        if (t == 0) f += (j == 0) ? wrap_first : 0.0;
        if constexpr (FULL) {
            if (t == C - 1) f += last_chunk ? wrap_last : 0.0;
        } else {
            f += (t == nrow - 1) ? wrap_last : 0.0;
            f = t < nrow ? f : 0.0;
        }
        c[t] = f;
        nprev = ncur;
        ncur = nnext;
    });
}

// The Cahn-Hilliard right-hand side as a policy of the fused stepper.
struct ChRhs {
    static constexpr int R = 1;
    double alpha;
    struct State {};
    __device__ State lane_state(int64_t, int) const { return State{}; }
    template <int C, bool FULL>
    __device__ __forceinline__ void operator()(double (&c)[C], const Halo &h, int j,
                                               bool last_chunk, int nrow, const State &) const
    {
        ch_rhs<C, FULL>(c, h.l1, h.r1, h.e0, h.en1, alpha, j, last_chunk, nrow);
    }
};

// The Cahn-Hilliard right-hand side as the source of the long-system
// launches: rows of the state plus the neighbour row on each side (indices
// mod n), so no wrap term is needed beyond the halo.
struct ChLongSrc {
    const double *c;
    double alpha;
    template <int C>
    __device__ __forceinline__ void full(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, true>(v, c, row0, k, ld, n);
        const int left = row0 > 0 ? row0 - 1 : n - 1;
        const int right = row0 + C < n ? row0 + C : 0;
        const double cl = c[(int64_t)left * ld + k], cr = c[(int64_t)right * ld + k];
        ch_rhs<C, true>(v, cl, cr, 0.0, 0.0, alpha, 1, false, C);
    }
    // the last chunk: rows row0 .. n-1 (at least one, and row0 > 0)
    template <int C>
    __device__ __forceinline__ void tail(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, false>(v, c, row0, k, ld, n);
        const double cl = c[(int64_t)(row0 - 1) * ld + k], c0 = c[k];
        ch_rhs<C, false>(v, cl, 0.0, c0, 0.0, alpha, 1, true, n - row0);
    }
};

// lbar[s] = 1 + inv_m * sum over groups of partial[group][s], groups in
// order; the partial sums hold l - 1 per run (about <C^2>, a few thousandths
// early in a coarsening run), whose rounding the 1 would otherwise swamp.
__global__ void stats_fold(const double *__restrict__ partial, int64_t groups, int64_t samples,
                           double inv_m, double *__restrict__ lbar)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= samples) return;
    double acc = 0.0;
    for (int64_t r = 0; r < groups; ++r) acc += partial[r * samples + s];
    lbar[s] = fma(acc, inv_m, 1.0);
}

}  // namespace

hipError_t launch_ch_long(const double *table, const CyclicQ &q, const LongGeom &g, double alpha,
                          const double *c_in, double *c_out, hipStream_t s)
{
    return launch_long_k<2, true>(table, q, g, ChLongSrc{c_in, alpha}, c_out, s);
}

hipError_t launch_ch(const double *table, int64_t table_elems, const CyclicQ &q,
                     const SweepGeom &g, bool scalar, double alpha, int64_t steps,
                     const double *in, double *out, hipStream_t s, int64_t every,
                     int64_t samples, double *partial, double *lbar)
{
    if (!partial || samples < 1)
        return launch_stepper<ChRhs, 2, true>(table, table_elems, q, g, scalar, ChRhs{alpha},
                                              steps, in, out, s);
    StepStats st;
    st.partial = partial;
    st.every = every;
    st.samples = samples;
    st.inv_n = 1.0 / g.n;
    hipError_t e = launch_stepper<ChRhs, 2, true, true>(table, table_elems, q, g, scalar,
                                                        ChRhs{alpha}, steps, in, out, s, st);
    if (e != hipSuccess) return e;
    const int threads = 256;
    hipLaunchKernelGGL(stats_fold, dim3((unsigned)((samples + threads - 1) / threads)),
                       dim3(threads), 0, s, (const double *)partial, g.groups, samples,
                       1.0 / (double)g.m, lbar);
    return hipGetLastError();
}

}  // namespace bb
