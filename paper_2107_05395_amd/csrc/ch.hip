// ch.hip -- fused Cahn-Hilliard steps (Section 5.1) with the state kept in
// registers; building blocks in sweep_core.h.
#include "sweep_core.h"

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

template <int C, bool FULL>
__global__ __launch_bounds__(kMaxBlockThreads) void ch_kernel(const double *__restrict__ table,
                                                           int64_t table_elems, CyclicQ cq,
                                                           SweepGeom g, double alpha,
                                                           int64_t steps, const double *in,
                                                           double *out)
{
    extern __shared__ double smem_d[];
    stage_table(smem_d, table, table_elems);
    __syncthreads();

    const LaneGeom lg = lane_geom(g.log2P);
    const int lane = threadIdx.x % kWave;
    const int row0 = lg.j * C;
    const bool has_left = lg.j > 0, has_right = lg.j < lg.P - 1;
    const int left = has_left ? lane - lg.S : lane;
    const int right = has_right ? lane + lg.S : lane;
    const int exact = FULL || g.exact;
    const GroupRange gr = group_range(g.groups);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        double c[C];
        load_chunk<double, C, FULL>(c, in, row0, kval ? k : g.m - 1, g.ld, g.n);

        for (int64_t step = 0; step < steps; ++step) {
            double cl = shfl(c[C - 1], left), cr = shfl(c[0], right);
            if (!has_left) cl = 0.0;
            if (!has_right) cr = 0.0;
            double r0, r1, rn2, rn1;
            gather_ends<double, 2, C>(c, lg, g.n, exact, r0, r1, rn2, rn1);
            ch_rhs<C, FULL>(c, cl, cr, r0, rn1, alpha, lg.j, lg.j == lg.P - 1, opaque_v(g.n - row0));
            __builtin_amdgcn_sched_barrier(0);
            chunk_solve<double, 2, C, true>(c, smem_d, lg, g.n, exact, cq);
        }
        if (kval) store_chunk<double, C, FULL>(c, out, row0, k, g.ld, g.n);
    }
}

// The same steps with one chunk per wave: a workgroup of P = 2^QL waves holds
// one group of 64 systems, wave j their rows j*C .. j*C + C - 1.  Every lane
// of a wave then needs the same coefficient row at the same time, so the
// coefficients come from the global table through the scalar cache (no LDS
// staging, no LDS reads) and the chunk-boundary values go through the LDS
// exchange area: rows 0 and C-1 of every chunk for the stencil and the wrap
// terms, then the three phases of chunk_solve.
template <int C, int QL>
__global__ __launch_bounds__((kWave << QL) > kMaxBlockThreads ? (kWave << QL) : kMaxBlockThreads)
void ch_kernel_uniform(const double *__restrict__ table, CyclicQ cq, SweepGeom g, double alpha,
                       int64_t steps, const double *in, double *out)
{
    using Src = FromScalar<double>;
    extern __shared__ double smem_d[];
    double *xch = smem_d;                                   // chunk_solve phases
    double *xd = smem_d + split_exchange_len(QL);           // rows 0, C-1 per (chunk, slot)
    const typename Src::ptr tab = (typename Src::ptr)table;

    LaneGeom lg = lane_geom(QL, QL);
    lg.j = __builtin_amdgcn_readfirstlane(lg.j);            // the wave's chunk: uniform
    const int row0 = lg.j * C;
    const bool has_left = lg.j > 0, has_right = lg.j < lg.P - 1;
    const int PS = lg.P * kWave;   // xd: [2][P*64], rows 0 and C-1 of (chunk, slot)
    const int me = lg.j * kWave + lg.sl;
    const int lft = (has_left ? lg.j - 1 : lg.j) * kWave + lg.sl;
    const int rgt = (has_right ? lg.j + 1 : lg.j) * kWave + lg.sl;
    const int first = lg.sl, last = (lg.P - 1) * kWave + lg.sl;
    const GroupRange gr = group_range(g.groups, QL);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * kWave + lg.sl;
        const bool kval = k < g.m;
        double c[C];
        load_chunk<double, C, true>(c, in, row0, kval ? k : g.m - 1, g.ld, g.n);

        for (int64_t step = 0; step < steps; ++step) {
            xd[me] = c[0];
            xd[PS + me] = c[C - 1];
            __syncthreads();
            const double cl = has_left ? xd[PS + lft] : 0.0;
            const double cr = has_right ? xd[rgt] : 0.0;
            ch_rhs<C, true>(c, cl, cr, xd[first], xd[PS + last], alpha, lg.j, !has_right, C);
            __builtin_amdgcn_sched_barrier(0);
            chunk_solve<double, 2, C, true, true, Src>(c, tab, lg, g.n, 1, cq, xch);
        }
        if (kval) store_chunk<double, C, true>(c, out, row0, k, g.ld, g.n);
    }
}

}  // namespace

hipError_t launch_ch(const double *table, int64_t table_elems, const CyclicQ &q,
                     const SweepGeom &g, double alpha, int64_t steps, const double *in,
                     double *out, hipStream_t s)
{
    if (g.log2Q > 0) {
        // one chunk per wave (host checks: full decomposition, log2Q == log2P)
        if (g.C != 64 || g.log2Q != g.log2P || g.log2Q > 3 || !is_full(g)) return hipErrorInvalidValue;
        const size_t xl = (size_t)(split_exchange_len(g.log2Q) + (2LL * kWave << g.log2Q)) * sizeof(double);
        switch (g.log2Q) {
        case 1: return launch_grid_split(ch_kernel_uniform<64, 1>, xl, g.groups, 2, s, table, q, g, alpha, steps, in, out);
        case 2: return launch_grid_split(ch_kernel_uniform<64, 2>, xl, g.groups, 4, s, table, q, g, alpha, steps, in, out);
        default: return launch_grid_split(ch_kernel_uniform<64, 3>, xl, g.groups, 8, s, table, q, g, alpha, steps, in, out);
        }
    }
    const size_t lds = (size_t)table_elems * sizeof(double);
#define BB_CH(CC)                                                                              \
    case CC:                                                                                   \
        return is_full(g) ? launch_grid(ch_kernel<CC, true>, lds, g.groups, s, table,           \
                                        table_elems, q, g, alpha, steps, in, out)               \
                          : launch_grid(ch_kernel<CC, false>, lds, g.groups, s, table,          \
                                        table_elems, q, g, alpha, steps, in, out);
    switch (g.C) {
        BB_CH(4)
        BB_CH(8)
        BB_CH(16)
        BB_CH(32)
        BB_CH(64)
        BB_CH(128)
    default: return hipErrorInvalidValue;
    }
#undef BB_CH
}

}  // namespace bb
