// ch_forced.hip -- fused steps of the forced Cahn-Hilliard equation in the
// frame of the travelling wave (the forced flow-pattern section, numerical
// scheme): the Section 5.1 right-hand side plus an advection term,
// differenced with the fifth-order Hamilton-Jacobi WENO scheme the paper
// cites, and a sinusoidal forcing; each run has its own advection speed and
// forcing.  A right-hand-side policy of the fused stepper (stepper.h).
#include <cmath>

#include "long_core.h"
#include "stepper.h"

namespace bb {
namespace {

__device__ __forceinline__ double nl3(double c) { return fma(c * c, c, -c); }

// dx times the one-sided WENO5 derivative from the five one-sided
// differences v1..v5 ordered from the far upwind end (Jiang and Peng): three
// third-order candidates blended with weights 0.1, 0.6, 0.3 over
// (smoothness + eps)^2, eps = 1e-6 max v_q^2 + 1e-99.
__device__ __forceinline__ double weno5(double v1, double v2, double v3, double v4, double v5)
{
    const double p1 = fma(v1, 1.0 / 3.0, fma(v2, -7.0 / 6.0, v3 * (11.0 / 6.0)));
    const double p2 = fma(v2, -1.0 / 6.0, fma(v3, 5.0 / 6.0, v4 * (1.0 / 3.0)));
    const double p3 = fma(v3, 1.0 / 3.0, fma(v4, 5.0 / 6.0, v5 * (-1.0 / 6.0)));
    const double a = v1 - 2.0 * v2 + v3, b = v1 - 4.0 * v2 + 3.0 * v3;
    const double c = v2 - 2.0 * v3 + v4, d = v2 - v4;
    const double e = v3 - 2.0 * v4 + v5, g = 3.0 * v3 - 4.0 * v4 + v5;
    const double s1 = fma(13.0 / 12.0, a * a, 0.25 * b * b);
    const double s2 = fma(13.0 / 12.0, c * c, 0.25 * d * d);
    const double s3 = fma(13.0 / 12.0, e * e, 0.25 * g * g);
    const double vm = fmax(fmax(fmax(v1 * v1, v2 * v2), fmax(v3 * v3, v4 * v4)), v5 * v5);
    const double eps = fma(1e-6, vm, 1e-99);
    const double t1 = s1 + eps, t2 = s2 + eps, t3 = s3 + eps;
    // 1/t_k from one division: t_k >= 1e-99, so t1 t2 t3 >= 1e-297 stays a
    // normal double (and below 1e8 for differences of O(1) states)
    const double inv = 1.0 / (t1 * t2 * t3);
    const double r1 = t2 * t3 * inv, r2 = t1 * t3 * inv, r3 = t1 * t2 * inv;
    const double w1 = 0.1 * r1 * r1, w2 = 0.6 * r2 * r2, w3 = 0.3 * r3 * r3;
    return fma(w1, p1, fma(w2, p2, w3 * p3)) / (w1 + w2 + w3);
}

// f_i = C_i + alpha (N_{i-1} - 2 N_i + N_{i+1}) + beta W_i(C) + amp cos(kdx i),
// N = C^3 - C, periodic, W upwinded for dC/dt = v dC/deta (beta > 0:
// right-biased differences).  The scheme's per-run coefficients follow from
// the physical parameters of run k when its group is loaded: the advection
// term dt v dC/deta with the WENO derivative W/dx gives beta = dt v / dx, the
// forcing dt f0 k cos(k eta) at eta_i = i dx gives amp = dt f0 k and
// kdx = k dx.
struct ForcedChRhs {
    static constexpr int R = 3;
    double alpha, dt, dx;
    const double *v, *f0, *k;   // device, one per run
    struct State {
        double beta, amp, c0, s0, cd, sd;   // cos, sin of kdx * row0 and of kdx
    };
    __device__ State lane_state(int64_t run, int row0) const
    {
        State st;
        const double kr = k[run];
        st.beta = dt * v[run] / dx;
        st.amp = dt * f0[run] * kr;
        const double kd = kr * dx;
        sincos(kd * (double)row0, &st.s0, &st.c0);
        sincos(kd, &st.sd, &st.cd);
        return st;
    }

    template <int C, bool FULL>
    __device__ __forceinline__ void operator()(double (&c)[C], const Halo &h, int j,
                                               bool last_chunk, int nrow, const State &st) const
    {
        // rows j*C - 1 .. j*C - 3: the previous chunk, or rows n-1 .. n-3
        double m1 = h.l1, m2 = h.l2, m3 = h.l3;
        if (j == 0) {
            m1 = h.en1;
            m2 = h.en2;
            m3 = h.en3;
        }
        // rows j*C + C .. j*C + C + 2: the next chunk, or rows 0 .. 2 after
        // the last chunk of a full decomposition
        double q1 = h.r1, q2 = h.r2, q3 = h.r3;
        if constexpr (FULL) {
            if (last_chunk) {
                q1 = h.e0;
                q2 = h.e1;
                q3 = h.e2;
            }
        }
        // row t + d of the chunk (d = 1..3) before this step
        auto ahead = [&](int t, int d) -> double {
            const int u = t + d;
            double x = u < C ? c[u < C ? u : C - 1] : (u == C ? q1 : (u == C + 1 ? q2 : q3));
            if constexpr (!FULL) {
                const int w = u - nrow;   // ragged: past row n-1 come rows 0, 1, 2
                x = w < 0 ? x : (w == 0 ? h.e0 : (w == 1 ? h.e1 : h.e2));
            }
            return x;
        };
        const bool plus = st.beta > 0.0;
        double nprev = nl3(m1), ncur = nl3(c[0]);
        double cs = st.c0, sn = st.s0;
        rows_up<C>([&](int t) {
            const double cur = c[t];
            const double p1 = ahead(t, 1), p2 = ahead(t, 2), p3 = ahead(t, 3);
            const double nnext = nl3(p1);
            double f = fma(alpha, fma(-2.0, ncur, nprev) + nnext, cur);
            // one-sided differences from the far upwind end
            const double v1 = plus ? p3 - p2 : m2 - m3;
            const double v2 = plus ? p2 - p1 : m1 - m2;
            const double v3 = plus ? p1 - cur : cur - m1;
            const double v4 = plus ? cur - m1 : p1 - cur;
            const double v5 = plus ? m1 - m2 : p2 - p1;
            f = fma(st.beta, weno5(v1, v2, v3, v4, v5), f);
            f = fma(st.amp, cs, f);
            if constexpr (!FULL) f = t < nrow ? f : 0.0;
            c[t] = f;
            m3 = m2;
            m2 = m1;
            m1 = cur;
            nprev = ncur;
            ncur = nnext;
            const double cn = fma(cs, st.cd, -sn * st.sd);   // rotate to row t + 1
            sn = fma(sn, st.cd, cs * st.sd);
            cs = cn;
        });
    }
};

// The forced right-hand side as the source of the long-system launches
// (one step per call): a chunk's rows and the three rows on each side of it,
// indices mod n, read from the state before the step.  The halo takes the
// place of the wrap rows, so the policy sees every chunk as an inner one.
struct ForcedLongSrc {
    ForcedChRhs rhs;
    const double *c;
    __device__ __forceinline__ double row(int i, int64_t k, int64_t ld, int n) const
    {
        i = i < 0 ? i + n : (i >= n ? i - n : i);
        return c[(int64_t)i * ld + k];
    }
    template <int C>
    __device__ __forceinline__ void full(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, true>(v, c, row0, k, ld, n);
        Halo h{};
        h.l1 = row(row0 - 1, k, ld, n);
        h.l2 = row(row0 - 2, k, ld, n);
        h.l3 = row(row0 - 3, k, ld, n);
        h.r1 = row(row0 + C, k, ld, n);
        h.r2 = row(row0 + C + 1, k, ld, n);
        h.r3 = row(row0 + C + 2, k, ld, n);
        rhs.template operator()<C, true>(v, h, 1, false, C, rhs.lane_state(k, row0));
    }
    // the last chunk: rows row0 .. n-1 (row0 >= C >= 16); past row n-1 come
    // rows 0, 1, 2
    template <int C>
    __device__ __forceinline__ void tail(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, false>(v, c, row0, k, ld, n);
        Halo h{};
        h.l1 = row(row0 - 1, k, ld, n);
        h.l2 = row(row0 - 2, k, ld, n);
        h.l3 = row(row0 - 3, k, ld, n);
        h.e0 = c[k];
        h.e1 = c[ld + k];
        h.e2 = c[2 * ld + k];
        rhs.template operator()<C, false>(v, h, 1, false, n - row0, rhs.lane_state(k, row0));
    }
};

}  // namespace

hipError_t launch_ch_forced_long(const double *table, const CyclicQ &q, const LongGeom &g,
                                 double alpha, double dt, double dx, const double *v,
                                 const double *f0, const double *k, const double *in, double *out,
                                 hipStream_t s)
{
    ForcedChRhs r;
    r.alpha = alpha;
    r.dt = dt;
    r.dx = dx;
    r.v = v;
    r.f0 = f0;
    r.k = k;
    return launch_long_k<2, true>(table, q, g, ForcedLongSrc{r, in}, out, s);
}

hipError_t launch_ch_forced(const double *table, int64_t table_elems, const CyclicQ &q,
                            const SweepGeom &g, bool scalar, double alpha, double dt, double dx,
                            const double *v, const double *f0, const double *k, int64_t steps,
                            const double *in, double *out, hipStream_t s)
{
    ForcedChRhs r;
    r.alpha = alpha;
    r.dt = dt;
    r.dx = dx;
    r.v = v;
    r.f0 = f0;
    r.k = k;
    return launch_stepper<ForcedChRhs, 2, true>(table, table_elems, q, g, scalar, r, steps, in,
                                                out, s);
}

}  // namespace bb
