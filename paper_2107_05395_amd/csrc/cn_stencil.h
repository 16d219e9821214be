// cn_stencil.h -- the right-hand side of a Crank-Nicolson step as a policy of
// the fused stepper (stepper.h): periodic diffusion (Section 3 benchmark
// problem, K = 1) and periodic hyperdiffusion (Section 4 benchmark problem,
// K = 2), and their non-periodic forms.  cn_tri.hip and cn_penta.hip
// instantiate it.
#pragma once

#include "long_core.h"
#include "stepper.h"

namespace bb {
namespace {

// f_i = sum_{d=-K..K} w[d+K] c_{i+d}: the explicit half B of the scheme, a
// constant stencil of 2K+1 weights.  Periodic (CYC): indices wrap mod n like
// the matrix.  Otherwise the terms whose row falls outside the system are left
// out.  The sum is one fma chain from the leftmost term, so every kernel that
// uses the policy rounds it the same way.
template <int K, bool CYC>
struct StencilRhs {
    static constexpr int R = K;
    double w[2 * K + 1];
    struct State {};
    __device__ State lane_state(int64_t, int) const { return State{}; }

    template <int C, bool FULL>
    __device__ __forceinline__ void operator()(double (&c)[C], const Halo &h, int j,
                                               bool last_chunk, int nrow, const State &) const
    {
        // rows j*C - 1, j*C - 2: the previous chunk, or rows n-1, n-2 (periodic)
        double m1 = h.l1, m2 = h.l2;
        if (j == 0) {
            m1 = CYC ? h.en1 : 0.0;
            m2 = CYC ? h.en2 : 0.0;
        }
        // rows j*C + C, j*C + C + 1: the next chunk, or rows 0, 1 (periodic)
        // after the last chunk of a full decomposition
        double q1 = h.r1, q2 = h.r2;
        if constexpr (FULL) {
            if (last_chunk) {
                q1 = CYC ? h.e0 : 0.0;
                q2 = CYC ? h.e1 : 0.0;
            }
        }
        // ragged: rows past n-1 of the system are rows 0, 1 (periodic) or absent
        const double past0 = CYC ? h.e0 : 0.0, past1 = CYC ? h.e1 : 0.0;
        rows_up<C>([&](int t) {
            const double cur = c[t];
            double p1 = t + 1 < C ? c[t + 1] : q1;
            if constexpr (!FULL) p1 = t + 1 < nrow ? p1 : (t + 1 == nrow ? past0 : past1);
            double f;
            if constexpr (K == 1) {
                f = fma(w[2], p1, fma(w[1], cur, w[0] * m1));
            } else {
                double p2 = t + 2 < C ? c[t + 2] : (t + 2 == C ? q1 : q2);
                if constexpr (!FULL) p2 = t + 2 < nrow ? p2 : (t + 2 == nrow ? past0 : past1);
                f = fma(w[4], p2, fma(w[3], p1, fma(w[2], cur, fma(w[1], m1, w[0] * m2))));
            }
            if constexpr (!FULL) f = t < nrow ? f : 0.0;
            c[t] = f;
            m2 = m1;
            m1 = cur;
        });
    }
};

// traj_stride > 0: store the state after every step s at out + s * traj_stride
// (a trajectory) instead of only the last one.
template <int K, bool CYC>
hipError_t launch_cn_kc(const double *table, int64_t table_elems, const CyclicQ &q,
                        const SweepGeom &g, bool scalar, const double *w, int64_t steps,
                        int64_t traj_stride, const double *in, double *out, hipStream_t s)
{
    StencilRhs<K, CYC> r;
    for (int d = 0; d <= 2 * K; ++d) r.w[d] = w[d];
    if (traj_stride > 0) {
        StepStats st;
        st.traj_stride = traj_stride;
        return launch_stepper<StencilRhs<K, CYC>, K, CYC, false, true>(table, table_elems, q, g, scalar,
                                                                      r, steps, in, out, s, st);
    }
    return launch_stepper<StencilRhs<K, CYC>, K, CYC>(table, table_elems, q, g, scalar, r, steps, in,
                                                      out, s);
}

// The stencil as the source of the long-system launches (one step per call):
// a chunk's rows and the K rows on each side of it, read from the state
// before the step -- wrapped mod n (periodic) or zero outside the system.
// The halo takes the place of the wrap rows, so the policy sees every chunk
// as an inner one.
template <int K, bool CYC>
struct StencilLongSrc {
    StencilRhs<K, CYC> rhs;
    const double *c;
    __device__ __forceinline__ double row(int i, int64_t k, int64_t ld, int n) const
    {
        if constexpr (CYC) {
            i = i < 0 ? i + n : (i >= n ? i - n : i);
        } else {
            if (i < 0 || i >= n) return 0.0;
        }
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
        h.r1 = row(row0 + C, k, ld, n);
        h.r2 = row(row0 + C + 1, k, ld, n);
        rhs.template operator()<C, true>(v, h, 1, false, C, typename StencilRhs<K, CYC>::State{});
    }
    // the last chunk: rows row0 .. n-1 (row0 >= C); past row n-1 come rows
    // 0, 1 (periodic) or nothing
    template <int C>
    __device__ __forceinline__ void tail(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, false>(v, c, row0, k, ld, n);
        Halo h{};
        h.l1 = row(row0 - 1, k, ld, n);
        h.l2 = row(row0 - 2, k, ld, n);
        if constexpr (CYC) {
            h.e0 = c[k];
            h.e1 = c[ld + k];
        }
        rhs.template operator()<C, false>(v, h, 1, false, n - row0,
                                          typename StencilRhs<K, CYC>::State{});
    }
};

template <int K>
hipError_t launch_cn_long_k(bool cyclic, const double *table, const CyclicQ &q, const LongGeom &g,
                            const double *w, const double *in, double *out, hipStream_t s)
{
    if (cyclic) {
        StencilLongSrc<K, true> src{{}, in};
        for (int d = 0; d <= 2 * K; ++d) src.rhs.w[d] = w[d];
        return launch_long_k<K, true>(table, q, g, src, out, s);
    }
    StencilLongSrc<K, false> src{{}, in};
    for (int d = 0; d <= 2 * K; ++d) src.rhs.w[d] = w[d];
    return launch_long_k<K, false>(table, q, g, src, out, s);
}

template <int K>
hipError_t launch_cn_k(bool cyclic, const double *table, int64_t table_elems, const CyclicQ &q,
                       const SweepGeom &g, bool scalar, const double *w, int64_t steps,
                       int64_t traj_stride, const double *in, double *out, hipStream_t s)
{
    return cyclic ? launch_cn_kc<K, true>(table, table_elems, q, g, scalar, w, steps, traj_stride, in, out, s)
                  : launch_cn_kc<K, false>(table, table_elems, q, g, scalar, w, steps, traj_stride, in, out, s);
}

}  // namespace
}  // namespace bb
