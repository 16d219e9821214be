// refine_kernel.h -- FP32 sweeps with one FP64-residual refinement in a
// single kernel, for double or FP32 right-hand sides (the kernel and its
// dispatch templates; instantiated in refine.hip and refine_f32rhs.hip so
// the two compile in parallel).  Building blocks in sweep_core.h.
#pragma once

#include "sweep_core.h"

namespace bb {
namespace {

// ---------------------------------------------------------------- refine
// x0 = solve_f32(b); r = b - A x0 in double with the original bands;
// x = x0 + solve_f32(r), stored as double.
// QL > 0: split groups as in sweep_kernel; the exchange area holds the three
// phases of chunk_solve followed by rows 0, 1, C-2, C-1 of every chunk.
// TB: type of the right-hand sides in memory -- double, or float when the
// right-hand sides are FP32 data (promoted exactly for the residual).
template <int K, int C, bool CYC, bool FULL, int QL, typename TB>
__global__ __launch_bounds__((kWave << QL) > kMaxBlockThreads ? (kWave << QL) : kMaxBlockThreads)
void refine_kernel(
    const float *__restrict__ table, int64_t table_elems, const double *__restrict__ band_table,
    int64_t band_elems, CyclicQ cq, Corners cn, SweepGeom g, const TB *in, double *out)
{
    static_assert(QL == 0 || (FULL && C >= 2), "split groups are full decompositions");
    extern __shared__ double smem_d[];
    double *lds_band = smem_d;
    float *lds = reinterpret_cast<float *>(smem_d + band_elems);
    stage_table(lds_band, band_table, band_elems);
    stage_table(lds, table, table_elems);
    __syncthreads();
    float *xch = lds + table_elems;

    const LaneGeom lg = lane_geom(g.log2P, QL);
    const int lane = threadIdx.x % kWave;
    const int L = lg.P * (C + 1);
    const int row0 = lg.j * C;
    const bool has_left = lg.j > 0, has_right = lg.j < lg.P - 1;
    const int left = has_left ? lane - lg.S : lane;
    const int right = has_right ? lane + lg.S : lane;
    const int exact = FULL || g.exact;
    const GroupRange gr = group_range(g.groups, QL, g.linear);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        TB b[C];
        load_chunk<TB, C, FULL>(b, in, row0, kval ? k : g.m - 1, g.ld, g.n);
        float x0[C];
#pragma unroll
        for (int t = 0; t < C; ++t) x0[t] = (float)b[t];
        chunk_solve<float, K, C, CYC, (QL > 0)>(x0, lds, lg, g.n, exact, cq, xch);
        __builtin_amdgcn_sched_barrier(0);

        // neighbours across the chunk boundaries (zero outside the matrix) and,
        // periodic, rows 0, 1, n-2, n-1 of the system
        float xl1, xl2, xr1, xr2, r0 = 0.f, r1 = 0.f, rn2 = 0.f, rn1 = 0.f;
        if constexpr (QL > 0) {
            const int PS = lg.P * lg.S;
            float *xd = xch + 8 * PS;   // [4][P*S]: rows 0, 1, C-2, C-1 of (chunk, slot)
            const int me = lg.j * lg.S + lg.sl;
            xd[me] = x0[0];
            xd[PS + me] = x0[1];
            xd[2 * PS + me] = x0[C - 2];
            xd[3 * PS + me] = x0[C - 1];
            __syncthreads();
            const int lft = (has_left ? lg.j - 1 : lg.j) * lg.S + lg.sl;
            const int rgt = (has_right ? lg.j + 1 : lg.j) * lg.S + lg.sl;
            xl1 = has_left ? xd[3 * PS + lft] : 0.f;
            xl2 = has_left ? xd[2 * PS + lft] : 0.f;
            xr1 = has_right ? xd[rgt] : 0.f;
            xr2 = has_right ? xd[PS + rgt] : 0.f;
            if constexpr (CYC) {
                const int first = lg.sl, last = (lg.P - 1) * lg.S + lg.sl;
                r0 = xd[first];
                r1 = xd[PS + first];
                rn2 = xd[2 * PS + last];
                rn1 = xd[3 * PS + last];
            }
        } else {
            xl1 = shfl(x0[C - 1], left);
            xl2 = shfl(x0[C - 2], left);
            xr1 = shfl(x0[0], right);
            xr2 = shfl(x0[1], right);
            if (!has_left) xl1 = xl2 = 0.f;
            if (!has_right) xr1 = xr2 = 0.f;
            if constexpr (CYC) gather_ends<float, K, C>(x0, lg, g.n, exact, r0, r1, rn2, rn1);
        }
        double ctop0 = 0.0, ctop1 = 0.0, cbot2 = 0.0, cbot1 = 0.0;
        if constexpr (CYC) {
            if constexpr (K == 1) {
                ctop0 = cn.top[0][1] * (double)rn1;
                cbot1 = cn.bot[1][0] * (double)r0;
            } else {
                ctop0 = fma(cn.top[0][1], (double)rn1, cn.top[0][0] * (double)rn2);
                ctop1 = fma(cn.top[1][1], (double)rn1, cn.top[1][0] * (double)rn2);
                cbot2 = fma(cn.bot[0][1], (double)r1, cn.bot[0][0] * (double)r0);
                cbot1 = fma(cn.bot[1][1], (double)r1, cn.bot[1][0] * (double)r0);
            }
        }
        const int nrow = opaque_v(g.n - row0);   // this chunk's row index of row n (may be <= 0 or > C)
        const double *band[5];
        {
            const int off = opaque_v(lg.j * (C + 1));
#pragma unroll
            for (int q = 0; q < 2 * K + 1; ++q) band[q] = lds_band + q * L + off;
        }
        float dx[C];
        rows_up<C>([&](int t) {
            const double xm1 = t >= 1 ? (double)x0[t - 1] : (double)xl1;
            const double xp1 = t + 1 < C ? (double)x0[t + 1] : (double)xr1;
            double ax = band[K][t] * (double)x0[t];
            ax = fma(band[K - 1][t], xm1, ax);
            ax = fma(band[K + 1][t], xp1, ax);
            if constexpr (K == 2) {
                const double xm2 = t >= 2 ? (double)x0[t - 2] : (t == 1 ? (double)xl1 : (double)xl2);
                const double xp2 = t + 2 < C ? (double)x0[t + 2]
                                             : (t + 1 < C ? (double)xr1 : (double)xr2);
                ax = fma(band[0][t], xm2, ax);
                ax = fma(band[4][t], xp2, ax);
            }
            double r = (double)b[t] - ax;
            if constexpr (CYC) {
                // corner terms of the periodic matrix: rows 0, 1 (chunk 0) and n-2, n-1
                if (t == 0) r -= (lg.j == 0) ? ctop0 : 0.0;
                if constexpr (K == 2) {
                    if (t == 1) r -= (lg.j == 0) ? ctop1 : 0.0;
                    r -= (t == nrow - 2) ? cbot2 : 0.0;
                }
                r -= (t == nrow - 1) ? cbot1 : 0.0;
            }
            if constexpr (!FULL) r = t < nrow ? r : 0.0;
            dx[t] = (float)r;
        });
        __builtin_amdgcn_sched_barrier(0);
        chunk_solve<float, K, C, CYC, (QL > 0)>(dx, lds, lg, g.n, exact, cq, xch);
        if (kval)
            store_chunk_fn<C, FULL>([&](int t) { return (double)x0[t] + (double)dx[t]; }, out, row0,
                                    k, g.ld, g.n);
    }
}

template <int K, bool CYC, int C, typename TB>
hipError_t refine_c(const void *table, int64_t table_elems, const double *band,
                    int64_t band_elems, const CyclicQ &q, const Corners &cn, const SweepGeom &g,
                    const void *in, void *out, hipStream_t stream)
{
    const size_t lds = (size_t)band_elems * sizeof(double) + (size_t)table_elems * sizeof(float);
    if (g.log2Q > 0) {
        if constexpr (C >= 32) {
            if (!is_full(g) || g.log2Q > max_log2q(C, true) || g.log2Q > g.log2P)
                return hipErrorInvalidValue;
            const size_t xl = (size_t)(split_exchange_len(g.log2Q) + (4LL * kWave << g.log2Q)) * sizeof(float);
            if (g.log2Q == 1)
                return launch_grid_split(refine_kernel<K, C, CYC, true, 1, TB>, lds + xl, g.groups, 2,
                                         stream, (const float *)table, table_elems, band,
                                         band_elems, q, cn, g, (const TB *)in, (double *)out);
            if (g.log2Q == 2)
                return launch_grid_split(refine_kernel<K, C, CYC, true, 2, TB>, lds + xl, g.groups, 4,
                                         stream, (const float *)table, table_elems, band,
                                         band_elems, q, cn, g, (const TB *)in, (double *)out);
            if constexpr (C <= 32)
                return launch_grid_split(refine_kernel<K, C, CYC, true, 3, TB>, lds + xl, g.groups, 8,
                                         stream, (const float *)table, table_elems, band,
                                         band_elems, q, cn, g, (const TB *)in, (double *)out);
        }
        return hipErrorInvalidValue;
    }
    if (is_full(g))
        return launch_grid(refine_kernel<K, C, CYC, true, 0, TB>, lds, g.groups, stream,
                           (const float *)table, table_elems, band, band_elems, q, cn, g,
                           (const TB *)in, (double *)out);
    return launch_grid(refine_kernel<K, C, CYC, false, 0, TB>, lds, g.groups, stream,
                       (const float *)table, table_elems, band, band_elems, q, cn, g,
                       (const TB *)in, (double *)out);
}

template <int K, bool CYC, typename TB>
hipError_t refine_dispatch(const void *table, int64_t te, const double *band, int64_t be,
                           const CyclicQ &q, const Corners &cn, const SweepGeom &g,
                           const void *in, void *out, hipStream_t s)
{
    switch (g.C) {
    case 4: return refine_c<K, CYC, 4, TB>(table, te, band, be, q, cn, g, in, out, s);
    case 8: return refine_c<K, CYC, 8, TB>(table, te, band, be, q, cn, g, in, out, s);
    case 16: return refine_c<K, CYC, 16, TB>(table, te, band, be, q, cn, g, in, out, s);
    case 32: return refine_c<K, CYC, 32, TB>(table, te, band, be, q, cn, g, in, out, s);
    case 64: return refine_c<K, CYC, 64, TB>(table, te, band, be, q, cn, g, in, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace bb
