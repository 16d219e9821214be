// stepper.h -- fused implicit time steps with the state kept on chip: every
// step builds the right-hand side of a system from its current state (an
// explicit stencil, possibly nonlinear) and solves the shared banded LHS,
// `steps` times per launch, reading the batch once and writing it once.
// The right-hand-side rule is a policy (Rhs); ch.hip (Cahn-Hilliard, Section
// 5.1) and cn.hip (Crank-Nicolson diffusion and hyperdiffusion, Sections 3
// and 4 benchmark problems) instantiate it.
//
// An Rhs policy provides
//   static constexpr int R;   // rows of halo it reads on each side (1, 2 or 3)
//   struct State;             // per-lane data of the system it works on
//   State lane_state(int64_t k, int row0) const;   // system k, chunk from row0
//   template <int C, bool FULL>
//   void operator()(double (&c)[C], const Halo &h, int j, bool last_chunk, int nrow,
//                   const State &s) const;
// which overwrites the chunk c (rows j*C .. j*C + C - 1 of the system) with
// the right-hand side.  nrow = n - j*C (rows of the chunk that are real when
// the decomposition is ragged); last_chunk: j == P - 1.
#pragma once

#include <type_traits>

#include "sweep_core.h"

namespace bb {
namespace {

// Values around a chunk: the R rows above it (l1 = row j*C - 1, l2, l3;
// 0 for the first chunk) and below it (r1 = row j*C + C, r2, r3; 0 past the
// last chunk), and rows 0, 1, 2, n-3, n-2, n-1 of the system (for periodic
// wrap-around).  Entries a smaller R does not read stay 0.
struct Halo {
    double l1, l2, l3, r1, r2, r3;
    double e0, e1, e2, en3, en2, en1;
};

// Optional per-run statistic of the fused steps (Cahn-Hilliard coarsening,
// Section 5, batched 1D scaling), compiled in only where asked for (STATS):
// after every `every` steps, each system's typical domain size
// 1 / (1 - <c^2>), <c^2> = (1/n) sum_i c_i^2, summed over the systems of its
// group in a fixed order and stored at [group][sample] of `partial` (each
// entry written once; no read-modify-write inside the step loop).
struct StepStats {
    double *partial = nullptr;
    int64_t every = 1, samples = 0;
    double inv_n = 0.0;
    int64_t traj_stride = 0;   // TRAJ: elements between the states of consecutive steps in `out`
};

// sum of squares of this lane's rows (padding rows hold 0): four interleaved
// partial sums (rows t mod 4) keep the dependency chain short, combined in a
// fixed order
template <int C>
__device__ __forceinline__ double chunk_sum_sq(const double (&c)[C])
{
    double ss[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < C; ++t) ss[t & 3] = fma(c[t], c[t], ss[t & 3]);
    return (ss[0] + ss[1]) + (ss[2] + ss[3]);
}

// Sum of v over the S lanes of each block of S consecutive lanes (S a power
// of two), a fixed butterfly: every lane of the block gets the same sum.
__device__ __forceinline__ double block_sum(double v, int S)
{
    for (int off = 1; off < S; off <<= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One lane per chunk; the lanes of a system sit in one wave (shuffles) and
// the coefficient table is staged in LDS.
// TRAJ: the state after every step s (0-based) is stored at
// out + s * st.traj_stride instead of only the last one at out.
template <class Rhs, int K, bool CYC, int C, bool FULL, bool STATS, bool TRAJ>
__global__ __launch_bounds__(kMaxBlockThreads) void step_kernel(const double *__restrict__ table,
                                                             int64_t table_elems, CyclicQ cq,
                                                             SweepGeom g, Rhs rhs, int64_t steps,
                                                             StepStats st, const double *in,
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
    const GroupRange gr = group_range(g.groups, 0, STATS ? 0 : g.linear);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        double c[C];
        load_chunk<double, C, FULL>(c, in, row0, kval ? k : g.m - 1, g.ld, g.n);
        const typename Rhs::State ls = rhs.lane_state(kval ? k : g.m - 1, row0);

        for (int64_t step = 0; step < steps; ++step) {
            Halo h = {};
            h.l1 = shfl(c[C - 1], left);
            h.r1 = shfl(c[0], right);
            if (!has_left) h.l1 = 0.0;
            if (!has_right) h.r1 = 0.0;
            if constexpr (Rhs::R >= 2) {
                h.l2 = shfl(c[C - 2], left);
                h.r2 = shfl(c[1], right);
                if (!has_left) h.l2 = 0.0;
                if (!has_right) h.r2 = 0.0;
            }
            if constexpr (Rhs::R >= 3) {
                h.l3 = shfl(c[C - 3], left);
                h.r3 = shfl(c[2], right);
                if (!has_left) h.l3 = 0.0;
                if (!has_right) h.r3 = 0.0;
            }
            gather_ends<double, 2, C>(c, lg, g.n, exact, h.e0, h.e1, h.en2, h.en1);
            if constexpr (Rhs::R >= 3) {
                h.e2 = shfl(c[2], lg.sl);
                h.en3 = exact ? shfl(c[C - 3], (g.n / C - 1) * lg.S + lg.sl)
                              : shfl(pick(c, (g.n - 3) % C), ((g.n - 3) / C) * lg.S + lg.sl);
            }
            rhs.template operator()<C, FULL>(c, h, lg.j, lg.j == lg.P - 1, opaque_v(g.n - row0), ls);
            __builtin_amdgcn_sched_barrier(0);
            chunk_solve<double, K, C, CYC>(c, smem_d, lg, g.n, exact, cq);
            if (STATS && (step + 1) % st.every == 0) {
                // chunks of a system: lanes j*S + sl of this wave, summed in chunk order
                const double ss = chunk_sum_sq<C>(c);
                double tot = 0.0;
                for (int i = 0; i < lg.P; ++i) tot += shfl(ss, i * lg.S + lg.sl);
                // l - 1 = <C^2> / (1 - <C^2>): summed without the 1 of every run,
                // so the ensemble sum keeps the digits that l - 1 carries
                const double msq = tot * st.inv_n;
                const double ell = kval ? msq / (1.0 - msq) : 0.0;
                const double sum = block_sum(ell, lg.S);   // the group: lanes 0 .. S-1
                if (lane == 0) st.partial[grp * st.samples + (step + 1) / st.every - 1] = sum;
            }
            if constexpr (TRAJ) {
                if (kval) store_chunk<double, C, FULL>(c, out + step * st.traj_stride, row0, k, g.ld, g.n);
            }
        }
        if constexpr (!TRAJ) {
            if (kval) store_chunk<double, C, FULL>(c, out, row0, k, g.ld, g.n);
        }
    }
}

// The same steps with a system group split over the Q = 2^QL waves of a
// workgroup (chunks tile n exactly): wave q holds chunks q*P/Q ..
// (q+1)*P/Q - 1 of S = 64Q/P systems, and every chunk-boundary value goes
// through the LDS exchange area: the first and last R rows of every chunk
// for the stencil and the wrap-around, then the phases of chunk_solve.
// SCALAR (one chunk per wave, P == Q): every lane of a wave needs the same
// coefficient row at the same time, so the coefficients come from the global
// table through the scalar cache (no LDS staging, no LDS reads).  Otherwise
// the table is staged in LDS ahead of the exchange area.
template <class Rhs, int K, bool CYC, int C, int QL, bool SCALAR, bool STATS, bool TRAJ>
__global__ __launch_bounds__((kWave << QL) > kMaxBlockThreads ? (kWave << QL) : kMaxBlockThreads)
void step_kernel_split(const double *__restrict__ table, int64_t table_elems, CyclicQ cq,
                       SweepGeom g, Rhs rhs, int64_t steps, StepStats st, const double *in,
                       double *out)
{
    using Src = typename std::conditional<SCALAR, FromScalar<double>, FromLds<double>>::type;
    constexpr int R = Rhs::R;
    extern __shared__ double smem_d[];
    const int64_t tl = SCALAR ? 0 : table_elems;
    double *xch = smem_d + tl;                              // chunk_solve phases
    double *xd = xch + split_exchange_len(QL);              // [2R][P*S]: rows 0, C-1, 1, C-2, 2, C-3
    double *xs = xd + ((2LL * R * kWave) << QL);            // [P*S]: sums of squares
    typename Src::ptr tab;
    if constexpr (SCALAR) {
        tab = (typename Src::ptr)table;
    } else {
        stage_table(smem_d, table, table_elems);
        __syncthreads();
        tab = smem_d;
    }

    // SCALAR: P == Q (the host checks log2P == QL), so the geometry is known
    // at compile time: S = 64, one chunk per wave
    LaneGeom lg = lane_geom(SCALAR ? QL : g.log2P, QL);
    if constexpr (SCALAR) lg.j = __builtin_amdgcn_readfirstlane(lg.j);   // the wave's chunk
    const int row0 = lg.j * C;
    const bool has_left = lg.j > 0, has_right = lg.j < lg.P - 1;
    const int PS = lg.P * lg.S;
    const int me = lg.j * lg.S + lg.sl;
    const int lft = (has_left ? lg.j - 1 : lg.j) * lg.S + lg.sl;
    const int rgt = (has_right ? lg.j + 1 : lg.j) * lg.S + lg.sl;
    const int first = lg.sl, last = (lg.P - 1) * lg.S + lg.sl;
    // STATS launches are persistent unless forced (the mapping code costs the
    // statistic kernel its third wave per SIMD); the persistent mapping also
    // serves a forced one-per-group grid
    const GroupRange gr = group_range(g.groups, QL, STATS ? 0 : g.linear);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        double c[C];
        load_chunk<double, C, true>(c, in, row0, kval ? k : g.m - 1, g.ld, g.n);
        const typename Rhs::State ls = rhs.lane_state(kval ? k : g.m - 1, row0);

        for (int64_t step = 0; step < steps; ++step) {
            xd[me] = c[0];
            xd[PS + me] = c[C - 1];
            if constexpr (R >= 2) {
                xd[2 * PS + me] = c[1];
                xd[3 * PS + me] = c[C - 2];
            }
            if constexpr (R >= 3) {
                xd[4 * PS + me] = c[2];
                xd[5 * PS + me] = c[C - 3];
            }
            __syncthreads();
            Halo h = {};
            h.l1 = has_left ? xd[PS + lft] : 0.0;
            h.r1 = has_right ? xd[rgt] : 0.0;
            h.e0 = xd[first];
            h.en1 = xd[PS + last];
            if constexpr (R >= 2) {
                h.l2 = has_left ? xd[3 * PS + lft] : 0.0;
                h.r2 = has_right ? xd[2 * PS + rgt] : 0.0;
                h.e1 = xd[2 * PS + first];
                h.en2 = xd[3 * PS + last];
            }
            if constexpr (R >= 3) {
                h.l3 = has_left ? xd[5 * PS + lft] : 0.0;
                h.r3 = has_right ? xd[4 * PS + rgt] : 0.0;
                h.e2 = xd[4 * PS + first];
                h.en3 = xd[5 * PS + last];
            }
            rhs.template operator()<C, true>(c, h, lg.j, !has_right, C, ls);
            __builtin_amdgcn_sched_barrier(0);
            chunk_solve<double, K, C, CYC, true, Src>(c, tab, lg, g.n, 1, cq, xch);
            if (STATS && (step + 1) % st.every == 0) {
                // chunks of a system through LDS, summed in chunk order, by
                // wave 0 (it holds chunk 0: lanes 0 .. S-1 are the group)
                xs[me] = chunk_sum_sq<C>(c);
                __syncthreads();
                if (threadIdx.x < kWave) {
                    double tot = 0.0;
                    for (int i = 0; i < lg.P; ++i) tot += xs[i * lg.S + lg.sl];
                    const double msq = tot * st.inv_n;   // l - 1, as above
                    const double ell = kval ? msq / (1.0 - msq) : 0.0;
                    const double sum = block_sum(ell, lg.S);
                    if (threadIdx.x == 0)
                        st.partial[grp * st.samples + (step + 1) / st.every - 1] = sum;
                }
            }
            if constexpr (TRAJ) {
                if (kval) store_chunk<double, C, true>(c, out + step * st.traj_stride, row0, k, g.ld, g.n);
            }
        }
        if constexpr (!TRAJ) {
            if (kval) store_chunk<double, C, true>(c, out, row0, k, g.ld, g.n);
        }
    }
}

// LDS bytes of the split kernel beyond the staged table: the chunk_solve
// exchange, 2R rows per (chunk, slot) and one sum of squares per (chunk, slot).
constexpr size_t split_step_lds(int QL, int R)
{
    return (size_t)(split_exchange_len(QL) + ((2LL * R * kWave) << QL) + (kWave << QL)) * sizeof(double);
}

// Launch `steps` fused steps.  g.log2Q > 0 selects the split kernel (full
// decomposition, log2Q <= 3), with the coefficients through the scalar cache
// when `scalar` (then log2Q == log2P and C is 16, 32 or 64); `scalar` with
// g.log2Q == g.log2P == 0 runs one-chunk systems the same way.  Otherwise the
// LDS kernel with one wave per group.  The scalar kernel's grid follows
// g.linear (it stages no table, so one workgroup per group costs nothing);
// the LDS kernels stage the table once per workgroup and stay persistent
// unless tuning grid_linear asks otherwise.  TRAJ: every step's state, see
// step_kernel.
template <class Rhs, int K, bool CYC, bool STATS = false, bool TRAJ = false>
hipError_t launch_stepper(const double *table, int64_t table_elems, const CyclicQ &q,
                          const SweepGeom &g, bool scalar, const Rhs &rhs, int64_t steps,
                          const double *in, double *out, hipStream_t s,
                          StepStats st = StepStats{})
{
    if (scalar) {
        // one chunk per wave: 16-, 32- or 64-row chunks tiling n into at most 8
        if ((g.C != 16 && g.C != 32 && g.C != 64) || g.log2Q != g.log2P || g.log2Q > 3 || !is_full(g))
            return hipErrorInvalidValue;
        const size_t xl = split_step_lds(g.log2Q, Rhs::R);
#define BB_SCALAR(CC)                                                                                    \
        case CC:                                                                                         \
            switch (g.log2Q) {                                                                           \
            case 0: return launch_grid_mode(step_kernel_split<Rhs, K, CYC, CC, 0, true, STATS, TRAJ>, xl, g.groups, 1, g.linear, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            case 1: return launch_grid_mode(step_kernel_split<Rhs, K, CYC, CC, 1, true, STATS, TRAJ>, xl, g.groups, 2, g.linear, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            case 2: return launch_grid_mode(step_kernel_split<Rhs, K, CYC, CC, 2, true, STATS, TRAJ>, xl, g.groups, 4, g.linear, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            default: return launch_grid_mode(step_kernel_split<Rhs, K, CYC, CC, 3, true, STATS, TRAJ>, xl, g.groups, 8, g.linear, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            }
        switch (g.C) {
            BB_SCALAR(16)
            BB_SCALAR(32)
            BB_SCALAR(64)
        default: return hipErrorInvalidValue;
        }
#undef BB_SCALAR
    }
    if (g.log2Q > 0) {
        // LDS table, group split over 2^log2Q waves: 32- and 64-row chunks
        if (g.log2Q > 3 || g.log2Q > g.log2P || !is_full(g)) return hipErrorInvalidValue;
        const size_t xl = (size_t)table_elems * sizeof(double) + split_step_lds(g.log2Q, Rhs::R);
#define BB_SPLIT(CC)                                                                                     \
        case CC:                                                                                         \
            switch (g.log2Q) {                                                                           \
            case 1: return launch_grid_split(step_kernel_split<Rhs, K, CYC, CC, 1, false, STATS, TRAJ>, xl, g.groups, 2, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            case 2: return launch_grid_split(step_kernel_split<Rhs, K, CYC, CC, 2, false, STATS, TRAJ>, xl, g.groups, 4, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            default: return launch_grid_split(step_kernel_split<Rhs, K, CYC, CC, 3, false, STATS, TRAJ>, xl, g.groups, 8, s, table, table_elems, q, g, rhs, steps, st, in, out); \
            }
        switch (g.C) {
            BB_SPLIT(32)
            BB_SPLIT(64)
        default: return hipErrorInvalidValue;
        }
#undef BB_SPLIT
    }
    const size_t lds = (size_t)table_elems * sizeof(double);
#define BB_STEP(CC)                                                                            \
    case CC:                                                                                   \
        return is_full(g) ? launch_grid(step_kernel<Rhs, K, CYC, CC, true, STATS, TRAJ>, lds, g.groups, s,   \
                                        table, table_elems, q, g, rhs, steps, st, in, out)      \
                          : launch_grid(step_kernel<Rhs, K, CYC, CC, false, STATS, TRAJ>, lds, g.groups, s,  \
                                        table, table_elems, q, g, rhs, steps, st, in, out);
    switch (g.C) {
        BB_STEP(4)
        BB_STEP(8)
        BB_STEP(16)
        BB_STEP(32)
        BB_STEP(64)
    default: return hipErrorInvalidValue;
    }
#undef BB_STEP
}

}  // namespace
}  // namespace bb
