// adjoint_grad_kernel.h -- the adjoint recursion of a differentiated rollout
// fused with its band gradients (instantiated in adjoint_grad_tri.hip and
// adjoint_grad_penta.hip so the two compile in parallel).
//
// For the rollout u_t = A^{-1} u_{t-1} the adjoints are lam_t = A^{-T}
// lam_{t+1} and the gradient of the shared bands is
//   dL/dA[i][i+q-K] = -sum_t sum_k lam_t[i,k] u_t[i+q-K,k]
// (the adjoint of a batched solve, reduced over the batch and the steps).
// One launch steps the adjoints of a segment of the rollout with each chunk
// held in registers -- the fused stepper's decomposition and transposed-solve
// table, so every adjoint equals the adjoint trajectory's bitwise -- and after
// each step reduces the adjoint against the stored forward state of that
// step over the S systems of the chunk.  HBM sees one read of each forward
// state in place of a write of every adjoint and two reads by a separate
// band-gradient pass.
//
// The reduction of one step, in blocks of RB rows of the chunk: each lane
// forms its V = RB (2K+1) products; NH halving rounds across the top slot
// bits (lanes sl and sl ^ S/2, then sl ^ S/4, add their values, each lane
// keeping one half) leave each lane V / 2^NH values summed over 2^NH
// systems; the lanes stage them in the wave's LDS area, and one lane per
// (chunk, row, band) entry adds the S / 2^NH staged values in slot order to
// its sum over the steps.  At the end of a system group its sums are stored
// at part[group][band][row]; a fold adds the groups in a fixed order.  Every
// sum has a fixed order, so the gradients repeat bitwise.
#pragma once

#include <type_traits>

#include "sweep_core.h"

namespace bb {
namespace {

// Rows per reduction block: the entries of a block (W chunks per wave x RB
// rows x 2K+1 bands) fit the 64 lanes that sum them.
template <int K, int SL>
constexpr int grad_rows()
{
    constexpr int cap = K == 1 ? 8 : 4;
    constexpr int fit = (K == 1 ? 16 : 8) * (1 << SL) / kWave;
    return fit < cap ? fit : cap;
}

// Halving rounds in registers: two where both have a lane-swap instruction
// (64 systems per chunk) or the LDS area must stay small (pentadiagonal).
template <int K, int SL>
constexpr int grad_halvings()
{
    return (SL == 6 || K == 2) ? 2 : 1;
}

// Double halves, for the 32-bit cross-lane operations.
__device__ __forceinline__ double join_d(unsigned lo, unsigned hi)
{
    return __hiloint2double((int)hi, (int)lo);
}

// One halving round across lane bit X (a wave-uniform power of two, X < 64):
// a lane with that bit clear keeps values [0, N/2), the other half [N/2, N),
// each adding its partner's copy.  X = 32 and 16 use the swap instructions
// (v_permlane32_swap swaps the upper 32 lanes of its first operand with the
// lower 32 of its second; v_permlane16_swap the odd 16-lane rows of the first
// with the even rows of the second), which hand every lane its own value and
// its partner's in one step; other X a shuffle and two selects per value.
template <int N, int X>
__device__ __forceinline__ void halve(const double (&v)[N], double (&out)[N / 2], int lane)
{
    constexpr int H = N / 2;
    if constexpr (X == 32 || X == 16) {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const unsigned alo = (unsigned)__double2loint(v[i]), ahi = (unsigned)__double2hiint(v[i]);
            const unsigned blo = (unsigned)__double2loint(v[i + H]), bhi = (unsigned)__double2hiint(v[i + H]);
            if constexpr (X == 32) {
                const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
                const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
                out[i] = join_d(lo[0], hi[0]) + join_d(lo[1], hi[1]);
            } else {
                const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
                const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
                out[i] = join_d(lo[0], hi[0]) + join_d(lo[1], hi[1]);
            }
        }
    } else {
        const bool top = (lane & X) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const double send = top ? v[i] : v[i + H];
            const double keep = top ? v[i + H] : v[i];
            out[i] = keep + __shfl_xor(send, X, kWave);
        }
    }
}

// Orders this wave's LDS staging writes before its reads by other lanes (and
// the reads before the next block's writes): a wave's LDS instructions run in
// program order, so a fence at wavefront scope is all that is needed.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Staging area per wave, in doubles: (S / 2^NH) rows of E + 1 (odd stride).
template <int K, int SL>
constexpr int grad_stage_len()
{
    constexpr int S = 1 << SL, W = kWave / S;
    constexpr int E = W * grad_rows<K, SL>() * (2 * K + 1);
    return (S >> grad_halvings<K, SL>()) * (E + 1);
}

// QL: log2 of the waves per system group; SL: log2 of the systems per group
// (S = 64 Q / P); SCALAR: one chunk per wave with the coefficients through
// the scalar cache (then P == Q and S = 64), else the table staged in LDS.
template <int K, int C, int QL, bool CYC, bool SCALAR, int SL>
__global__ __launch_bounds__((kWave << QL) > kMaxBlockThreads ? (kWave << QL) : kMaxBlockThreads)
void adjoint_grad_kernel(const double *__restrict__ table, int64_t table_elems, CyclicQ cq,
                         SweepGeom g, int64_t steps, const double *lam_in,
                         const double *traj, int64_t traj_stride, double *lam_out,
                         double *__restrict__ part)
{
    using Src = typename std::conditional<SCALAR, FromScalar<double>, FromLds<double>>::type;
    constexpr int NB = 2 * K + 1;
    constexpr int S = 1 << SL, W = kWave / S;
    constexpr int RB = grad_rows<K, SL>(), NH = grad_halvings<K, SL>();
    constexpr int V = RB * NB;          // products per lane and block
    constexpr int HV = V >> NH;         // values per lane after the halvings
    constexpr int HS = S >> NH;         // staged partial sums per entry
    constexpr int E = W * V, EP = E + 1;
    constexpr int NBLK = C / RB;
    static_assert(SL >= 1 && SL <= 6 && C % RB == 0 && (HV << NH) == V && E <= kWave, "geometry");

    extern __shared__ double smem_d[];
    const int64_t tl = SCALAR ? 0 : table_elems;
    double *xch = smem_d + tl;
    double *stage = xch + split_exchange_len(QL) + (int64_t)(threadIdx.x / kWave) * grad_stage_len<K, SL>();
    typename Src::ptr tab;
    if constexpr (SCALAR) {
        tab = (typename Src::ptr)table;
    } else {
        stage_table(smem_d, table, table_elems);
        __syncthreads();
        tab = smem_d;
    }

    LaneGeom lg = lane_geom(SCALAR ? QL : g.log2P, QL);
    if constexpr (SCALAR) lg.j = __builtin_amdgcn_readfirstlane(lg.j);
    const int lane = threadIdx.x % kWave;
    const int n = g.n;
    const int row0 = lg.j * C;
    const int wl = lane >> SL;                      // this lane's chunk within the wave
    // where this lane's halved values go: slot bits below the halved ones,
    // and the offset of the kept part of the V products
    const int h = lg.sl & (HS - 1);
    int off = 0;
#pragma unroll
    for (int r = 1; r <= NH; ++r) off += ((lg.sl >> (SL - r)) & 1) * (V >> r);
    double *my_stage = stage + h * EP + wl * V + off;
    // the entry this lane sums (lanes below E): chunk, row in the block, band
    const int wl_e = lane / V, v_e = lane % V;
    const int j_e = lg.j - wl + wl_e, r_e = v_e / NB, q_e = v_e % NB;
    const GroupRange gr = group_range(g.groups, QL, g.linear);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        const int64_t kk = kval ? k : g.m - 1;
        double c[C];
        load_chunk<double, C, true>(c, lam_in, row0, kk, g.ld, n);
        double acc[NBLK];
#pragma unroll
        for (int b = 0; b < NBLK; ++b) acc[b] = 0.0;

        for (int64_t step = 0; step < steps; ++step) {
            // the forward state paired with this step's adjoint: rows row0 - K
            // .. row0 + C + K - 1 of system k (outside the matrix: 0, or mod
            // n when periodic; padding systems: 0).  The first block's rows
            // are loaded before the transposed solve, so they arrive during
            // it; each later block's rows are loaded while the block before
            // it is reduced (one block in flight ahead: measured 1.65 against
            // 1.74 ms for 10 steps at n = 1024, m = 2^16), their row index
            // passed through an opaque value so that the compiler cannot
            // hoist every row's load to the top of the step and hold them all
            // at once.
            const int64_t ld = opaque_s(g.ld);
            const double *ucol = traj + (steps - 1 - step) * traj_stride + kk;
            auto urow = [&](int t) -> double {   // row row0 + t, t in [-K, C + K)
                const int i = row0 + t + opaque_v(0);
                if (t >= 0 && t < C) {
                    const double x = ucol[(int64_t)i * ld];
                    return kval ? x : 0.0;
                }
                const bool out = i < 0 || i >= n;
                const int w = i < 0 ? i + n : (i >= n ? i - n : i);
                const double x = ucol[(int64_t)w * ld];
                return (kval && (CYC || !out)) ? x : 0.0;
            };
            double win[RB + 2 * K];
#pragma unroll
            for (int t = 0; t < RB + 2 * K; ++t) win[t] = urow(t - K);
            __builtin_amdgcn_sched_barrier(0);
            chunk_solve<double, K, C, CYC, true, Src>(c, tab, lg, n, 1, cq, xch);
            __builtin_amdgcn_sched_barrier(0);
            double nxt[RB];
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                if (b > 0) {
#pragma unroll
                    for (int t = 0; t < 2 * K; ++t) win[t] = win[t + RB];
#pragma unroll
                    for (int t = 2 * K; t < RB + 2 * K; ++t) win[t] = nxt[t - 2 * K];
                }
                if (b + 1 < NBLK) {
#pragma unroll
                    for (int t = 0; t < RB; ++t) nxt[t] = urow((b + 1) * RB + K + t);
                }
                double p[V];
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int q = 0; q < NB; ++q) p[r * NB + q] = c[b * RB + r] * win[r + q];
                double p1[V / 2];
                halve<V, S / 2>(p, p1, lane);
                double hv[HV];
                if constexpr (NH == 2) {
                    halve<V / 2, S / 4>(p1, hv, lane);
                } else {
#pragma unroll
                    for (int i = 0; i < HV; ++i) hv[i] = p1[i];
                }
#pragma unroll
                for (int i = 0; i < HV; ++i) my_stage[i] = hv[i];
                wave_lds_sync();
                if (lane < E) {
                    double sum = 0.0;
#pragma unroll
                    for (int s = 0; s < HS; ++s) sum += stage[s * EP + lane];
                    acc[b] += sum;
                }
                wave_lds_sync();
            }
        }
        if (kval) store_chunk<double, C, true>(c, lam_out, row0, k, g.ld, n);
        if (lane < E) {
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                const int i = j_e * C + b * RB + r_e;
                const int col = i + q_e - K;
                const bool inside = CYC || (col >= 0 && col < n);
                part[(grp * NB + q_e) * (int64_t)n + i] = inside ? -acc[b] : 0.0;
            }
        }
    }
}

// The kernels this file builds: the LDS-table split kernel for 32- and 64-row
// chunks in groups of 4 or 8 waves (S = 16 tri only, or 32), and the scalar
// kernel for 32- and 64-row chunks (S = 64).
template <int K>
constexpr bool grad_lds_slots_ok(int SL)
{
    return SL == 5 || (K == 1 && SL == 4);
}

template <int K, bool CYC, int C, int QL, bool SCALAR, int SL>
hipError_t adjoint_grad_go(const double *table, int64_t table_elems, const CyclicQ &q,
                           const SweepGeom &g, int64_t steps, const double *lam_in,
                           const double *traj, int64_t traj_stride, double *lam_out, double *part,
                           size_t lds, hipStream_t s)
{
    auto kern = adjoint_grad_kernel<K, C, QL, CYC, SCALAR, SL>;
    if (SCALAR)
        return launch_grid_mode(kern, lds, g.groups, 1 << QL, g.linear, s, table, table_elems, q, g,
                                steps, lam_in, traj, traj_stride, lam_out, part);
    // one workgroup per group in launch order (no persistent loop): in a
    // rollout's backward the recomputation of the next segment runs beside
    // this launch, and workgroups that end free their CU for it (rollout step
    // n = 1024, m = 2^16: 38.9 against 39.6 ms persistent); the table staged
    // per workgroup costs 42 KB of L2 reads per group of 32 systems
    SweepGeom gl = g;
    gl.linear = 1;
    return launch_grid_mode(kern, lds, g.groups, 1 << QL, true, s, table, table_elems, q, gl, steps,
                            lam_in, traj, traj_stride, lam_out, part);
}

template <int K, bool CYC>
hipError_t adjoint_grad_dispatch(const double *table, int64_t table_elems, const CyclicQ &q,
                                 const SweepGeom &g, bool scalar, int64_t steps,
                                 const double *lam_in, const double *traj, int64_t traj_stride,
                                 double *lam_out, double *part, size_t lds, hipStream_t s)
{
#define BB_AG(C, QL, SC, SL)                                                                       \
    return adjoint_grad_go<K, CYC, C, QL, SC, SL>(table, table_elems, q, g, steps, lam_in, traj, \
                                                  traj_stride, lam_out, part, lds, s)
    if (scalar) {
        if (g.log2P != g.log2Q) return hipErrorInvalidValue;
        if (g.C == 64) {
            switch (g.log2Q) {
            case 0: BB_AG(64, 0, true, 6);
            case 1: BB_AG(64, 1, true, 6);
            case 2: BB_AG(64, 2, true, 6);
            case 3: BB_AG(64, 3, true, 6);
            default: return hipErrorInvalidValue;
            }
        }
        if (g.C == 32) {
            switch (g.log2Q) {
            case 0: BB_AG(32, 0, true, 6);
            case 1: BB_AG(32, 1, true, 6);
            case 2: BB_AG(32, 2, true, 6);
            case 3: BB_AG(32, 3, true, 6);
            default: return hipErrorInvalidValue;
            }
        }
        return hipErrorInvalidValue;
    }
    const int sl = 6 - (g.log2P - g.log2Q);
    if (g.C == 64) {
        if (g.log2Q == 2 && sl == 5) BB_AG(64, 2, false, 5);
        if (g.log2Q == 3 && sl == 5) BB_AG(64, 3, false, 5);
        if constexpr (K == 1) {
            if (g.log2Q == 2 && sl == 4) BB_AG(64, 2, false, 4);
            if (g.log2Q == 3 && sl == 4) BB_AG(64, 3, false, 4);
        }
    }
    if (g.C == 32) {
        if (g.log2Q == 2 && sl == 5) BB_AG(32, 2, false, 5);
        if (g.log2Q == 3 && sl == 5) BB_AG(32, 3, false, 5);
        if constexpr (K == 1) {
            if (g.log2Q == 2 && sl == 4) BB_AG(32, 2, false, 4);
            if (g.log2Q == 3 && sl == 4) BB_AG(32, 3, false, 4);
        }
    }
    return hipErrorInvalidValue;
#undef BB_AG
}

}  // namespace
}  // namespace bb
