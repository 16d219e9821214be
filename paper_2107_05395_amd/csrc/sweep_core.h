// sweep_core.h -- device building blocks shared by the gfx950 kernels of
// libbandbatch (sweep.hip, refine.hip, ch.hip): the per-lane chunk solve of a
// banded LU with one shared LHS, the lane/workgroup geometry, coefficient
// table sources, chunk loads and stores, and the persistent-grid launcher.
//
// Forward elimination + back substitution of the Thomas algorithm (Section
// 3.1; Appendix A batched sweep) and of the pentadiagonal LR solve (Section
// 4.1; Appendix B), on right-hand sides interleaved with the batch index
// fastest (Section 2).  The decomposition of a system over P lanes, the
// coefficient table and its LDS layout are described in internal.h.
//
// Per lane: load the C rows of its chunk (one coalesced wave-wide load per
// row), run the two recurrences in registers with the chunk-boundary scans,
// apply the periodic correction if any, store once.  HBM traffic is one read
// of the right-hand side and one write of the solution; coefficients come
// from LDS (staged once per workgroup) or through the scalar cache.
#pragma once

#include "internal.h"

namespace bb {
namespace {

template <typename T>
__device__ __forceinline__ T shfl(T v, int src)
{
    return __shfl(v, src, kWave);
}

// Opaque copies of loop-invariant values.  The persistent loops below would
// otherwise let the compiler hoist every per-row LDS coefficient read and
// every per-row address offset out of the loop and keep them all live in
// registers; re-reading them each iteration is what the design wants.
__device__ __forceinline__ int opaque_v(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ int64_t opaque_s(int64_t x)
{
    asm volatile("" : "+s"(x));
    return x;
}

__device__ __forceinline__ int opaque_u(int x)   // wave-uniform (SGPR) copy
{
    asm volatile("" : "+s"(x));
    return x;
}

// Where a kernel reads its coefficient table: from LDS, staged once per
// workgroup (the lanes of a wave work on different chunks), or -- when every
// lane of a wave works on the same chunk -- straight from the global table
// through the scalar cache, the coefficient of each row arriving in SGPRs as
// an operand of the lanes' FMAs.  base() re-derives the pointer from a value
// the compiler cannot see through, so coefficient reads are not hoisted out
// of the persistent loop.
template <typename T>
struct FromLds {
    using ptr = const T *;
    __device__ static ptr base(ptr p) { return p + opaque_v(0); }
};

template <typename T>
struct FromScalar {
    typedef const T __attribute__((address_space(4))) elem;   // constant address space
    using ptr = elem *;
    __device__ static ptr base(ptr p) { return p + opaque_u(0); }
};

// A branch the compiler cannot fold (always taken, on a uniform value it
// cannot see).  Each pass runs in blocks of kFenceRows rows, each block inside
// such a branch: a separate basic block, so the coefficient reads of one block
// are not hoisted above the work of the previous one and only a few rows of
// coefficients are live at a time.
constexpr int kFenceRows = 8;
__device__ __forceinline__ bool opaque_true()
{
    int x = 1;
    asm volatile("" : "+s"(x));
    return x != 0;
}

// body(t) for t = 0 .. C-1 (rows_up) or C-1 .. 0 (rows_down), fully
// unrolled, in fenced blocks of kFenceRows rows.
template <int C, typename F>
__device__ __forceinline__ void rows_up(F &&body)
{
    constexpr int B = C < kFenceRows ? C : kFenceRows;
#pragma unroll
    for (int t0 = 0; t0 < C; t0 += B) {
        if (opaque_true()) {
#pragma unroll
            for (int tt = 0; tt < B; ++tt) body(t0 + tt);
        }
    }
}

template <int C, typename F>
__device__ __forceinline__ void rows_down(F &&body)
{
    constexpr int B = C < kFenceRows ? C : kFenceRows;
#pragma unroll
    for (int t0 = C - B; t0 >= 0; t0 -= B) {
        if (opaque_true()) {
#pragma unroll
            for (int tt = B - 1; tt >= 0; --tt) body(t0 + tt);
        }
    }
}

// runtime-indexed read of a register array without spilling it: C selects
template <typename T, int C>
__device__ __forceinline__ T pick(const T (&v)[C], int t)
{
    T r = T(0);
#pragma unroll
    for (int q = 0; q < C; ++q) r = (q == t) ? v[q] : r;
    return r;
}

// Where this lane sits: chunk j (of P) of system slot sl (of S) in its group.
struct LaneGeom {
    int j, sl, S, P;
};

// This lane's view of a coefficient table (layout in internal.h); Ptr is the
// pointer type of the table's source (LDS or scalar).
template <typename Ptr>
struct LaneTable {
    Ptr wE1, wE2, wS1, wS2;   // boundary-state weights (pass 1)
    Ptr s, l1, l2;            // forward recurrence (pass 2), l stored negated
    Ptr u1, u2;               // backward recurrence (pass 3), stored negated
    Ptr z0, z1;               // periodic correction, stored negated
    Ptr Mf, Mb, G;            // per-chunk KxK matrices
};

template <typename T, int K, int C, bool CYC, typename Ptr>
__device__ __forceinline__ LaneTable<Ptr> lane_table(Ptr tab, int P, int j)
{
    const int L = P * (C + 1);
    const int off = j * (C + 1);
    LaneTable<Ptr> tb;
    int q = 0;
    tb.wE1 = tab + (q++) * L + off;
    tb.wE2 = (K == 2) ? tab + (q++) * L + off : nullptr;
    tb.wS1 = tab + (q++) * L + off;
    tb.wS2 = (K == 2) ? tab + (q++) * L + off : nullptr;
    tb.s = tab + (q++) * L + off;
    tb.l1 = tab + (q++) * L + off;
    tb.l2 = (K == 2) ? tab + (q++) * L + off : nullptr;
    tb.u1 = tab + (q++) * L + off;
    tb.u2 = (K == 2) ? tab + (q++) * L + off : nullptr;
    tb.z0 = CYC ? tab + (q++) * L + off : nullptr;
    tb.z1 = (CYC && K == 2) ? tab + (q++) * L + off : nullptr;
    tb.Mf = tab + q * L;
    tb.Mb = tb.Mf + P * K * K;
    tb.G = tb.Mb + P * K * K;
    return tb;
}

// Gather rows 0, 1, n-2, n-1 of the system this lane works on (every lane of
// the system gets the same four values).  Row n-1 / n-2 sit at a compile-time
// position when the chunks tile n exactly, else they are picked at run time.
template <typename T, int K, int C>
__device__ __forceinline__ void gather_ends(const T (&v)[C], const LaneGeom &lg, int n, int exact,
                                            T &r0, T &r1, T &rn2, T &rn1)
{
    r0 = shfl(v[0], lg.sl);
    r1 = (K == 2) ? shfl(v[1], lg.sl) : T(0);
    if (exact) {
        const int src = (n / C - 1) * lg.S + lg.sl;
        rn1 = shfl(v[C - 1], src);
        rn2 = (K == 2) ? shfl(v[C - 2], src) : T(0);
    } else {
        rn1 = shfl(pick(v, (n - 1) % C), ((n - 1) / C) * lg.S + lg.sl);
        rn2 = (K == 2) ? shfl(pick(v, (n - 2) % C), ((n - 2) / C) * lg.S + lg.sl) : T(0);
    }
}

// y <- M y + e for a KxK matrix M (row-major) and K-vectors
template <typename T, int K, typename Ptr>
__device__ __forceinline__ void affine(Ptr M, T &y1, T &y2, T e1, T e2)
{
    if constexpr (K == 1) {
        y1 = fma(M[0], y1, e1);
    } else {
        const T n1 = fma(M[1], y2, fma(M[0], y1, e1));
        const T n2 = fma(M[3], y2, fma(M[2], y1, e2));
        y1 = n1;
        y2 = n2;
    }
}

// s = Q (r0, r1, rn2, rn1): the periodic correction scalars, with every
// product-sum written as an explicit fma chain so the rounding does not
// depend on how the compiler contracts a particular kernel.
template <typename T, int K>
__device__ __forceinline__ void correction_scalars(const CyclicQ &cq, T r0, T r1, T rn2, T rn1,
                                                   T &c0, T &c1)
{
    if constexpr (K == 1) {
        c0 = fma(T(cq.q[0][1]), rn1, T(cq.q[0][0]) * r0);
    } else {
        c0 = fma(T(cq.q[0][3]), rn1, fma(T(cq.q[0][2]), rn2, fma(T(cq.q[0][1]), r1, T(cq.q[0][0]) * r0)));
        c1 = fma(T(cq.q[1][3]), rn1, fma(T(cq.q[1][2]), rn2, fma(T(cq.q[1][1]), r1, T(cq.q[1][0]) * r0)));
    }
}

// Solve this lane's chunk in place: v holds the right-hand side rows on entry
// and the solution rows on exit.  All 64 lanes of the wave must call it
// together (the scans shuffle across the wave).
//
//   pass 1: the chunk's zero-history forward end state e and the zero-future
//           backward start state o of that forward solution, both linear in
//           the right-hand side: dot products with precomputed weights (no
//           dependency chain, nothing written);
//   scans:  history H_j (prefix over chunks, H_{i+1} = e_i + Mf_i H_i), then
//           S_j = o_j + G_j H_j and the future F_j (suffix, F_{i-1} = S_i + Mb_i F_i);
//   pass 2: forward recurrence from H_j, writing y;
//   pass 3: backward recurrence from F_j, writing x (periodic correction fused
//           when the chunks tile n exactly, else applied afterwards).
// Each pass re-derives its table pointers (LDS or scalar) from an opaque base
// so the compiler re-reads coefficients instead of keeping C of them live
// across passes.
//
// SPLIT: the group spans several waves of the workgroup; boundary states go
// through the exchange area xch (split_exchange_len elements, plus
// split_ends_len when the chunks do not tile n exactly in a periodic solve)
// with workgroup barriers, so every wave of the workgroup must call it the
// same number of times.
template <typename T, int K, int C, bool CYC, bool SPLIT = false, typename Src = FromLds<T>>
__device__ __forceinline__ void chunk_solve(T (&v)[C], typename Src::ptr tab, const LaneGeom &lg,
                                            int n, int exact, const CyclicQ &cq, T *xch = nullptr)
{
    T e1 = T(0), e2 = T(0), o1 = T(0), o2 = T(0);
    {
        const auto tb = lane_table<T, K, C, CYC>(Src::base(tab), lg.P, lg.j);
        rows_up<C>([&](int t) {
            e1 = fma(tb.wE1[t], v[t], e1);
            o1 = fma(tb.wS1[t], v[t], o1);
            if constexpr (K == 2) {
                e2 = fma(tb.wE2[t], v[t], e2);
                o2 = fma(tb.wS2[t], v[t], o2);
            }
        });
    }
    __builtin_amdgcn_sched_barrier(0);
    // history of this chunk: H_j = true (y_{start-1}, y_{start-2})
    const auto tb = lane_table<T, K, C, CYC>(Src::base(tab), lg.P, lg.j);
    T h1 = T(0), h2 = T(0);
    // exchange area: structure of arrays of P*S entries, (chunk, slot) at
    // chunk*S + slot, so a wave's accesses are consecutive words
    const int me = lg.j * lg.S + lg.sl;
    const int PS = lg.P * lg.S;
    if constexpr (SPLIT) {
        T *xa = xch;   // [2][P*S]
        xa[me] = e1;
        xa[PS + me] = e2;
        __syncthreads();
        for (int i = 0; i < lg.j; ++i) {
            const int src = i * lg.S + lg.sl;
            affine<T, K>(tb.Mf + i * K * K, h1, h2, xa[src], xa[PS + src]);
        }
    } else {
        for (int i = 0; i < lg.P; ++i) {
            const int src = i * lg.S + lg.sl;
            const T a1 = shfl(e1, src);
            const T a2 = (K == 2) ? shfl(e2, src) : T(0);
            if (i < lg.j) affine<T, K>(tb.Mf + i * K * K, h1, h2, a1, a2);
        }
    }
    // zero-future start state of the true forward solution of this chunk
    T s1 = o1, s2 = o2;
    {
        const auto Gm = tb.G + lg.j * K * K;
        if constexpr (K == 1) {
            s1 = fma(Gm[0], h1, o1);
        } else {
            s1 = fma(Gm[1], h2, fma(Gm[0], h1, o1));
            s2 = fma(Gm[3], h2, fma(Gm[2], h1, o2));
        }
    }
    // future of this chunk: F_j = true (x_{end+1}, x_{end+2})
    T f1 = T(0), f2 = T(0);
    if constexpr (SPLIT) {
        T *xb = xch + 2 * PS;   // [2][P*S]
        xb[me] = s1;
        xb[PS + me] = s2;
        __syncthreads();
        for (int i = lg.P - 1; i > lg.j; --i) {
            const int src = i * lg.S + lg.sl;
            affine<T, K>(tb.Mb + i * K * K, f1, f2, xb[src], xb[PS + src]);
        }
    } else {
        for (int i = lg.P - 1; i >= 0; --i) {
            const int src = i * lg.S + lg.sl;
            const T a1 = shfl(s1, src);
            const T a2 = (K == 2) ? shfl(s2, src) : T(0);
            if (i > lg.j) affine<T, K>(tb.Mb + i * K * K, f1, f2, a1, a2);
        }
    }
    // periodic correction x = y - Z s, s = Q (y_0..y_{K-1}, y_{n-K}..y_{n-1}), from
    // the scan results when the chunks tile n exactly
    T c0 = T(0), c1 = T(0);
    if constexpr (CYC) {
        if (exact) {
            // rows 0, 1: start state of chunk 0 = S_0 + Mb_0 F_0
            T x0 = s1, x1 = s2;
            {
                T g1 = f1, g2 = f2;
                affine<T, K>(tb.Mb + lg.j * K * K, g1, g2, s1, s2);
                x0 = g1;
                x1 = g2;
            }
            // rows n-1, n-2: the last real chunk's true forward end state (its
            // future is zero, so x_{n-1} = y_{n-1}, x_{n-2} = y_{n-2} - u1 y_{n-1})
            T y1 = h1, y2 = h2;
            affine<T, K>(tb.Mf + lg.j * K * K, y1, y2, e1, e2);
            const int last = (n / C - 1) * lg.S + lg.sl;
            T r0, r1, rn1, rn2;
            if constexpr (SPLIT) {
                T *xc = xch + 4 * PS;   // [4][P*S]
                xc[me] = x0;
                xc[PS + me] = x1;
                xc[2 * PS + me] = y1;
                xc[3 * PS + me] = y2;
                __syncthreads();
                r0 = xc[lg.sl];
                r1 = xc[PS + lg.sl];
                rn1 = xc[2 * PS + last];
                rn2 = (K == 2) ? fma(T(cq.u1_nm2), rn1, xc[3 * PS + last]) : T(0);
            } else {
                r0 = shfl(x0, lg.sl);
                r1 = (K == 2) ? shfl(x1, lg.sl) : T(0);
                rn1 = shfl(y1, last);
                rn2 = (K == 2) ? fma(T(cq.u1_nm2), rn1, shfl(y2, last)) : T(0);
            }
            correction_scalars<T, K>(cq, r0, r1, rn2, rn1, c0, c1);
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    // pass 2: forward recurrence from the true history
    {
        const auto tp = lane_table<T, K, C, CYC>(Src::base(tab), lg.P, lg.j);
        T y1 = h1, y2 = h2;
        rows_up<C>([&](int t) {
            T y = tp.s[t] * v[t];
            if constexpr (K == 2) y = fma(tp.l2[t], y2, y);
            y = fma(tp.l1[t], y1, y);
            v[t] = y;
            y2 = y1;
            y1 = y;
        });
    }
    __builtin_amdgcn_sched_barrier(0);
    // pass 3: backward recurrence from the true future (+ fused periodic correction)
    {
        const auto tp = lane_table<T, K, C, CYC>(Src::base(tab), lg.P, lg.j);
        T x1 = f1, x2 = f2;
        rows_down<C>([&](int t) {
            T x = v[t];
            if constexpr (K == 2) x = fma(tp.u2[t], x2, x);
            x = fma(tp.u1[t], x1, x);
            x2 = x1;
            x1 = x;
            if constexpr (CYC) {
                x = fma(tp.z0[t], c0, x);
                if constexpr (K == 2) x = fma(tp.z1[t], c1, x);
            }
            v[t] = x;
        });
    }
    if constexpr (CYC) {
        if (!exact) {
            __builtin_amdgcn_sched_barrier(0);
            T r0, r1, rn2, rn1;
            if constexpr (SPLIT) {
                // rows 0, 1 (chunk 0) and n-2, n-1 (wherever they sit) through
                // the fourth phase of the exchange area
                T *xd = xch + 8 * PS;   // [4][P*S]
                xd[me] = v[0];
                xd[PS + me] = v[1];
                xd[2 * PS + me] = pick(v, (n - 2) % C);
                xd[3 * PS + me] = pick(v, (n - 1) % C);
                __syncthreads();
                r0 = xd[lg.sl];
                r1 = (K == 2) ? xd[PS + lg.sl] : T(0);
                rn2 = (K == 2) ? xd[2 * PS + ((n - 2) / C) * lg.S + lg.sl] : T(0);
                rn1 = xd[3 * PS + ((n - 1) / C) * lg.S + lg.sl];
            } else {
                gather_ends<T, K, C>(v, lg, n, exact, r0, r1, rn2, rn1);
            }
            correction_scalars<T, K>(cq, r0, r1, rn2, rn1, c0, c1);
            const auto tp = lane_table<T, K, C, CYC>(Src::base(tab), lg.P, lg.j);
            rows_up<C>([&](int t) {
                T x = fma(tp.z0[t], c0, v[t]);
                if constexpr (K == 2) x = fma(tp.z1[t], c1, x);
                v[t] = x;
            });
        }
    }
}

// Workgroup -> group-of-systems mapping.  A workgroup of W waves works on
// W consecutive groups at a time (one per wave); workgroups are dealt
// round-robin to the 8 XCDs, and each XCD gets a contiguous range of these
// blocks of groups, so segments that share 128 B lines are read inside one L2.
// The trip count of the loop over blocks is uniform across the workgroup, so a
// workgroup barrier inside it is reached by every wave the same number of times.
struct GroupRange {
    int64_t first, end, stride;   // blocks of W groups
    int W, wave;
};

__device__ __forceinline__ GroupRange group_range(int64_t groups, int log2Q = 0, int linear = 0)
{
    constexpr int kXcd = 8;
    GroupRange r;
    r.W = (blockDim.x / kWave) >> log2Q;     // groups per workgroup
    r.wave = (threadIdx.x / kWave) >> log2Q; // this wave's group in the workgroup
    const int64_t blocks = (groups + r.W - 1) / r.W;
    if (linear) {   // the host launched one workgroup per block of groups
        r.first = blockIdx.x;
        r.end = r.first < blocks ? r.first + 1 : r.first;
        r.stride = 1;
        return r;
    }
    const int xcd = blockIdx.x % kXcd;
    const int64_t per_xcd = (blocks + kXcd - 1) / kXcd;
    const int64_t base = (int64_t)xcd * per_xcd;
    r.first = base + blockIdx.x / kXcd;
    r.end = base + per_xcd < blocks ? base + per_xcd : blocks;
    r.stride = gridDim.x / kXcd;   // host launches a multiple of 8
    return r;
}

// Start of one iteration of the persistent loop.  With `lockstep`, the waves
// of a workgroup start their loads together, so the two halves of a 128 B
// line that two waves read (64 B segments) are requested close in time and
// the second request hits in L2 instead of refetching the line.
__device__ __forceinline__ int64_t begin_block(const GroupRange &r, int64_t b, int lockstep)
{
    if (lockstep) __syncthreads();
    return b * r.W + r.wave;
}

// Copy the shared table into LDS: four loads in flight per thread per round.
template <typename T>
__device__ __forceinline__ void stage_table(T *lds, const T *__restrict__ table, int64_t elems)
{
    const int64_t stride = blockDim.x;
    int64_t e = threadIdx.x;
    for (; e + 3 * stride < elems; e += 4 * stride) {
        const T a = table[e], b = table[e + stride], c = table[e + 2 * stride], d = table[e + 3 * stride];
        lds[e] = a;
        lds[e + stride] = b;
        lds[e + 2 * stride] = c;
        lds[e + 3 * stride] = d;
    }
    for (; e < elems; e += stride) lds[e] = table[e];
}

// Load the C rows of this lane's chunk; column k must be in bounds.
// FULL: every row of every chunk is a real row, no predicates at all.
// Ragged: the row pointer stops at row n-1 (in bounds) and rows past n read 0.
// The stride is laundered once per call so the C row offsets are recomputed
// here rather than hoisted out of the persistent loop and kept live.
template <typename T, int C, bool FULL>
__device__ __forceinline__ void load_chunk(T (&v)[C], const T *base, int row0, int64_t k,
                                           int64_t ld, int n)
{
    ld = opaque_s(ld);
    if constexpr (FULL) {
        const T *p = base + (int64_t)row0 * ld + k;
#pragma unroll
        for (int t = 0; t < C; ++t) v[t] = p[(int64_t)t * ld];
    } else {
        const int nv = opaque_v(n - row0);   // rows of this chunk that are real
        const T *p = base + (int64_t)(row0 < n ? row0 : n - 1) * ld + k;
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const T x = *p;
            v[t] = t < nv ? x : T(0);
            p += (t + 1 < nv) ? ld : 0;
        }
    }
}

// Store the chunk; the caller masks out lanes whose column is past m.  Ragged:
// the pointer stops at row n-1 and the rows past n rewrite row n-1 with its
// own value, so no store is predicated per row.
template <typename T, int C, bool FULL>
__device__ __forceinline__ void store_chunk(const T (&v)[C], T *base, int row0, int64_t k,
                                            int64_t ld, int n)
{
    ld = opaque_s(ld);
    if constexpr (FULL) {
        T *p = base + (int64_t)row0 * ld + k;
#pragma unroll
        for (int t = 0; t < C; ++t) p[(int64_t)t * ld] = v[t];
    } else if (row0 < n) {
        const int nv = opaque_v(n - row0);
        T *p = base + (int64_t)row0 * ld + k;
        T keep = v[0];
#pragma unroll
        for (int t = 0; t < C; ++t) {
            keep = t < nv ? v[t] : keep;
            *p = keep;
            p += (t + 1 < nv) ? ld : 0;
        }
    }
}

// store_chunk of value(t), computed row by row inside the fenced row blocks,
// so the values need not all be live at once.
template <int C, bool FULL, typename F>
__device__ __forceinline__ void store_chunk_fn(F &&value, double *base, int row0, int64_t k,
                                               int64_t ld, int n)
{
    ld = opaque_s(ld);
    if constexpr (FULL) {
        double *p = base + (int64_t)row0 * ld + k;
        rows_up<C>([&](int t) { p[(int64_t)t * ld] = value(t); });
    } else if (row0 < n) {
        const int nv = opaque_v(n - row0);
        double *p = base + (int64_t)row0 * ld + k;
        double keep = value(0);
        rows_up<C>([&](int t) {
            keep = t < nv ? value(t) : keep;
            *p = keep;
            p += (t + 1 < nv) ? ld : 0;
        });
    }
}

// Lane coordinates: a wave holds P/Q chunks of S = 64Q/P systems,
// lane = (chunk within the wave) * S + slot; wave q of a split group holds
// chunks q*P/Q .. (q+1)*P/Q - 1.
__device__ __forceinline__ LaneGeom lane_geom(int log2P, int log2Q = 0)
{
    LaneGeom lg;
    const int lw = log2P - log2Q;   // log2 of chunks per wave
    lg.P = 1 << log2P;
    lg.S = kWave >> lw;
    const int lane = threadIdx.x % kWave;
    const int q = (threadIdx.x / kWave) & ((1 << log2Q) - 1);
    lg.j = (q << lw) + (lane >> (6 - lw));
    lg.sl = lane & (lg.S - 1);
    return lg;
}

// ---------------------------------------------------------------- launch helpers
int cu_count()
{
    static int cached = 0;
    if (!cached) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            cached = cus;
        else
            return 256;
    }
    return cached;
}

// Persistent-style launch: as many workgroups as can be resident at once
// (rounded to a multiple of the 8 XCDs), each looping over groups of systems.
// split_waves > 0: a split group of that many waves is the whole workgroup.
// Tuning grid_linear = 1: non-persistent grids for the kernels launched
// through launch_grid_split; the host sets SweepGeom::linear to match.
inline bool grid_linear() { return tuning(kTuneGridLinear) == 1; }

// linear: one workgroup per block of groups (the kernel's SweepGeom::linear
// must be set); otherwise a persistent grid of at most one wave of resident
// workgroups, each walking the blocks of its XCD's share (group_range).
template <typename... KArgs, typename... Args>
hipError_t launch_grid_mode(void (*kern)(KArgs...), size_t lds, int64_t groups, int split_waves,
                            bool linear, hipStream_t s, Args... args)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // waves per workgroup: the workgroup is the unit that moves in step (see
    // begin_block); tuning waves_per_block (1, 2 or 4) overrides
    int waves_per_block = kBlockThreads / kWave;
    if (tuning(kTuneWavesPerBlock) > 0) waves_per_block = (int)tuning(kTuneWavesPerBlock);
    int groups_per_block = waves_per_block;
    if (split_waves > 0) {
        waves_per_block = split_waves;
        groups_per_block = 1;
    }
    const int threads = waves_per_block * kWave;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int64_t need = (groups + groups_per_block - 1) / groups_per_block;
    int64_t cap = (int64_t)cu_count() * per_cu;
    int64_t blocks = need < cap ? need : cap;
    if (linear) blocks = need;
    blocks = ((blocks + 7) / 8) * 8;   // multiple of the XCD count, see group_range
    if (blocks < 8) blocks = 8;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), lds, s, args...);
    return hipGetLastError();
}

template <typename... KArgs, typename... Args>
hipError_t launch_grid_split(void (*kern)(KArgs...), size_t lds, int64_t groups, int split_waves,
                             hipStream_t s, Args... args)
{
    return launch_grid_mode(kern, lds, groups, split_waves, grid_linear(), s, args...);
}

template <typename... KArgs, typename... Args>
hipError_t launch_grid(void (*kern)(KArgs...), size_t lds, int64_t groups, hipStream_t s,
                       Args... args)
{
    return launch_grid_split(kern, lds, groups, 0, s, args...);
}

bool is_full(const SweepGeom &g) { return ((int64_t)g.C << g.log2P) == g.n; }

}  // namespace
}  // namespace bb
