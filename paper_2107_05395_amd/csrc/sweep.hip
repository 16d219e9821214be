// sweep.hip -- gfx950 kernels for batched banded solves with one shared LHS.
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
// from LDS, where each workgroup stages the shared table once.
#include <cstdlib>

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
// through the exchange area xch (split_exchange_len elements) with workgroup
// barriers, so every wave of the workgroup must call it the same number of
// times.  Split groups are always full decompositions (exact).
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
    const int me = lg.j * lg.S + lg.sl;   // (chunk, slot) index in the exchange area
    if constexpr (SPLIT) {
        T *xa = xch;
        xa[2 * me] = e1;
        xa[2 * me + 1] = e2;
        __syncthreads();
        for (int i = 0; i < lg.j; ++i) {
            const int src = 2 * (i * lg.S + lg.sl);
            affine<T, K>(tb.Mf + i * K * K, h1, h2, xa[src], xa[src + 1]);
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
        T *xb = xch + 2 * lg.P * lg.S;
        xb[2 * me] = s1;
        xb[2 * me + 1] = s2;
        __syncthreads();
        for (int i = lg.P - 1; i > lg.j; --i) {
            const int src = 2 * (i * lg.S + lg.sl);
            affine<T, K>(tb.Mb + i * K * K, f1, f2, xb[src], xb[src + 1]);
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
                T *xc = xch + 4 * lg.P * lg.S;
                xc[4 * me] = x0;
                xc[4 * me + 1] = x1;
                xc[4 * me + 2] = y1;
                xc[4 * me + 3] = y2;
                __syncthreads();
                r0 = xc[4 * lg.sl];
                r1 = xc[4 * lg.sl + 1];
                rn1 = xc[4 * last + 2];
                rn2 = (K == 2) ? fma(T(cq.u1_nm2), rn1, xc[4 * last + 3]) : T(0);
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
    if constexpr (CYC && !SPLIT) {
        if (!exact) {
            __builtin_amdgcn_sched_barrier(0);
            T r0, r1, rn2, rn1;
            gather_ends<T, K, C>(v, lg, n, exact, r0, r1, rn2, rn1);
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

__device__ __forceinline__ GroupRange group_range(int64_t groups, int log2Q = 0)
{
    constexpr int kXcd = 8;
    GroupRange r;
    r.W = (blockDim.x / kWave) >> log2Q;     // groups per workgroup
    r.wave = (threadIdx.x / kWave) >> log2Q; // this wave's group in the workgroup
    const int64_t blocks = (groups + r.W - 1) / r.W;
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

// ---------------------------------------------------------------- solve
// QL = log2 of the waves per system group (0: one wave per group).  With
// QL > 0 the workgroup is exactly one group (2^QL waves): every wave of it has
// the same group index, so the exchange barriers are reached uniformly.
template <typename T, int K, int C, bool CYC, bool FULL, int QL>
__global__ __launch_bounds__((kWave << QL) > kMaxBlockThreads ? (kWave << QL) : kMaxBlockThreads)
void sweep_kernel(const T *__restrict__ table, int64_t table_elems, CyclicQ cq, SweepGeom g,
                  const T *in, T *out)
{
    static_assert(QL == 0 || FULL, "split groups are full decompositions");
    extern __shared__ double smem_d[];
    T *lds = reinterpret_cast<T *>(smem_d);
    stage_table(lds, table, table_elems);
    __syncthreads();
    T *xch = lds + table_elems;   // exchange area of the split group (QL > 0)

    const LaneGeom lg = lane_geom(g.log2P, QL);
    const int row0 = lg.j * C;
    const GroupRange gr = group_range(g.groups, QL);
    for (int64_t b = gr.first; b < gr.end; b += gr.stride) {
        const int64_t grp = begin_block(gr, b, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        T v[C];
        load_chunk<T, C, FULL>(v, in, row0, kval ? k : g.m - 1, g.ld, g.n);
        chunk_solve<T, K, C, CYC, (QL > 0)>(v, lds, lg, g.n, FULL || g.exact, cq, xch);
        if (kval) store_chunk<T, C, FULL>(v, out, row0, k, g.ld, g.n);
    }
}

// ---------------------------------------------------------------- refine
// x0 = solve_f32(b); r = b - A x0 in double with the original bands;
// x = x0 + solve_f32(r), stored as double.
// QL > 0: split groups as in sweep_kernel; the exchange area holds the three
// phases of chunk_solve followed by rows 0, 1, C-2, C-1 of every chunk.
template <int K, int C, bool CYC, bool FULL, int QL>
__global__ __launch_bounds__(kMaxBlockThreads) void refine_kernel(
    const float *__restrict__ table, int64_t table_elems, const double *__restrict__ band_table,
    int64_t band_elems, CyclicQ cq, Corners cn, SweepGeom g, const double *in, double *out)
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
    const GroupRange gr = group_range(g.groups, QL);

    for (int64_t blk = gr.first; blk < gr.end; blk += gr.stride) {
        const int64_t grp = begin_block(gr, blk, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        double b[C];
        load_chunk<double, C, FULL>(b, in, row0, kval ? k : g.m - 1, g.ld, g.n);
        float x0[C];
#pragma unroll
        for (int t = 0; t < C; ++t) x0[t] = (float)b[t];
        chunk_solve<float, K, C, CYC, (QL > 0)>(x0, lds, lg, g.n, exact, cq, xch);
        __builtin_amdgcn_sched_barrier(0);

        // neighbours across the chunk boundaries (zero outside the matrix) and,
        // periodic, rows 0, 1, n-2, n-1 of the system
        float xl1, xl2, xr1, xr2, r0 = 0.f, r1 = 0.f, rn2 = 0.f, rn1 = 0.f;
        if constexpr (QL > 0) {
            float *xd = xch + 8 * lg.P * lg.S;
            const int me = 4 * (lg.j * lg.S + lg.sl);
            xd[me] = x0[0];
            xd[me + 1] = x0[1];
            xd[me + 2] = x0[C - 2];
            xd[me + 3] = x0[C - 1];
            __syncthreads();
            const int lft = 4 * ((has_left ? lg.j - 1 : lg.j) * lg.S + lg.sl);
            const int rgt = 4 * ((has_right ? lg.j + 1 : lg.j) * lg.S + lg.sl);
            xl1 = has_left ? xd[lft + 3] : 0.f;
            xl2 = has_left ? xd[lft + 2] : 0.f;
            xr1 = has_right ? xd[rgt] : 0.f;
            xr2 = has_right ? xd[rgt + 1] : 0.f;
            if constexpr (CYC) {
                const int first = 4 * lg.sl, last = 4 * ((lg.P - 1) * lg.S + lg.sl);
                r0 = xd[first];
                r1 = xd[first + 1];
                rn2 = xd[last + 2];
                rn1 = xd[last + 3];
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
            double r = b[t] - ax;
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
    const int me = 2 * (lg.j * kWave + lg.sl);
    const int lft = 2 * ((has_left ? lg.j - 1 : lg.j) * kWave + lg.sl) + 1;
    const int rgt = 2 * ((has_right ? lg.j + 1 : lg.j) * kWave + lg.sl);
    const int first = 2 * lg.sl, last = 2 * ((lg.P - 1) * kWave + lg.sl) + 1;
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
            xd[me + 1] = c[C - 1];
            __syncthreads();
            const double cl = has_left ? xd[lft] : 0.0;
            const double cr = has_right ? xd[rgt] : 0.0;
            ch_rhs<C, true>(c, cl, cr, xd[first], xd[last], alpha, lg.j, !has_right, C);
            __builtin_amdgcn_sched_barrier(0);
            chunk_solve<double, 2, C, true, true, Src>(c, tab, lg, g.n, 1, cq, xch);
        }
        if (kval) store_chunk<double, C, true>(c, out, row0, k, g.ld, g.n);
    }
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
template <typename... KArgs, typename... Args>
hipError_t launch_grid_split(void (*kern)(KArgs...), size_t lds, int64_t groups, int split_waves,
                             hipStream_t s, Args... args)
{
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void *)kern,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    // waves per workgroup: the workgroup is the unit that moves in step (see
    // begin_block); BANDBATCH_WAVES_PER_BLOCK (1, 2 or 4) overrides (tuning)
    int waves_per_block = kBlockThreads / kWave;
    if (const char *env = std::getenv("BANDBATCH_WAVES_PER_BLOCK")) {
        const int w = std::atoi(env);
        if (w == 1 || w == 2 || w == 4) waves_per_block = w;
    }
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
    blocks = ((blocks + 7) / 8) * 8;   // multiple of the XCD count, see group_range
    if (blocks < 8) blocks = 8;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), lds, s, args...);
    return hipGetLastError();
}

template <typename... KArgs, typename... Args>
hipError_t launch_grid(void (*kern)(KArgs...), size_t lds, int64_t groups, hipStream_t s,
                       Args... args)
{
    return launch_grid_split(kern, lds, groups, 0, s, args...);
}

bool is_full(const SweepGeom &g) { return ((int64_t)g.C << g.log2P) == g.n; }

template <typename T, int K, bool CYC, int C, int QL>
hipError_t sweep_split(const void *table, int64_t table_elems, const CyclicQ &q,
                       const SweepGeom &g, const void *in, void *out, hipStream_t stream)
{
    const size_t lds = (size_t)(table_elems + split_exchange_len(QL)) * sizeof(T);
    return launch_grid_split(sweep_kernel<T, K, C, CYC, true, QL>, lds, g.groups, 1 << QL, stream,
                             (const T *)table, table_elems, q, g, (const T *)in, (T *)out);
}

template <typename T, int K, bool CYC, int C>
hipError_t sweep_c(const void *table, int64_t table_elems, const CyclicQ &q, const SweepGeom &g,
                   const void *in, void *out, hipStream_t stream)
{
    if (g.log2Q > 0) {
        // split groups: full decompositions with 64 or 128 rows per lane only
        if constexpr (C >= 64) {
            if (!is_full(g) || g.log2Q > max_log2q(C, false) || g.log2Q > g.log2P)
                return hipErrorInvalidValue;
            if (g.log2Q == 1) return sweep_split<T, K, CYC, C, 1>(table, table_elems, q, g, in, out, stream);
            if (g.log2Q == 2) return sweep_split<T, K, CYC, C, 2>(table, table_elems, q, g, in, out, stream);
            if constexpr (C <= 64) return sweep_split<T, K, CYC, C, 3>(table, table_elems, q, g, in, out, stream);
        }
        return hipErrorInvalidValue;
    }
    const size_t lds = (size_t)table_elems * sizeof(T);
    if (is_full(g))
        return launch_grid(sweep_kernel<T, K, C, CYC, true, 0>, lds, g.groups, stream,
                           (const T *)table, table_elems, q, g, (const T *)in, (T *)out);
    return launch_grid(sweep_kernel<T, K, C, CYC, false, 0>, lds, g.groups, stream,
                       (const T *)table, table_elems, q, g, (const T *)in, (T *)out);
}

template <int K, bool CYC, int C>
hipError_t refine_c(const void *table, int64_t table_elems, const double *band,
                    int64_t band_elems, const CyclicQ &q, const Corners &cn, const SweepGeom &g,
                    const void *in, void *out, hipStream_t stream)
{
    const size_t lds = (size_t)band_elems * sizeof(double) + (size_t)table_elems * sizeof(float);
    if (g.log2Q > 0) {
        if constexpr (C >= 64) {
            if (!is_full(g) || g.log2Q > max_log2q(C, true) || g.log2Q > g.log2P)
                return hipErrorInvalidValue;
            const size_t xl = (size_t)(split_exchange_len(g.log2Q) + (4LL * kWave << g.log2Q)) * sizeof(float);
            if (g.log2Q == 1)
                return launch_grid_split(refine_kernel<K, C, CYC, true, 1>, lds + xl, g.groups, 2,
                                         stream, (const float *)table, table_elems, band,
                                         band_elems, q, cn, g, (const double *)in, (double *)out);
            return launch_grid_split(refine_kernel<K, C, CYC, true, 2>, lds + xl, g.groups, 4,
                                     stream, (const float *)table, table_elems, band, band_elems,
                                     q, cn, g, (const double *)in, (double *)out);
        }
        return hipErrorInvalidValue;
    }
    if (is_full(g))
        return launch_grid(refine_kernel<K, C, CYC, true, 0>, lds, g.groups, stream,
                           (const float *)table, table_elems, band, band_elems, q, cn, g,
                           (const double *)in, (double *)out);
    return launch_grid(refine_kernel<K, C, CYC, false, 0>, lds, g.groups, stream,
                       (const float *)table, table_elems, band, band_elems, q, cn, g,
                       (const double *)in, (double *)out);
}

template <typename T, int K, bool CYC>
hipError_t sweep_dispatch(const void *table, int64_t te, const CyclicQ &q, const SweepGeom &g,
                          const void *in, void *out, hipStream_t s)
{
    switch (g.C) {
    case 4: return sweep_c<T, K, CYC, 4>(table, te, q, g, in, out, s);
    case 8: return sweep_c<T, K, CYC, 8>(table, te, q, g, in, out, s);
    case 16: return sweep_c<T, K, CYC, 16>(table, te, q, g, in, out, s);
    case 32: return sweep_c<T, K, CYC, 32>(table, te, q, g, in, out, s);
    case 64: return sweep_c<T, K, CYC, 64>(table, te, q, g, in, out, s);
    case 128: return sweep_c<T, K, CYC, 128>(table, te, q, g, in, out, s);
    default: return hipErrorInvalidValue;
    }
}

template <int K, bool CYC>
hipError_t refine_dispatch(const void *table, int64_t te, const double *band, int64_t be,
                           const CyclicQ &q, const Corners &cn, const SweepGeom &g,
                           const void *in, void *out, hipStream_t s)
{
    switch (g.C) {
    case 4: return refine_c<K, CYC, 4>(table, te, band, be, q, cn, g, in, out, s);
    case 8: return refine_c<K, CYC, 8>(table, te, band, be, q, cn, g, in, out, s);
    case 16: return refine_c<K, CYC, 16>(table, te, band, be, q, cn, g, in, out, s);
    case 32: return refine_c<K, CYC, 32>(table, te, band, be, q, cn, g, in, out, s);
    case 64: return refine_c<K, CYC, 64>(table, te, band, be, q, cn, g, in, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_sweep(int K, bool cyclic, Op op, bool f32, const void *table,
                        int64_t table_elems, const double *band_table, int64_t band_elems,
                        const CyclicQ &q, const Corners &cn, const SweepGeom &g, const void *in,
                        void *out, hipStream_t s)
{
    if (op == Op::Refine) {
        if (K == 1) return cyclic ? refine_dispatch<1, true>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s)
                                  : refine_dispatch<1, false>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s);
        return cyclic ? refine_dispatch<2, true>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s)
                      : refine_dispatch<2, false>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s);
    }
    if (f32) {
        if (K == 1) return cyclic ? sweep_dispatch<float, 1, true>(table, table_elems, q, g, in, out, s)
                                  : sweep_dispatch<float, 1, false>(table, table_elems, q, g, in, out, s);
        return cyclic ? sweep_dispatch<float, 2, true>(table, table_elems, q, g, in, out, s)
                      : sweep_dispatch<float, 2, false>(table, table_elems, q, g, in, out, s);
    }
    if (K == 1) return cyclic ? sweep_dispatch<double, 1, true>(table, table_elems, q, g, in, out, s)
                              : sweep_dispatch<double, 1, false>(table, table_elems, q, g, in, out, s);
    return cyclic ? sweep_dispatch<double, 2, true>(table, table_elems, q, g, in, out, s)
                  : sweep_dispatch<double, 2, false>(table, table_elems, q, g, in, out, s);
}

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
