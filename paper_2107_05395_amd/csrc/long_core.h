// long_core.h -- batched solves of long systems, whose rows a workgroup
// cannot hold at once: the chunked decomposition of internal.h spread over
// three launches instead of one wave or workgroup per system group.
//
// A system of n rows is cut into P chunks of C rows; chunks 0 .. P-2 are full
// and chunk P-1 (the tail) holds the remaining nr = n - (P-1) C rows (1 .. C).
// The recurrences, coefficient table (internal.h layout, any P) and
// chunk-boundary algebra are those of the one-launch sweep (sweep_core.h):
//
//   reduce (one wave per full chunk and group of 64 systems): the chunk's
//          zero-history forward end state e_j and zero-future backward start
//          state o_j (dot products with the table's weights), written to rows
//          r0 .. r0+2K-1 of the solution array x, which serves as the scratch
//          of the launch sequence;
//   scan   (one lane per system, or one wave per system for small
//          batches, long_scan_spread): H_j (prefix over the full chunks,
//          H_{j+1} = e_j + Mf_j H_j) written over e_j; the tail chunk solved
//          in registers from its history H_{P-1}; then S_j = o_j + G_j H_j and
//          the future F_j (suffix, F_{j-1} = S_j + Mb_j F_j, F_{P-2} = the
//          tail's start state) written over o_j; for periodic systems the
//          correction scalars c = Q (w_0, w_1, w_{n-2}, w_{n-1}) written to
//          rows r0+2K .. r0+3K-1 of every full chunk; the tail's solution
//          stored (and corrected, periodic);
//   solve  (one wave per full chunk and group): forward pass from H_j,
//          backward pass from F_j with the correction fused, solution stored
//          over the chunk (the reads of H_j, F_j and c come first).
//
// Every wave of reduce and solve works on one chunk of 64 systems (one
// 512-byte segment per row, or two 256-byte ones for large batches), so
// every coefficient is the same for the whole wave: the table is read
// through the scalar cache and may have any size.  HBM traffic: the right-hand side read twice and the solution
// written once (24 B per row in double) plus 2K doubles per chunk of
// scratch, against 16 B for the one-launch sweep.  x must not overlap the
// right-hand side.
#pragma once

#include "sweep_core.h"

namespace bb {
namespace {

// Right-hand-side source of the plain solve: the rows of rhs.
struct PlainSrc {
    const double *rhs;
    template <int C>
    __device__ __forceinline__ void full(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, true>(v, rhs, row0, k, ld, n);
    }
    template <int C>
    __device__ __forceinline__ void tail(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        load_chunk<double, C, false>(v, rhs, row0, k, ld, n);
    }
};

template <int K, int C, bool CYC>
using LongTable = LaneTable<typename FromScalar<double>::ptr>;

template <int K, int C, bool CYC>
__device__ __forceinline__ LongTable<K, C, CYC> long_table(const double *table, int P, int j)
{
    using Src = FromScalar<double>;
    return lane_table<double, K, C, CYC>(Src::base((typename Src::ptr)table), P, j);
}

// Wave w of a reduce or solve launch: chunk j = w / groups (wave-uniform)
// and group w % groups of 64 systems, neighbouring waves on neighbouring
// systems of the same rows.  With g.halves the 64 lanes of group p are
// systems 32p .. 32p+31 and 32(groups + p) .. 32(groups + p)+31: two
// 256-byte segments per row instead of one 512-byte one, which large batches
// stream faster (tri n = 8192, m = 2^16: 2.37 against 2.86 ms per solve;
// slower at m = 4096).
struct LongWave {
    int j;
    int64_t k;
    bool valid;   // false: the wave has no chunk (grid rounding)
};

__device__ __forceinline__ LongWave long_wave(const LongGeom &g)
{
    LongWave lw;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t total = (int64_t)(g.P - 1) * g.groups;
    lw.valid = w < total;
    const int64_t ww = lw.valid ? w : 0;
    lw.j = __builtin_amdgcn_readfirstlane((int)(ww / g.groups));
    const int64_t grp = ww % g.groups;
    const int lane = threadIdx.x % kWave;
    if (g.halves)
        lw.k = lane < kWave / 2 ? grp * (kWave / 2) + lane
                                : (g.groups + grp) * (kWave / 2) + (lane - kWave / 2);
    else
        lw.k = grp * kWave + lane;
    return lw;
}

template <int K, int C, bool CYC, class Src>
__global__ __launch_bounds__(256) void long_reduce(const double *__restrict__ table, LongGeom g,
                                                   Src src, double *x)
{
    const LongWave lw = long_wave(g);
    if (!lw.valid) return;   // whole waves
    const bool kval = lw.k < g.m;
    const int64_t kk = kval ? lw.k : g.m - 1;
    const int row0 = lw.j * C;
    double v[C];
    src.template full<C>(v, row0, kk, g.ld, g.n);
    const auto tb = long_table<K, C, CYC>(table, g.P, lw.j);
    double e1 = 0.0, e2 = 0.0, o1 = 0.0, o2 = 0.0;
    rows_up<C>([&](int t) {
        e1 = fma(tb.wE1[t], v[t], e1);
        o1 = fma(tb.wS1[t], v[t], o1);
        if constexpr (K == 2) {
            e2 = fma(tb.wE2[t], v[t], e2);
            o2 = fma(tb.wS2[t], v[t], o2);
        }
    });
    if (kval) {
        double *p = x + (int64_t)row0 * g.ld + lw.k;
        p[0] = e1;
        if constexpr (K == 2) p[g.ld] = e2;
        p[(int64_t)K * g.ld] = o1;
        if constexpr (K == 2) p[(int64_t)(K + 1) * g.ld] = o2;
    }
}

// Full chunks per block of the scan.  The chain over a system's chunks is
// bound by load latency, so everything a block needs is loaded before the
// chain runs over it: each chunk's scratch values (per lane) and the block's
// chunk matrices, which are the same for every system -- one vector load
// spreads them over the wave's lanes and the chain reads them back with
// readlane (a scalar load per chunk would put one round trip per chunk into
// the chain).  SB K x K matrices fill at most the 64 lanes.
template <int K>
constexpr int scan_block() { return K == 1 ? 32 : 16; }

// the double held by lane l of the wave (l wave-uniform)
__device__ __forceinline__ double lane_value(double v, int l)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// M_j = mats[(j0 + b) K^2 ..] for b = 0 .. SB-1, lane b K^2 + q holding
// element q of chunk j0 + b (clamped to the last full chunk).
template <int K, int SB>
__device__ __forceinline__ double load_block_mats(const double *mats, int j0, int full, int lane)
{
    const int b = lane / (K * K) < SB ? lane / (K * K) : SB - 1;
    const int j = j0 + b < full ? j0 + b : full - 1;
    return mats[(int64_t)j * K * K + lane % (K * K)];
}

// y <- e + M_b y with M_b the matrix of chunk b of the block in `mats`.
template <int K>
__device__ __forceinline__ void affine_lanes(double mats, int b, double &y1, double &y2,
                                             double e1, double e2)
{
    if constexpr (K == 1) {
        y1 = fma(lane_value(mats, b), y1, e1);
    } else {
        const double m0 = lane_value(mats, 4 * b), m1 = lane_value(mats, 4 * b + 1);
        const double m2 = lane_value(mats, 4 * b + 2), m3 = lane_value(mats, 4 * b + 3);
        const double n1 = fma(m1, y2, fma(m0, y1, e1));
        const double n2 = fma(m3, y2, fma(m2, y1, e2));
        y1 = n1;
        y2 = n2;
    }
}

// One lane per system (k): the forward scan over the full chunks, the tail
// chunk, the backward scan and the periodic correction scalars, reading and
// writing the scratch rows of x.  Every lane of a launched wave runs (lanes
// past m on system m-1, storing nothing), so readlane sees loaded values.
template <int K, int C, bool CYC, class Src>
__global__ __launch_bounds__(256) void long_scan(const double *__restrict__ table, CyclicQ cq,
                                                 LongGeom g, Src src, double *x)
{
    using SP = FromScalar<double>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t kmax = g.groups * kWave;
    if ((int64_t)blockIdx.x * blockDim.x >= kmax) return;   // whole workgroups past the batch
    const bool kval = k < g.m;
    const int64_t kk = kval ? k : g.m - 1;
    const int lane = threadIdx.x % kWave;
    const int64_t ld = g.ld;
    const int full = g.P - 1;
    const int na = num_arrays(K, CYC);
    const int64_t L = (int64_t)g.P * (C + 1);
    const typename SP::ptr tabs = SP::base((typename SP::ptr)table);
    // the chunk matrices, read with vector loads
    const double *Mf = table + opaque_v(0) + na * L;
    const double *Mb = Mf + (int64_t)g.P * K * K;
    const double *Gm = Mb + (int64_t)g.P * K * K;
    constexpr int SB = scan_block<K>();

    // forward: H_j written over e_j
    double h1 = 0.0, h2 = 0.0;
    for (int j0 = 0; j0 < full; j0 += SB) {
        double a1[SB], a2[SB];
        const double mats = load_block_mats<K, SB>(Mf, j0, full, lane);
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int j = j0 + b < full ? j0 + b : full - 1;
            const double *p = x + (int64_t)j * C * ld + kk;
            a1[b] = p[0];
            a2[b] = K == 2 ? p[ld] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            if (j0 + b < full) {
                double *p = x + (int64_t)(j0 + b) * C * ld + k;
                if (kval) {
                    p[0] = h1;
                    if constexpr (K == 2) p[ld] = h2;
                }
                affine_lanes<K>(mats, b, h1, h2, a1[b], a2[b]);
            }
        }
    }

    // the tail chunk from its history, stored (uncorrected if periodic); its
    // rows are not scratch rows of any full chunk
    const int trow0 = full * C;
    const int nr = g.n - trow0;
    double yn1, yn2, f1, f2;   // y_{n-1}, y_{n-2}; the tail's start state
    {
        double v[C];
        src.template tail<C>(v, trow0, kk, ld, g.n);
        const auto tp = lane_table<double, K, C, CYC>(SP::base(tabs), g.P, full);
        double y1 = h1, y2 = h2;
        rows_up<C>([&](int t) {
            double y = tp.s[t] * v[t];
            if constexpr (K == 2) y = fma(tp.l2[t], y2, y);
            y = fma(tp.l1[t], y1, y);
            v[t] = y;
            y2 = y1;
            y1 = y;
        });
        yn1 = pick(v, nr - 1);
        yn2 = nr >= 2 ? pick(v, nr - 2) : h1;
        double x1 = 0.0, x2 = 0.0;
        rows_down<C>([&](int t) {
            double xx = v[t];
            if constexpr (K == 2) xx = fma(tp.u2[t], x2, xx);
            xx = fma(tp.u1[t], x1, xx);
            x2 = x1;
            x1 = xx;
            v[t] = xx;
        });
        f1 = v[0];
        f2 = K == 2 ? v[1] : 0.0;
        if (kval) store_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
    }

    // backward: S_j = o_j + G_j H_j, F_j written over o_j
    for (int j1 = full - 1; j1 >= 0; j1 -= SB) {
        // chunks j1, j1-1, .. j1-SB+1 are entries SB-1 .. 0 of the block
        // starting at j1 - SB + 1 (clamped at 0 by the loads)
        const int jb = j1 - SB + 1;
        double hh1[SB], hh2[SB], oo1[SB], oo2[SB];
        const double gms = load_block_mats<K, SB>(Gm, jb < 0 ? 0 : jb, full, lane);
        const double mbs = load_block_mats<K, SB>(Mb, jb < 0 ? 0 : jb, full, lane);
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int j = j1 - b >= 0 ? j1 - b : 0;
            const double *p = x + (int64_t)j * C * ld + kk;
            hh1[b] = p[0];
            hh2[b] = K == 2 ? p[ld] : 0.0;
            oo1[b] = p[(int64_t)K * ld];
            oo2[b] = K == 2 ? p[(int64_t)(K + 1) * ld] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < SB; ++b) {
            const int j = j1 - b;
            if (j >= 0) {
                const int e = j - (jb < 0 ? 0 : jb);   // entry of chunk j in the block
                double s1, s2 = 0.0;
                if constexpr (K == 1) {
                    s1 = fma(lane_value(gms, e), hh1[b], oo1[b]);
                } else {
                    const double g0 = lane_value(gms, 4 * e), g1 = lane_value(gms, 4 * e + 1);
                    const double g2 = lane_value(gms, 4 * e + 2), g3 = lane_value(gms, 4 * e + 3);
                    s1 = fma(g1, hh2[b], fma(g0, hh1[b], oo1[b]));
                    s2 = fma(g3, hh2[b], fma(g2, hh1[b], oo2[b]));
                }
                if (kval) {
                    double *p = x + (int64_t)j * C * ld + k;
                    p[(int64_t)K * ld] = f1;
                    if constexpr (K == 2) p[(int64_t)(K + 1) * ld] = f2;
                }
                affine_lanes<K>(mbs, e, f1, f2, s1, s2);
            }
        }
    }

    if constexpr (CYC) {
        const double rn1 = yn1;
        const double rn2 = K == 2 ? fma(cq.u1_nm2, rn1, yn2) : 0.0;
        double c0 = 0.0, c1 = 0.0;
        correction_scalars<double, K>(cq, f1, f2, rn2, rn1, c0, c1);
        if (kval) {
            for (int j = 0; j < full; ++j) {
                double *p = x + ((int64_t)j * C + 2 * K) * ld + k;
                p[0] = c0;
                if constexpr (K == 2) p[ld] = c1;
            }
            // the tail again, corrected (this lane stored it above)
            double v[C];
            load_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
            const auto tp = lane_table<double, K, C, CYC>(SP::base(tabs), g.P, full);
            rows_up<C>([&](int t) {
                double xx = fma(tp.z0[t], c0, v[t]);
                if constexpr (K == 2) xx = fma(tp.z1[t], c1, xx);
                v[t] = xx;
            });
            store_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
        }
    }
}

template <int K, int C, bool CYC, class Src>
__global__ __launch_bounds__(256) void long_solve(const double *__restrict__ table, LongGeom g,
                                                  Src src, double *x)
{
    const LongWave lw = long_wave(g);
    if (!lw.valid) return;
    const bool kval = lw.k < g.m;
    const int64_t kk = kval ? lw.k : g.m - 1;
    const int row0 = lw.j * C;
    const int64_t ld = g.ld;
    // scratch of this chunk: H (rows 0..K-1), F (K..2K-1), c (2K..3K-1)
    const double *p = x + (int64_t)row0 * ld + kk;
    const double h1 = p[0], h2 = K == 2 ? p[ld] : 0.0;
    const double f1 = p[(int64_t)K * ld], f2 = K == 2 ? p[(int64_t)(K + 1) * ld] : 0.0;
    double c0 = 0.0, c1 = 0.0;
    if constexpr (CYC) {
        c0 = p[(int64_t)2 * K * ld];
        if constexpr (K == 2) c1 = p[(int64_t)(2 * K + 1) * ld];
    }
    double v[C];
    src.template full<C>(v, row0, kk, ld, g.n);
    __builtin_amdgcn_sched_barrier(0);
    {
        const auto tp = long_table<K, C, CYC>(table, g.P, lw.j);
        double y1 = h1, y2 = h2;
        rows_up<C>([&](int t) {
            double y = tp.s[t] * v[t];
            if constexpr (K == 2) y = fma(tp.l2[t], y2, y);
            y = fma(tp.l1[t], y1, y);
            v[t] = y;
            y2 = y1;
            y1 = y;
        });
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        const auto tp = long_table<K, C, CYC>(table, g.P, lw.j);
        double x1 = f1, x2 = f2;
        rows_down<C>([&](int t) {
            double xx = v[t];
            if constexpr (K == 2) xx = fma(tp.u2[t], x2, xx);
            xx = fma(tp.u1[t], x1, xx);
            x2 = x1;
            x1 = xx;
            if constexpr (CYC) {
                xx = fma(tp.z0[t], c0, xx);
                if constexpr (K == 2) xx = fma(tp.z1[t], c1, xx);
            }
            v[t] = xx;
        });
    }
    if (kval) store_chunk<double, C, true>(v, x, row0, lw.k, ld, g.n);
}

// ---------------------------------------------------------------- small batches
// The scan with one wave per system, for batches too small for the
// lane-per-system scan to keep more than a few lanes busy.  The lanes load
// the values of 64 consecutive full chunks at once (lane l: chunk j0 + l),
// keep the loads of the next two such blocks in flight while the current one
// is scanned, and run the chain over a block as a scan of the chunks' affine
// maps across the wave (6 rounds instead of 64 dependent steps); lane l
// stores the state entering its chunk.  The composition rounds differently
// from the lane scan's step-by-step chain (to a few units in the last place
// of the chunk-boundary states); each round trip to memory serves 64 chunks.

// one full chunk's scratch values and matrices, in the lane that holds it
template <int K>
struct SpreadFwd {
    double e1, e2, m[K * K];   // e_j; Mf_j
};
template <int K>
struct SpreadBwd {
    double s1, s2, m[K * K];   // S_j = o_j + G_j H_j; Mb_j
};

template <int K, int C>
__device__ __forceinline__ SpreadFwd<K> spread_fwd(const double *x, const double *Mf, int j,
                                                   int64_t k, int64_t ld)
{
    SpreadFwd<K> v;
    const double *p = x + (int64_t)j * C * ld + k;
    v.e1 = p[0];
    v.e2 = K == 2 ? p[ld] : 0.0;
#pragma unroll
    for (int q = 0; q < K * K; ++q) v.m[q] = Mf[(int64_t)j * K * K + q];
    return v;
}

template <int K, int C>
__device__ __forceinline__ SpreadBwd<K> spread_bwd(const double *x, const double *Mb,
                                                   const double *Gm, int j, int64_t k, int64_t ld)
{
    SpreadBwd<K> v;
    const double *p = x + (int64_t)j * C * ld + k;
    const double h1 = p[0], h2 = K == 2 ? p[ld] : 0.0;
    const double o1 = p[(int64_t)K * ld], o2 = K == 2 ? p[(int64_t)(K + 1) * ld] : 0.0;
    double g[K * K];
#pragma unroll
    for (int q = 0; q < K * K; ++q) {
        g[q] = Gm[(int64_t)j * K * K + q];
        v.m[q] = Mb[(int64_t)j * K * K + q];
    }
    if constexpr (K == 1) {
        v.s1 = fma(g[0], h1, o1);
        v.s2 = 0.0;
    } else {
        v.s1 = fma(g[1], h2, fma(g[0], h1, o1));
        v.s2 = fma(g[3], h2, fma(g[2], h1, o2));
    }
    return v;
}

// The affine map y -> c + M y of one chunk.
template <int K>
struct ChunkMap {
    double m[K * K], c[K];
};

template <int K>
__device__ __forceinline__ ChunkMap<K> identity_map()
{
    ChunkMap<K> a;
#pragma unroll
    for (int q = 0; q < K * K; ++q) a.m[q] = (q % (K + 1) == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int q = 0; q < K; ++q) a.c[q] = 0.0;
    return a;
}

// a <- a after b (b applied first): c = c_a + M_a c_b, M = M_a M_b
template <int K>
__device__ __forceinline__ void compose_after(ChunkMap<K> &a, const ChunkMap<K> &b)
{
    if constexpr (K == 1) {
        a.c[0] = fma(a.m[0], b.c[0], a.c[0]);
        a.m[0] = a.m[0] * b.m[0];
    } else {
        const double c0 = fma(a.m[1], b.c[1], fma(a.m[0], b.c[0], a.c[0]));
        const double c1 = fma(a.m[3], b.c[1], fma(a.m[2], b.c[0], a.c[1]));
        const double m0 = fma(a.m[1], b.m[2], a.m[0] * b.m[0]);
        const double m1 = fma(a.m[1], b.m[3], a.m[0] * b.m[1]);
        const double m2 = fma(a.m[3], b.m[2], a.m[2] * b.m[0]);
        const double m3 = fma(a.m[3], b.m[3], a.m[2] * b.m[1]);
        a.c[0] = c0;
        a.c[1] = c1;
        a.m[0] = m0;
        a.m[1] = m1;
        a.m[2] = m2;
        a.m[3] = m3;
    }
}

template <int K>
__device__ __forceinline__ ChunkMap<K> shfl_up_map(const ChunkMap<K> &a, int d)
{
    ChunkMap<K> b;
#pragma unroll
    for (int q = 0; q < K * K; ++q) b.m[q] = __shfl_up(a.m[q], d, kWave);
#pragma unroll
    for (int q = 0; q < K; ++q) b.c[q] = __shfl_up(a.c[q], d, kWave);
    return b;
}

// The chain over one block: lane l holds the map of the l-th chunk in the
// chain's order (the identity past the block's last chunk).  An inclusive
// scan of the maps across the wave (log2(64) rounds of composition with the
// lane d below) gives every lane the composition of the maps up to its own;
// lane l's entering state is the composition up to lane l-1 applied to y,
// and y leaves as the composition of all 64.
template <int K>
__device__ __forceinline__ void chain_block(ChunkMap<K> a, int lane, double &y1, double &y2,
                                            double &my1, double &my2)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const ChunkMap<K> b = shfl_up_map<K>(a, d);
        if (lane >= d) compose_after<K>(a, b);
    }
    ChunkMap<K> p = shfl_up_map<K>(a, 1);
    if (lane == 0) p = identity_map<K>();
    if constexpr (K == 1) {
        my1 = fma(p.m[0], y1, p.c[0]);
        my2 = 0.0;
        y1 = fma(__shfl(a.m[0], kWave - 1, kWave), y1, __shfl(a.c[0], kWave - 1, kWave));
    } else {
        my1 = fma(p.m[1], y2, fma(p.m[0], y1, p.c[0]));
        my2 = fma(p.m[3], y2, fma(p.m[2], y1, p.c[1]));
        const double t0 = __shfl(a.m[0], kWave - 1, kWave), t1 = __shfl(a.m[1], kWave - 1, kWave);
        const double t2 = __shfl(a.m[2], kWave - 1, kWave), t3 = __shfl(a.m[3], kWave - 1, kWave);
        const double c0 = __shfl(a.c[0], kWave - 1, kWave), c1 = __shfl(a.c[1], kWave - 1, kWave);
        const double n1 = fma(t1, y2, fma(t0, y1, c0));
        const double n2 = fma(t3, y2, fma(t2, y1, c1));
        y1 = n1;
        y2 = n2;
    }
}

// Grid: exactly m workgroups of one wave (system k = blockIdx.x).
template <int K, int C, bool CYC, class Src>
__global__ __launch_bounds__(64) void long_scan_spread(const double *__restrict__ table, CyclicQ cq,
                                                       LongGeom g, Src src, double *x)
{
    using SP = FromScalar<double>;
    const int64_t k = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t ld = g.ld;
    const int full = g.P - 1;
    const int na = num_arrays(K, CYC);
    const int64_t L = (int64_t)g.P * (C + 1);
    const typename SP::ptr tabs = SP::base((typename SP::ptr)table);
    const double *Mf = table + opaque_v(0) + na * L;
    const double *Mb = Mf + (int64_t)g.P * K * K;
    const double *Gm = Mb + (int64_t)g.P * K * K;

    // forward: H_j written over e_j; lane l of block j0 holds chunk j0 + l
    // (clamped to the last full chunk for the loads past it)
    double h1 = 0.0, h2 = 0.0;
    auto fwd_at = [&](int j) { return spread_fwd<K, C>(x, Mf, j < full ? j : full - 1, k, ld); };
    SpreadFwd<K> cur = fwd_at(lane), nxt = fwd_at(kWave + lane);
    for (int j0 = 0; j0 < full; j0 += kWave) {
        const int cnt = full - j0 < kWave ? full - j0 : kWave;
        // two blocks in flight ahead of the chain
        const SpreadFwd<K> nn = fwd_at(j0 + 2 * kWave + lane);
        ChunkMap<K> a = identity_map<K>();
        if (lane < cnt) {
#pragma unroll
            for (int q = 0; q < K * K; ++q) a.m[q] = cur.m[q];
            a.c[0] = cur.e1;
            if constexpr (K == 2) a.c[1] = cur.e2;
        }
        double my1, my2;
        chain_block<K>(a, lane, h1, h2, my1, my2);
        if (lane < cnt) {
            double *p = x + (int64_t)(j0 + lane) * C * ld + k;
            p[0] = my1;
            if constexpr (K == 2) p[ld] = my2;
        }
        cur = nxt;
        nxt = nn;
    }
    // the H_j stored by one lane are read back by another below
    __threadfence_block();

    // the tail chunk (every lane the same; lane 0 stores it, uncorrected if
    // periodic)
    const int trow0 = full * C;
    const int nr = g.n - trow0;
    double yn1, yn2, f1, f2;
    {
        double v[C];
        src.template tail<C>(v, trow0, k, ld, g.n);
        const auto tp = lane_table<double, K, C, CYC>(SP::base(tabs), g.P, full);
        double y1 = h1, y2 = h2;
        rows_up<C>([&](int t) {
            double y = tp.s[t] * v[t];
            if constexpr (K == 2) y = fma(tp.l2[t], y2, y);
            y = fma(tp.l1[t], y1, y);
            v[t] = y;
            y2 = y1;
            y1 = y;
        });
        yn1 = pick(v, nr - 1);
        yn2 = nr >= 2 ? pick(v, nr - 2) : h1;
        double x1 = 0.0, x2 = 0.0;
        rows_down<C>([&](int t) {
            double xx = v[t];
            if constexpr (K == 2) xx = fma(tp.u2[t], x2, xx);
            xx = fma(tp.u1[t], x1, xx);
            x2 = x1;
            x1 = xx;
            v[t] = xx;
        });
        f1 = v[0];
        f2 = K == 2 ? v[1] : 0.0;
        if (lane == 0) store_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
    }

    // backward: F_j written over o_j; lane l of block jt holds chunk jt - l
    // (clamped to chunk 0)
    auto bwd_at = [&](int j) { return spread_bwd<K, C>(x, Mb, Gm, j >= 0 ? j : 0, k, ld); };
    SpreadBwd<K> bcur = bwd_at(full - 1 - lane), bnxt = bwd_at(full - 1 - kWave - lane);
    for (int jt = full - 1; jt >= 0; jt -= kWave) {
        const int cnt = jt + 1 < kWave ? jt + 1 : kWave;
        const SpreadBwd<K> bnn = bwd_at(jt - 2 * kWave - lane);
        ChunkMap<K> a = identity_map<K>();
        if (lane < cnt) {
#pragma unroll
            for (int q = 0; q < K * K; ++q) a.m[q] = bcur.m[q];
            a.c[0] = bcur.s1;
            if constexpr (K == 2) a.c[1] = bcur.s2;
        }
        double my1, my2;
        chain_block<K>(a, lane, f1, f2, my1, my2);
        if (lane < cnt) {
            double *p = x + (int64_t)(jt - lane) * C * ld + k;
            p[(int64_t)K * ld] = my1;
            if constexpr (K == 2) p[(int64_t)(K + 1) * ld] = my2;
        }
        bcur = bnxt;
        bnxt = bnn;
    }

    if constexpr (CYC) {
        const double rn1 = yn1;
        const double rn2 = K == 2 ? fma(cq.u1_nm2, rn1, yn2) : 0.0;
        double c0 = 0.0, c1 = 0.0;
        correction_scalars<double, K>(cq, f1, f2, rn2, rn1, c0, c1);
        for (int j = lane; j < full; j += kWave) {
            double *p = x + ((int64_t)j * C + 2 * K) * ld + k;
            p[0] = c0;
            if constexpr (K == 2) p[ld] = c1;
        }
        if (lane == 0) {
            // the tail again, corrected (this lane stored it above)
            double v[C];
            load_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
            const auto tp = lane_table<double, K, C, CYC>(SP::base(tabs), g.P, full);
            rows_up<C>([&](int t) {
                double xx = fma(tp.z0[t], c0, v[t]);
                if constexpr (K == 2) xx = fma(tp.z1[t], c1, xx);
                v[t] = xx;
            });
            store_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
        }
    }
}

template <int K, int C, bool CYC, class Src>
hipError_t launch_long_c(const double *table, const CyclicQ &q, const LongGeom &g, const Src &src,
                         double *x, hipStream_t s)
{
    constexpr int threads = 256;
    const int64_t waves = (int64_t)(g.P - 1) * g.groups;
    const int64_t blocks = (waves * kWave + threads - 1) / threads;
    const int64_t sblocks = (g.groups * kWave + threads - 1) / threads;
    hipLaunchKernelGGL((long_reduce<K, C, CYC, Src>), dim3((unsigned)blocks), dim3(threads), 0, s,
                       table, g, src, x);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.spread)
        hipLaunchKernelGGL((long_scan_spread<K, C, CYC, Src>), dim3((unsigned)g.m), dim3(kWave), 0,
                           s, table, q, g, src, x);
    else
        hipLaunchKernelGGL((long_scan<K, C, CYC, Src>), dim3((unsigned)sblocks), dim3(threads), 0,
                           s, table, q, g, src, x);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((long_solve<K, C, CYC, Src>), dim3((unsigned)blocks), dim3(threads), 0, s,
                       table, g, src, x);
    return hipGetLastError();
}

template <int K, bool CYC, class Src>
hipError_t launch_long_k(const double *table, const CyclicQ &q, const LongGeom &g, const Src &src,
                         double *x, hipStream_t s)
{
    switch (g.C) {
    case 16: return launch_long_c<K, 16, CYC>(table, q, g, src, x, s);
    case 32: return launch_long_c<K, 32, CYC>(table, q, g, src, x, s);
    case 64: return launch_long_c<K, 64, CYC>(table, q, g, src, x, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace bb
