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
//   scan   (one lane per system): H_j (prefix over the full chunks,
//          H_{j+1} = e_j + Mf_j H_j) written over e_j; the tail chunk solved
//          in registers from its history H_{P-1}; then S_j = o_j + G_j H_j and
//          the future F_j (suffix, F_{j-1} = S_j + Mb_j F_j, F_{P-2} = the
//          tail's start state) written over o_j; for periodic systems the
//          correction scalars c = Q (w_0, w_1, w_{n-2}, w_{n-1}) written to
//          rows r0+2K .. r0+3K-1 of every full chunk; the tail's solution
//          stored;
//   solve  (one wave per full chunk and group): forward pass from H_j,
//          backward pass from F_j with the correction fused, solution stored
//          over the chunk (the reads of H_j, F_j and c come first).
//
// Every wave of reduce and solve works on one chunk of 64 systems, so each
// row is one 512-byte coalesced access and every coefficient is the same for
// the whole wave: the table is read through the scalar cache and may have
// any size.  HBM traffic: the right-hand side read twice and the solution
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

// Wave w of a reduce or solve launch: chunk j = w / groups (wave-uniform),
// group w % groups, so neighbouring waves read neighbouring 512-byte
// segments of the same rows.
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
    lw.k = (ww % g.groups) * kWave + threadIdx.x % kWave;
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
// The scan with one wave per system: lane l owns full chunks
// [l * cpl, (l + 1) * cpl), composes their affine maps, the wave scans the
// 64 compositions (shuffles, log2(64) steps), and each lane re-walks its
// chunks with its exact history / future.  Every scratch value is loaded at
// once, so the chain over the chunks costs a few round trips instead of one
// per block of chunks; used when the batch is too small for the
// lane-per-system scan to fill the device.  Same scratch protocol and results
// (up to the rounding of the composition order) as long_scan.
constexpr int kWaveScanMax = 8;       // full chunks per lane at most
constexpr int64_t kWaveScanBatch = 256;  // systems up to which the wave scan is used

// y <- M y + e composed as maps: (M, c) after (Ma, ca) is (M Ma, M ca + c)
template <int K>
struct Affine {
    double m[4], c[2];
    __device__ __forceinline__ void identity()
    {
        m[0] = 1.0; m[1] = 0.0; m[2] = 0.0; m[3] = 1.0;
        c[0] = 0.0; c[1] = 0.0;
    }
    // this <- this after a (apply a first)
    __device__ __forceinline__ void after(const Affine &a)
    {
        if constexpr (K == 1) {
            c[0] = fma(m[0], a.c[0], c[0]);
            m[0] = m[0] * a.m[0];
        } else {
            const double c0 = fma(m[1], a.c[1], fma(m[0], a.c[0], c[0]));
            const double c1 = fma(m[3], a.c[1], fma(m[2], a.c[0], c[1]));
            const double m0 = fma(m[1], a.m[2], m[0] * a.m[0]);
            const double m1 = fma(m[1], a.m[3], m[0] * a.m[1]);
            const double m2 = fma(m[3], a.m[2], m[2] * a.m[0]);
            const double m3 = fma(m[3], a.m[3], m[2] * a.m[1]);
            c[0] = c0; c[1] = c1;
            m[0] = m0; m[1] = m1; m[2] = m2; m[3] = m3;
        }
    }
    // this <- (M, e) after this, M a table matrix (row-major K x K)
    template <typename Ptr>
    __device__ __forceinline__ void then(Ptr M, double e1, double e2)
    {
        Affine t;
        t.m[0] = M[0];
        if constexpr (K == 2) { t.m[1] = M[1]; t.m[2] = M[2]; t.m[3] = M[3]; }
        t.c[0] = e1;
        t.c[1] = e2;
        t.after(*this);
        *this = t;
    }
    __device__ __forceinline__ Affine shfl_from(int src) const
    {
        Affine r;
        r.c[0] = __shfl(c[0], src, kWave);
        r.m[0] = __shfl(m[0], src, kWave);
        if constexpr (K == 2) {
            r.c[1] = __shfl(c[1], src, kWave);
            r.m[1] = __shfl(m[1], src, kWave);
            r.m[2] = __shfl(m[2], src, kWave);
            r.m[3] = __shfl(m[3], src, kWave);
        } else {
            r.c[1] = 0.0; r.m[1] = 0.0; r.m[2] = 0.0; r.m[3] = 1.0;
        }
        return r;
    }
};

template <int K, int C, bool CYC, class Src>
__global__ __launch_bounds__(64) void long_scan_wave(const double *__restrict__ table, CyclicQ cq,
                                                     LongGeom g, Src src, double *x)
{
    using SP = FromScalar<double>;
    const int64_t k = blockIdx.x;   // one system per workgroup of one wave
    if (k >= g.m) return;
    const int lane = threadIdx.x;
    const int64_t ld = g.ld;
    const int full = g.P - 1;
    const int cpl = (full + kWave - 1) / kWave;   // <= kWaveScanMax (host checks)
    const int j0 = lane * cpl;
    const int nb = j0 < full ? (full - j0 < cpl ? full - j0 : cpl) : 0;
    const int na = num_arrays(K, CYC);
    const int64_t L = (int64_t)g.P * (C + 1);
    const typename SP::ptr tabs = SP::base((typename SP::ptr)table);
    const typename SP::ptr Mf = tabs + na * L;
    const typename SP::ptr Mb = Mf + (int64_t)g.P * K * K;
    const typename SP::ptr Gm = Mb + (int64_t)g.P * K * K;

    // every scratch value of this lane's chunks, and the tail's rows
    double e1[kWaveScanMax], e2[kWaveScanMax], o1[kWaveScanMax], o2[kWaveScanMax];
#pragma unroll
    for (int b = 0; b < kWaveScanMax; ++b) {
        const int j = b < nb ? j0 + b : 0;
        const double *p = x + (int64_t)j * C * ld + k;
        e1[b] = b < nb ? p[0] : 0.0;
        e2[b] = (K == 2 && b < nb) ? p[ld] : 0.0;
        o1[b] = b < nb ? p[(int64_t)K * ld] : 0.0;
        o2[b] = (K == 2 && b < nb) ? p[(int64_t)(K + 1) * ld] : 0.0;
    }
    const int trow0 = full * C;
    const int nr = g.n - trow0;
    double v[C];
    src.template tail<C>(v, trow0, k, ld, g.n);

    // forward: this lane's composition, the wave's exclusive scan, re-walk
    Affine<K> a;
    a.identity();
    for (int b = 0; b < nb; ++b) {
        const int j = j0 + b;
        a.then(Mf + j * K * K, e1[b], e2[b]);
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Affine<K> o = a.shfl_from(lane >= d ? lane - d : lane);
        if (lane >= d) a.after(o);
    }
    const int prev = lane > 0 ? lane - 1 : 0;
    double h1 = __shfl(a.c[0], prev, kWave), h2 = K == 2 ? __shfl(a.c[1], prev, kWave) : 0.0;
    if (lane == 0) h1 = h2 = 0.0;
    double hh1[kWaveScanMax], hh2[kWaveScanMax];
#pragma unroll
    for (int b = 0; b < kWaveScanMax; ++b) {
        hh1[b] = h1;
        hh2[b] = h2;
        if (b < nb) {
            double *p = x + (int64_t)(j0 + b) * C * ld + k;
            p[0] = h1;
            if constexpr (K == 2) p[ld] = h2;
            const auto M = Mf + (j0 + b) * K * K;
            affine<double, K>(M, h1, h2, e1[b], e2[b]);
        }
    }
    // history of the tail: the inclusive composition of the last lane
    const double th1 = __shfl(a.c[0], kWave - 1, kWave);
    const double th2 = K == 2 ? __shfl(a.c[1], kWave - 1, kWave) : 0.0;

    // the tail, as in long_scan (every lane, identical)
    double yn1, yn2;
    {
        const auto tp = lane_table<double, K, C, CYC>(SP::base(tabs), g.P, full);
        double y1 = th1, y2 = th2;
        rows_up<C>([&](int t) {
            double y = tp.s[t] * v[t];
            if constexpr (K == 2) y = fma(tp.l2[t], y2, y);
            y = fma(tp.l1[t], y1, y);
            v[t] = y;
            y2 = y1;
            y1 = y;
        });
        yn1 = pick(v, nr - 1);
        yn2 = nr >= 2 ? pick(v, nr - 2) : th1;
        double x1 = 0.0, x2 = 0.0;
        rows_down<C>([&](int t) {
            double xx = v[t];
            if constexpr (K == 2) xx = fma(tp.u2[t], x2, xx);
            xx = fma(tp.u1[t], x1, xx);
            x2 = x1;
            x1 = xx;
            v[t] = xx;
        });
    }

    // backward: S_j, this lane's composition (last chunk first), the wave's
    // exclusive scan from the top lane down, re-walk
    double s1[kWaveScanMax], s2[kWaveScanMax];
    Affine<K> bk;
    bk.identity();
#pragma unroll
    for (int b = kWaveScanMax - 1; b >= 0; --b) {
        s1[b] = 0.0;
        s2[b] = 0.0;
        if (b < nb) {
            const auto G = Gm + (j0 + b) * K * K;
            if constexpr (K == 1) {
                s1[b] = fma(G[0], hh1[b], o1[b]);
            } else {
                s1[b] = fma(G[1], hh2[b], fma(G[0], hh1[b], o1[b]));
                s2[b] = fma(G[3], hh2[b], fma(G[2], hh1[b], o2[b]));
            }
            bk.then(Mb + (j0 + b) * K * K, s1[b], s2[b]);
        }
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Affine<K> o = bk.shfl_from(lane + d < kWave ? lane + d : lane);
        if (lane + d < kWave) bk.after(o);
    }
    // F entering this lane's last chunk: the lanes above applied to the
    // tail's start state
    const double ts1 = v[0], ts2 = K == 2 ? v[1] : 0.0;
    const int nxt = lane + 1 < kWave ? lane + 1 : lane;
    Affine<K> up = bk.shfl_from(nxt);
    double f1 = ts1, f2 = ts2;
    if (lane + 1 < kWave) {
        if constexpr (K == 1) {
            f1 = fma(up.m[0], ts1, up.c[0]);
        } else {
            f1 = fma(up.m[1], ts2, fma(up.m[0], ts1, up.c[0]));
            f2 = fma(up.m[3], ts2, fma(up.m[2], ts1, up.c[1]));
        }
    }
#pragma unroll
    for (int b = kWaveScanMax - 1; b >= 0; --b) {
        if (b < nb) {
            double *p = x + (int64_t)(j0 + b) * C * ld + k;
            p[(int64_t)K * ld] = f1;
            if constexpr (K == 2) p[(int64_t)(K + 1) * ld] = f2;
            affine<double, K>(Mb + (j0 + b) * K * K, f1, f2, s1[b], s2[b]);
        }
    }
    // (w_0, w_1): the start state of chunk 0, on lane 0
    double c0 = 0.0, c1 = 0.0;
    if constexpr (CYC) {
        const double w0 = __shfl(f1, 0, kWave), w1 = K == 2 ? __shfl(f2, 0, kWave) : 0.0;
        const double rn1 = yn1;
        const double rn2 = K == 2 ? fma(cq.u1_nm2, rn1, yn2) : 0.0;
        correction_scalars<double, K>(cq, w0, w1, rn2, rn1, c0, c1);
        for (int b = 0; b < nb; ++b) {
            double *p = x + ((int64_t)(j0 + b) * C + 2 * K) * ld + k;
            p[0] = c0;
            if constexpr (K == 2) p[ld] = c1;
        }
        const auto tp = lane_table<double, K, C, CYC>(SP::base(tabs), g.P, full);
        rows_up<C>([&](int t) {
            double xx = fma(tp.z0[t], c0, v[t]);
            if constexpr (K == 2) xx = fma(tp.z1[t], c1, xx);
            v[t] = xx;
        });
    }
    if (lane == 0) store_chunk<double, C, false>(v, x, trow0, k, ld, g.n);
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
    // The wave-per-system scan (long_scan_wave) is not launched: its first
    // GPU run faulted on a periodic pentadiagonal batch (n = 1025, m = 65)
    // and the cause has not been found; every batch takes the lane scan.
    hipLaunchKernelGGL((long_scan<K, C, CYC, Src>), dim3((unsigned)sblocks), dim3(threads), 0, s,
                       table, q, g, src, x);
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
