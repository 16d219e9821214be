// api.cpp -- the extern "C" boundary of libbandbatch (declared in
// include/bandbatch.h): argument checks, choice of the sweep decomposition,
// lazy upload of the factor's coefficient tables, kernel dispatch.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bandbatch.h"
#include "adjoint_grad.h"
#include "factor.h"
#include "precision.h"

struct bb_factor_s {
    bb::Factor f;
};

namespace {

thread_local std::string g_last_error;

bb_status fail(bb_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

bb_status from_internal(int st, const std::string &err)
{
    switch (st) {
    case bb::kOk: return BB_OK;
    case bb::kErrPivot: return fail(BB_ERR_ZERO_PIVOT, err);
    case bb::kErrCapacitance: return fail(BB_ERR_SINGULAR_CAPACITANCE, err);
    default: return fail(BB_ERR_ARG, err);
    }
}

bb_status hip_fail(hipError_t e, const char *where)
{
    return fail(BB_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Tuning overrides (bb_set_tuning), read at each call; -1 = automatic.
std::atomic<int64_t> g_tuning[bb::kTuneCount] = {{-1}, {-1}, {-1}, {-1}, {-1}, {-1}, {-1}};
const char *const kTuneNames[bb::kTuneCount] = {"max_chunk", "waves_per_system", "waves_per_block",
                                                "lockstep", "ch_uniform", "grid_linear",
                                                "long_spread"};

bool tune_valid(int key, int64_t v)
{
    if (v == -1) return true;
    switch (key) {
    case bb::kTuneMaxChunk: return v >= bb::kChunkMin && v <= bb::kChunkMax && (v & (v - 1)) == 0;
    case bb::kTuneWavesPerSystem: return v == 1 || v == 2 || v == 4 || v == 8;
    case bb::kTuneWavesPerBlock: return v == 1 || v == 2 || v == 4;
    default: return v == 0 || v == 1;
    }
}

// Upper bound on rows per lane.  The sweeps hold C rows of the right-hand side
// per lane in registers; the refinement kernel holds the double input, the
// float first solution and the float correction at once, so it gets half.
// Tuning max_chunk lowers the bound.
int max_chunk(bb_precision p)
{
    int c = bb::kChunkMax;
    if (bb::tuning(bb::kTuneMaxChunk) > 0) c = (int)bb::tuning(bb::kTuneMaxChunk);
    if ((p == BB_F32_REFINE || p == BB_F32_RHS_REFINE) && c > bb::kChunkMaxRefine) c = bb::kChunkMaxRefine;
    return c;
}

// Small batches: with fewer than 2^16 lanes of 64-row chunks in flight (one
// wave per SIMD) a solve or a time step is bound by the latency of its
// dependency chain -- about 3C rows of the three passes plus the scans over
// the P chunks -- not by bandwidth, and shorter chunks win: C = the power of
// two >= 2 sqrt(n), at most 32, as long as that leaves at most 32 chunks per
// system.  Measured (solves captured in a HIP graph, us per tri solve, C = 64
// vs the rule): n = 64, m = 2^12: 6.5 vs 4.0; n = 256, m = 2^10: 7.4 vs 5.9;
// n = 1024, m = 2^6: 14.5 vs 11.3; n = 1024, m = 2^10: 15.5 vs 14.4; not
// applied at n = 2048, m = 2^8 (15.8 at 64 rows, 22.3 at 32).  Fused
// Crank-Nicolson steps, ms per 1000 (m = 2^6 and 2^12): tri n = 64 1.72 vs
// 2.58; n = 256 2.95 vs 3.61; n = 1024 6.2 vs 7.8; penta n = 64 2.35 vs
// 4.14; n = 256 5.5 vs 6.3; n = 1024 12.0 vs 13.6.
int latency_chunk(int64_t n, int64_t m, int C)
{
    if (m * bb::lanes_for(n, C) >= (int64_t(1) << 16)) return C;
    int c = bb::kChunkMin;
    while (c < 32 && (int64_t)c * c < 4 * n) c *= 2;
    const int cc = bb::choose_chunk(n, c);
    return (cc < C && bb::lanes_for(n, cc) <= 32) ? cc : C;
}

// Rows per lane of a solve: 64 (about 170 VGPRs, two waves per SIMD), with
// the system groups split over 4 or 8 waves from 8 chunks on (split_log2).
// Measured against 128 rows per lane (FP64, 4 GiB batches, GB/s, best split
// each): tri n = 512 4881 vs 4749; n = 1024 4771 vs 4490; n = 2048 3975 vs
// 3406; penta n = 1024 4269 vs 3949; ragged tri n = 1000 3992 vs 3701,
// n = 2000 3635 vs 3200, penta n = 1000 3994 vs 3328.  Systems of 64 rows or
// fewer take one lane; small batches follow latency_chunk.
// Tuning max_chunk overrides.
int solve_chunk(int64_t n, int64_t m, bb_precision p)
{
    const int cmax = max_chunk(p);
    if (bb::tuning(bb::kTuneMaxChunk) > 0) return bb::choose_chunk(n, cmax);
    const int C = bb::choose_chunk(n, std::min(cmax, 64));
    return m > 0 ? latency_chunk(n, m, C) : C;
}

// Keep the waves of a workgroup in step at every iteration of the persistent
// loop.  When one wave's segment of a row is shorter than a 128 B line the
// neighbouring wave reads the rest of the line; in step, the second request
// hits in L2 (measured: 64 B segments otherwise re-read 1.7x the bytes).  It
// measured no worse with full-line segments, so it is on for one-wave groups.
// A split group of the solve kernel is its whole workgroup and its exchange
// barriers already keep the waves together: there the extra barrier only
// costs (measured tri n = 1024, m = 2^16: 0.267 vs 0.293 ms), so it is off.
// The refinement kernel keeps it (penta n = 1024 with FP32 right-hand sides:
// 1.46 vs 1.56 ms without).
// Tuning lockstep = 0/1 overrides.
// Grid shape.  Persistent grids (at most one wave of resident workgroups,
// each walking its XCD's share of the groups) serve the kernels that stage
// a coefficient table in LDS, once per workgroup.  The scalar-coefficient
// stepper stages nothing and runs one workgroup per group in launch order
// (measured, CH n = 256, m = 2^20, one step per launch: 0.855 vs 0.953 ms;
// the LDS kernels lose: tri FP32+refine n = 512, m = 2^20 2.64 vs 2.04 ms,
// penta n = 1024 FP64 1.04 vs 0.99 ms).  Tuning grid_linear = 0/1 forces
// persistent / one-per-group grids everywhere (tuning; the launcher reads the
// same setting for the LDS kernels).  Returns -1 when unset.
int grid_linear() { return (int)bb::tuning(bb::kTuneGridLinear); }

int lockstep_for(bool split)
{
    if (bb::tuning(bb::kTuneLockstep) >= 0) return (int)bb::tuning(bb::kTuneLockstep);
    return split ? 0 : 1;
}

// Waves per system group (log2) for C >= 64 (the refinement kernel: full
// decompositions only) -- see internal.h.  Measured on 2^29-element batches and on the 2^16-system
// differentiated workload: the sweep at 64 rows per lane runs fastest with
// 4-wave groups at P = 8 (S = 32) and 8-wave groups from P = 16 on (S = 32,
// 16); at 128 rows (one wave per SIMD) with 4-wave groups from P = 8; the
// refinement kernel (64 rows, one wave per SIMD) with S = 16, i.e. Q = P/4;
// with FP32 right-hand sides (two waves per SIMD for tri) with 4-wave groups
// from P = 4 (tri n = 512: 1.59 vs 1.80 ms at Q = 2).  P <= 4 otherwise keeps
// one wave.
// Tuning waves_per_system = 1, 2, 4 or 8 forces the group size where it is
// valid; otherwise the automatic choice stands.
int split_log2(int log2P, int C, int n, bb::Op op, bool f32_in = false)
{
    const bool refine = op != bb::Op::Solve;
    if (C < 32 || (refine && ((int64_t)C << log2P) != n)) return 0;
    const int lmax = bb::max_log2q(C, refine);
    int l = 0;
    if (op == bb::Op::RefineF32Rhs)   // float input: fewer registers, 4-wave groups from P = 4
        l = log2P >= 2 ? 2 : 0;
    else if (refine)
        l = log2P > 2 ? log2P - 2 : 0;
    else if (C > 64)
        l = log2P >= 3 ? 2 : 0;
    else if (C == 64 && f32_in)
        // FP32 right-hand sides into the FP64 sweep: one chunk of 64 systems
        // per wave from 4 to 8 chunks, so each row is a 256-byte float
        // segment.  Measured, ms (groups of 64 systems against the FP64
        // rule's): tri n = 512, m = 2^20 1.32 vs 1.50; n = 256, m = 2^21
        // 1.33 vs 1.48; penta n = 256, m = 2^20 0.67 vs 0.76; n = 512,
        // m = 2^19 0.71 vs 0.78; not at 2 chunks (tri n = 128: 1.35 vs 1.31)
        l = log2P >= 4 ? 3 : log2P >= 2 ? log2P : 0;
    else if (C == 64)
        l = log2P >= 4 ? 3 : log2P == 3 ? 2 : 0;
    if (l > lmax) l = lmax;
    if (bb::tuning(bb::kTuneWavesPerSystem) > 0) {
        const int64_t q = bb::tuning(bb::kTuneWavesPerSystem);
        const int fl = q == 1 ? 0 : q == 2 ? 1 : q == 4 ? 2 : 3;
        if (fl <= log2P && fl <= lmax) l = fl;
    }
    return l;
}

// Decomposition of the fused steppers (Cahn-Hilliard, Crank-Nicolson).
struct StepPlan {
    int C, P, log2P, log2Q;
    bool scalar;   // one chunk per wave, coefficients through the scalar cache
};

// Rows per lane: 64 (two waves per SIMD), or latency_chunk for small
// batches, or 32 below two waves per SIMD where that keeps one chunk per wave.  Systems split over several waves when the chunks tile n: one
// chunk per wave with scalar coefficients up to 8 chunks, else the LDS table
// with 32 systems per group (4 waves at P = 8, 8 waves from P = 16; n = 1024,
// m = 2^16: 0.063 vs 0.096 ms per tri step over one wave per group).
// Tuning max_chunk, ch_uniform = 0 (no scalar kernel) and waves_per_system =
// 1/2/4/8 override (tuning, testing).
StepPlan step_plan(int64_t n, int64_t m)
{
    int C = bb::choose_chunk(n, std::min(max_chunk(BB_F64), bb::kChunkMaxCH));
    if (bb::tuning(bb::kTuneMaxChunk) < 0) {
        const int64_t lanes64 = m * bb::lanes_for(n, C);
        C = latency_chunk(n, m, C);
        // Fewer than two waves per SIMD at 64 rows: 32-row chunks (still one
        // per wave, scalar coefficients) double the waves.  Measured, ms per
        // 200 fused steps, 64 vs 32 rows: penta n = 64, m = 2^16 0.84 vs
        // 0.71; n = 128, m = 2^15 1.18 vs 0.80; n = 256, m = 2^14 1.22 vs
        // 0.98; CH n = 64, m = 2^16 0.87 vs 0.67; equal or worse from 2^17
        // lanes on.
        if (C == 64 && lanes64 < (int64_t(1) << 17) && 32LL * bb::lanes_for(n, 32) == n &&
            bb::lanes_for(n, 32) <= 8)
            C = 32;
    }
    StepPlan pl;
    pl.C = C;
    pl.P = bb::lanes_for(n, C);
    pl.log2P = 0;
    while ((1 << pl.log2P) < pl.P) ++pl.log2P;
    const bool full = (int64_t)C * pl.P == n;
    pl.scalar = full && C >= 16 && pl.log2P <= 3 && bb::tuning(bb::kTuneChUniform) != 0;
    pl.log2Q = 0;
    if (pl.scalar)
        pl.log2Q = pl.log2P;
    else if (full && C >= 32 && pl.log2P >= 3)
        pl.log2Q = pl.log2P >= 4 ? 3 : 2;
    if (bb::tuning(bb::kTuneWavesPerSystem) > 0 && !pl.scalar && full && C >= 32) {
        const int64_t q = bb::tuning(bb::kTuneWavesPerSystem);
        const int fl = q == 1 ? 0 : q == 2 ? 1 : q == 4 ? 2 : 3;
        if (fl <= pl.log2P) pl.log2Q = fl;
    }
    return pl;
}

bb::SweepGeom step_geom(int64_t n, int64_t m, int64_t ld, const StepPlan &pl)
{
    bb::SweepGeom g;
    g.n = (int)n;
    g.C = pl.C;
    g.log2P = pl.log2P;
    g.exact = (n % pl.C) == 0;
    g.m = m;
    g.ld = ld;
    g.log2Q = pl.log2Q;
    const int S = (bb::kWave << g.log2Q) / pl.P;
    g.groups = (m + S - 1) / S;
    g.lockstep = lockstep_for(g.log2Q > 0);
    g.linear = grid_linear() < 0 ? pl.scalar : grid_linear();
    return g;
}

// Long systems: n above what one workgroup holds (tri 2048, penta 1024: the
// one-launch kernels stage the whole coefficient table in LDS) go through the
// three launches of long_core.h.
bool is_long(const bb::Factor &f) { return f.n > (f.K == 1 ? bb::kMaxN : bb::kMaxNPenta); }

// Rows per chunk of a long solve: 64 for large batches (fewer chunks, so less
// scratch traffic and a shorter scan), 32 for small ones, whose time is the
// latency of a chunk's passes and of the scan.  Tuning max_chunk = 16, 32 or
// 64 overrides.
int long_chunk(int64_t m)
{
    const int64_t v = bb::tuning(bb::kTuneMaxChunk);
    if (v == 16 || v == 32 || v == 64) return (int)v;
    return (m == 0 || m >= 4096) ? 64 : 32;
}

bb::LongGeom long_geom(const bb::Factor &f, int64_t m, int64_t ld, int C)
{
    bb::LongGeom g;
    g.n = (int)f.n;
    g.C = C;
    g.P = (int)((f.n + C - 1) / C);
    g.m = m;
    g.ld = ld;
    g.groups = (m + bb::kWave - 1) / bb::kWave;
    // the scan: one wave per system while that leaves the batch's waves on
    // few enough SIMDs that they run at once (a chain over the chunks in
    // each, 64 chunks per round trip to memory), else one lane per system
    const int64_t sp = bb::tuning(bb::kTuneLongSpread);
    g.spread = sp >= 0 ? sp == 1 : m <= bb::kSpreadMax;
    g.halves = m >= bb::kHalvesMin;
    return g;
}

// Decomposition, device table (the factor's own primal FP64 table for that
// chunk size, shared with the solves) and launch geometry of a fused stepper.
bb_status stepper_setup(bb::Factor &f, int dev, int64_t m, int64_t ld, StepPlan *pl,
                        bb::DeviceTable *tab, bb::SweepGeom *g, bool adjoint = false);

bb_status make(int kind, const double *a, const double *b, const double *c, const double *d,
               const double *e, int64_t n, bb_factor *out)
{
    if (!out) return fail(BB_ERR_ARG, "out is NULL");
    const bool penta = (kind == bb::kPenta || kind == bb::kPentaCyclic);
    if (!a || !b || !c || (penta && (!d || !e))) return fail(BB_ERR_ARG, "band pointer is NULL");
    const int64_t nmin = kind == bb::kTriCyclic ? 3 : kind == bb::kPentaCyclic ? 5 : 1;
    if (n < nmin) return fail(BB_ERR_ARG, "n = " + std::to_string(n) + " is below the minimum " + std::to_string(nmin));
    if (n > bb::kMaxNLong)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(n) + " exceeds bb_max_n() = " +
                                            std::to_string(bb::kMaxNLong));
    bb_factor f = new (std::nothrow) bb_factor_s;
    if (!f) return fail(BB_ERR_OOM, "host allocation");
    const double *bands[5] = {a, b, c, d, e};
    std::string err;
    int st;
    try {
        st = bb::make_factor(kind, bands, n, f->f, err);
    } catch (const std::bad_alloc &) {
        delete f;
        return fail(BB_ERR_OOM, "host allocation");
    }
    if (st != bb::kOk) {
        delete f;
        return from_internal(st, err);
    }
    *out = f;
    g_last_error.clear();
    return BB_OK;
}

bb_status current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return BB_OK;
}

// Device copy of a host table, created on first use per (device, key).
template <typename Key, typename Build>
bb_status device_table(bb::Factor &f, std::map<Key, bb::DeviceTable> &cache, const Key &key,
                       bool as_float, Build build, bb::DeviceTable *out)
{
    std::lock_guard<std::mutex> lock(f.mu);
    auto it = cache.find(key);
    if (it != cache.end()) { *out = it->second; return BB_OK; }
    std::vector<double> host = build();
    bb::DeviceTable t;
    t.elems = (int64_t)host.size();
    const size_t bytes = host.size() * (as_float ? sizeof(float) : sizeof(double));
    hipError_t e = hipMalloc(&t.ptr, bytes ? bytes : 8);
    if (e != hipSuccess) { (void)hipGetLastError(); return fail(BB_ERR_OOM, "hipMalloc of the coefficient table"); }
    if (as_float) {
        std::vector<float> hf(host.begin(), host.end());
        e = hipMemcpy(t.ptr, hf.data(), bytes, hipMemcpyHostToDevice);
    } else {
        e = hipMemcpy(t.ptr, host.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) { (void)hipFree(t.ptr); return hip_fail(e, "hipMemcpy of the coefficient table"); }
    cache[key] = t;
    *out = t;
    return BB_OK;
}

// The table of a long solve: any number of chunks, read through the scalar
// cache (key slot 4 = 2 keeps it apart from the one-launch tables).
bb_status long_table(bb::Factor &f, int dev, bool adjoint, int C, bb::DeviceTable *tab)
{
    const int P = (int)((f.n + C - 1) / C);
    const bb::Direction &dir = adjoint ? f.adjoint : f.primal;
    return device_table(f, f.dev, std::make_tuple(dev, (int)adjoint, 0, C, 2), false,
                        [&] { return bb::build_table(dir, f.K, f.cyclic, f.n, C, P); }, tab);
}

bb_status stepper_too_long(const bb::Factor &f)
{
    return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                        ": the fused steppers hold a system on chip (tri n <= " +
                                        std::to_string(bb::kMaxN) + ", penta n <= " +
                                        std::to_string(bb::kMaxNPenta) + ")");
}

bb_status stepper_setup(bb::Factor &f, int dev, int64_t m, int64_t ld, StepPlan *pl,
                        bb::DeviceTable *tab, bb::SweepGeom *g, bool adjoint)
{
    if (is_long(f)) return stepper_too_long(f);
    *pl = step_plan(f.n, m);
    const int C = pl->C, P = pl->P;
    // the same table as a solve (or adjoint solve) with this chunk size
    const bb::Direction &dir = adjoint ? f.adjoint : f.primal;
    bb_status st = device_table(f, f.dev, std::make_tuple(dev, (int)adjoint, 0, C, 0), false,
                                [&] { return bb::build_table(dir, f.K, f.cyclic, f.n, C, P); },
                                tab);
    if (st != BB_OK) return st;
    *g = step_geom(f.n, m, ld, *pl);
    return BB_OK;
}

bb_status check_batch(bb_factor f, const void *in, const void *out, int64_t m, int64_t ld)
{
    if (!f) return fail(BB_ERR_ARG, "factor is NULL");
    if (m < 0) return fail(BB_ERR_ARG, "m < 0");
    if (ld < (m > 1 ? m : 1)) return fail(BB_ERR_ARG, "ld < max(m, 1)");
    if (m > 0 && (!in || !out)) return fail(BB_ERR_ARG, "device pointer is NULL");
    if (ld > (int64_t(1) << 40)) return fail(BB_ERR_ARG, "ld too large");
    return BB_OK;
}

bb_status solve(bb_factor fh, const void *in, void *out, int64_t m, int64_t ld, bb_precision p,
                void *stream, bool adjoint, int want_k, int want_cyclic)
{
    bb_status st = check_batch(fh, in, out, m, ld);
    if (st != BB_OK) return st;
    bb::Factor &f = fh->f;
    if (f.K != want_k) return fail(BB_ERR_ARG, want_k == 1 ? "not a tridiagonal factor" : "not a pentadiagonal factor");
    if (want_cyclic == 1 && !f.cyclic) return fail(BB_ERR_ARG, "not a cyclic factor");
    if (p != BB_F64 && p != BB_F32_REFINE && p != BB_F32 && p != BB_F32_RHS_REFINE &&
        p != BB_F32_RHS_F64)
        return fail(BB_ERR_ARG, "unknown precision");
    if ((p == BB_F32_RHS_REFINE || p == BB_F32_RHS_F64) && m > 0 && in == out)
        return fail(BB_ERR_ARG, "BB_F32_RHS_REFINE and BB_F32_RHS_F64 read float and write double: "
                                "rhs and x must not overlap");
    if (is_long(f) && p != BB_F64 && p != BB_F32_RHS_F64)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): only BB_F64 and BB_F32_RHS_F64 are "
                                             "built for it");
    if (is_long(f) && m > 0 && in == out)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): x serves as scratch and must not "
                                             "overlap rhs");
    if (m == 0) { g_last_error.clear(); return BB_OK; }
    int dev;
    if ((st = current_device(&dev)) != BB_OK) return st;

    if (is_long(f)) {
        const int C = long_chunk(m);
        bb::DeviceTable tab;
        if ((st = long_table(f, dev, adjoint, C, &tab)) != BB_OK) return st;
        const bb::Direction &dir = adjoint ? f.adjoint : f.primal;
        const bb::LongGeom lg = long_geom(f, m, ld, C);
        hipError_t e = p == BB_F32_RHS_F64
            ? bb::launch_long_solve_f32in(f.K, f.cyclic, (const double *)tab.ptr, dir.cor.q, lg,
                                          (const float *)in, (double *)out, (hipStream_t)stream)
            : bb::launch_long_solve(f.K, f.cyclic, (const double *)tab.ptr, dir.cor.q, lg,
                                    (const double *)in, (double *)out, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "long-system launch");
        g_last_error.clear();
        return BB_OK;
    }

    const int C = solve_chunk(f.n, m, p);
    const int P = bb::lanes_for(f.n, C);
    int log2P = 0;
    while ((1 << log2P) < P) ++log2P;
    const bool f32 = (p != BB_F64 && p != BB_F32_RHS_F64);   // float table
    const bb::Direction &dir = adjoint ? f.adjoint : f.primal;
    bb::DeviceTable tab, band;
    st = device_table(f, f.dev, std::make_tuple(dev, (int)adjoint, (int)f32, C, 0), f32,
                      [&] { return bb::build_table(dir, f.K, f.cyclic, f.n, C, P); }, &tab);
    if (st != BB_OK) return st;
    bb::Corners corners = f.corners;
    bb::Op op = bb::Op::Solve;
    if (p == BB_F32_REFINE || p == BB_F32_RHS_REFINE) {
        op = p == BB_F32_REFINE ? bb::Op::Refine : bb::Op::RefineF32Rhs;
        if (adjoint) {
            // residual of the transposed system: bands and corners of A^T
            st = device_table(f, f.dev, std::make_tuple(dev, 1, 0, C, 1), false,
                              [&] {
                                  bb::Factor t;
                                  t.n = f.n;
                                  t.K = f.K;
                                  const int nb = 2 * f.K + 1;
                                  for (int q = 0; q < nb; ++q) {
                                      t.band[q].assign(f.n, 0.0);
                                      const int off = q - f.K;
                                      // A^T[i][i+off] = A[i+off][i] = band[K-off][i+off]
                                      for (int64_t i = 0; i < f.n; ++i)
                                          if (i + off >= 0 && i + off < f.n)
                                              t.band[q][i] = f.band[2 * f.K - q][i + off];
                                  }
                                  return bb::build_band_table(t, C, P);
                              },
                              &band);
            for (int r = 0; r < 2; ++r)
                for (int q = 0; q < 2; ++q) {
                    // A^T top-right block = (A bottom-left block)^T, and vice versa
                    corners.top[r][q] = f.corners.bot[q][r];
                    corners.bot[r][q] = f.corners.top[q][r];
                }
            if (f.K == 1) {
                corners = bb::Corners{};
                corners.top[0][1] = f.corners.bot[1][0];
                corners.bot[1][0] = f.corners.top[0][1];
            }
        } else {
            st = device_table(f, f.dev, std::make_tuple(dev, 0, 0, C, 1), false,
                              [&] { return bb::build_band_table(f, C, P); }, &band);
        }
        if (st != BB_OK) return st;
    }
    bb::SweepGeom g;
    g.n = (int)f.n;
    g.C = C;
    g.log2P = log2P;
    g.exact = (f.n % C) == 0;
    g.m = m;
    g.ld = ld;
    g.log2Q = split_log2(log2P, C, (int)f.n, op, p == BB_F32_RHS_F64);
    const int S = (bb::kWave << g.log2Q) / P;
    g.groups = (m + S - 1) / S;
    g.lockstep = lockstep_for(g.log2Q > 0 && op == bb::Op::Solve);
    g.linear = grid_linear() > 0;
    hipError_t e = p == BB_F32_RHS_F64
        ? bb::launch_sweep_f32in(f.K, f.cyclic, tab.ptr, tab.elems, dir.cor.q, g, (const float *)in,
                                 (double *)out, (hipStream_t)stream)
        : bb::launch_sweep(f.K, f.cyclic, op, f32 && p == BB_F32, tab.ptr, tab.elems,
                           (const double *)band.ptr, band.elems, dir.cor.q, corners, g, in, out,
                           (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "sweep launch");
    g_last_error.clear();
    return BB_OK;
}

}  // namespace

int64_t bb::tuning(bb::TuneKey key) { return g_tuning[key].load(std::memory_order_relaxed); }

extern "C" {

bb_status bb_set_tuning(const char *name, int64_t value)
{
    if (!name) return fail(BB_ERR_ARG, "name is NULL");
    for (int k = 0; k < bb::kTuneCount; ++k)
        if (std::strcmp(name, kTuneNames[k]) == 0) {
            if (!tune_valid(k, value))
                return fail(BB_ERR_ARG, "value " + std::to_string(value) + " is not valid for " + name);
            g_tuning[k].store(value, std::memory_order_relaxed);
            g_last_error.clear();
            return BB_OK;
        }
    return fail(BB_ERR_ARG, std::string("unknown tuning name: ") + name);
}

int64_t bb_get_tuning(const char *name)
{
    if (name)
        for (int k = 0; k < bb::kTuneCount; ++k)
            if (std::strcmp(name, kTuneNames[k]) == 0) return g_tuning[k].load(std::memory_order_relaxed);
    return -2;
}

bb_status bb_factor_shared_tri(const double *a, const double *b, const double *c, int64_t n,
                               bb_factor *out)
{
    return make(bb::kTri, a, b, c, nullptr, nullptr, n, out);
}

bb_status bb_factor_shared_tri_cyclic(const double *a, const double *b, const double *c, int64_t n,
                                      bb_factor *out)
{
    return make(bb::kTriCyclic, a, b, c, nullptr, nullptr, n, out);
}

bb_status bb_factor_shared_penta(const double *a, const double *b, const double *c, const double *d,
                                 const double *e, int64_t n, bb_factor *out)
{
    return make(bb::kPenta, a, b, c, d, e, n, out);
}

bb_status bb_factor_shared_penta_cyclic(const double *a, const double *b, const double *c,
                                        const double *d, const double *e, int64_t n,
                                        bb_factor *out)
{
    return make(bb::kPentaCyclic, a, b, c, d, e, n, out);
}

bb_status bb_factor_destroy(bb_factor f)
{
    delete f;
    return BB_OK;
}

bb_status bb_factor_upload(bb_factor fh, void *stream)
{
    (void)stream;   // the upload is a blocking copy; it is complete when this returns
    if (!fh) return fail(BB_ERR_ARG, "factor is NULL");
    bb::Factor &f = fh->f;
    int dev;
    bb_status st = current_device(&dev);
    if (st != BB_OK) return st;
    if (is_long(f)) {
        bb::DeviceTable t;
        for (int adj = 0; adj < 2; ++adj)
            if ((st = long_table(f, dev, adj != 0, long_chunk(0), &t)) != BB_OK) return st;
        g_last_error.clear();
        return BB_OK;
    }
    for (bb_precision p : {BB_F64, BB_F32_REFINE}) {
        const int C = solve_chunk(f.n, 0, p);
        const int P = bb::lanes_for(f.n, C);
        const int f32 = p != BB_F64;
        for (int adj = 0; adj < 2; ++adj) {
            const bb::Direction &dir = adj ? f.adjoint : f.primal;
            bb::DeviceTable t;
            st = device_table(f, f.dev, std::make_tuple(dev, adj, f32, C, 0), f32 != 0,
                              [&] { return bb::build_table(dir, f.K, f.cyclic, f.n, C, P); }, &t);
            if (st != BB_OK) return st;
        }
    }
    g_last_error.clear();
    return BB_OK;
}

bb_status bb_plan(bb_factor fh, int64_t m, int32_t what, bb_precision p, int32_t *chunk,
                  int32_t *lanes, int32_t *waves, int32_t *scalar)
{
    if (!fh) return fail(BB_ERR_ARG, "factor is NULL");
    if (m < 1) return fail(BB_ERR_ARG, "m < 1");
    if (what != 0 && what != 1) return fail(BB_ERR_ARG, "what must be 0 (solve) or 1 (fused steps)");
    if (p != BB_F64 && p != BB_F32_REFINE && p != BB_F32 && p != BB_F32_RHS_REFINE &&
        p != BB_F32_RHS_F64)
        return fail(BB_ERR_ARG, "unknown precision");
    const bb::Factor &f = fh->f;
    int C, P, log2Q, sc = 0;
    if (is_long(f)) {
        // three launches, one chunk of 64 systems per wave, coefficients
        // through the scalar cache
        C = long_chunk(m);
        P = (int)((f.n + C - 1) / C);
        log2Q = 0;
        sc = 1;
    } else if (what == 0) {
        C = solve_chunk(f.n, m, p);
        P = bb::lanes_for(f.n, C);
        int log2P = 0;
        while ((1 << log2P) < P) ++log2P;
        const bb::Op op = p == BB_F32_REFINE ? bb::Op::Refine
                        : p == BB_F32_RHS_REFINE ? bb::Op::RefineF32Rhs : bb::Op::Solve;
        log2Q = split_log2(log2P, C, (int)f.n, op, p == BB_F32_RHS_F64);
    } else {
        const StepPlan pl = step_plan(f.n, m);
        C = pl.C;
        P = pl.P;
        log2Q = pl.log2Q;
        sc = pl.scalar ? 1 : 0;
    }
    if (chunk) *chunk = C;
    if (lanes) *lanes = P;
    if (waves) *waves = 1 << log2Q;
    if (scalar) *scalar = sc;
    g_last_error.clear();
    return BB_OK;
}

bb_status bb_factor_info(bb_factor fh, int64_t *n, int32_t *kind, int32_t *chunk)
{
    if (!fh) return fail(BB_ERR_ARG, "factor is NULL");
    if (n) *n = fh->f.n;
    if (kind) *kind = fh->f.kind;
    if (chunk) *chunk = is_long(fh->f) ? long_chunk(0) : solve_chunk(fh->f.n, 0, BB_F64);
    return BB_OK;
}

int64_t bb_max_n(void) { return bb::kMaxNLong; }

bb_status bb_solve_batch_tri(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                             bb_precision p, void *stream)
{
    return solve(f, rhs, x, m, ld, p, stream, false, 1, -1);
}

bb_status bb_solve_batch_penta(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                               bb_precision p, void *stream)
{
    return solve(f, rhs, x, m, ld, p, stream, false, 2, -1);
}

bb_status bb_solve_batch_tri_cyclic(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                                    bb_precision p, void *stream)
{
    return solve(f, rhs, x, m, ld, p, stream, false, 1, 1);
}

bb_status bb_solve_batch_penta_cyclic(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                                      bb_precision p, void *stream)
{
    return solve(f, rhs, x, m, ld, p, stream, false, 2, 1);
}

bb_status bb_solve_batch_tri_adjoint(bb_factor f, const void *g, void *lam, int64_t m, int64_t ld,
                                     bb_precision p, void *stream)
{
    return solve(f, g, lam, m, ld, p, stream, true, 1, -1);
}

bb_status bb_solve_batch_penta_adjoint(bb_factor f, const void *g, void *lam, int64_t m,
                                       int64_t ld, bb_precision p, void *stream)
{
    return solve(f, g, lam, m, ld, p, stream, true, 2, -1);
}

bb_status bb_solve_batch_tri_thread_per_system(bb_factor fh, const double *rhs, double *x,
                                               int64_t m, int64_t ld, void *stream)
{
    bb_status st = check_batch(fh, rhs, x, m, ld);
    if (st != BB_OK) return st;
    bb::Factor &f = fh->f;
    if (f.kind != bb::kTri) return fail(BB_ERR_ARG, "needs a non-cyclic tridiagonal factor");
    if (m == 0) return BB_OK;
    int dev;
    if ((st = current_device(&dev)) != BB_OK) return st;
    bb::DeviceTable t;
    st = device_table(f, f.dev_paper, dev, false,
                      [&] {
                          std::vector<double> h(f.rhat);
                          h.insert(h.end(), f.aprime.begin(), f.aprime.end());
                          h.insert(h.end(), f.chat.begin(), f.chat.end());
                          return h;
                      },
                      &t);
    if (st != BB_OK) return st;
    const double *base = (const double *)t.ptr;
    hipError_t e = bb::launch_tri_thread_per_system(base, base + f.n, base + 2 * f.n, (int)f.n, m,
                                                    ld, rhs, x, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "thread-per-system launch");
    return BB_OK;
}

size_t bb_band_grad_workspace_bytes(bb_factor f, int64_t m)
{
    if (!f || m <= 0) return 0;
    return bb::band_grad_workspace(2 * f->f.K + 1, (int)f->f.n, m);
}

bb_status bb_band_grad(bb_factor fh, const double *lam, const double *x, int64_t m, int64_t ld,
                       double *grad_bands, void *workspace, size_t workspace_bytes, void *stream)
{
    bb_status st = check_batch(fh, lam, x, m, ld);
    if (st != BB_OK) return st;
    if (!grad_bands) return fail(BB_ERR_ARG, "grad_bands is NULL");
    if (m == 0) return BB_OK;
    const bb::Factor &f = fh->f;
    const int nb = 2 * f.K + 1;
    const size_t need = bb::band_grad_workspace(nb, (int)f.n, m);
    if (workspace_bytes < need || (need && !workspace))
        return fail(BB_ERR_ARG, "workspace smaller than bb_band_grad_workspace_bytes()");
    hipError_t e = bb::launch_band_grad(nb, f.cyclic, (int)f.n, m, ld, lam, x, grad_bands,
                                        workspace, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "band-gradient launch");
    return BB_OK;
}

bb_status bb_band_grad_noalloc(bb_factor fh, const double *lam, const double *x, int64_t m,
                               int64_t ld, double *grad_bands, void *stream)
{
    bb_status st = check_batch(fh, lam, x, m, ld);
    if (st != BB_OK) return st;
    if (!grad_bands) return fail(BB_ERR_ARG, "grad_bands is NULL");
    const bb::Factor &f = fh->f;
    const int nb = 2 * f.K + 1;
    if ((size_t)nb * (size_t)f.n * sizeof(double) > bb::kGradScratchBytes)
        return fail(BB_ERR_UNSUPPORTED, "bands x n exceed the library's band-gradient scratch (" +
                                            std::to_string(bb::kGradScratchBytes) + " bytes)");
    if (m == 0) { g_last_error.clear(); return BB_OK; }
    hipError_t e = bb::launch_band_grad_scratch(nb, f.cyclic, (int)f.n, m, ld, lam, x, grad_bands,
                                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "band-gradient launch (library scratch)");
    g_last_error.clear();
    return BB_OK;
}

int64_t bb_band_grad_scratch_bytes(void) { return (int64_t)bb::kGradScratchBytes; }

namespace {

// One row of `samples` partial sums per group of systems of the stepper.
size_t ch_stats_bytes(int64_t n, int64_t m, int64_t samples)
{
    if (samples < 1 || m < 1) return 0;
    const StepPlan pl = step_plan(n, m);
    const bb::SweepGeom g = step_geom(n, m, m, pl);
    return (size_t)g.groups * (size_t)samples * sizeof(double);
}

bb_status ch_steps(bb_factor fh, const double *c_in, double *c_out, int64_t m, int64_t ld,
                   double alpha, int64_t steps, int64_t every, double *lbar, void *workspace,
                   size_t workspace_bytes, void *stream)
{
    bb_status st = check_batch(fh, c_in, c_out, m, ld);
    if (st != BB_OK) return st;
    bb::Factor &f = fh->f;
    if (f.kind != bb::kPentaCyclic) return fail(BB_ERR_ARG, "needs a cyclic pentadiagonal factor");
    if (steps < 1) return fail(BB_ERR_ARG, "steps < 1");
    if (!std::isfinite(alpha)) return fail(BB_ERR_ARG, "alpha is not finite");
    if (every < 1) return fail(BB_ERR_ARG, "every < 1");
    const int64_t samples = lbar ? steps / every : 0;
    if (is_long(f) && (steps != 1 || samples > 0))
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): one step per call, without the "
                                             "statistic");
    if (is_long(f) && m > 0 && c_in == c_out)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): c_out must not overlap c_in");
    if (m == 0) { g_last_error.clear(); return BB_OK; }
    if (samples > 0) {
        if (!workspace) return fail(BB_ERR_ARG, "workspace is NULL");
        if (workspace_bytes < ch_stats_bytes(f.n, m, samples))
            return fail(BB_ERR_ARG, "workspace too small (bb_ch_stats_workspace_bytes)");
    }
    int dev;
    if ((st = current_device(&dev)) != BB_OK) return st;
    if (is_long(f)) {
        const int C = long_chunk(m);
        bb::DeviceTable tab;
        if ((st = long_table(f, dev, false, C, &tab)) != BB_OK) return st;
        hipError_t e = bb::launch_ch_long((const double *)tab.ptr, f.primal.cor.q,
                                          long_geom(f, m, ld, C), alpha, c_in, c_out,
                                          (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "long Cahn-Hilliard launch");
        g_last_error.clear();
        return BB_OK;
    }
    // The fused steps are bound by arithmetic and coefficient reads, not HBM
    // (64 rows per lane, two waves per SIMD: 0.39 vs 0.52 ms per step at
    // n = 256, m = 2^20 against 128 rows per lane); see step_plan.
    StepPlan pl;
    bb::DeviceTable tab;
    bb::SweepGeom g;
    if ((st = stepper_setup(f, dev, m, ld, &pl, &tab, &g)) != BB_OK) return st;
    // with the statistic the persistent grid measured faster (coarsening
    // n = 256, m = 2^20, 2000 steps per launch: 0.209 vs 0.226 ms per step)
    if (samples > 0 && grid_linear() < 0) g.linear = 0;
    hipError_t e = bb::launch_ch((const double *)tab.ptr, tab.elems, f.primal.cor.q, g, pl.scalar,
                                 alpha, steps, c_in, c_out, (hipStream_t)stream, every, samples,
                                 (double *)workspace, lbar);
    if (e != hipSuccess) return hip_fail(e, "Cahn-Hilliard launch");
    g_last_error.clear();
    return BB_OK;
}

}  // namespace

bb_status bb_ch_step(bb_factor fh, const double *c_in, double *c_out, int64_t m, int64_t ld,
                     double alpha, int64_t steps, void *stream)
{
    return ch_steps(fh, c_in, c_out, m, ld, alpha, steps, 1, nullptr, nullptr, 0, stream);
}

size_t bb_ch_stats_workspace_bytes(bb_factor f, int64_t m, int64_t samples)
{
    if (!f || m < 1 || samples < 1) return 0;
    return ch_stats_bytes(f->f.n, m, samples);
}

bb_status bb_ch_step_stats(bb_factor fh, const double *c_in, double *c_out, int64_t m, int64_t ld,
                           double alpha, int64_t steps, int64_t every, double *lbar,
                           void *workspace, size_t workspace_bytes, void *stream)
{
    if (!lbar) return fail(BB_ERR_ARG, "lbar is NULL");
    return ch_steps(fh, c_in, c_out, m, ld, alpha, steps, every, lbar, workspace, workspace_bytes,
                    stream);
}

bb_status bb_ch_forced_step(bb_factor fh, const double *c_in, double *c_out, int64_t m,
                            int64_t ld, double dt, double dx, const double *v, const double *f0,
                            const double *k, int64_t steps, void *stream)
{
    bb_status st = check_batch(fh, c_in, c_out, m, ld);
    if (st != BB_OK) return st;
    bb::Factor &f = fh->f;
    if (f.kind != bb::kPentaCyclic) return fail(BB_ERR_ARG, "needs a cyclic pentadiagonal factor");
    if (steps < 1) return fail(BB_ERR_ARG, "steps < 1");
    if (!(dt > 0.0) || !(dx > 0.0) || !std::isfinite(dt) || !std::isfinite(dx))
        return fail(BB_ERR_ARG, "dt and dx must be finite and positive");
    // the scheme's explicit second difference: dt d2 N ~ (dt / dx^2) (N_{i-1} - 2 N_i + N_{i+1})
    const double alpha = dt / (dx * dx);
    if (!std::isfinite(alpha)) return fail(BB_ERR_ARG, "dt / dx^2 is not finite");
    if (m > 0 && (!v || !f0 || !k)) return fail(BB_ERR_ARG, "parameter pointer is NULL");
    if (is_long(f) && steps != 1)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): one step per call");
    if (is_long(f) && m > 0 && c_in == c_out)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): c_out must not overlap c_in");
    if (m == 0) { g_last_error.clear(); return BB_OK; }
    int dev;
    if ((st = current_device(&dev)) != BB_OK) return st;
    if (is_long(f)) {
        const int C = long_chunk(m);
        bb::DeviceTable tab;
        if ((st = long_table(f, dev, false, C, &tab)) != BB_OK) return st;
        hipError_t e = bb::launch_ch_forced_long((const double *)tab.ptr, f.primal.cor.q,
                                                 long_geom(f, m, ld, C), alpha, dt, dx, v, f0, k,
                                                 c_in, c_out, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "long forced Cahn-Hilliard launch");
        g_last_error.clear();
        return BB_OK;
    }
    StepPlan pl;
    bb::DeviceTable tab;
    bb::SweepGeom g;
    if ((st = stepper_setup(f, dev, m, ld, &pl, &tab, &g)) != BB_OK) return st;
    hipError_t e = bb::launch_ch_forced((const double *)tab.ptr, tab.elems, f.primal.cor.q, g,
                                        pl.scalar, alpha, dt, dx, v, f0, k, steps, c_in, c_out,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "forced Cahn-Hilliard launch");
    g_last_error.clear();
    return BB_OK;
}

bb_status bb_factor_ch(int64_t n, double length, double gamma, double dt, bb_factor *out,
                       double *sigma, double *alpha)
{
    if (!out) return fail(BB_ERR_ARG, "out is NULL");
    if (n < 5) return fail(BB_ERR_ARG, "n must be at least 5");
    if (!(length > 0.0) || !(gamma > 0.0) || !(dt > 0.0) || !std::isfinite(length) ||
        !std::isfinite(gamma) || !std::isfinite(dt))
        return fail(BB_ERR_ARG, "length, gamma and dt must be finite and positive");
    // n periodic points on [0, L): dx = L / n; implicit hyperdiffusion
    // dt gamma d4 C ~ sigma (C_{i-2} - 4 C_{i-1} + 6 C_i - 4 C_{i+1} + C_{i+2})
    const double dx = length / (double)n;
    const double dx2 = dx * dx;
    const double s = gamma * dt / (dx2 * dx2);
    const double a = dt / dx2;
    if (!std::isfinite(s) || !std::isfinite(a)) return fail(BB_ERR_ARG, "coefficients overflow");
    std::vector<double> e(n, s), d(n, -4.0 * s), c(n, 1.0 + 6.0 * s);
    bb_status st = make(bb::kPentaCyclic, e.data(), d.data(), c.data(), d.data(), e.data(), n, out);
    if (st != BB_OK) return st;
    if (sigma) *sigma = s;
    if (alpha) *alpha = a;
    return BB_OK;
}

}  // extern "C"

namespace {

// Fused Crank-Nicolson steps; traj: store every step's state (step s at
// out + s * n * ld) rather than only the last.
bb_status cn_steps(bb_factor fh, const double *w, const double *c_in, double *out, int64_t m,
                   int64_t ld, int64_t steps, bool traj, void *stream, bool adjoint = false)
{
    bb_status st = check_batch(fh, c_in, out, m, ld);
    if (st != BB_OK) return st;
    bb::Factor &f = fh->f;
    if (!w) return fail(BB_ERR_ARG, "stencil pointer is NULL");
    for (int d = 0; d <= 2 * f.K; ++d)
        if (!std::isfinite(w[d])) return fail(BB_ERR_ARG, "stencil weight is not finite");
    if (steps < 1) return fail(BB_ERR_ARG, "steps < 1");
    const int64_t stride = traj ? f.n * ld : 0;
    if (traj && steps > (int64_t(1) << 62) / stride) return fail(BB_ERR_ARG, "steps * n * ld overflows");
    if (is_long(f) && !traj && steps != 1)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): one step per call");
    if (is_long(f) && m > 0 && !traj && c_in == out)
        return fail(BB_ERR_UNSUPPORTED, "n = " + std::to_string(f.n) +
                                             " (long system): c_out must not overlap c_in");
    if (m == 0) { g_last_error.clear(); return BB_OK; }
    int dev;
    if ((st = current_device(&dev)) != BB_OK) return st;
    if (is_long(f)) {
        // one three-launch step per step, each out of place: a trajectory
        // steps from each stored state to the next
        const int C = long_chunk(m);
        bb::DeviceTable tab;
        if ((st = long_table(f, dev, adjoint, C, &tab)) != BB_OK) return st;
        const bb::LongGeom lg = long_geom(f, m, ld, C);
        const bb::CyclicQ &q = adjoint ? f.adjoint.cor.q : f.primal.cor.q;
        double wk[5] = {0, 0, 0, 0, 0};
        for (int d = 0; d <= 2 * f.K; ++d) wk[d] = w[d];
        const double *src = c_in;
        for (int64_t s = 0; s < steps; ++s) {
            double *dst = out + s * stride;
            hipError_t e = f.K == 1
                ? bb::launch_cn_tri_long(f.cyclic, (const double *)tab.ptr, q, lg, wk, src, dst,
                                         (hipStream_t)stream)
                : bb::launch_cn_penta_long(f.cyclic, (const double *)tab.ptr, q, lg, wk, src, dst,
                                           (hipStream_t)stream);
            if (e != hipSuccess) return hip_fail(e, "long-system Crank-Nicolson launch");
            src = dst;
        }
        g_last_error.clear();
        return BB_OK;
    }
    StepPlan pl;
    bb::DeviceTable tab;
    bb::SweepGeom g;
    if ((st = stepper_setup(f, dev, m, ld, &pl, &tab, &g, adjoint)) != BB_OK) return st;
    double wk[5] = {0, 0, 0, 0, 0};
    for (int d = 0; d <= 2 * f.K; ++d) wk[d] = w[d];
    const bb::CyclicQ &q = adjoint ? f.adjoint.cor.q : f.primal.cor.q;
    hipError_t e = f.K == 1
        ? bb::launch_cn_tri(f.cyclic, (const double *)tab.ptr, tab.elems, q, g, pl.scalar, wk,
                            steps, stride, c_in, out, (hipStream_t)stream)
        : bb::launch_cn_penta(f.cyclic, (const double *)tab.ptr, tab.elems, q, g, pl.scalar, wk,
                              steps, stride, c_in, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "Crank-Nicolson launch");
    g_last_error.clear();
    return BB_OK;
}

}  // namespace

extern "C" {

bb_status bb_cn_step(bb_factor fh, const double *w, const double *c_in, double *c_out, int64_t m,
                     int64_t ld, int64_t steps, void *stream)
{
    return cn_steps(fh, w, c_in, c_out, m, ld, steps, false, stream);
}

bb_status bb_cn_trajectory(bb_factor fh, const double *w, const double *c_in, double *traj,
                           int64_t m, int64_t ld, int64_t steps, void *stream)
{
    return cn_steps(fh, w, c_in, traj, m, ld, steps, true, stream);
}

bb_status bb_adjoint_trajectory(bb_factor fh, const double *g, double *traj, int64_t m,
                                int64_t ld, int64_t steps, void *stream)
{
    if (!fh) return fail(BB_ERR_ARG, "factor is NULL");
    double id[5] = {0, 0, 0, 0, 0};
    id[fh->f.K] = 1.0;   // the identity stencil: every step is a plain transposed solve
    return cn_steps(fh, id, g, traj, m, ld, steps, true, stream, true);
}

}  // extern "C"

namespace {

// How bb_adjoint_band_grad runs a batch: the fused kernel where it covers the
// fused stepper's decomposition (and its LDS fits one workgroup), else one
// transposed step and one band-gradient pass per step.  Host only.
struct AdjGradPlan {
    bool fused = false;
    StepPlan pl{};
    bb::SweepGeom g{};
    size_t bytes = 0;   // workspace
};

constexpr size_t kLdsBytes = 160 * 1024;   // LDS of one CU (gfx950)

AdjGradPlan adjoint_grad_plan(const bb::Factor &f, int64_t m, int64_t ld)
{
    AdjGradPlan a;
    const int nb = 2 * f.K + 1;
    if (!is_long(f) && m > 0) {
        a.pl = step_plan(f.n, m);
        a.g = step_geom(f.n, m, ld, a.pl);
        if (bb::adjoint_grad_supported(f.K, a.g, a.pl.scalar)) {
            const int64_t te = bb::table_len(f.K, f.cyclic, a.pl.C, a.pl.P);
            a.fused = bb::adjoint_grad_lds(f.K, a.g, a.pl.scalar, te) <= kLdsBytes;
        }
    }
    if (m <= 0) return a;
    if (a.fused)
        a.bytes = (size_t)a.g.groups * nb * f.n * sizeof(double);
    else   // one adjoint state, then the band-gradient partial sums
        a.bytes = (size_t)f.n * ld * sizeof(double) + bb::band_grad_workspace(nb, (int)f.n, m);
    return a;
}

}  // namespace

extern "C" {

int32_t bb_adjoint_band_grad_fused(bb_factor f, int64_t m)
{
    if (!f || m <= 0) return 0;
    return adjoint_grad_plan(f->f, m, m).fused ? 1 : 0;
}

size_t bb_adjoint_band_grad_workspace_bytes(bb_factor f, int64_t m, int64_t ld)
{
    if (!f || m <= 0 || ld < m) return 0;
    return adjoint_grad_plan(f->f, m, ld).bytes;
}

bb_status bb_adjoint_band_grad(bb_factor fh, const double *g, const double *traj, double *lam,
                               int64_t m, int64_t ld, int64_t steps, double *grad_bands,
                               void *workspace, size_t workspace_bytes, void *stream)
{
    bb_status st = check_batch(fh, g, lam, m, ld);
    if (st != BB_OK) return st;
    if (m > 0 && !traj) return fail(BB_ERR_ARG, "traj is NULL");
    if (!grad_bands) return fail(BB_ERR_ARG, "grad_bands is NULL");
    if (steps < 1) return fail(BB_ERR_ARG, "steps < 1");
    bb::Factor &f = fh->f;
    const int64_t stride = f.n * ld;
    if (steps > (int64_t(1) << 62) / stride) return fail(BB_ERR_ARG, "steps * n * ld overflows");
    if (m == 0) { g_last_error.clear(); return BB_OK; }
    {
        // lam is written while other groups still read traj: no overlap
        const uintptr_t l0 = (uintptr_t)lam, l1 = l0 + (uintptr_t)stride * sizeof(double);
        const uintptr_t t0 = (uintptr_t)traj, t1 = t0 + (uintptr_t)(steps * stride) * sizeof(double);
        if (l0 < t1 && t0 < l1) return fail(BB_ERR_ARG, "lam must not overlap traj");
    }
    const AdjGradPlan a = adjoint_grad_plan(f, m, ld);
    if (workspace_bytes < a.bytes || !workspace)
        return fail(BB_ERR_ARG, "workspace smaller than bb_adjoint_band_grad_workspace_bytes()");
    const int nb = 2 * f.K + 1;
    const hipStream_t s = (hipStream_t)stream;
    if (a.fused) {
        int dev;
        if ((st = current_device(&dev)) != BB_OK) return st;
        StepPlan pl;
        bb::DeviceTable tab;
        bb::SweepGeom geo;
        if ((st = stepper_setup(f, dev, m, ld, &pl, &tab, &geo, true)) != BB_OK) return st;
        double *part = (double *)workspace;
        hipError_t e = bb::launch_adjoint_grad(f.K, f.cyclic, (const double *)tab.ptr, tab.elems,
                                               f.adjoint.cor.q, geo, pl.scalar, steps, g, traj,
                                               stride, lam, part, s);
        if (e != hipSuccess) return hip_fail(e, "fused adjoint and band-gradient launch");
        e = bb::launch_grad_fold((int64_t)nb * f.n, geo.groups, part, grad_bands, s);
        if (e != hipSuccess) return hip_fail(e, "band-gradient fold");
        g_last_error.clear();
        return BB_OK;
    }
    // step by step: the adjoints alternate between the workspace and lam (the
    // first step writes the workspace, so lam may be g), each followed by
    // its band gradients against the state it pairs with
    double *w = (double *)workspace;
    void *bws = (char *)workspace + (size_t)stride * sizeof(double);
    double id[5] = {0, 0, 0, 0, 0};
    id[f.K] = 1.0;   // the identity stencil: plain transposed solves
    const double *src = g;
    for (int64_t t = 1; t <= steps; ++t) {
        double *dst = (t % 2 == 1) ? w : lam;
        if ((st = cn_steps(fh, id, src, dst, m, ld, 1, false, stream, true)) != BB_OK) return st;
        const double *u = traj + (steps - t) * stride;
        hipError_t e = bb::launch_band_grad(nb, f.cyclic, (int)f.n, m, ld, dst, u, grad_bands, bws, s);
        if (e != hipSuccess) return hip_fail(e, "band-gradient launch");
        src = dst;
    }
    if (src != lam) {
        hipError_t e = hipMemcpy2DAsync(lam, ld * sizeof(double), src, ld * sizeof(double),
                                        m * sizeof(double), f.n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "copy of the last adjoint");
    }
    g_last_error.clear();
    return BB_OK;
}

bb_status bb_copy_rows(const double *src, double *dst, int64_t n, int64_t m, int64_t ld,
                       void *stream)
{
    if (n < 0 || m < 0 || n % 128 || m % 32 || n > bb::kMaxNLong)
        return fail(BB_ERR_ARG, "n must be a multiple of 128 and m of 32");
    if (ld < m || ld > (int64_t(1) << 40)) return fail(BB_ERR_ARG, "ld out of range");
    if (n == 0 || m == 0) { g_last_error.clear(); return BB_OK; }
    if (!src || !dst) return fail(BB_ERR_ARG, "NULL pointer");
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    const uintptr_t bytes = (uintptr_t)(n * ld) * sizeof(double);
    if (a < b + bytes && b < a + bytes) return fail(BB_ERR_ARG, "source and destination overlap");
    hipError_t e = bb::launch_copy_rows(src, dst, (int)n, m, ld, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    g_last_error.clear();
    return BB_OK;
}

bb_status bb_copy_tiles(const void *src, void *dst, int64_t bytes, void *stream)
{
    if (bytes < 0 || bytes % 16) return fail(BB_ERR_ARG, "bytes must be a non-negative multiple of 16");
    if (bytes == 0) { g_last_error.clear(); return BB_OK; }
    if (!src || !dst) return fail(BB_ERR_ARG, "NULL pointer");
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(BB_ERR_ARG, "pointers must be 16-byte aligned");
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (bytes > 0 && a < b + (uintptr_t)bytes && b < a + (uintptr_t)bytes)
        return fail(BB_ERR_ARG, "source and destination overlap");
    hipError_t e = bb::launch_copy_tiles(src, dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    g_last_error.clear();
    return BB_OK;
}

size_t bb_mse_workspace_bytes(int64_t n, int64_t m)
{
    if (n <= 0 || m <= 0) return 0;
    return bb::mse_workspace(n, m);
}

bb_status bb_mse_loss_grad(const double *u, const double *target, double *grad, double *loss_dev,
                           int64_t n, int64_t m, int64_t ld, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    if (n < 1 || n > bb::kMaxNLong || m < 1 || ld < m) return fail(BB_ERR_ARG, "bad n, m or ld");
    if (!u || !target || !grad || !loss_dev) return fail(BB_ERR_ARG, "device pointer is NULL");
    const size_t need = bb::mse_workspace(n, m);
    if (workspace_bytes < need || !workspace) return fail(BB_ERR_ARG, "workspace too small");
    hipError_t e = bb::launch_mse(u, target, grad, loss_dev, (int)n, m, ld, workspace,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mse launch");
    return BB_OK;
}

const char *bb_status_string(bb_status s)
{
    switch (s) {
    case BB_OK: return "success";
    case BB_ERR_ARG: return "invalid argument";
    case BB_ERR_ZERO_PIVOT: return "zero or non-finite pivot";
    case BB_ERR_SINGULAR_CAPACITANCE: return "singular periodic-correction capacitance";
    case BB_ERR_HIP: return "HIP runtime error";
    case BB_ERR_OOM: return "out of memory";
    case BB_ERR_UNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

const char *bb_last_error_message(void) { return g_last_error.c_str(); }

}  // extern "C"
