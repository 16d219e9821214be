// internal.h -- layouts and launch interfaces shared by the host side
// (factor.cpp, api.cpp) and the gfx950 kernels (*.hip) of libbandbatch.
//
// Work decomposition ("chunked sweep")
// ------------------------------------
// The paper gives every system one GPU thread that walks all n rows forward
// and back (Section 2; Appendix A/B batched sweeps), keeping the forward
// intermediate in global memory.  Here a system is split into P contiguous
// chunks of C rows and each chunk is owned by one lane that holds its rows in
// registers, so the right-hand side is read once and the solution written
// once.  A wave of 64 lanes holds S = 64/P systems: lane = chunk * S + sys.
//
// Both sweeps of a banded LU are order-K linear recurrences (K = 1 tri,
// K = 2 penta):
//   forward  y_i = s_i f_i - l1_i y_{i-1} - l2_i y_{i-2}
//   backward x_i = y_i - u1_i x_{i+1} - u2_i x_{i+2}
// The lanes of one system couple only through K numbers at each chunk
// boundary.  Because the matrix is shared, everything about that coupling
// that depends only on A is precomputed once on the host:
//   * the zero-history forward end state e_j and the zero-future backward
//     start state o_j of a chunk are linear in its right-hand side, so each
//     lane gets them as dot products with weight vectors;
//   * chunk transfer matrices Mf_j, Mb_j (KxK) carry a history forward / a
//     future backward across a chunk, and G_j carries the history into the
//     backward start state;
// so a solve is: one dot-product pass, two scans over the P chunks of a
// system (shuffles inside the wave), one forward and one backward pass.
//
// Split groups: when P is large, S = 64/P systems per wave make short row
// segments (S*8 bytes per load instruction).  A system group can instead span
// Q = 2^log2Q waves of one workgroup: each wave holds P/Q chunks of
// S = 64Q/P systems, and the scans read the other waves' boundary states
// through a small LDS exchange area (barriers instead of shuffles).  The
// solve kernel splits any decomposition with C >= 64, the refinement kernel
// only full ones (P*C == n); the fused steppers (stepper.h) split full 32- and
// 64-row decompositions, into one chunk per wave with the coefficients in
// scalar registers up to P = 8, else with the table in LDS.
//
// Coefficient table (one per direction, precision and chunk size)
// ----------------------------------------------------------------
// NA arrays, each L = P*(C+1) elements long; row r = j*C + t of array q is
// element [q*L + j*(C+1) + t] (one pad element per chunk keeps the P chunks of
// a wave in different LDS banks).  Array order (bracketed: K = 2 / cyclic):
//   wE1, [wE2]   weights of e: e_r = sum_t wE_r[t] f_t   (e = (y_end, y_end-1))
//   wS1, [wS2]   weights of o: o_r = sum_t wS_r[t] f_t   (o = (x_start, x_start+1))
//   s, -l1, [-l2], -u1, [-u2], [-z0, [-z1]]
// (off-diagonal coefficients and z stored negated: every step is one fma)
// followed by Mf[P][K][K], Mb[P][K][K], G[P][K][K] (row-major KxK):
//   Mf_j[r][c]: response of y_{end_j - r} to the history component c
//               (history = (y_{end_{j-1}}, y_{end_{j-1}-1}));
//   Mb_j[r][c]: response of x_{start_j + r} to the future component c
//               (future = (x_{start_{j+1}}, x_{start_{j+1}+1}));
//   G_j[r][c]:  response of the zero-future backward start state o_r of the
//               chunk to the forward history component c.
// Rows r >= n are padding: every coefficient 0, so they hold 0 and couple to
// nothing.  Periodic systems: A = A' + U V^T; the table describes A' and the
// correction x = y - Z s, s = Q (y_0..y_{K-1}, y_{n-K}..y_{n-1}) uses the
// per-row z arrays and the K x 2K matrix Q passed by value.
//
// Residual table (refinement only, double): the 2K+1 bands of the original
// matrix in the same padded layout (entries outside the matrix 0; periodic
// corners are passed separately as 'corner').
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bb {

constexpr int kWave = 64;
constexpr int kBlockThreads = 128;      // 2 waves per workgroup for the sweep kernels (measured best)
constexpr int kMaxBlockThreads = 256;   // launch bound: up to 4 waves per workgroup (tuning)

// chunk sizes the sweep kernels are instantiated for
constexpr int kChunkMin = 4;
constexpr int kChunkMax = 128;
constexpr int kChunkMaxRefine = 64;   // the refinement kernel holds 4 words per row
constexpr int kChunkMaxCH = 64;       // fused Cahn-Hilliard steps: two waves per SIMD
// Largest system sizes.  The coefficient tables of a workgroup live in LDS
// (160 KB per CU): a tridiagonal table has up to 6 arrays of n (+pad) values,
// a pentadiagonal one up to 11; at these limits the largest tables (periodic,
// double) take 100 KB (tri, n = 2048) and 92 KB (penta, n = 1024).
constexpr int64_t kMaxN = 2048;
constexpr int64_t kMaxNPenta = 1024;

__host__ __device__ constexpr int num_arrays(int K, bool cyclic) { return 4 * K + 1 + (cyclic ? K : 0); }

inline int64_t table_len(int K, bool cyclic, int C, int P)
{
    return (int64_t)num_arrays(K, cyclic) * P * (C + 1) + 3LL * P * K * K;
}

// Uniform arguments of a sweep launch.
struct SweepGeom {
    int n;          // rows per system
    int C;          // rows per lane (template parameter of the kernel, repeated for checks)
    int log2P;      // lanes per system = 1 << log2P
    int exact;      // n == (number of non-padding chunks) * C
    int64_t m;      // systems
    int64_t ld;     // leading dimension (elements) of the interleaved arrays
    int64_t groups; // ceil(m / S): groups of S systems (one wave each, or 2^log2Q waves when split)
    int lockstep;   // workgroup barrier at the start of every persistent-loop iteration
    int log2Q;      // waves per system group (0: a group is one wave)
    int linear = 0; // one workgroup per block of groups, in launch order (no persistent loop)
};

// Split groups of up to 4 waves, or 8 when the kernel runs two waves per SIMD
// (solve: C <= 64; refinement: C <= 32).
constexpr int kMaxLog2Q = 3;
inline int max_log2q(int C, bool refine) { return (refine ? C > 32 : C > 64) ? 2 : 3; }

// LDS elements of the exchange area of one split group: three phases
// (forward scan: 2 per lane, backward scan: 2, periodic end values: 4).
__host__ __device__ constexpr int64_t split_exchange_len(int log2Q) { return 8LL * kWave << log2Q; }
// ... and of a fourth phase: rows 0, 1, n-2, n-1 of every (chunk, slot).
__host__ __device__ constexpr int64_t split_ends_len(int log2Q) { return 4LL * kWave << log2Q; }

// Tuning overrides of the automatic decomposition choices (measurement and
// tests), process-wide, set through bb_set_tuning; -1 means automatic.
enum TuneKey : int {
    kTuneMaxChunk = 0,       // rows per lane: power of two 4 .. 128
    kTuneWavesPerSystem,     // split-group width 1, 2, 4 or 8 where valid
    kTuneWavesPerBlock,      // waves per workgroup of unsplit sweeps: 1, 2 or 4
    kTuneLockstep,           // 0 / 1: workgroup barrier per persistent iteration
    kTuneChUniform,          // 0: no scalar-coefficient stepper kernel
    kTuneGridLinear,         // 0 / 1: persistent or one-workgroup-per-group grids
    kTuneLongSpread,         // 0 / 1: long-system scan with one lane or one wave per system
    kTuneCount
};
int64_t tuning(TuneKey key);   // api.cpp

struct CyclicQ {
    double q[2][4];   // K x 2K, uses q[0][0..1] for K = 1
    double u1_nm2;    // -u1 of row n-2 (x_{n-2} = y_{n-2} - u1 y_{n-1} at the last chunk)
};

struct Corners {      // periodic corner entries of the original matrix (refinement residual)
    double top[2][2];  // K = 2: A[0][n-2], A[0][n-1]; A[1][n-2], A[1][n-1].  K = 1: top[0][1] = A[0][n-1]
    double bot[2][2];  // K = 2: A[n-2][0], A[n-2][1]; A[n-1][0], A[n-1][1].  K = 1: bot[1][0] = A[n-1][0]
};

// Refine: double right-hand sides; RefineF32Rhs: FP32 right-hand sides.
enum class Op : int { Solve = 0, Refine = 1, RefineF32Rhs = 2 };

// Launch the chunked sweep kernel.
//   T_io / T_sweep: double/double (FP64), float/float (FP32), double/float (refine)
//   table:          device coefficient table in T_sweep (layout above)
//   band_table:     device residual table (double) -- refine only, else nullptr
hipError_t launch_sweep(int K, bool cyclic, Op op, bool f32, const void *table,
                        int64_t table_elems, const double *band_table, int64_t band_elems,
                        const CyclicQ &q, const Corners &corners, const SweepGeom &g,
                        const void *in, void *out, hipStream_t stream);

// Float solves (sweep_f32.hip); launch_sweep forwards f32 here.
hipError_t launch_sweep_f32(int K, bool cyclic, const void *table, int64_t table_elems,
                            const CyclicQ &q, const SweepGeom &g, const void *in, void *out,
                            hipStream_t stream);

// FP32 sweeps + one FP64-residual refinement (refine.hip); launch_sweep
// forwards Op::Refine and Op::RefineF32Rhs here.
hipError_t launch_refine(int K, bool cyclic, bool f32_rhs, const void *table, int64_t table_elems,
                         const double *band_table, int64_t band_elems, const CyclicQ &q,
                         const Corners &corners, const SweepGeom &g, const void *in, void *out,
                         hipStream_t stream);

// The FP32-right-hand-side instantiation (refine_f32rhs.hip); launch_refine
// forwards f32_rhs here.
hipError_t launch_refine_f32rhs(int K, bool cyclic, const void *table, int64_t table_elems,
                                const double *band_table, int64_t band_elems, const CyclicQ &q,
                                const Corners &corners, const SweepGeom &g, const void *in,
                                void *out, hipStream_t stream);

// Cahn-Hilliard steps with the state resident on chip (cyclic penta, double).
// scalar: one 64-row chunk per wave with scalar coefficients (log2Q ==
// log2P <= 3); else log2Q > 0 splits a full decomposition (C = 32, 64) over
// 2^log2Q waves with the table in LDS, and log2Q == 0 keeps one wave per group.
// With partial != nullptr and samples >= 1, also the typical domain size:
// lbar[s] = mean over the m runs of 1 / (1 - <c^2>) after (s + 1) * every
// steps; partial is a workspace of g.groups * samples doubles.
hipError_t launch_ch(const double *table, int64_t table_elems, const CyclicQ &q,
                     const SweepGeom &g, bool scalar, double alpha, int64_t steps,
                     const double *in, double *out, hipStream_t stream, int64_t every = 1,
                     int64_t samples = 0, double *partial = nullptr, double *lbar = nullptr);

// Forced Cahn-Hilliard steps in the frame of the travelling wave
// (ch_forced.hip): per run, the speed v[k], forcing amplitude f0[k] and
// wavenumber k[k] (device arrays of m doubles); alpha = dt / dx^2; scalar /
// log2Q as for launch_ch.
hipError_t launch_ch_forced(const double *table, int64_t table_elems, const CyclicQ &q,
                            const SweepGeom &g, bool scalar, double alpha, double dt, double dx,
                            const double *v, const double *f0, const double *k, int64_t steps,
                            const double *in, double *out, hipStream_t stream);

// Crank-Nicolson steps x <- A^{-1} (B x) with B a constant (2K+1)-point
// stencil w (host array of 2K+1, copied into the kernel arguments), state on
// chip (cn_tri.hip, cn_penta.hip); scalar / log2Q as for launch_ch.
// traj_stride > 0: every step's state, step s at out + s * traj_stride.
hipError_t launch_cn_tri(bool cyclic, const double *table, int64_t table_elems, const CyclicQ &q,
                         const SweepGeom &g, bool scalar, const double *w, int64_t steps,
                         int64_t traj_stride, const double *in, double *out, hipStream_t stream);
hipError_t launch_cn_penta(bool cyclic, const double *table, int64_t table_elems,
                           const CyclicQ &q, const SweepGeom &g, bool scalar, const double *w,
                           int64_t steps, int64_t traj_stride, const double *in, double *out,
                           hipStream_t stream);

// Long systems (long_core.h): n above what one workgroup's LDS table and
// registers hold, solved in three launches (reduce, scan, solve) with the
// solution array as their scratch; FP64 only, x must not overlap the input.
struct LongGeom {
    int n, C, P;        // rows, rows per chunk, chunks (P >= 2; chunk P-1 is the tail)
    int64_t m, ld;      // systems, leading dimension
    int64_t groups;     // groups of 64 systems
    bool spread;        // scan with one wave per system (small batches, m <= kSpreadMax)
    bool halves;        // reduce / solve waves on two 32-system segments (m >= kHalvesMin)
};
constexpr int64_t kHalvesMin = 8192;
// One wave per system scans faster than one lane per system up to 2048 systems
// (32-row chunks) and slower from 4096 on (64-row chunks): the same boundary
// as the chunk size.
constexpr int64_t kSpreadMax = 4095;
constexpr int64_t kMaxNLong = int64_t(1) << 18;
hipError_t launch_long_solve(int K, bool cyclic, const double *table, const CyclicQ &q,
                             const LongGeom &g, const double *rhs, double *x, hipStream_t stream);
// One Cahn-Hilliard step (Section 5.1) of long periodic systems: the
// right-hand side C + alpha d2(C^3 - C) is formed from c_in (with its
// neighbour rows) wherever the launches read it; c_out must not overlap c_in.
hipError_t launch_ch_long(const double *table, const CyclicQ &q, const LongGeom &g, double alpha,
                          const double *c_in, double *c_out, hipStream_t stream);
// One forced Cahn-Hilliard step of long periodic systems (the travelling-wave
// scheme: the Section 5.1 right-hand side plus per-run WENO advection and
// forcing), the right-hand side formed from c_in like launch_ch_long's;
// v, f0, k: device, one per run; c_out must not overlap c_in.
hipError_t launch_ch_forced_long(const double *table, const CyclicQ &q, const LongGeom &g,
                                 double alpha, double dt, double dx, const double *v,
                                 const double *f0, const double *k, const double *c_in,
                                 double *c_out, hipStream_t stream);
// One Crank-Nicolson step of long systems (A c' = B c, B the stencil w of
// 2K+1 weights, periodic when the factor is), the right-hand side formed
// from c_in wherever the long-system launches read it; out must not overlap
// in.
hipError_t launch_cn_tri_long(bool cyclic, const double *table, const CyclicQ &q, const LongGeom &g,
                              const double *w, const double *in, double *out, hipStream_t s);
hipError_t launch_cn_penta_long(bool cyclic, const double *table, const CyclicQ &q, const LongGeom &g,
                                const double *w, const double *in, double *out, hipStream_t s);

// Copy of `bytes` (a multiple of 16) in contiguous 16 KB tiles per workgroup:
// the streaming reference the sweeps' HBM rate is compared with.
hipError_t launch_copy_tiles(const void *src, void *dst, int64_t bytes, hipStream_t stream);
// Copy of an interleaved n x m double array (n a multiple of 128, m of 32)
// with the access pattern of the 64-row-chunk sweeps: their own streaming
// reference.
hipError_t launch_copy_rows(const double *src, double *dst, int n, int64_t m, int64_t ld,
                            hipStream_t stream);

// The paper's thread-per-system mapping (Appendix A), kept as a measured
// baseline design: forward intermediate written to and re-read from `x`.
hipError_t launch_tri_thread_per_system(const double *rhat, const double *aprime,
                                        const double *chat, int n, int64_t m, int64_t ld,
                                        const double *rhs, double *x, hipStream_t stream);

// Batch-reduced band gradients: partial sums per (k-block, band, row), then a
// fixed-order fold into grad (+=).
size_t band_grad_workspace(int nb, int n, int64_t m);
hipError_t launch_band_grad(int nb, bool cyclic, int n, int64_t m, int64_t ld, const double *lam,
                            const double *x, double *grad, void *ws, hipStream_t stream);

// The same reduction with the partial sums in the library's own device array
// (`scratch` in aux.hip, kGradScratchBytes per device, held until the process
// ends): k-blocks per wave raised until the partial sums fit.  No allocation;
// calls that overlap on one device race on the array.
constexpr size_t kGradScratchBytes = (size_t)4 << 20;
hipError_t launch_band_grad_scratch(int nb, bool cyclic, int n, int64_t m, int64_t ld,
                                    const double *lam, const double *x, double *grad,
                                    hipStream_t stream);

size_t mse_workspace(int64_t n, int64_t m);
hipError_t launch_mse(const double *u, const double *target, double *grad, double *loss, int n,
                      int64_t m, int64_t ld, void *ws, hipStream_t stream);

}  // namespace bb
