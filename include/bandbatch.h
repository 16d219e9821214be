/*
 * bandbatch.h -- C ABI of libbandbatch: batched solution of many tridiagonal or
 * pentadiagonal systems A x_k = b_k, k = 0..m-1, that all share one
 * left-hand-side matrix A, on an AMD Instinct MI355X (gfx950).
 *
 * Method: Carroll, Gloster, Bustamante, O Naraigh, "A Batched GPU Methodology
 * for Numerical Solutions of Partial Differential Equations", arXiv:2107.05395.
 *   - A is factorised once on the host (Section 3.1 Thomas pre-factorisation,
 *     Section 4.1 LR factorisation; Appendix A and B pre-factorisation steps)
 *     and one copy of the factor is kept in device memory (Section 2).
 *   - The right-hand sides are interleaved, batch index fastest (Section 2):
 *     element i of system k lives at [i*ld + k], 0 <= i < n, 0 <= k < m <= ld.
 *   - Every system is swept forward then backward (Section 3.1, 4.1; Appendix A
 *     and B batched sweeps).  Periodic matrices take a Sherman-Morrison
 *     correction (Section 3.3) or its rank-2 Woodbury analogue (Section 5.1
 *     matrix).
 *
 * Conventions for every entry point
 *   - Every call returns a bb_status; no C++ exception crosses the ABI.
 *   - Argument, pivot and capacitance checks run synchronously on the host
 *     before anything is enqueued; on error nothing is enqueued and
 *     bb_last_error_message() (thread-local) says what was wrong.
 *   - Device work is enqueued on `stream` (a hipStream_t; NULL = the default
 *     stream) and the call returns without waiting.  A fault in device code is
 *     reported as BB_ERR_HIP by a later call or by the caller's stream sync.
 *   - Pointers named rhs, x, g, lam, c_in, c_out, grad_bands and workspace are
 *     DEVICE pointers owned by the caller.  Band pointers given to the factor
 *     constructors are HOST pointers, read during the call and not kept.
 *   - In place is allowed wherever input and output have the same type and
 *     layout (x == rhs, lam == g, c_out == c_in); partial overlap is not.
 *   - A bb_factor is immutable after construction and may be used from several
 *     host threads and streams at once.  It owns its host and device memory,
 *     released by bb_factor_destroy().
 */
#ifndef BANDBATCH_H
#define BANDBATCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BB_OK = 0,
    BB_ERR_ARG = -1,                  /* bad size, pointer, precision or factor kind */
    BB_ERR_ZERO_PIVOT = -2,           /* a pivot (b^_i or alpha_i) is 0 or not finite; the method does not pivot */
    BB_ERR_SINGULAR_CAPACITANCE = -3, /* 1 + V.z (or I + V^T Z) of a periodic correction is singular */
    BB_ERR_HIP = -4,                  /* a HIP runtime call failed */
    BB_ERR_OOM = -5,                  /* host or device allocation failed */
    BB_ERR_UNSUPPORTED = -6           /* size outside what the kernels are built for (see bb_max_n) */
} bb_status;

typedef enum {
    BB_F64 = 0,        /* rhs, x and all arithmetic in double */
    BB_F32_REFINE = 1, /* double rhs and x; sweeps in float with the factor rounded to float, then one
                          residual r = b - A x0 in double with the original bands and a float correction
                          sweep: x = x0 + A^{-1} r.  Relative error ~ (kappa eps32)^2 + kappa eps64. */
    BB_F32 = 2,        /* float rhs and x, float sweeps; no refinement */
    BB_F32_RHS_REFINE = 3, /* float rhs (FP32 data, 4 B per entry read), double x: the BB_F32_REFINE
                          sweeps and refinement, the residual taken with the rhs promoted exactly to
                          double.  rhs and x must not overlap. */
    BB_F32_RHS_F64 = 4 /* float rhs (FP32 data, 4 B per entry read), double x: the rhs promoted
                          exactly and solved with the FP64 sweeps and factor of BB_F64 (same
                          decomposition), so x is the FP64 solution of the FP32 data.  rhs and x
                          must not overlap. */
} bb_precision;

typedef struct bb_factor_s *bb_factor;

/* ---------------------------------------------------------------- factors
 * Factorise a shared matrix once, on the host, in double (Section 3.1
 * pre-factorisation; Section 4.1 steps 1-14; Appendix A/B).  The device copy
 * is made lazily on the first solve, or by bb_factor_upload().
 *
 * Tridiagonal row i:   a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = rhs[i].
 *   Non-cyclic: a[0] and c[n-1] are ignored.
 *   Cyclic (indices mod n): a[0] is A[0][n-1], c[n-1] is A[n-1][0] (Section 3.3).
 * Pentadiagonal row i: a[i] x[i-2] + b[i] x[i-1] + c[i] x[i] + d[i] x[i+1] + e[i] x[i+2].
 *   Non-cyclic: a[0], a[1], b[0], d[n-1], e[n-2], e[n-1] are ignored.
 *   Cyclic (indices mod n): those six are the corners (Section 5.1 matrix).
 *
 * Sizes: 1 <= n <= bb_max_n(); cyclic needs 3 <= n (tri) or 5 <= n (penta).
 * Up to n = 2048 (tri) and 1024 (penta) every system of a batch is solved
 * on chip in one launch (its coefficient table staged in LDS).  Longer
 * ("long") systems are solved in three launches (a pass over every chunk of
 * C rows, a scan along each system, a second pass) with the solution array
 * as their scratch: FP64 only, out of place, one (forced) Cahn-Hilliard or
 * Crank-Nicolson step per call (trajectories: one such step per stored state);
 * other requests return BB_ERR_UNSUPPORTED.
 * Errors: BB_ERR_ARG (null pointer, n out of range), BB_ERR_ZERO_PIVOT,
 *         BB_ERR_SINGULAR_CAPACITANCE (cyclic), BB_ERR_OOM.  *out is set only on BB_OK. */
bb_status bb_factor_shared_tri(const double *a, const double *b, const double *c, int64_t n,
                               bb_factor *out);
bb_status bb_factor_shared_tri_cyclic(const double *a, const double *b, const double *c, int64_t n,
                                      bb_factor *out);
bb_status bb_factor_shared_penta(const double *a, const double *b, const double *c, const double *d,
                                 const double *e, int64_t n, bb_factor *out);
bb_status bb_factor_shared_penta_cyclic(const double *a, const double *b, const double *c,
                                        const double *d, const double *e, int64_t n, bb_factor *out);

/* Release a factor and its device copies.  NULL is accepted.  The caller must
 * make sure no enqueued work still uses it (synchronise the streams first). */
bb_status bb_factor_destroy(bb_factor f);

/* Copy the factor's coefficient tables for large batches to the current
 * device now, instead of on the first solve.  The copy is synchronous: the
 * tables are on the device when the call returns, and `stream` is not used
 * (kept so that the call can later be made asynchronous without an ABI
 * change).  A call whose decomposition differs (a small batch: fewer than
 * 2^16 lanes of 64-row chunks; the fused steppers) builds its own table on
 * first use.  That first call allocates device memory; make it before
 * capturing the calls in a HIP graph. */
bb_status bb_factor_upload(bb_factor f, void *stream);

/* Matrix size, kind (0 tri, 1 tri cyclic, 2 penta, 3 penta cyclic) and the
 * number of unknowns per lane ("chunk") the sweeps use for this n on large
 * batches (small batches take shorter chunks).  Any out pointer may be NULL. */
bb_status bb_factor_info(bb_factor f, int64_t *n, int32_t *kind, int32_t *chunk);

/* Largest n a factor may have (262144).  Above n = 2048 (tri) / 1024
 * (penta) the solves take the three-launch path described with the factors. */
int64_t bb_max_n(void);

/* The decomposition a call with m systems takes, without running it: rows per
 * lane (chunk), lanes per system (lanes, a power of two, chunk * lanes >= n),
 * waves per system group (waves: 1, 2, 4 or 8), and for the fused steppers
 * whether the coefficients are read through the scalar cache (scalar; one
 * chunk per wave).  what = 0: a solve or adjoint of precision p; what = 1:
 * the fused steppers (bb_ch_step, bb_ch_step_stats, bb_ch_forced_step,
 * bb_cn_step, bb_cn_trajectory; p is ignored).  Host only: no device is touched.  The tuning
 * variables of the library are honoured.  Any out pointer may be NULL.
 * Errors: BB_ERR_ARG (NULL factor, m < 1, what or p unknown). */
bb_status bb_plan(bb_factor f, int64_t m, int32_t what, bb_precision p, int32_t *chunk,
                  int32_t *lanes, int32_t *waves, int32_t *scalar);

/* ---------------------------------------------------------------- solves
 * x[:,k] = A^{-1} rhs[:,k] for 0 <= k < m (Appendix A/B batched sweeps, with
 * the periodic correction of Section 3.3 when the factor is cyclic).
 * rhs, x: device, interleaved [i*ld + k]; double for BB_F64 and BB_F32_REFINE,
 * float for BB_F32; float rhs and double x for BB_F32_RHS_REFINE and
 * BB_F32_RHS_F64 (same ld).
 * m >= 0 (m == 0 enqueues nothing), ld >= max(m, 1).
 * The tri entry point requires a tri factor (cyclic or not), the penta one a
 * penta factor; the _cyclic names additionally require a cyclic factor.
 * Long systems (n above 2048 tri / 1024 penta): three launches, x is written
 * as scratch before it receives the solution, so x must not overlap rhs;
 * BB_F64 and BB_F32_RHS_F64 only.
 * Errors: BB_ERR_ARG (wrong factor kind, null pointer, m or ld out of range,
 * unknown precision, rhs == x with BB_F32_RHS_REFINE or BB_F32_RHS_F64), BB_ERR_UNSUPPORTED
 * (long system: another precision, or rhs == x), BB_ERR_HIP, BB_ERR_OOM
 * (first upload). */
bb_status bb_solve_batch_tri(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                             bb_precision p, void *stream);
bb_status bb_solve_batch_penta(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                               bb_precision p, void *stream);
bb_status bb_solve_batch_tri_cyclic(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                                    bb_precision p, void *stream);
bb_status bb_solve_batch_penta_cyclic(bb_factor f, const void *rhs, void *x, int64_t m, int64_t ld,
                                      bb_precision p, void *stream);

/* Adjoint (transposed) solve lam[:,k] = A^{-T} g[:,k] with the same shared
 * factor: A = L U gives A^T = U^T L^T, so the sweeps run with the factor's
 * transposed coefficients (for periodic factors the Sherman-Morrison /
 * Woodbury correction is transposed as well).  This is the backward pass of a
 * batched solve: for x = A^{-1} b and a loss L, dL/db = A^{-T} dL/dx.
 * Same layouts, sizes, precisions and errors as the solves. */
bb_status bb_solve_batch_tri_adjoint(bb_factor f, const void *g, void *lam, int64_t m, int64_t ld,
                                     bb_precision p, void *stream);
bb_status bb_solve_batch_penta_adjoint(bb_factor f, const void *g, void *lam, int64_t m,
                                       int64_t ld, bb_precision p, void *stream);

/* The paper's own work mapping, kept as a measured baseline design (Appendix A
 * batched sweep): one thread per system walks all n rows, writing the forward
 * intermediate to x and reading it back in the backward sweep.  Non-cyclic
 * tridiagonal factor, double only; same layouts and errors as the solves.
 * Moves twice the bytes of bb_solve_batch_tri, which keeps every system's
 * intermediate on chip. */
bb_status bb_solve_batch_tri_thread_per_system(bb_factor f, const double *rhs, double *x,
                                               int64_t m, int64_t ld, void *stream);

/* Band gradients of a batched solve: for x = A^{-1} b and lam = A^{-T} dL/dx,
 * dL/dA_ij = -sum_k lam[i,k] x[j,k].  For each band (a..c for tri, a..e for
 * penta, in that order) and row i:
 *     grad_bands[band*n + i] += -sum_k lam[i,k] * x[i + band - nb/2, k]
 * where nb = 3 or 5; entries outside the matrix receive nothing unless the
 * factor is cyclic, where column indices wrap mod n.  Accumulates (+=) into
 * grad_bands (device, nb*n doubles), so calls for several time steps sum.
 * The batch sum runs in a fixed order: results are bitwise reproducible.
 * workspace: device scratch of at least bb_band_grad_workspace_bytes(f, m)
 * bytes, caller-owned; it may be NULL when that size is 0.
 * Errors: BB_ERR_ARG, BB_ERR_HIP. */
size_t bb_band_grad_workspace_bytes(bb_factor f, int64_t m);
bb_status bb_band_grad(bb_factor f, const double *lam, const double *x, int64_t m, int64_t ld,
                       double *grad_bands, void *workspace, size_t workspace_bytes, void *stream);

/* bb_band_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * gradients, accumulated (+=) into grad_bands, with the batch's partial sums
 * kept in a device array of the library instead of a caller workspace.  The
 * array holds bb_band_grad_scratch_bytes() bytes (4 MiB) per device, is made
 * when the library is loaded and lives until the process ends; the call
 * allocates nothing and needs no factor upload.  The batch is cut into at
 * most as many partial groups as fit the array, so the sum order (fixed, and
 * bitwise reproducible from call to call) can differ from bb_band_grad's; the
 * two agree to rounding.  Every call on a device shares that device's array:
 * calls that overlap in time on one device (several streams or host threads)
 * race and must be serialised by the caller.
 * Errors: as bb_band_grad; BB_ERR_UNSUPPORTED when (2K+1) * n doubles exceed
 * the array (n above 174762 for tri, 104857 for penta: beyond every size the
 * solves support). */
bb_status bb_band_grad_noalloc(bb_factor f, const double *lam, const double *x, int64_t m,
                               int64_t ld, double *grad_bands, void *stream);
int64_t bb_band_grad_scratch_bytes(void);

/* ---------------------------------------------------------------- Cahn-Hilliard
 * `steps` semi-implicit Cahn-Hilliard steps (Section 5.1) of m periodic
 * systems:  C^{n+1} + dt gamma d4 C^{n+1} = C^n + dt d2 (C^3 - C)^n, i.e.
 * C^{n+1} = A^{-1} f with f_i = C_i + alpha (N_{i-1} - 2 N_i + N_{i+1}),
 * N = C^3 - C, alpha = dt/dx^2, indices mod n.  `f` must be the cyclic penta
 * factor of the LHS (a = e = sigma, b = d = -4 sigma, c = 1 + 6 sigma,
 * sigma = gamma dt / dx^4).  All `steps` steps of a system run inside one
 * kernel with the state held on chip, reading c_in once and writing c_out once.
 * c_in, c_out: device double, interleaved, same ld.  steps >= 1.
 * Long systems (n > 1024): one step per call, in three launches that form the
 * right-hand side from c_in and its neighbour rows wherever they read it;
 * c_out must not overlap c_in.
 * Errors: BB_ERR_ARG (not a cyclic penta factor, sizes), BB_ERR_UNSUPPORTED
 * (long system with steps > 1 or c_out == c_in), BB_ERR_HIP. */
bb_status bb_ch_step(bb_factor f, const double *c_in, double *c_out, int64_t m, int64_t ld,
                     double alpha, int64_t steps, void *stream);

/* Cahn-Hilliard steps as bb_ch_step plus the coarsening statistic of the
 * ensemble (Section 5, batched 1D scaling): the typical domain size of run k,
 * l_k = 1 / (1 - <C^2>_k) with <C^2>_k = (1/n) sum_i C[i,k]^2, averaged over
 * the m runs, after every `every` steps, computed inside the stepping kernel
 * from the state on chip:
 *     lbar[s] = (1/m) sum_k l_k  after (s + 1) * every steps,  s < steps / every.
 * lbar: device, steps / every doubles (nothing is written when that is 0).
 * workspace: device scratch of at least bb_ch_stats_workspace_bytes(f, m,
 * steps / every) bytes, caller-owned: one row of partial sums per group of
 * runs the kernel handles together (at most m rows, 8 bytes per sample; m/64
 * rows when the chunks tile n into at most 8).  The sums run in a fixed
 * order that does not depend on the device: lbar is bitwise reproducible,
 * and c_out is bitwise what bb_ch_step writes.
 * Errors: as bb_ch_step; BB_ERR_ARG also for every < 1, lbar NULL, or a
 * smaller workspace. */
size_t bb_ch_stats_workspace_bytes(bb_factor f, int64_t m, int64_t samples);
bb_status bb_ch_step_stats(bb_factor f, const double *c_in, double *c_out, int64_t m, int64_t ld,
                           double alpha, int64_t steps, int64_t every, double *lbar,
                           void *workspace, size_t workspace_bytes, void *stream);

/* Forced Cahn-Hilliard steps in the frame of the travelling wave eta = x - vt
 * (the forced flow-pattern section, numerical scheme):
 *     C^{n+1} + dt gamma d4 C^{n+1} = C^n + dt [d2 (C^3 - C)^n + v dC^n/deta
 *                                              + f0 k cos(k eta)],
 * with the second difference of bb_ch_step (alpha = dt / dx^2), the advection
 * term dt v dC/deta taken as (dt v / dx) W_i(C), W_i dx times the fifth-order
 * Hamilton-Jacobi WENO derivative of the run's state at row i, upwinded for
 * dC/dt = v dC/deta (right-biased differences when v > 0, left-biased when
 * v < 0), and the forcing at eta_i = i dx.
 * Per run k: speed v[k], forcing amplitude f0[k] and wavenumber k[k] (device,
 * m doubles each); dt and dx are shared.  `f` must be the cyclic penta factor
 * of the Cahn-Hilliard LHS for the same dt and dx (bb_factor_ch).
 * c_in, c_out: device double, interleaved, same ld; in place allowed.  All
 * `steps` steps run inside one kernel with the state on chip.  Long systems
 * (n > 1024): one step per call in the three long-system launches, the
 * right-hand side formed inside them from c_in; out of place.
 * Errors: BB_ERR_ARG (not a cyclic penta factor, NULL parameters, dt or dx not
 * finite and positive, sizes), BB_ERR_UNSUPPORTED (long system with
 * steps != 1 or c_out == c_in), BB_ERR_HIP. */
bb_status bb_ch_forced_step(bb_factor f, const double *c_in, double *c_out, int64_t m, int64_t ld,
                            double dt, double dx, const double *v, const double *f0,
                            const double *k, int64_t steps, void *stream);

/* The semi-implicit Cahn-Hilliard scheme of Section 5.1 on n periodic grid
 * points of a domain of length L (dx = L / n): factorise its left-hand side,
 * the cyclic pentadiagonal matrix with a = e = sigma, b = d = -4 sigma,
 * c = 1 + 6 sigma, sigma = gamma dt / dx^4 (the implicit fourth difference),
 * and return sigma and alpha = dt / dx^2 (the explicit second difference of
 * C^3 - C, the alpha of bb_ch_step).  sigma, alpha: host, may be NULL.
 * Errors: BB_ERR_ARG (n < 5, length, gamma or dt not finite and positive),
 * BB_ERR_UNSUPPORTED (n above bb_max_n()), BB_ERR_OOM. */
bb_status bb_factor_ch(int64_t n, double length, double gamma, double dt, bb_factor *out,
                       double *sigma, double *alpha);

/* ---------------------------------------------------------------- Crank-Nicolson
 * `steps` Crank-Nicolson steps of m systems (Section 3 benchmark problem:
 * periodic diffusion; Section 4 benchmark problem: periodic hyperdiffusion):
 *     A C^{n+1} = B C^n,   (B C)_i = sum_{d=-K..K} w[d+K] C_{i+d},
 * with A the factor's matrix, K = 1 (tridiagonal factor) or 2 (pentadiagonal).
 * Cyclic factor: the indices of B wrap mod n like A.  Otherwise the terms of
 * B whose row falls outside 0..n-1 are left out (zero boundary values).
 *   diffusion:      A rows (-s, 1 + 2s, -s),           w = (s, 1 - 2s, s),            s = dt/(2 dx^2)
 *   hyperdiffusion: A rows (s, -4s, 1 + 6s, -4s, s),   w = (-s, 4s, 1 - 6s, 4s, -s),  s = dt/(2 dx^4)
 * All `steps` steps of a system run inside one kernel with the state held on
 * chip, reading c_in once and writing c_out once; steps = 1 per call gives the
 * one-launch-per-step form (one read and one write of the batch per step).
 * w: host, 2K+1 finite doubles, read before the call returns.
 * c_in, c_out: device double, interleaved, same ld; c_in == c_out is allowed
 * (in place), any other overlap is not.  steps >= 1.  Long systems: one step
 * per call (three launches, the right-hand side formed inside them), out of
 * place.
 * Errors: BB_ERR_ARG (w NULL or not finite, steps, sizes), BB_ERR_UNSUPPORTED
 * (long system with steps != 1 or c_out == c_in), BB_ERR_HIP. */
bb_status bb_cn_step(bb_factor f, const double *w, const double *c_in, double *c_out, int64_t m,
                     int64_t ld, int64_t steps, void *stream);

/* The same steps, keeping every state: the state after step s (s = 0 ..
 * steps-1) goes to traj + s * n * ld, each an interleaved n x ld array like
 * c_in.  One kernel for all steps, reading c_in once and writing each state
 * once; the states are bitwise those of `steps` calls of bb_cn_step with
 * steps = 1 (same kernel and decomposition).  With w the identity (w[K] = 1,
 * the rest 0) this is a trajectory of implicit solves A u_{s+1} = u_s, which
 * the recomputation between checkpoints of a differentiated rollout uses.
 * traj: device double, steps * n * ld elements, not overlapping c_in.  Long
 * systems: one three-launch step per state, each from the state before it.
 * Errors: as bb_cn_step, and BB_ERR_ARG if steps * n * ld overflows. */
bb_status bb_cn_trajectory(bb_factor f, const double *w, const double *c_in, double *traj,
                           int64_t m, int64_t ld, int64_t steps, void *stream);

/* The adjoint recursion of `steps` implicit steps, lam_{s+1} = A^{-T} lam_s
 * (s = 0 .. steps-1, lam_0 = g), with the same shared factor as the solves
 * (A^T = U^T L^T, the transposed solve of bb_solve_batch_*_adjoint), in one
 * launch of the fused stepper with the state on chip: lam_{s+1} goes to
 * traj + s * n * ld.  This is the backward pass of a rollout
 * u_{t+1} = A^{-1} u_t: for a loss of u_T, lam_s = dL/du_{T-s}.  Reads g once
 * and writes each state once (long systems: one three-launch transposed
 * solve per state).  Same sizes, layouts and errors as bb_cn_trajectory
 * (g, traj: device double; traj must not overlap g). */
bb_status bb_adjoint_trajectory(bb_factor f, const double *g, double *traj, int64_t m,
                                int64_t ld, int64_t steps, void *stream);

/* The backward pass over one stretch of a rollout u_t = A^{-1} u_{t-1}
 * (t = 1 .. T, T = steps), adjoints and band gradients together: the adjoint
 * recursion of bb_adjoint_trajectory, d_{t-1} = A^{-T} d_t from d_T = g
 * (d_t = dL/du_t), fused with the reduction of bb_band_grad for every step,
 *     grad_bands[band*n + i] += -sum_t sum_k d_{t-1}[i,k] u_t[i + band - nb/2, k]
 * (the adjoint of each solve is A^{-T} d_t = d_{t-1}; nb = 3 or 5; entries
 * outside a non-cyclic matrix receive nothing, cyclic column indices wrap mod
 * n).  This is the FP64 backward of a checkpointed differentiable rollout
 * (the adjoint recursion and its gradient with respect to the shared bands,
 * the extension of the batched solves to gradients).  Outputs d_0 = dL/du_0 at lam.
 * traj: the forward states u_1 .. u_T, state u_t at traj + (t-1) * n * ld
 * (what bb_cn_trajectory writes from u_0 with the identity stencil); g, lam:
 * interleaved n x ld, lam may be g, traj must not overlap lam.
 * Where the fused steppers hold a system on chip in split groups or one chunk
 * per wave (bb_adjoint_band_grad_fused), one kernel steps the adjoints with
 * each chunk in registers and reduces d_{t-1} u_t over each group's systems
 * after every step: it reads g and every u_t once and writes lam and the
 * groups' partial sums once (no adjoint states in memory), then a
 * fixed-order fold adds the groups into grad_bands.  Otherwise each step is a
 * transposed solve into the workspace or lam followed by bb_band_grad's
 * reduction.  The adjoints equal bb_adjoint_trajectory's bitwise; the band
 * gradients sum in a fixed order (bitwise reproducible), which differs
 * between the two paths, so they agree with bb_band_grad's to rounding.
 * workspace: device scratch of at least
 * bb_adjoint_band_grad_workspace_bytes(f, m, ld) bytes, caller-owned.
 * Errors: BB_ERR_ARG (null pointer, sizes, steps < 1, workspace too small,
 * lam overlapping traj), BB_ERR_HIP, BB_ERR_OOM (first table upload). */
bb_status bb_adjoint_band_grad(bb_factor f, const double *g, const double *traj, double *lam,
                               int64_t m, int64_t ld, int64_t steps, double *grad_bands,
                               void *workspace, size_t workspace_bytes, void *stream);
size_t bb_adjoint_band_grad_workspace_bytes(bb_factor f, int64_t m, int64_t ld);
/* 1 if bb_adjoint_band_grad with m systems runs the fused kernel, else 0
 * (host only). */
int32_t bb_adjoint_band_grad_fused(bb_factor f, int64_t m);

/* ---------------------------------------------------------------- measurement
 * A measurement utility, not part of the method: copy `bytes` from src to
 * dst (device, 16-byte aligned, not overlapping; bytes a multiple of 16) with
 * each workgroup moving one contiguous 16 KB tile, its loads issued before
 * its stores -- the fastest plain read + write stream found on this part,
 * which benchmarks time beside the sweeps as their HBM reference.  bytes = 0
 * does nothing (the pointers may then be NULL).
 * Errors: BB_ERR_ARG (NULL, alignment, size, overlap), BB_ERR_HIP. */
bb_status bb_copy_tiles(const void *src, void *dst, int64_t bytes, void *stream);

/* A measurement utility, not part of the method: copy the interleaved n x m
 * double array src (element (i,k) at [i*ld + k]) to dst with the access
 * pattern of the FP64 sweeps -- every wave moves 64 rows of two 32-system
 * segments 64 rows apart (256 contiguous bytes per segment and row), all its
 * loads issued before its stores -- the ceiling that pattern sets on a solve
 * that reads b and writes x once.  n a multiple of 128, m of 32, ld >= m;
 * src and dst must not overlap (n * ld doubles each).
 * Errors: BB_ERR_ARG, BB_ERR_HIP. */
bb_status bb_copy_rows(const double *src, double *dst, int64_t n, int64_t m, int64_t ld,
                       void *stream);

/* ---------------------------------------------------------------- loss
 * Mean-squared-error loss of a batch against a target and its gradient:
 *   grad[i,k] = 2 (u[i,k] - target[i,k]) / (n m),
 *   partial sums of (u - target)^2 are written to workspace and folded in a
 *   fixed order into *loss_dev = sum (u - target)^2 / (n m)   (device double).
 * grad may alias u.  workspace: bb_mse_workspace_bytes(n, m) bytes.
 * Errors: BB_ERR_ARG, BB_ERR_HIP. */
size_t bb_mse_workspace_bytes(int64_t n, int64_t m);
bb_status bb_mse_loss_grad(const double *u, const double *target, double *grad, double *loss_dev,
                           int64_t n, int64_t m, int64_t ld, void *workspace,
                           size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- tuning
 * Process-wide overrides of the decomposition choices, for measurement and
 * tests; results never depend on them beyond rounding (on max_chunk) and not
 * at all on the others.  value -1 restores the automatic choice.
 *   "max_chunk"         rows per lane, power of two 4 .. 128 (long systems: 16,
 *                       32 or 64; other values leave them automatic)
 *   "waves_per_system"  waves per split system group: 1, 2, 4 or 8 where valid
 *   "waves_per_block"   waves per workgroup of unsplit sweeps: 1, 2 or 4
 *   "lockstep"          0 / 1: a workgroup barrier at every persistent iteration
 *   "ch_uniform"        0: the fused steppers never read coefficients through
 *                       the scalar cache
 *   "grid_linear"       0 / 1: persistent grids / one workgroup per group
 *   "long_spread"       0 / 1: the scan of long systems with one lane per system
 *                       / one wave per system (automatic: a wave for m < 4096)
 * The settings are read when a call enqueues its launches; change them only
 * between calls.  Errors: BB_ERR_ARG (unknown name, invalid value). */
bb_status bb_set_tuning(const char *name, int64_t value);
/* The current value of a setting (-1: automatic), or -2 for an unknown name. */
int64_t bb_get_tuning(const char *name);

/* ---------------------------------------------------------------- errors */
const char *bb_status_string(bb_status s);
/* Detail of the last error raised on the calling thread ("" if none). */
const char *bb_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* BANDBATCH_H */
