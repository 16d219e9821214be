// adjoint_grad.h -- host interface of adjoint_grad.hip: the adjoint recursion
// of a differentiated rollout fused with its band gradients, and the fold of
// per-group partial sums into the gradient (aux.hip).
#pragma once

#include "internal.h"

namespace bb {

// Whether the fused kernel runs the stepper decomposition g (split groups or
// one chunk per wave with scalar coefficients; full decomposition), and its
// LDS bytes.  table_elems: elements of the LDS-staged table (ignored when
// scalar).
bool adjoint_grad_supported(int K, const SweepGeom &g, bool scalar);
size_t adjoint_grad_lds(int K, const SweepGeom &g, bool scalar, int64_t table_elems);

// `steps` transposed solves lam <- A^{-T} lam of the batch (the stepper's
// decomposition and table: each step equals a step of the adjoint trajectory
// bitwise), starting from lam_in; step s (0-based) pairs its adjoint with
// the state at traj + (steps - 1 - s) * traj_stride.  Every group g of S
// systems stores
//   part[(g * (2K+1) + q) * n + i] = -sum_s sum_{k in g} lam_s[i,k] u_s[i+q-K,k]
// (columns outside a non-cyclic matrix: 0) and the last adjoint at lam_out.
// part: g.groups * (2K+1) * n doubles.
hipError_t launch_adjoint_grad(int K, bool cyclic, const double *table, int64_t table_elems,
                               const CyclicQ &q, const SweepGeom &g, bool scalar, int64_t steps,
                               const double *lam_in, const double *traj, int64_t traj_stride,
                               double *lam_out, double *part, hipStream_t s);

// grad[e] += sum over g < groups of part[g * total + e], in a fixed order.
hipError_t launch_grad_fold(int64_t total, int64_t groups, const double *part, double *grad,
                            hipStream_t s);

}  // namespace bb
