// cn_tri.hip -- fused Crank-Nicolson steps with a tridiagonal LHS (periodic
// diffusion, Section 3 benchmark problem); the policy is in cn_stencil.h.
#include "cn_stencil.h"

namespace bb {

hipError_t launch_cn_tri(bool cyclic, const double *table, int64_t table_elems, const CyclicQ &q,
                         const SweepGeom &g, bool scalar, const double *w, int64_t steps,
                         int64_t traj_stride, const double *in, double *out, hipStream_t s)
{
    return launch_cn_k<1>(cyclic, table, table_elems, q, g, scalar, w, steps, traj_stride, in, out, s);
}

hipError_t launch_cn_tri_long(bool cyclic, const double *table, const CyclicQ &q, const LongGeom &g,
                              const double *w, const double *in, double *out, hipStream_t s)
{
    return launch_cn_long_k<1>(cyclic, table, q, g, w, in, out, s);
}

}  // namespace bb
