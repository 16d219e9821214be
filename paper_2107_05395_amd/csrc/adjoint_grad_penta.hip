// adjoint_grad_penta.hip -- pentadiagonal instances of the fused adjoint and
// band gradient of a rollout (adjoint_grad_kernel.h).
#include "adjoint_grad.h"
#include "adjoint_grad_kernel.h"

namespace bb {

hipError_t launch_adjoint_grad_penta(bool cyclic, const double *table, int64_t table_elems,
                                     const CyclicQ &q, const SweepGeom &g, bool scalar,
                                     int64_t steps, const double *lam_in, const double *traj,
                                     int64_t traj_stride, double *lam_out, double *part,
                                     size_t lds, hipStream_t s)
{
    if (cyclic)
        return adjoint_grad_dispatch<2, true>(table, table_elems, q, g, scalar, steps, lam_in, traj,
                                              traj_stride, lam_out, part, lds, s);
    return adjoint_grad_dispatch<2, false>(table, table_elems, q, g, scalar, steps, lam_in, traj,
                                           traj_stride, lam_out, part, lds, s);
}

}  // namespace bb
