// adjoint_grad_tri.hip -- the fused adjoint and band gradient of a rollout
// (adjoint_grad_kernel.h): tridiagonal instances, the geometry checks and
// the dispatch on the band count.
#include "adjoint_grad.h"
#include "adjoint_grad_kernel.h"

namespace bb {

hipError_t launch_adjoint_grad_penta(bool cyclic, const double *table, int64_t table_elems,
                                     const CyclicQ &q, const SweepGeom &g, bool scalar,
                                     int64_t steps, const double *lam_in, const double *traj,
                                     int64_t traj_stride, double *lam_out, double *part,
                                     size_t lds, hipStream_t s);

namespace {
int grad_slots_log2(const SweepGeom &g, bool scalar)
{
    return scalar ? 6 : 6 - (g.log2P - g.log2Q);
}
}  // namespace

bool adjoint_grad_supported(int K, const SweepGeom &g, bool scalar)
{
    if (((int64_t)g.C << g.log2P) != g.n) return false;   // chunks tile n
    if (scalar) return g.log2P == g.log2Q && g.log2Q <= 3 && (g.C == 32 || g.C == 64);
    if ((g.C != 32 && g.C != 64) || (g.log2Q != 2 && g.log2Q != 3) || g.log2Q > g.log2P)
        return false;
    const int sl = grad_slots_log2(g, false);
    return K == 1 ? grad_lds_slots_ok<1>(sl) : grad_lds_slots_ok<2>(sl);
}

size_t adjoint_grad_lds(int K, const SweepGeom &g, bool scalar, int64_t table_elems)
{
    const int sl = grad_slots_log2(g, scalar);
    int stage;
    if (K == 1)
        stage = sl == 4 ? grad_stage_len<1, 4>() : sl == 5 ? grad_stage_len<1, 5>() : grad_stage_len<1, 6>();
    else
        stage = sl == 5 ? grad_stage_len<2, 5>() : grad_stage_len<2, 6>();
    const int64_t elems = (scalar ? 0 : table_elems) + split_exchange_len(g.log2Q) +
                          ((int64_t)stage << g.log2Q);
    return (size_t)elems * sizeof(double);
}

hipError_t launch_adjoint_grad(int K, bool cyclic, const double *table, int64_t table_elems,
                               const CyclicQ &q, const SweepGeom &g, bool scalar, int64_t steps,
                               const double *lam_in, const double *traj, int64_t traj_stride,
                               double *lam_out, double *part, hipStream_t s)
{
    if (!adjoint_grad_supported(K, g, scalar) || steps < 1) return hipErrorInvalidValue;
    const size_t lds = adjoint_grad_lds(K, g, scalar, table_elems);
    if (K == 2)
        return launch_adjoint_grad_penta(cyclic, table, table_elems, q, g, scalar, steps, lam_in,
                                         traj, traj_stride, lam_out, part, lds, s);
    if (cyclic)
        return adjoint_grad_dispatch<1, true>(table, table_elems, q, g, scalar, steps, lam_in, traj,
                                              traj_stride, lam_out, part, lds, s);
    return adjoint_grad_dispatch<1, false>(table, table_elems, q, g, scalar, steps, lam_in, traj,
                                           traj_stride, lam_out, part, lds, s);
}

}  // namespace bb
