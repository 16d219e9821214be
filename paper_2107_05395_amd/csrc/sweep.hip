// sweep.hip -- launcher of the batched solve; double instantiations here,
// float ones in sweep_f32.hip, the kernel in sweep_kernel.h.
#include "sweep_kernel.h"

namespace bb {

hipError_t launch_sweep(int K, bool cyclic, Op op, bool f32, const void *table,
                        int64_t table_elems, const double *band_table, int64_t band_elems,
                        const CyclicQ &q, const Corners &cn, const SweepGeom &g, const void *in,
                        void *out, hipStream_t s)
{
    if (op != Op::Solve)
        return launch_refine(K, cyclic, op == Op::RefineF32Rhs, table, table_elems, band_table,
                             band_elems, q, cn, g, in, out, s);
    if (f32) return launch_sweep_f32(K, cyclic, table, table_elems, q, g, in, out, s);
    if (K == 1) return cyclic ? sweep_dispatch<double, 1, true>(table, table_elems, q, g, in, out, s)
                              : sweep_dispatch<double, 1, false>(table, table_elems, q, g, in, out, s);
    return cyclic ? sweep_dispatch<double, 2, true>(table, table_elems, q, g, in, out, s)
                  : sweep_dispatch<double, 2, false>(table, table_elems, q, g, in, out, s);
}

}  // namespace bb
