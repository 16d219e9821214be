// refine.hip -- FP32 sweeps with one FP64-residual refinement, double
// right-hand sides; kernel in refine_kernel.h.
#include "refine_kernel.h"

namespace bb {

hipError_t launch_refine(int K, bool cyclic, bool f32_rhs, const void *table, int64_t table_elems,
                         const double *band_table, int64_t band_elems, const CyclicQ &q,
                         const Corners &cn, const SweepGeom &g, const void *in, void *out,
                         hipStream_t s)
{
    if (f32_rhs)
        return launch_refine_f32rhs(K, cyclic, table, table_elems, band_table, band_elems, q, cn, g,
                                    in, out, s);
    if (K == 1)
        return cyclic ? refine_dispatch<1, true, double>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s)
                      : refine_dispatch<1, false, double>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s);
    return cyclic ? refine_dispatch<2, true, double>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s)
                  : refine_dispatch<2, false, double>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s);
}

}  // namespace bb
