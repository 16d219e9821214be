// refine_f32rhs.hip -- FP32 sweeps with one FP64-residual refinement for
// FP32 right-hand sides (promoted exactly for the residual), double solution;
// kernel in refine_kernel.h.
#include "refine_kernel.h"

namespace bb {

hipError_t launch_refine_f32rhs(int K, bool cyclic, const void *table, int64_t table_elems,
                                const double *band_table, int64_t band_elems, const CyclicQ &q,
                                const Corners &cn, const SweepGeom &g, const void *in, void *out,
                                hipStream_t s)
{
    if (K == 1)
        return cyclic ? refine_dispatch<1, true, float>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s)
                      : refine_dispatch<1, false, float>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s);
    return cyclic ? refine_dispatch<2, true, float>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s)
                  : refine_dispatch<2, false, float>(table, table_elems, band_table, band_elems, q, cn, g, in, out, s);
}

}  // namespace bb
