// sweep_f32.hip -- float instantiations of the batched solve (BB_F32);
// kernel in sweep_kernel.h.
#include "sweep_kernel.h"

namespace bb {

hipError_t launch_sweep_f32(int K, bool cyclic, const void *table, int64_t table_elems,
                            const CyclicQ &q, const SweepGeom &g, const void *in, void *out,
                            hipStream_t s)
{
    if (K == 1) return cyclic ? sweep_dispatch<float, 1, true>(table, table_elems, q, g, in, out, s)
                              : sweep_dispatch<float, 1, false>(table, table_elems, q, g, in, out, s);
    return cyclic ? sweep_dispatch<float, 2, true>(table, table_elems, q, g, in, out, s)
                  : sweep_dispatch<float, 2, false>(table, table_elems, q, g, in, out, s);
}

}  // namespace bb
