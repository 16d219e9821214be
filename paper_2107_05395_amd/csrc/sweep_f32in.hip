// sweep_f32in.hip -- FP32 right-hand sides solved with the FP64 sweeps and
// factor (BB_F32_RHS_F64): each value is promoted exactly on load, so the
// result is the FP64 solve of the FP32 data, with 4 instead of 8 bytes read
// per row; kernel in sweep_kernel.h.
#include "precision.h"
#include "sweep_kernel.h"

namespace bb {

hipError_t launch_sweep_f32in(int K, bool cyclic, const void *table, int64_t table_elems,
                              const CyclicQ &q, const SweepGeom &g, const float *in, double *out,
                              hipStream_t s)
{
    if (K == 1)
        return cyclic ? sweep_dispatch<double, 1, true, float>(table, table_elems, q, g, in, out, s)
                      : sweep_dispatch<double, 1, false, float>(table, table_elems, q, g, in, out, s);
    return cyclic ? sweep_dispatch<double, 2, true, float>(table, table_elems, q, g, in, out, s)
                  : sweep_dispatch<double, 2, false, float>(table, table_elems, q, g, in, out, s);
}

}  // namespace bb
