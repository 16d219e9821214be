// long_sweep.hip -- batched solves of long tridiagonal and pentadiagonal
// systems in three launches (long_core.h): the plain right-hand side.
#include "long_core.h"

namespace bb {

hipError_t launch_long_solve(int K, bool cyclic, const double *table, const CyclicQ &q,
                             const LongGeom &g, const double *rhs, double *x, hipStream_t s)
{
    const PlainSrc src{rhs};
    if (K == 1)
        return cyclic ? launch_long_k<1, true>(table, q, g, src, x, s)
                      : launch_long_k<1, false>(table, q, g, src, x, s);
    return cyclic ? launch_long_k<2, true>(table, q, g, src, x, s)
                  : launch_long_k<2, false>(table, q, g, src, x, s);
}

}  // namespace bb
