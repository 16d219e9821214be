// long_f32in.hip -- long systems (long_core.h) with FP32 right-hand sides
// solved in FP64 (BB_F32_RHS_F64): each value promoted exactly wherever the
// three launches read the right-hand side, 4 instead of 8 bytes per read.
#include "long_core.h"
#include "precision.h"

namespace bb {
namespace {

struct F32Src {
    const float *rhs;
    template <int C>
    __device__ __forceinline__ void full(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        float w[C];
        load_chunk<float, C, true>(w, rhs, row0, k, ld, n);
#pragma unroll
        for (int t = 0; t < C; ++t) v[t] = (double)w[t];
    }
    template <int C>
    __device__ __forceinline__ void tail(double (&v)[C], int row0, int64_t k, int64_t ld,
                                         int n) const
    {
        float w[C];
        load_chunk<float, C, false>(w, rhs, row0, k, ld, n);
#pragma unroll
        for (int t = 0; t < C; ++t) v[t] = (double)w[t];
    }
};

}  // namespace

hipError_t launch_long_solve_f32in(int K, bool cyclic, const double *table, const CyclicQ &q,
                                   const LongGeom &g, const float *rhs, double *x, hipStream_t s)
{
    const F32Src src{rhs};
    if (K == 1)
        return cyclic ? launch_long_k<1, true>(table, q, g, src, x, s)
                      : launch_long_k<1, false>(table, q, g, src, x, s);
    return cyclic ? launch_long_k<2, true>(table, q, g, src, x, s)
                  : launch_long_k<2, false>(table, q, g, src, x, s);
}

}  // namespace bb
