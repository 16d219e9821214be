// precision.h -- host interface of sweep_f32in.hip and long_f32in.hip: FP32
// right-hand sides solved with the FP64 sweeps and the FP64 table.
#pragma once

#include "internal.h"

namespace bb {

// x = A^{-1} b for float b (promoted exactly) with the double table and
// sweeps of launch_sweep's FP64 solve (same decomposition g), double x.
hipError_t launch_sweep_f32in(int K, bool cyclic, const void *table, int64_t table_elems,
                              const CyclicQ &q, const SweepGeom &g, const float *in, double *out,
                              hipStream_t s);

// The same for long systems: launch_long_solve's three launches with each
// right-hand-side read promoted from float (x must not overlap rhs).
hipError_t launch_long_solve_f32in(int K, bool cyclic, const double *table, const CyclicQ &q,
                                   const LongGeom &g, const float *rhs, double *x, hipStream_t s);

}  // namespace bb
