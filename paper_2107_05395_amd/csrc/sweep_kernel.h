// sweep_kernel.h -- the batched solve kernel (FP64 or FP32 sweeps, primal or
// adjoint table) and its dispatch templates; instantiated for double in
// sweep.hip, for float in sweep_f32.hip and for float right-hand sides with
// double sweeps in sweep_f32in.hip, so they compile in parallel.  Building
// blocks in sweep_core.h.
#pragma once

#include <type_traits>

#include "sweep_core.h"

namespace bb {
namespace {

// ---------------------------------------------------------------- solve
// QL = log2 of the waves per system group (0: one wave per group).  With
// QL > 0 the workgroup is exactly one group (2^QL waves): every wave of it has
// the same group index, so the exchange barriers are reached uniformly.
// TI: type of the right-hand sides in memory (T, or float read into double
// sweeps: FP32 data solved in FP64, exact promotion).
template <typename T, int K, int C, bool CYC, bool FULL, int QL, typename TI = T>
__global__ __launch_bounds__((kWave << QL) > kMaxBlockThreads ? (kWave << QL) : kMaxBlockThreads)
void sweep_kernel(const T *__restrict__ table, int64_t table_elems, CyclicQ cq, SweepGeom g,
                  const TI *in, T *out)
{
    extern __shared__ double smem_d[];
    T *lds = reinterpret_cast<T *>(smem_d);
    stage_table(lds, table, table_elems);
    __syncthreads();
    T *xch = lds + table_elems;   // exchange area of the split group (QL > 0)

    const LaneGeom lg = lane_geom(g.log2P, QL);
    const int row0 = lg.j * C;
    const GroupRange gr = group_range(g.groups, QL, g.linear);
    for (int64_t b = gr.first; b < gr.end; b += gr.stride) {
        const int64_t grp = begin_block(gr, b, g.lockstep);
        if (grp >= g.groups) continue;
        const int64_t k = grp * lg.S + lg.sl;
        const bool kval = k < g.m;
        T v[C];
        if constexpr (std::is_same<TI, T>::value) {
            load_chunk<T, C, FULL>(v, in, row0, kval ? k : g.m - 1, g.ld, g.n);
        } else {
            TI w[C];
            load_chunk<TI, C, FULL>(w, in, row0, kval ? k : g.m - 1, g.ld, g.n);
#pragma unroll
            for (int t = 0; t < C; ++t) v[t] = (T)w[t];
        }
        chunk_solve<T, K, C, CYC, (QL > 0)>(v, lds, lg, g.n, FULL || g.exact, cq, xch);
        if (kval) store_chunk<T, C, FULL>(v, out, row0, k, g.ld, g.n);
    }
}

template <typename T, int K, bool CYC, int C, int QL, typename TI = T>
hipError_t sweep_split(const void *table, int64_t table_elems, const CyclicQ &q,
                       const SweepGeom &g, const void *in, void *out, hipStream_t stream)
{
    const size_t lds =
        (size_t)(table_elems + split_exchange_len(QL) + (CYC ? split_ends_len(QL) : 0)) * sizeof(T);
    if (is_full(g))
        return launch_grid_split(sweep_kernel<T, K, C, CYC, true, QL, TI>, lds, g.groups, 1 << QL,
                                 stream, (const T *)table, table_elems, q, g, (const TI *)in,
                                 (T *)out);
    return launch_grid_split(sweep_kernel<T, K, C, CYC, false, QL, TI>, lds, g.groups, 1 << QL,
                             stream, (const T *)table, table_elems, q, g, (const TI *)in, (T *)out);
}

template <typename T, int K, bool CYC, int C, typename TI = T>
hipError_t sweep_c(const void *table, int64_t table_elems, const CyclicQ &q, const SweepGeom &g,
                   const void *in, void *out, hipStream_t stream)
{
    if (g.log2Q > 0) {
        // split groups: 32, 64 or 128 rows per lane
        if constexpr (C >= 32) {
            if (g.log2Q > max_log2q(C, false) || g.log2Q > g.log2P) return hipErrorInvalidValue;
            if (g.log2Q == 1) return sweep_split<T, K, CYC, C, 1, TI>(table, table_elems, q, g, in, out, stream);
            if (g.log2Q == 2) return sweep_split<T, K, CYC, C, 2, TI>(table, table_elems, q, g, in, out, stream);
            if constexpr (C <= 64) return sweep_split<T, K, CYC, C, 3, TI>(table, table_elems, q, g, in, out, stream);
        }
        return hipErrorInvalidValue;
    }
    const size_t lds = (size_t)table_elems * sizeof(T);
    if (is_full(g))
        return launch_grid(sweep_kernel<T, K, C, CYC, true, 0, TI>, lds, g.groups, stream,
                           (const T *)table, table_elems, q, g, (const TI *)in, (T *)out);
    return launch_grid(sweep_kernel<T, K, C, CYC, false, 0, TI>, lds, g.groups, stream,
                       (const T *)table, table_elems, q, g, (const TI *)in, (T *)out);
}

template <typename T, int K, bool CYC, typename TI = T>
hipError_t sweep_dispatch(const void *table, int64_t te, const CyclicQ &q, const SweepGeom &g,
                          const void *in, void *out, hipStream_t s)
{
    switch (g.C) {
    case 4: return sweep_c<T, K, CYC, 4, TI>(table, te, q, g, in, out, s);
    case 8: return sweep_c<T, K, CYC, 8, TI>(table, te, q, g, in, out, s);
    case 16: return sweep_c<T, K, CYC, 16, TI>(table, te, q, g, in, out, s);
    case 32: return sweep_c<T, K, CYC, 32, TI>(table, te, q, g, in, out, s);
    case 64: return sweep_c<T, K, CYC, 64, TI>(table, te, q, g, in, out, s);
    case 128: return sweep_c<T, K, CYC, 128, TI>(table, te, q, g, in, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace bb
