// aux.hip -- the remaining gfx950 kernels of libbandbatch:
//   * band gradients of a batched solve, reduced over the batch in a fixed order
//   * mean-squared-error loss and gradient
//   * the paper's thread-per-system tridiagonal sweep (Appendix A batched
//     sweep), kept as the measured baseline design
#include <mutex>

#include "adjoint_grad.h"
#include "internal.h"

namespace bb {

// Device memory of the allocation-free band gradient: the partial sums of
// its groups of systems.  One copy per device, alive until the process ends.
// Host code never uses this name as an address (on the host it is only a
// stand-in for the symbol): band_grad_scratch_ptr() asks the runtime for the
// device address once per device.
static __device__ __align__(256) double scratch[kGradScratchBytes / sizeof(double)];

namespace {

constexpr int kGradR = 4;          // systems per lane in the band-gradient kernel
constexpr int kGradRows = 32;      // rows per wave strip
constexpr int kGradSys = kWave * kGradR;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One wave: rows [i0, i0 + kGradRows) x the k-blocks kg*kpw .. (kg+1)*kpw - 1
// of kGradSys systems each (blockIdx.x = kg).
// part[kg][band][i] = -sum over those systems of lam[i,k] x[i+off,k], the
// k-blocks added in ascending order.  Within a k-block the loads of row i+1
// are issued before row i is reduced (one row in flight ahead); lane i - i0
// keeps row i's sum and the strip is stored at the end, one coalesced store
// per band.
template <int NB>
__global__ __launch_bounds__(256) void band_grad_partial(int n, int cyclic, int64_t m, int64_t ld,
                                                         int64_t kpw,
                                                         const double *__restrict__ lam,
                                                         const double *__restrict__ x,
                                                         double *__restrict__ part)
{
    static_assert(kGradRows <= kWave, "one row per lane at the store");
    constexpr int H = NB / 2;
    const int lane = threadIdx.x % kWave;
    const int strip = blockIdx.y * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int i0 = strip * kGradRows;
    if (i0 >= n) return;
    const int i1 = i0 + kGradRows < n ? i0 + kGradRows : n;
    const int64_t kblocks = (m + kGradSys - 1) / kGradSys;
    const int64_t kb0 = (int64_t)blockIdx.x * kpw;
    const int64_t kb1 = kb0 + kpw < kblocks ? kb0 + kpw : kblocks;
    double keep[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) keep[q] = 0.0;
    for (int64_t kb = kb0; kb < kb1; ++kb) {
        int64_t ks[kGradR];
        bool kv[kGradR];
#pragma unroll
        for (int r = 0; r < kGradR; ++r) {
            ks[r] = kb * kGradSys + r * kWave + lane;
            kv[r] = ks[r] < m;
        }
        auto load_x = [&](int row, int r) -> double {
            if (row < 0 || row >= n) {
                if (!cyclic) return 0.0;
                row = (row % n + n) % n;
            }
            return kv[r] ? x[(int64_t)row * ld + ks[r]] : 0.0;
        };
        auto load_l = [&](int row, int r) -> double {
            return (kv[r] && row < n) ? lam[(int64_t)row * ld + ks[r]] : 0.0;
        };
        // sliding window of x rows i-H .. i+H, and the next row's operands
        double win[NB][kGradR], xn[kGradR], ln[kGradR];
#pragma unroll
        for (int w = 0; w < NB - 1; ++w)
#pragma unroll
            for (int r = 0; r < kGradR; ++r) win[w + 1][r] = load_x(i0 - H + w, r);
#pragma unroll
        for (int r = 0; r < kGradR; ++r) {
            xn[r] = load_x(i0 + H, r);
            ln[r] = load_l(i0, r);
        }
        for (int i = i0; i < i1; ++i) {
            double l[kGradR];
#pragma unroll
            for (int r = 0; r < kGradR; ++r) {
#pragma unroll
                for (int w = 0; w < NB - 1; ++w) win[w][r] = win[w + 1][r];
                win[NB - 1][r] = xn[r];
                l[r] = ln[r];
            }
            if (i + 1 < i1) {
#pragma unroll
                for (int r = 0; r < kGradR; ++r) {
                    xn[r] = load_x(i + 1 + H, r);
                    ln[r] = load_l(i + 1, r);
                }
            }
            double acc[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) acc[q] = 0.0;
#pragma unroll
            for (int r = 0; r < kGradR; ++r)
#pragma unroll
                for (int q = 0; q < NB; ++q) acc[q] = fma(l[r], win[q][r], acc[q]);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const double sum = wave_sum(acc[q]);
                if (lane == i - i0) keep[q] -= sum;
            }
        }
    }
    double *dst = part + (int64_t)blockIdx.x * NB * n;
    if (lane < i1 - i0) {
        const int i = i0 + lane;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            // entries outside a non-cyclic matrix have no gradient
            const bool inside = cyclic || (i + q - H >= 0 && i + q - H < n);
            dst[(int64_t)q * n + i] = inside ? keep[q] : 0.0;
        }
    }
}

// grad[e] += sum over the partial groups g of part[g][e]: the 16 waves of a
// block each sum every 16th group (ascending), and the 16 sums are added in
// a fixed order -- the same result on every run.
constexpr int kFoldSubs = 16;
__global__ __launch_bounds__(kFoldSubs * kWave) void band_grad_fold(int64_t total, int64_t groups,
                                                                  const double *__restrict__ part,
                                                                  double *__restrict__ grad)
{
    __shared__ double red[kFoldSubs][kWave];
    const int lane = threadIdx.x % kWave, sub = threadIdx.x / kWave;
    const int64_t e = (int64_t)blockIdx.x * kWave + lane;
    double s = 0.0;
    if (e < total)
        for (int64_t g = sub; g < groups; g += kFoldSubs) s += part[g * total + e];
    red[sub][lane] = s;
    __syncthreads();
    if (sub == 0 && e < total) {
        double t = red[0][lane];
#pragma unroll
        for (int q = 1; q < kFoldSubs; ++q) t += red[q][lane];
        grad[e] += t;
    }
}

// ---------------------------------------------------------------- MSE
constexpr int kMseCols = 1024;   // systems per block (4 per thread)

// One block per (row, 1024 systems): the block grid is (columns, n).
__global__ __launch_bounds__(256) void mse_partial(int64_t n, int64_t m, int64_t ld, double scale,
                                                   const double *u,
                                                   const double *__restrict__ y,
                                                   double *grad,
                                                   double *__restrict__ part)
{
    __shared__ double red[256 / kWave];
    // rows over grid y and z (a grid dimension y holds at most 65535 blocks)
    const int row = (int)(blockIdx.z * gridDim.y + blockIdx.y);
    if (row >= (int)n) return;   // whole blocks
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kMseCols / 256; ++r) {
        const int64_t k = (int64_t)blockIdx.x * kMseCols + r * 256 + threadIdx.x;
        if (k < m) {
            const int64_t idx = (int64_t)row * ld + k;
            const double d = u[idx] - y[idx];
            grad[idx] = 2.0 * scale * d;
            acc = fma(d, d, acc);
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < 256 / kWave; ++w) s += red[w];
        part[(int64_t)row * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void mse_fold(int64_t parts, double scale,
                                                const double *__restrict__ part,
                                                double *__restrict__ loss)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < parts; e += 256) s += part[e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * scale;
}

// ---------------------------------------------------------------- baseline
// One thread per system walks all n rows: forward sweep into x, backward
// sweep reading x back (the forward intermediate goes through memory).
// Coefficients are wave-uniform (scalar loads).
__global__ __launch_bounds__(256) void tri_thread_per_system(const double *__restrict__ rhat,
                                                             const double *__restrict__ aprime,
                                                             const double *__restrict__ chat,
                                                             int n, int64_t m, int64_t ld,
                                                             const double *rhs, double *x)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    double prev = rhs[k] * rhat[0];
    x[k] = prev;
    for (int i = 1; i < n; ++i) {
        prev = fma(-aprime[i], prev, rhs[(int64_t)i * ld + k] * rhat[i]);
        x[(int64_t)i * ld + k] = prev;
    }
    for (int i = n - 2; i >= 0; --i) {
        prev = fma(-chat[i], prev, x[(int64_t)i * ld + k]);
        x[(int64_t)i * ld + k] = prev;
    }
}

// Streaming reference for the roofline (not part of the method): each
// workgroup of 256 threads copies one contiguous 16 KB tile, four 16-byte
// loads per thread issued before its four stores.
typedef double copy_vec __attribute__((ext_vector_type(2)));
constexpr int kCopyPerThread = 4;

__global__ __launch_bounds__(256) void copy_tiles(const copy_vec *__restrict__ in,
                                                  copy_vec *__restrict__ out, int64_t n2)
{
    const int64_t base = (int64_t)blockIdx.x * 256 * kCopyPerThread + threadIdx.x;
    copy_vec v[kCopyPerThread];
#pragma unroll
    for (int u = 0; u < kCopyPerThread; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n2) v[u] = in[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyPerThread; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n2) out[i] = v[u];
    }
}

// Streaming reference with the access pattern of the FP64 sweeps (not part
// of the method): an interleaved n x m array copied by waves that each move
// 64 rows of two 32-system segments 64 rows apart -- one 8-byte load per
// lane per row, 256-byte segments, every load issued before any store --
// like a 64-row-chunk sweep wave holding two chunks of 32 systems.
constexpr int kRowsPerLane = 64, kSegSystems = 32;

__global__ __launch_bounds__(256) void copy_rows(const double *__restrict__ in,
                                                 double *__restrict__ out, int n, int64_t ld,
                                                 int64_t m)
{
    const int lane = threadIdx.x % kWave;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t cblocks = m / kSegSystems;
    const int64_t rblocks = n / (2 * kRowsPerLane);
    if (wave >= cblocks * rblocks) return;
    const int64_t cb = wave % cblocks;   // neighbouring waves: neighbouring segments
    const int64_t rb = wave / cblocks;
    const int64_t col = cb * kSegSystems + lane % kSegSystems;
    const int64_t row0 = rb * 2 * kRowsPerLane + (lane / kSegSystems) * kRowsPerLane;
    const double *p = in + row0 * ld + col;
    double *q = out + row0 * ld + col;
    double v[kRowsPerLane];
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) v[t] = p[(int64_t)t * ld];
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) q[(int64_t)t * ld] = v[t];
}

}  // namespace

hipError_t launch_copy_rows(const double *src, double *dst, int n, int64_t m, int64_t ld,
                            hipStream_t s)
{
    const int64_t waves = (m / kSegSystems) * (n / (2 * kRowsPerLane));
    const int64_t blocks = (waves * kWave + 255) / 256;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_rows, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n, ld, m);
    return hipGetLastError();
}

hipError_t launch_copy_tiles(const void *src, void *dst, int64_t bytes, hipStream_t s)
{
    const int64_t n2 = bytes / 16;
    const int64_t blocks = (n2 + 256 * kCopyPerThread - 1) / (256 * kCopyPerThread);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_tiles, dim3((unsigned)blocks), dim3(256), 0, s, (const copy_vec *)src,
                       (copy_vec *)dst, n2);
    return hipGetLastError();
}

// k-blocks per wave: enough waves (about 8192, four per SIMD on 256 CUs) to
// keep HBM busy, few enough partial sums that the fold stays short.
int64_t band_grad_kpw(int n, int64_t m)
{
    const int64_t kblocks = (m + kGradSys - 1) / kGradSys;
    const int64_t strips = (n + kGradRows - 1) / kGradRows;
    int64_t kpw = kblocks * strips / 8192;
    return kpw < 1 ? 1 : kpw;
}

size_t band_grad_workspace(int nb, int n, int64_t m)
{
    const int64_t kblocks = (m + kGradSys - 1) / kGradSys;
    const int64_t kpw = band_grad_kpw(n, m);
    const int64_t groups = (kblocks + kpw - 1) / kpw;
    return (size_t)groups * nb * n * sizeof(double);
}

namespace {

hipError_t band_grad_launch(int nb, bool cyclic, int n, int64_t m, int64_t ld, const double *lam,
                            const double *x, double *grad, double *part, int64_t kpw,
                            hipStream_t s)
{
    const int64_t kblocks = (m + kGradSys - 1) / kGradSys;
    const int64_t groups = (kblocks + kpw - 1) / kpw;
    const int strips = (n + kGradRows - 1) / kGradRows;
    const int waves = 256 / kWave;
    dim3 grid((unsigned)groups, (unsigned)((strips + waves - 1) / waves));
    if (nb == 3)
        hipLaunchKernelGGL(band_grad_partial<3>, grid, dim3(256), 0, s, n, (int)cyclic, m, ld, kpw,
                           lam, x, part);
    else
        hipLaunchKernelGGL(band_grad_partial<5>, grid, dim3(256), 0, s, n, (int)cyclic, m, ld, kpw,
                           lam, x, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = (int64_t)nb * n;
    hipLaunchKernelGGL(band_grad_fold, dim3((unsigned)((total + kWave - 1) / kWave)),
                       dim3(kFoldSubs * kWave), 0, s, total, groups, (const double *)part, grad);
    return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy at its own address).
constexpr int kMaxDevices = 64;
hipError_t band_grad_scratch_ptr(double **out)
{
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = (double *)p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t launch_band_grad(int nb, bool cyclic, int n, int64_t m, int64_t ld, const double *lam,
                            const double *x, double *grad, void *ws, hipStream_t s)
{
    return band_grad_launch(nb, cyclic, n, m, ld, lam, x, grad, (double *)ws, band_grad_kpw(n, m),
                            s);
}

// Every entry of the partial sums that the fold reads is written by
// band_grad_partial in the same call, so nothing in the array needs clearing.
hipError_t launch_band_grad_scratch(int nb, bool cyclic, int n, int64_t m, int64_t ld,
                                    const double *lam, const double *x, double *grad,
                                    hipStream_t s)
{
    const int64_t cap = (int64_t)(kGradScratchBytes / sizeof(double)) / ((int64_t)nb * n);
    if (cap < 1) return hipErrorInvalidValue;   // the host checks nb * n first
    const int64_t kblocks = (m + kGradSys - 1) / kGradSys;
    int64_t kpw = band_grad_kpw(n, m);
    if ((kblocks + kpw - 1) / kpw > cap) kpw = (kblocks + cap - 1) / cap;
    double *part = nullptr;
    hipError_t e = band_grad_scratch_ptr(&part);
    if (e != hipSuccess) return e;
    return band_grad_launch(nb, cyclic, n, m, ld, lam, x, grad, part, kpw, s);
}

hipError_t launch_grad_fold(int64_t total, int64_t groups, const double *part, double *grad,
                            hipStream_t s)
{
    if (total <= 0 || groups <= 0) return hipSuccess;
    hipLaunchKernelGGL(band_grad_fold, dim3((unsigned)((total + kWave - 1) / kWave)),
                       dim3(kFoldSubs * kWave), 0, s, total, groups, part, grad);
    return hipGetLastError();
}

size_t mse_workspace(int64_t n, int64_t m)
{
    return (size_t)n * (size_t)((m + kMseCols - 1) / kMseCols) * sizeof(double);
}

hipError_t launch_mse(const double *u, const double *target, double *grad, double *loss, int n,
                      int64_t m, int64_t ld, void *ws, hipStream_t s)
{
    const int64_t cols = (m + kMseCols - 1) / kMseCols;
    const double scale = 1.0 / ((double)n * (double)m);
    const int ny = n < 32768 ? n : 32768;
    hipLaunchKernelGGL(mse_partial, dim3((unsigned)cols, (unsigned)ny, (unsigned)((n + ny - 1) / ny)),
                       dim3(256), 0, s, (int64_t)n, m, ld, scale, u, target, grad, (double *)ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mse_fold, dim3(1), dim3(256), 0, s, (int64_t)n * cols, scale,
                       (const double *)ws, loss);
    return hipGetLastError();
}

hipError_t launch_tri_thread_per_system(const double *rhat, const double *aprime,
                                        const double *chat, int n, int64_t m, int64_t ld,
                                        const double *rhs, double *x, hipStream_t s)
{
    const int64_t blocks = (m + 255) / 256;
    hipLaunchKernelGGL(tri_thread_per_system, dim3((unsigned)blocks), dim3(256), 0, s, rhat,
                       aprime, chat, n, m, ld, rhs, x);
    return hipGetLastError();
}

}  // namespace bb
