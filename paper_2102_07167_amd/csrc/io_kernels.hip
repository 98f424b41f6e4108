// io_kernels.hip -- device-side data movement of the device-pointer calls (user order <-> block
// order, the phase split into wrapped value, compensation term and winding count) and the order
// parameter of an arbitrary phase vector with its vector-Jacobian product.
//
// Order parameter (Sec. 2, eq. OrderParameter): r e^{i psi} = (1/N) sum_m e^{i theta_m}. With
// C = (1/N) sum cos theta and S = (1/N) sum sin theta, r = sqrt(C^2 + S^2), psi = atan2(S, C), and
//     dr/dtheta_m   = sin(psi - theta_m) / N,
//     dpsi/dtheta_m = cos(psi - theta_m) / (N r),
// both taken as 0 when r = 0.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kur_device.hpp"
#include "kur_io.hpp"

namespace kur {

namespace {

constexpr int kIoThreads = 256;

inline unsigned io_blocks(int64_t n) { return (unsigned)((n + kIoThreads - 1) / kIoThreads); }

// dst[perm[u]] = src[u]
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_scatter_in(int64_t n, const int32_t *__restrict__ perm,
                                                         const T *__restrict__ src, T *__restrict__ dst)
{
    const int64_t u = (int64_t)blockIdx.x * kIoThreads + threadIdx.x;
    if (u < n) dst[perm[u]] = src[u];
}

// dst[perm[u]] = x reduced to [-pi, pi] in FP64 (remainder by 2 pi), then rounded to T
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_reduce_in(int64_t n, const int32_t *__restrict__ perm,
                                                        const T *__restrict__ src, T *__restrict__ dst)
{
    const int64_t u = (int64_t)blockIdx.x * kIoThreads + threadIdx.x;
    if (u < n) dst[perm[u]] = (T)remainder((double)src[u], 2.0 * TwoPi<double>::PI);
}

// The phase split of the host path in FP64 with the context type's two-part 2 pi (p1 + p2):
// q = nearest integer to x / (2 pi), red = (x - q p1) - q p2, hi = T(red), lo = T(red - hi),
// winding q. No contraction into fused multiply-adds, so the split is the host's bit for bit.
// Non-finite x gives a non-finite hi (winding 0); |q| is clamped to the int32 range.
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_phase_in(int64_t n, const int32_t *__restrict__ perm,
                                                       const T *__restrict__ theta, double p1, double p2,
                                                       T *__restrict__ hi, T *__restrict__ lo, int32_t *__restrict__ wind)
{
#pragma clang fp contract(off)
    const int64_t u = (int64_t)blockIdx.x * kIoThreads + threadIdx.x;
    if (u >= n) return;
    const double x = (double)theta[u];
    const int32_t m = perm[u];
    double q = rint(x / (2.0 * TwoPi<double>::PI));
    if (!(q == q)) q = 0.0;
    q = fmin(fmax(q, -2147483647.0), 2147483647.0);
    const double red = (x - q * p1) - q * p2;
    const T h = (T)red;
    hi[m] = h;
    lo[m] = (T)(red - (double)h);
    wind[m] = (int32_t)q;
}

// dst[u] = TD(src[perm[u]])
template <typename TS, typename TD>
__global__ __launch_bounds__(kIoThreads) void k_gather_out(int64_t n, const int32_t *__restrict__ perm,
                                                         const TS *__restrict__ src, TD *__restrict__ dst)
{
    const int64_t u = (int64_t)blockIdx.x * kIoThreads + threadIdx.x;
    if (u < n) dst[u] = (TD)src[perm[u]];
}

// The phases of user node u from the block-order state, in FP64 as on the host: x = hi + lo,
// then either wrapped to [-pi, pi) or unwrapped by the winding count (x + (w p1 + w p2)).
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_phase_out_user(int64_t n, const int32_t *__restrict__ perm,
                                                             const T *__restrict__ hi, const T *__restrict__ lo,
                                                             const int32_t *__restrict__ wind, int wrapped, double p1,
                                                             double p2, T *__restrict__ out)
{
#pragma clang fp contract(off)
    const int64_t u = (int64_t)blockIdx.x * kIoThreads + threadIdx.x;
    if (u >= n) return;
    const int32_t m = perm[u];
    double x = (double)hi[m] + (double)lo[m];
    if (wrapped) {
        x = remainder(x, 2.0 * TwoPi<double>::PI);
        if (x >= TwoPi<double>::PI) x -= 2.0 * TwoPi<double>::PI;
    } else {
        const double w = (double)wind[m];
        x = x + (w * p1 + w * p2);
    }
    out[u] = (T)x;
}

// out[0] = T(sum of part[0..count)), one workgroup, fixed order
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_fold_sum(int64_t count, const double *__restrict__ part, T *__restrict__ out)
{
    __shared__ double red[kIoThreads];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += kIoThreads) a += part[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = kIoThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (T)red[0];
}

// Partial sums (sum cos theta, sum sin theta) in FP64: workgroup b takes the entries
// b, b + G, b + 2G, ... in chunks of kIoThreads (G = the fixed grid size), so the order of the
// sums does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_op_part(int64_t n, const T *__restrict__ theta, double *__restrict__ part)
{
    __shared__ double rc[kIoThreads / 64], rs[kIoThreads / 64];
    double c = 0.0, s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kIoThreads;
    for (int64_t m = (int64_t)blockIdx.x * kIoThreads + threadIdx.x; m < n; m += stride) {
        double sn, cs;
        sincos((double)theta[m], &sn, &cs);
        c += cs;
        s += sn;
    }
    c = wave_sum(c);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) {
        rc[threadIdx.x >> 6] = c;
        rs[threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tc = 0.0, ts = 0.0;
        for (int w = 0; w < kIoThreads / 64; ++w) {
            tc += rc[w];
            ts += rs[w];
        }
        part[2 * blockIdx.x] = tc;
        part[2 * blockIdx.x + 1] = ts;
    }
}

// out = (r, psi) from the partials of k_op_part, one workgroup
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_op_fold(int nblk, const double *__restrict__ part, double inv_n,
                                                       T *__restrict__ out)
{
    __shared__ double rc[kIoThreads], rs[kIoThreads];
    double c = 0.0, s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kIoThreads) {
        c += part[2 * b];
        s += part[2 * b + 1];
    }
    rc[threadIdx.x] = c;
    rs[threadIdx.x] = s;
    __syncthreads();
    for (int w = kIoThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            rc[threadIdx.x] += rc[threadIdx.x + w];
            rs[threadIdx.x] += rs[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double C = rc[0] * inv_n, S = rs[0] * inv_n;
        out[0] = (T)sqrt(C * C + S * S);
        out[1] = (T)atan2(S, C);
    }
}

// out[m] (+)= g_r sin(psi - theta_m) / N + g_psi cos(psi - theta_m) / (N r), 0 when r = 0
template <typename T>
__global__ __launch_bounds__(kIoThreads) void k_op_vjp(int64_t n, const T *__restrict__ theta, const T *__restrict__ rpsi,
                                                      const T *__restrict__ grad, double inv_n, int accumulate,
                                                      T *__restrict__ out)
{
    const int64_t m = (int64_t)blockIdx.x * kIoThreads + threadIdx.x;
    if (m >= n) return;
    const double r = (double)rpsi[0], psi = (double)rpsi[1];
    double v = 0.0;
    if (r > 0.0) {
        double sn, cs;
        sincos(psi - (double)theta[m], &sn, &cs);
        v = ((double)grad[0] * sn + (double)grad[1] * cs / r) * inv_n;
    }
    out[m] = accumulate ? (T)((double)out[m] + v) : (T)v;
}

}  // namespace

template <typename T>
hipError_t launch_scatter_in(int64_t n, const int32_t *perm, const void *src, void *dst, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_scatter_in<T>), dim3(io_blocks(n)), dim3(kIoThreads), 0, st, n, perm, (const T *)src, (T *)dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce_in(int64_t n, const int32_t *perm, const void *src, void *dst, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_reduce_in<T>), dim3(io_blocks(n)), dim3(kIoThreads), 0, st, n, perm, (const T *)src, (T *)dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phase_in(int64_t n, const int32_t *perm, const void *theta, double p1, double p2, void *hi, void *lo,
                           int32_t *wind, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_phase_in<T>), dim3(io_blocks(n)), dim3(kIoThreads), 0, st, n, perm, (const T *)theta, p1, p2,
                       (T *)hi, (T *)lo, wind);
    return hipGetLastError();
}

template <typename TS, typename TD>
hipError_t launch_gather_out(int64_t n, const int32_t *perm, const void *src, void *dst, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_gather_out<TS, TD>), dim3(io_blocks(n)), dim3(kIoThreads), 0, st, n, perm, (const TS *)src,
                       (TD *)dst);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phase_out_user(int64_t n, const int32_t *perm, const void *hi, const void *lo, const int32_t *wind,
                                 int wrapped, double p1, double p2, void *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_phase_out_user<T>), dim3(io_blocks(n)), dim3(kIoThreads), 0, st, n, perm, (const T *)hi,
                       (const T *)lo, wind, wrapped, p1, p2, (T *)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fold_sum(int64_t count, const double *part, void *out, hipStream_t st)
{
    hipLaunchKernelGGL((k_fold_sum<T>), dim3(1), dim3(kIoThreads), 0, st, count, part, (T *)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_order_param(int64_t n, const void *theta, double *part, void *out, hipStream_t st)
{
    if (n <= 0) return hipErrorInvalidValue;
    const int64_t want = (n + kIoThreads - 1) / kIoThreads;
    const int nblk = (int)(want < kOpParts ? want : kOpParts);
    hipLaunchKernelGGL((k_op_part<T>), dim3(nblk), dim3(kIoThreads), 0, st, n, (const T *)theta, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_op_fold<T>), dim3(1), dim3(kIoThreads), 0, st, nblk, (const double *)part, 1.0 / (double)n,
                       (T *)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_order_param_vjp(int64_t n, const void *theta, const void *rpsi, const void *grad, int accumulate,
                                  void *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_op_vjp<T>), dim3(io_blocks(n)), dim3(kIoThreads), 0, st, n, (const T *)theta,
                       (const T *)rpsi, (const T *)grad, 1.0 / (double)n, accumulate, (T *)out);
    return hipGetLastError();
}

#define KUR_IO_INST(T)                                                                                                 \
    template hipError_t launch_scatter_in<T>(int64_t, const int32_t *, const void *, void *, hipStream_t);            \
    template hipError_t launch_reduce_in<T>(int64_t, const int32_t *, const void *, void *, hipStream_t);             \
    template hipError_t launch_phase_in<T>(int64_t, const int32_t *, const void *, double, double, void *, void *,    \
                                           int32_t *, hipStream_t);                                                   \
    template hipError_t launch_phase_out_user<T>(int64_t, const int32_t *, const void *, const void *,                \
                                                 const int32_t *, int, double, double, void *, hipStream_t);          \
    template hipError_t launch_fold_sum<T>(int64_t, const double *, void *, hipStream_t);                             \
    template hipError_t launch_order_param<T>(int64_t, const void *, double *, void *, hipStream_t);                  \
    template hipError_t launch_order_param_vjp<T>(int64_t, const void *, const void *, const void *, int, void *,     \
                                                  hipStream_t);
KUR_IO_INST(float)
KUR_IO_INST(double)
#undef KUR_IO_INST
template hipError_t launch_gather_out<float, float>(int64_t, const int32_t *, const void *, void *, hipStream_t);
template hipError_t launch_gather_out<double, double>(int64_t, const int32_t *, const void *, void *, hipStream_t);
template hipError_t launch_gather_out<double, float>(int64_t, const int32_t *, const void *, void *, hipStream_t);

}  // namespace kur
