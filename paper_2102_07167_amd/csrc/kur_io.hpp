// kur_io.hpp -- launchers of io_kernels.hip: user order <-> block order on the device, the phase
// split, and the order parameter of an arbitrary phase vector with its vector-Jacobian product.
// perm[u] is the block-order index of user node u. Every launcher enqueues on `st` only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kur {

// workgroups (and FP64 (cos, sin) partial pairs) of the order-parameter reduction
constexpr int kOpParts = 1024;

// dst[perm[u]] = src[u] (T arrays)
template <typename T>
hipError_t launch_scatter_in(int64_t n, const int32_t *perm, const void *src, void *dst, hipStream_t st);
// dst[perm[u]] = T(remainder(double(src[u]), 2 pi))
template <typename T>
hipError_t launch_reduce_in(int64_t n, const int32_t *perm, const void *src, void *dst, hipStream_t st);
// phases theta (user order, T) -> (hi, lo, wind) in block order, split with 2 pi = p1 + p2
template <typename T>
hipError_t launch_phase_in(int64_t n, const int32_t *perm, const void *theta, double p1, double p2, void *hi, void *lo,
                           int32_t *wind, hipStream_t st);
// dst[u] = TD(src[perm[u]])
template <typename TS, typename TD>
hipError_t launch_gather_out(int64_t n, const int32_t *perm, const void *src, void *dst, hipStream_t st);
// user-order phases from (hi, lo, wind): wrapped to [-pi, pi) or unwrapped
template <typename T>
hipError_t launch_phase_out_user(int64_t n, const int32_t *perm, const void *hi, const void *lo, const int32_t *wind,
                                 int wrapped, double p1, double p2, void *out, hipStream_t st);
// out[0] = T(sum of count FP64 values), fixed order
template <typename T>
hipError_t launch_fold_sum(int64_t count, const double *part, void *out, hipStream_t st);
// out[0] = r, out[1] = psi of theta[0..n) (T); part holds 2 kOpParts doubles of scratch
template <typename T>
hipError_t launch_order_param(int64_t n, const void *theta, double *part, void *out, hipStream_t st);
// out[m] (+)= grad[0] dr/dtheta_m + grad[1] dpsi/dtheta_m at (r, psi) = rpsi[0..2)
template <typename T>
hipError_t launch_order_param_vjp(int64_t n, const void *theta, const void *rpsi, const void *grad, int accumulate,
                                  void *out, hipStream_t st);

}  // namespace kur
