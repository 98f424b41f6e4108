// kur_device.hpp -- device helpers shared by the kernel files: (sin, cos), rounding, the two-part
// split of 2 pi used to wrap phases, the error-free sum, the per-oscillator bookkeeping of one
// classical RK4 stage, and wave-level sums.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kur {

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };

template <typename T> __device__ __forceinline__ void dev_sincos(T x, T *s, T *c);
template <> __device__ __forceinline__ void dev_sincos<float>(float x, float *s, float *c) { sincosf(x, s, c); }
template <> __device__ __forceinline__ void dev_sincos<double>(double x, double *s, double *c) { sincos(x, s, c); }

template <typename T> __device__ __forceinline__ T dev_rint(T x);
template <> __device__ __forceinline__ float dev_rint<float>(float x) { return rintf(x); }
template <> __device__ __forceinline__ double dev_rint<double>(double x) { return rint(x); }

template <typename T>
struct TwoPi;
template <> struct TwoPi<float> {
    // 2 pi = P1 + P2 + O(1e-10); P1 has 8 significant bits so q * P1 is exact for |q| < 2^16
    static constexpr float P1 = 6.28125f;
    static constexpr float P2 = 1.93530717958647692528676655900576839e-3f;
    static constexpr float INV = 0.159154943091895335768883763372514362f;
    static constexpr float PI = 3.14159265358979323846264338327950288f;
};
template <> struct TwoPi<double> {
    // P1 has 26 significant bits so q * P1 is exact for |q| < 2^27
    static constexpr double P1 = 6.283185362815857;  // 52707179 / 2^23
    static constexpr double P2 = -5.5636270456668466e-08;
    static constexpr double INV = 0.159154943091895335768883763372514362;
    static constexpr double PI = 3.14159265358979323846264338327950288;
};

// error-free sum a + b = s + e
template <typename T> __device__ __forceinline__ void two_sum(T a, T b, T &s, T &e)
{
    s = a + b;
    T bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Advance one oscillator's phase (th + lo, winding wind) by delta: with error-free sums when
// `compensate`, then wrapped to [-pi, pi) (the whole turns go to the winding count). Writes
// the new (hi, lo, wind) and returns the new hi.
template <typename T>
__device__ __forceinline__ T phase_advance(T th, T lo_in, int32_t wind_in, T delta, int compensate, T *hi_p, T *lo_p,
                                           int32_t *wind_p)
{
    T hi, lo;
    int wd = wind_in;
    if (compensate) {
        T d1, e1, s, e2;
        two_sum(delta, lo_in, d1, e1);
        two_sum(th, d1, s, e2);
        hi = s;
        lo = e1 + e2;
    } else {
        hi = th + delta;
        lo = T(0);
    }
    if (!(hi >= -TwoPi<T>::PI && hi < TwoPi<T>::PI)) {
        const T q = dev_rint<T>(hi * TwoPi<T>::INV);
        hi = hi - q * TwoPi<T>::P1;  // exact (Sterbenz)
        lo = lo - q * TwoPi<T>::P2;
        wd += (int)q;
    }
    T s2, e3;
    two_sum(hi, lo, s2, e3);
    *hi_p = s2;
    *lo_p = e3;
    *wind_p = wd;
    return s2;
}

// Bookkeeping of one oscillator given its stage derivative k, for classical RK4
// (y_{n+1} = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4)) and for the implicit midpoint rule
// (y_{n+1} = y_n + dt F((y_n + y_{n+1}) / 2), solved by fixed-point iteration on the midpoint).
//   stages 1-3   RK4: accumulate k1 + 2 k2 + 2 k3 in *ksum and return the next stage input
//                (theta + dt/2 k1, theta + dt/2 k2, theta + dt k3);
//   stage 4      RK4: advance the phase by dt/6 (ksum + k4);
//   stage 5      midpoint iterate: return theta + dt/2 k (the phase is not changed);
//   stage 6      midpoint final: advance the phase by dt k.
// The advance is phase_advance in place.
template <typename T>
__device__ __forceinline__ T rk4_stage(int stage, T k, T dt, T half_dt, T dt6, int compensate, T *ksum, T *hi_p,
                                       T *lo_p, int32_t *wind_p)
{
    const T th = *hi_p;
    if (stage == 1) {
        *ksum = k;
        return th + half_dt * k;
    }
    if (stage == 2) {
        *ksum += T(2) * k;
        return th + half_dt * k;
    }
    if (stage == 3) {
        *ksum += T(2) * k;
        return th + dt * k;
    }
    if (stage == 5) return th + half_dt * k;
    const T delta = stage == 6 ? dt * k : dt6 * (*ksum + k);
    return phase_advance<T>(th, *lo_p, *wind_p, delta, compensate, hi_p, lo_p, wind_p);
}

// Wave-level sums. wave_sum leaves the sum in every lane (butterfly of shuffles); the DPP forms
// use VALU cross-lane moves only, in a fixed order.
template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Cross-lane moves with DPP (VALU only, no LDS traffic). Rows are the 16-lane DPP rows of a
// wave64; lanes of disabled rows receive 0.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_mov(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_mov(double x)
{
    const int2 v = __builtin_bit_cast(int2, x);
    int2 o;
    o.x = __builtin_amdgcn_update_dpp(0, v.x, CTRL, ROWS, 0xf, false);
    o.y = __builtin_amdgcn_update_dpp(0, v.y, CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(double, o);
}

enum : int {
    DPP_XOR1 = 0xB1,        // quad_perm [1,0,3,2]
    DPP_XOR2 = 0x4E,        // quad_perm [2,3,0,1]
    DPP_HALF_MIRROR = 0x141,
    DPP_MIRROR = 0x140,
    DPP_BCAST15 = 0x142,
    DPP_BCAST31 = 0x143,
};

// Sum over aligned groups of G lanes (G a power of two, 2..64) in a fixed order; the result is
// valid in the last lane of every group (for G <= 16 in every lane of the group).
template <typename T>
__device__ __forceinline__ T group_sum_dpp(T v, int G)
{
    v += dpp_mov<DPP_XOR1>(v);
    if (G >= 4) v += dpp_mov<DPP_XOR2>(v);
    if (G >= 8) v += dpp_mov<DPP_HALF_MIRROR>(v);
    if (G >= 16) v += dpp_mov<DPP_MIRROR>(v);
    if (G >= 32) v += dpp_mov<DPP_BCAST15, 0xa>(v);
    if (G >= 64) v += dpp_mov<DPP_BCAST31, 0xc>(v);
    return v;
}

// Sum over the whole wave; valid in lane 63.
template <typename T>
__device__ __forceinline__ T wave_sum_dpp(T v)
{
    v += dpp_mov<DPP_XOR1>(v);
    v += dpp_mov<DPP_XOR2>(v);
    v += dpp_mov<DPP_HALF_MIRROR>(v);
    v += dpp_mov<DPP_MIRROR>(v);
    v += dpp_mov<DPP_BCAST15, 0xa>(v);
    v += dpp_mov<DPP_BCAST31, 0xc>(v);
    return v;
}

}  // namespace kur
