// persist_kernels.hip -- whole RK4 runs of small complete graphs in one workgroup (the classical
// model of Sec. 2 through its order parameter): no launch per stage, the state in registers.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kur_device.hpp"
#include "kur_kernels.hpp"

namespace kur {

// Classical RK4 on the complete graph in one workgroup (see PersistArgs). Thread t owns rows
// t + kPersistThreads j, j < kPersistMaxRows, and keeps their phase, compensation term, winding count, RK4
// accumulator and the (sin, cos) of the current stage input in registers for the whole run. The
// right-hand side of row m is omega_m + scale_m (S cos y_m - C sin y_m) with (S, C) the sums of
// (sin y, cos y) over all rows: the row's own term cancels, so this is the coupling to every
// other node (Sec. 2, eq. KuramotoReformulation). Each stage folds the waves' sums in wave order
// (every thread reads the same LDS slots), so all threads hold identical (S, C); the slots
// alternate between stages, so one barrier per stage orders the writes and reads.
template <typename T>
__global__ __launch_bounds__(kPersistThreads) void k_persist_complete(PersistArgs<T> a)
{
    constexpr int NW = kPersistThreads / 64, R = kPersistMaxRows;
    __shared__ T red_s[2][NW], red_c[2][NW];
    __shared__ double rd_s[2][NW], rd_c[2][NW];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t n = a.n;
    T th[R], lo[R], ks[R], om[R], scl[R], sn[R], cs[R];
    int32_t wd[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int64_t m = tid + (int64_t)kPersistThreads * j;
        const bool ok = m < n;
        th[j] = ok ? a.hi[m] : T(0);
        lo[j] = ok ? a.lo[m] : T(0);
        wd[j] = ok ? a.wind[m] : 0;
        om[j] = ok ? a.omega[m] : T(0);
        scl[j] = ok ? a.K * (a.unit ? a.unit[m] : a.inv_n) : T(0);
        ks[j] = T(0);
        dev_sincos<T>(th[j], &sn[j], &cs[j]);
        if (!ok) sn[j] = cs[j] = T(0);  // padding rows add nothing to the sums
    }
    int buf = 0;
    for (int64_t step = 0; step <= a.nsteps; ++step) {
        const bool sample = a.r_every > 0 && step % a.r_every == 0 && (step < a.nsteps || a.final_sample);
        if (a.ck && step < a.nsteps && (a.step0 + step) % a.ck_every == 0) {
            T *ck = a.ck + 2 * n * ((a.step0 + step) / a.ck_every);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int64_t m = tid + (int64_t)kPersistThreads * j;
                if (m < n) {
                    ck[m] = th[j];
                    ck[n + m] = lo[j];
                }
            }
        }
        if (step == a.nsteps && !sample) break;
        for (int stage = 1; stage <= 4; ++stage) {
            T ps = T(0), pc = T(0);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                ps += sn[j];
                pc += cs[j];
            }
            ps = wave_sum_dpp(ps);
            pc = wave_sum_dpp(pc);
            const bool smp = stage == 1 && sample;
            if (lane == 63) {
                red_s[buf][w] = ps;
                red_c[buf][w] = pc;
            }
            if (smp) {
                // the order parameter of the phases at this step, summed in FP64
                double ds = 0.0, dc = 0.0;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    ds += (double)sn[j];
                    dc += (double)cs[j];
                }
                ds = wave_sum_dpp(ds);
                dc = wave_sum_dpp(dc);
                if (lane == 63) {
                    rd_s[buf][w] = ds;
                    rd_c[buf][w] = dc;
                }
            }
            __syncthreads();
            T S = red_s[buf][0], C = red_c[buf][0];
#pragma unroll
            for (int i = 1; i < NW; ++i) {
                S += red_s[buf][i];
                C += red_c[buf][i];
            }
            if (smp && tid == 0) {
                // the mean (sin, cos); k_persist_samples turns it into (r, psi)
                double DS = rd_s[buf][0], DC = rd_c[buf][0];
                for (int i = 1; i < NW; ++i) {
                    DS += rd_s[buf][i];
                    DC += rd_c[buf][i];
                }
                const double inv = 1.0 / (double)n;
                const int64_t k = step / a.r_every;
                a.r_out[k] = DS * inv;
                a.psi_out[k] = DC * inv;
            }
            buf ^= 1;
            if (step == a.nsteps) break;  // the last sample only
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const T k = om[j] + scl[j] * (S * cs[j] - C * sn[j]);
                const T y = rk4_stage<T>(stage, k, a.dt, a.half_dt, a.dt6, a.compensate, &ks[j], &th[j], &lo[j], &wd[j]);
                dev_sincos<T>(y, &sn[j], &cs[j]);
                if (tid + (int64_t)kPersistThreads * j >= n) sn[j] = cs[j] = T(0);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int64_t m = tid + (int64_t)kPersistThreads * j;
        if (m < n) {
            a.hi[m] = th[j];
            a.lo[m] = lo[j];
            a.wind[m] = wd[j];
        }
    }
}

// Sum four values over the workgroup in a fixed order: wave sums (DPP), then the waves' sums
// folded in wave order by every thread from LDS (slots alternate between calls via buf).
template <typename T, int NW>
__device__ __forceinline__ void persist_sum4(T v[4], T (*red)[4][NW], int &buf)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = wave_sum_dpp(v[q]);
    if (lane == 63)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[buf][q][w] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        T t = red[buf][q][0];
        for (int i = 1; i < NW; ++i) t += red[buf][q][i];
        v[q] = t;
    }
    buf ^= 1;
}

// One launch of the reverse sweep (see PersistAdjArgs). Per reverse RK4 step, with lam the
// gradient at the end of the step and stages i = 4, 3, 2, 1 ((s, c) = (sin, cos) of the stage
// input Y_i, kept by the recompute; S and C their sums over all rows; u the row scale):
//   l_4 = dt/6 lam, l_3 = dt/3 lam + dt mu_4, l_2 = dt/3 lam + dt/2 mu_3, l_1 = dt/6 lam + dt/2 mu_2
//   w = K u l,  mu_i = c (sum_k w_k c_k) + s (sum_k w_k s_k) - w (c C + s S)   (= J(Y_i)^T l_i)
//   lam <- lam + mu_1 + mu_2 + mu_3 + mu_4,  dL/domega += sum_i l_i,  dL/dK += sum_i <l_i, u (S c - C s)>
// (for the complete graph A = 1 1^T - I the row's own terms cancel in mu and in dF/dK).
template <typename T>
__global__ __launch_bounds__(kPersistThreads) void k_persist_adjoint(PersistAdjArgs<T> a)
{
    constexpr int NW = kPersistThreads / 64, R = kPersistMaxRows;
    __shared__ T red[2][4][NW];
    const int tid = threadIdx.x;
    const int64_t n = a.n;
    T lam[R], om[R], u[R];
    double gw[R];
    bool ok[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int64_t m = tid + (int64_t)kPersistThreads * j;
        ok[j] = m < n;
        lam[j] = ok[j] ? a.lam[m] : T(0);
        gw[j] = ok[j] ? a.g_omega[m] : 0.0;
        om[j] = ok[j] ? a.omega[m] : T(0);
        u[j] = ok[j] ? (a.unit ? a.unit[m] : a.inv_n) : T(0);
    }
    double gk = a.gk_part[tid];
    int buf = 0;
    for (int64_t seg = a.seg_hi; seg >= a.seg_lo; --seg) {
        const int64_t s0 = seg * a.ck_every;
        const int64_t len = a.nsteps - s0 < a.ck_every ? a.nsteps - s0 : a.ck_every;
        // recompute the segment from its checkpoint, keeping every stage input y
        T th[R], lo[R], ks[R], sn[R], cs[R];
        int32_t wd[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int64_t m = tid + (int64_t)kPersistThreads * j;
            th[j] = ok[j] ? a.ck[2 * n * seg + m] : T(0);
            lo[j] = ok[j] ? a.ck[2 * n * seg + n + m] : T(0);
            wd[j] = 0;
            ks[j] = T(0);
        }
        for (int64_t k = 0; k < len; ++k) {
            T y[R];
#pragma unroll
            for (int j = 0; j < R; ++j) y[j] = th[j];
            for (int stage = 1; stage <= 4; ++stage) {
                T v[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int64_t m = tid + (int64_t)kPersistThreads * j;
                    dev_sincos<T>(y[j], &sn[j], &cs[j]);
                    if (!ok[j]) sn[j] = cs[j] = T(0);
                    if (ok[j]) {
                        T *st = a.ystore + 2 * (4 * k + stage - 1) * n;
                        st[m] = sn[j];
                        st[n + m] = cs[j];
                    }
                    v[0] += sn[j];
                    v[1] += cs[j];
                }
                persist_sum4<T, NW>(v, red, buf);
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const T kk = om[j] + a.K * u[j] * (v[0] * cs[j] - v[1] * sn[j]);
                    y[j] = rk4_stage<T>(stage, kk, a.dt, a.half_dt, a.dt6, a.compensate, &ks[j], &th[j], &lo[j], &wd[j]);
                }
            }
        }
        // reverse sweep of the segment
        for (int64_t k = len - 1; k >= 0; --k) {
            T acc[R], mu[R], l[R];
            for (int stage = 4; stage >= 1; --stage) {
                T v[4] = {T(0), T(0), T(0), T(0)};
                T w[R];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int64_t m = tid + (int64_t)kPersistThreads * j;
                    const T *st = a.ystore + 2 * (4 * k + stage - 1) * n;
                    sn[j] = ok[j] ? st[m] : T(0);
                    cs[j] = ok[j] ? st[n + m] : T(0);
                    if (stage == 4) {
                        l[j] = a.dt6 * lam[j];
                        acc[j] = lam[j];
                    } else {
                        const T cl = stage == 1 ? a.dt6 : a.dt3;
                        const T cm = stage == 3 ? a.dt : a.half_dt;
                        l[j] = cl * lam[j] + cm * mu[j];
                    }
                    w[j] = a.K * u[j] * l[j];
                    v[0] += sn[j];
                    v[1] += cs[j];
                    v[2] += w[j] * sn[j];
                    v[3] += w[j] * cs[j];
                }
                persist_sum4<T, NW>(v, red, buf);
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    mu[j] = cs[j] * v[3] + sn[j] * v[2] - w[j] * (cs[j] * v[1] + sn[j] * v[0]);
                    const T dfdk = u[j] * (v[0] * cs[j] - v[1] * sn[j]);
                    gw[j] += (double)l[j];
                    gk += (double)l[j] * (double)dfdk;
                    acc[j] += mu[j];
                }
            }
#pragma unroll
            for (int j = 0; j < R; ++j) lam[j] = acc[j];
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int64_t m = tid + (int64_t)kPersistThreads * j;
        if (ok[j]) {
            a.lam[m] = lam[j];
            a.g_omega[m] = gw[j];
        }
    }
    a.gk_part[tid] = gk;
}

// (mean sin, mean cos) of every sample -> (r, psi), in place
__global__ __launch_bounds__(256) void k_persist_samples(int64_t count, double *__restrict__ r, double *__restrict__ psi)
{
    for (int64_t k = threadIdx.x; k < count; k += 256) {
        const double s = r[k], c = psi[k];
        r[k] = sqrt(s * s + c * c);
        psi[k] = atan2(s, c);
    }
}

template <typename T>
hipError_t launch_persist_complete(const PersistArgs<T> &a, hipStream_t st)
{
    if (a.n < 1 || a.n > (int64_t)kPersistThreads * kPersistMaxRows) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_persist_complete<T>), dim3(1), dim3(kPersistThreads), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.r_every <= 0) return e;
    const int64_t count = (a.nsteps - 1) / a.r_every + 1 + (a.final_sample && a.nsteps % a.r_every == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_persist_samples, dim3(1), dim3(256), 0, st, a.nsteps > 0 ? count : 1, a.r_out, a.psi_out);
    return hipGetLastError();
}
template hipError_t launch_persist_complete<float>(const PersistArgs<float> &, hipStream_t);
template hipError_t launch_persist_complete<double>(const PersistArgs<double> &, hipStream_t);

template <typename T>
hipError_t launch_persist_adjoint(const PersistAdjArgs<T> &a, hipStream_t st)
{
    if (a.n < 1 || a.n > (int64_t)kPersistThreads * kPersistMaxRows || a.ck_every < 1 || a.seg_lo < 0 ||
        a.seg_hi < a.seg_lo || a.seg_hi * a.ck_every >= a.nsteps)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_persist_adjoint<T>), dim3(1), dim3(kPersistThreads), 0, st, a);
    return hipGetLastError();
}
template hipError_t launch_persist_adjoint<float>(const PersistAdjArgs<float> &, hipStream_t);
template hipError_t launch_persist_adjoint<double>(const PersistAdjArgs<double> &, hipStream_t);

}  // namespace kur
