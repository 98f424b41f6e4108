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

}  // namespace kur
