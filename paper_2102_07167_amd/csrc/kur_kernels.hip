// kur_kernels.hip -- gfx950 kernels of the Kuramoto-on-graphs right-hand side and RK4 stages.
//
// Data layout (block order, see kur_internal.hpp):
//   sc[m]      (sin y_m, cos y_m) of the current stage input y, as a 2-vector of T
//   part[t]    sum of sc over the rows of work tile t (deterministic, fixed order)
//   list       16-bit chunk-relative columns, segment per (block, chunk, row), padded to 8
//   inter      CSR over block-order columns outside the row's block
//
// One workgroup handles one tile (rows [r0, r1) of one diagonal block):
//   1. localised order parameters S_b, C_b of the block = fixed-order sum of the block's tile
//      partials (Sec. 3, eq. KuramotoGraphApproach: S_{M3,M4}, C_{M3,M4});
//   2. per column chunk: stage the chunk's (sin, cos) in LDS, then G lanes per row stream the
//      row's 16-bit list with 16-byte loads and gather from LDS; the zero entries of a dense
//      block are subtracted from (S_b, C_b), the one entries of a sparse block are added;
//   3. edges to other blocks: CSR gather from the global sc table;
//   4. epilogue, one lane per row: F_m = omega_m + scale_m ((sum A sin) cos y_m - (sum A cos) sin y_m)
//      (Sec. 3, eq. KuramotoGraphReformulation), then the RK4 stage bookkeeping, the next
//      stage input, its (sin, cos) and the tile partial for the next stage.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kur_internal.hpp"
#include "kur_kernels.hpp"

namespace kur {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };

template <typename T> __device__ __forceinline__ void dev_sincos(T x, T *s, T *c);
template <> __device__ __forceinline__ void dev_sincos<float>(float x, float *s, float *c) { sincosf(x, s, c); }
template <> __device__ __forceinline__ void dev_sincos<double>(double x, double *s, double *c) { sincos(x, s, c); }

template <typename T> __device__ __forceinline__ T dev_rint(T x);
template <> __device__ __forceinline__ float dev_rint<float>(float x) { return rintf(x); }
template <> __device__ __forceinline__ double dev_rint<double>(double x) { return rint(x); }

template <typename T> __device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T> __device__ __forceinline__ T group_sum(T v, int G)
{
    for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum v over the workgroup in a fixed order and store it to *out (thread 0).
template <typename T2, int NT>
__device__ __forceinline__ void block_sum_store(T2 v, T2 *red, T2 *out)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T2 s = red[0];
        for (int i = 1; i < NT / 64; ++i) {
            s.x += red[i].x;
            s.y += red[i].y;
        }
        *out = s;
    }
}

// (sin, cos) of the stage input and the tile partial: y from src (block order).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_sc_init(const Tile *__restrict__ tiles, const BlkInfo *__restrict__ blk,
                                                const T *__restrict__ y, typename V2<T>::type *__restrict__ sc,
                                                typename V2<T>::type *__restrict__ part)
{
    using T2 = typename V2<T>::type;
    __shared__ T2 red[NT / 64];
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const int row0 = blk[tl.block].row0 + tl.r0;
    const int nrows = tl.r1 - tl.r0;
    T2 acc;
    acc.x = T(0);
    acc.y = T(0);
    for (int r = threadIdx.x; r < nrows; r += NT) {
        T s, c;
        dev_sincos<T>(y[row0 + r], &s, &c);
        T2 v;
        v.x = s;
        v.y = c;
        sc[row0 + r] = v;
        acc.x += s;
        acc.y += c;
    }
    block_sum_store<T2, NT>(acc, red, part + t);
}

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

template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_rows(DevGraph g, RowArgs<T> a)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = g.W;
    T2 *lds_sc = reinterpret_cast<T2 *>(smem);                 // W + 1 slots, slot W is zero
    T *acc_s = reinterpret_cast<T *>(lds_sc + W + 1);          // tile_rows
    T *acc_c = acc_s + g.tile_rows;                            // tile_rows
    T2 *red = reinterpret_cast<T2 *>(acc_c + g.tile_rows);     // NT/64 + 1

    const int tile_id = g.order[blockIdx.x];
    const Tile tl = g.tiles[tile_id];
    const BlkInfo bi = g.blk[tl.block];
    const int nrows = tl.r1 - tl.r0;
    const int rowbase = bi.row0 + tl.r0;
    const T2 *__restrict__ sc_in = reinterpret_cast<const T2 *>(a.sc_in);
    const T2 *__restrict__ part_in = reinterpret_cast<const T2 *>(a.part_in);

    for (int r = threadIdx.x; r < nrows; r += NT) {
        acc_s[r] = T(0);
        acc_c[r] = T(0);
    }
    if (threadIdx.x == 0) {
        T2 z;
        z.x = T(0);
        z.y = T(0);
        lds_sc[W] = z;
    }
    // localised order parameters of the block: fixed-order sum of its tile partials
    if (bi.mode && threadIdx.x < 64) {
        T sx = T(0), sy = T(0);
        for (int i = threadIdx.x; i < bi.ntiles; i += 64) {
            T2 p = part_in[bi.tile0 + i];
            sx += p.x;
            sy += p.y;
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (threadIdx.x == 0) {
            T2 s;
            s.x = sx;
            s.y = sy;
            red[NT / 64] = s;
        }
    }
    __syncthreads();  // accumulators, pad slot and block sums visible to every wave

    // G > 0: G lanes per row (short rows); G == 0: every wave streams a contiguous run of rows
    const bool flat = tl.G == 0;
    const int G = flat ? 8 : tl.G;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int ngrp = NT / G;
    const T sign = bi.mode ? T(-1) : T(1);
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    const int ra = (int)(((int64_t)nrows * wv) / (NT / 64));
    const int rb = (int)(((int64_t)nrows * (wv + 1)) / (NT / 64));
    const uint32_t padw = (uint32_t)W | ((uint32_t)W << 16);

    for (int c = 0; c < bi.nchunk; ++c) {
        const int64_t sb = bi.segbase + (int64_t)c * bi.size;
        const int64_t e0 = g.seg_ptr[sb + tl.r0], e1 = g.seg_ptr[sb + tl.r1];
        if (e0 == e1) continue;  // uniform over the workgroup
        const int c0 = c * W;
        const int cw = min(W, bi.size - c0);
        __syncthreads();  // previous chunk's gathers are done
        for (int j = threadIdx.x; j < cw; j += NT) lds_sc[j] = sc_in[bi.row0 + c0 + j];
        __syncthreads();
        if (flat) {
            // rows [ra, rb) of this wave occupy the contiguous vectors [va, vb) of the chunk
            const int64_t *__restrict__ sp = g.seg_ptr + sb + tl.r0;
            const int64_t va = sp[ra] >> 3, vb = sp[rb] >> 3;
            if (va < vb) {
                const u32x4 *__restrict__ L = reinterpret_cast<const u32x4 *>(g.list);
                int r = ra;
                int64_t nbnd = sp[r + 1] >> 3;  // first vector after row r
                T as = T(0), ac = T(0);
                constexpr int U = 4;
                u32x4 q[U];
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int64_t vi = va + 64 * j + ln;
                    q[j] = vi < vb ? __builtin_nontemporal_load(L + vi) : u32x4{padw, padw, padw, padw};
                }
                for (int64_t base = va; base < vb; base += 64 * U) {
                    u32x4 qn[U];
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        const int64_t vi = base + 64 * (U + j) + ln;
                        qn[j] = vi < vb ? __builtin_nontemporal_load(L + vi) : u32x4{padw, padw, padw, padw};
                    }
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        const uint32_t w4[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
                        T ps = T(0), pc = T(0);
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const T2 t0 = lds_sc[w4[k] & 0xffffu];
                            const T2 t1 = lds_sc[w4[k] >> 16];
                            ps += t0.x;
                            pc += t0.y;
                            ps += t1.x;
                            pc += t1.y;
                        }
                        const int64_t s0 = base + 64 * j;
                        const int64_t vi = s0 + ln;
                        // rows ending inside (or right at the end of) this 64-vector span
                        while (nbnd <= s0 + 64 && r < rb) {
                            if (vi < nbnd) {
                                as += ps;
                                ac += pc;
                                ps = T(0);
                                pc = T(0);
                            }
                            const T ts = wave_sum(as), tc = wave_sum(ac);
                            if (ln == 0) {
                                acc_s[r] += sign * ts;
                                acc_c[r] += sign * tc;
                            }
                            as = T(0);
                            ac = T(0);
                            ++r;
                            nbnd = r < rb ? (sp[r + 1] >> 3) : INT64_MAX;
                        }
                        as += ps;
                        ac += pc;
                        q[j] = qn[j];
                    }
                }
            }
        } else {
            for (int r = grp; r < nrows; r += ngrp) {
                const int64_t s0 = g.seg_ptr[sb + tl.r0 + r], s1 = g.seg_ptr[sb + tl.r0 + r + 1];
                const u32x4 *__restrict__ p = reinterpret_cast<const u32x4 *>(g.list + s0);
                const int nv = (int)((s1 - s0) >> 3);
                T xs = T(0), xc = T(0);
                int v = lane;
                for (; v + G < nv; v += 2 * G) {
                    const u32x4 q0 = __builtin_nontemporal_load(p + v);
                    const u32x4 q1 = __builtin_nontemporal_load(p + v + G);
                    const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const T2 t0 = lds_sc[w[k] & 0xffffu];
                        const T2 t1 = lds_sc[w[k] >> 16];
                        xs += t0.x;
                        xc += t0.y;
                        xs += t1.x;
                        xc += t1.y;
                    }
                }
                if (v < nv) {
                    const u32x4 q0 = __builtin_nontemporal_load(p + v);
                    const uint32_t w[4] = {q0.x, q0.y, q0.z, q0.w};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const T2 t0 = lds_sc[w[k] & 0xffffu];
                        const T2 t1 = lds_sc[w[k] >> 16];
                        xs += t0.x;
                        xc += t0.y;
                        xs += t1.x;
                        xc += t1.y;
                    }
                }
                xs = group_sum(xs, G);
                xc = group_sum(xc, G);
                if (lane == 0) {
                    acc_s[r] += sign * xs;
                    acc_c[r] += sign * xc;
                }
            }
        }
    }

    // edges between blocks: straightforward summation from the global table. In streaming mode
    // another wave owns the row's accumulator above, so wait for those updates first.
    if (flat) __syncthreads();
    for (int r = grp; r < nrows; r += ngrp) {
        const int m = rowbase + r;
        const int64_t e0 = g.inter_ptr[m], e1 = g.inter_ptr[m + 1];
        if (e0 == e1) continue;  // uniform over the group
        T xs = T(0), xc = T(0);
        for (int64_t e = e0 + lane; e < e1; e += G) {
            const T2 t = sc_in[g.inter_col[e]];
            xs += t.x;
            xc += t.y;
        }
        xs = group_sum(xs, G);
        xc = group_sum(xc, G);
        if (lane == 0) {
            acc_s[r] += xs;
            acc_c[r] += xc;
        }
    }
    __syncthreads();

    T Sb = T(0), Cb = T(0);
    if (bi.mode) {
        Sb = red[NT / 64].x;
        Cb = red[NT / 64].y;
    }
    T2 part;
    part.x = T(0);
    part.y = T(0);
    for (int r = threadIdx.x; r < nrows; r += NT) {
        const int m = rowbase + r;
        const T2 scm = sc_in[m];
        const T As = Sb + acc_s[r];
        const T Ac = Cb + acc_c[r];
        const T scale = a.rowscale ? a.rowscale[m] : a.kscale;
        const T k = a.omega[m] + scale * (As * scm.y - Ac * scm.x);
        if (a.stage == 0) {
            a.kout[m] = k;
            continue;
        }
        const T th = a.hi[m];
        T y;
        if (a.stage == 1) {
            a.ksum[m] = k;
            y = th + a.half_dt * k;
        } else if (a.stage == 2) {
            a.ksum[m] += T(2) * k;
            y = th + a.half_dt * k;
        } else if (a.stage == 3) {
            a.ksum[m] += T(2) * k;
            y = th + a.dt * k;
        } else {
            const T delta = a.dt6 * (a.ksum[m] + k);
            T hi, lo;
            int wd = a.wind[m];
            if (a.compensate) {
                T d1, e1, s, e2;
                two_sum(delta, a.lo[m], d1, e1);
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
            hi = s2;
            lo = e3;
            a.hi[m] = hi;
            a.lo[m] = lo;
            a.wind[m] = wd;
            y = hi;
        }
        T s, c;
        dev_sincos<T>(y, &s, &c);
        T2 v;
        v.x = s;
        v.y = c;
        reinterpret_cast<T2 *>(a.sc_out)[m] = v;
        part.x += s;
        part.y += c;
    }
    if (a.stage != 0) block_sum_store<T2, NT>(part, red, reinterpret_cast<T2 *>(a.part_out) + tile_id);
}

// r e^{i psi} = (1/N) sum_m e^{i theta_m} from the tile partials (Sec. 2, eq. OrderParameter).
template <typename T>
__global__ __launch_bounds__(256) void k_order(const typename V2<T>::type *__restrict__ part, int ntiles, double inv_n,
                                               double *__restrict__ r_out, double *__restrict__ psi_out,
                                               int64_t idx)
{
    __shared__ double rs[4], rc[4];
    double s = 0.0, c = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 256) {
        s += (double)part[t].x;
        c += (double)part[t].y;
    }
    s = wave_sum(s);
    c = wave_sum(c);
    if ((threadIdx.x & 63) == 0) {
        rs[threadIdx.x >> 6] = s;
        rc[threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s = rs[0] + rs[1] + rs[2] + rs[3];
        c = rc[0] + rc[1] + rc[2] + rc[3];
        s *= inv_n;
        c *= inv_n;
        r_out[idx] = sqrt(s * s + c * c);
        psi_out[idx] = atan2(s, c);
    }
}

// out[m] = hi + lo (+ 2 pi wind)
template <typename T>
__global__ void k_phase_out(int64_t n, const T *__restrict__ hi, const T *__restrict__ lo, const int32_t *__restrict__ wind,
                            int unwrapped, T *__restrict__ out)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    T v = hi[m] + lo[m];
    if (unwrapped) v += (T)wind[m] * TwoPi<T>::P1 + (T)wind[m] * TwoPi<T>::P2;
    out[m] = v;
}

// ------------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------------

template <typename T>
hipError_t launch_sc_init(const DevGraph &g, int ntiles, const T *y, void *sc, void *part, int threads,
                          hipStream_t st)
{
    using T2 = typename V2<T>::type;
    if (ntiles <= 0) return hipSuccess;
    switch (threads) {
    case 256: hipLaunchKernelGGL((k_sc_init<T, 256>), dim3(ntiles), dim3(256), 0, st, g.tiles, g.blk, y, (T2 *)sc, (T2 *)part); break;
    case 1024: hipLaunchKernelGGL((k_sc_init<T, 1024>), dim3(ntiles), dim3(1024), 0, st, g.tiles, g.blk, y, (T2 *)sc, (T2 *)part); break;
    default: hipLaunchKernelGGL((k_sc_init<T, 512>), dim3(ntiles), dim3(512), 0, st, g.tiles, g.blk, y, (T2 *)sc, (T2 *)part); break;
    }
    return hipGetLastError();
}

size_t rows_lds_bytes(int elem_bytes, int W, int tile_rows, int threads)
{
    size_t b = (size_t)(W + 1) * 2 * elem_bytes + (size_t)2 * tile_rows * elem_bytes +
               (size_t)(threads / 64 + 1) * 2 * elem_bytes;
    return (b + 15) & ~size_t(15);
}

template <typename T>
hipError_t launch_rows(const DevGraph &g, int ntiles, const RowArgs<T> &a, int threads, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const size_t lds = rows_lds_bytes(sizeof(T), g.W, g.tile_rows, threads);
    static bool attr_done[3] = {false, false, false};
    const int slot = threads == 256 ? 0 : threads == 1024 ? 2 : 1;
    if (!attr_done[slot]) {
        const void *fn = threads == 256 ? reinterpret_cast<const void *>(&k_rows<T, 256>)
                         : threads == 1024 ? reinterpret_cast<const void *>(&k_rows<T, 1024>)
                                           : reinterpret_cast<const void *>(&k_rows<T, 512>);
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_done[slot] = true;
    }
    switch (threads) {
    case 256: hipLaunchKernelGGL((k_rows<T, 256>), dim3(ntiles), dim3(256), lds, st, g, a); break;
    case 1024: hipLaunchKernelGGL((k_rows<T, 1024>), dim3(ntiles), dim3(1024), lds, st, g, a); break;
    default: hipLaunchKernelGGL((k_rows<T, 512>), dim3(ntiles), dim3(512), lds, st, g, a); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_order(const void *part, int ntiles, int64_t n, double *r, double *psi, int64_t idx, hipStream_t st)
{
    using T2 = typename V2<T>::type;
    hipLaunchKernelGGL((k_order<T>), dim3(1), dim3(256), 0, st, (const T2 *)part, ntiles, 1.0 / (double)n, r, psi, idx);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phase_out(int64_t n, const void *hi, const void *lo, const int32_t *wind, int unwrapped, void *out,
                            hipStream_t st)
{
    const int bs = 256;
    hipLaunchKernelGGL((k_phase_out<T>), dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, n, (const T *)hi,
                       (const T *)lo, wind, unwrapped, (T *)out);
    return hipGetLastError();
}

template hipError_t launch_sc_init<float>(const DevGraph &, int, const float *, void *, void *, int, hipStream_t);
template hipError_t launch_sc_init<double>(const DevGraph &, int, const double *, void *, void *, int, hipStream_t);
template hipError_t launch_rows<float>(const DevGraph &, int, const RowArgs<float> &, int, hipStream_t);
template hipError_t launch_rows<double>(const DevGraph &, int, const RowArgs<double> &, int, hipStream_t);
template hipError_t launch_order<float>(const void *, int, int64_t, double *, double *, int64_t, hipStream_t);
template hipError_t launch_order<double>(const void *, int, int64_t, double *, double *, int64_t, hipStream_t);
template hipError_t launch_phase_out<float>(int64_t, const void *, const void *, const int32_t *, int, void *, hipStream_t);
template hipError_t launch_phase_out<double>(int64_t, const void *, const void *, const int32_t *, int, void *, hipStream_t);

double two_pi_p1(int elem_bytes) { return elem_bytes == 4 ? (double)TwoPi<float>::P1 : TwoPi<double>::P1; }
double two_pi_p2(int elem_bytes) { return elem_bytes == 4 ? (double)TwoPi<float>::P2 : TwoPi<double>::P2; }

}  // namespace kur
