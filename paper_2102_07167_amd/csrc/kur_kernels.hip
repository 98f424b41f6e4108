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

// LDS gather of the (sin, cos) pair at a byte offset into the staged chunk
template <typename T2>
__device__ __forceinline__ T2 lds_at(const T2 *base, uint32_t byte_off)
{
    return *reinterpret_cast<const T2 *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Accumulate the 8 list entries of one 16-byte vector (two 16-bit byte offsets per dword).
template <typename T, typename T2>
__device__ __forceinline__ void gather8(const T2 *lds, const u32x4 q, T &xs, T &xc)
{
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T2 t0 = lds_at(lds, w[k] & 0xffffu);
        const T2 t1 = lds_at(lds, w[k] >> 16);
        xs += t0.x;
        xc += t0.y;
        xs += t1.x;
        xc += t1.y;
    }
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
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8))) void k_rows(DevGraph g, RowArgs<T> a)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int W = g.W;
    T2 *lds_sc = reinterpret_cast<T2 *>(smem);                 // W + 1 slots, slot W is zero
    T *acc_s = reinterpret_cast<T *>(lds_sc + W + 1);          // tile_rows
    T *acc_c = acc_s + g.tile_rows;                            // tile_rows
    T2 *red = reinterpret_cast<T2 *>(acc_c + g.tile_rows);     // NT/64 + 1
    int *bnd = reinterpret_cast<int *>(red + NT / 64 + 1);     // tile_rows + 1 row starts (vectors)

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
    const int ln = threadIdx.x & 63;
    // this wave's rows [ra, rb) in streaming mode (wave-uniform, kept in scalar registers)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ra = (int)(((int64_t)nrows * wv) / (NT / 64));
    const int rb = (int)(((int64_t)nrows * (wv + 1)) / (NT / 64));

    for (int c = 0; c < bi.nchunk; ++c) {
        const int64_t sb = bi.segbase + (int64_t)c * bi.size;
        const int64_t e0 = g.seg_ptr[sb + tl.r0], e1 = g.seg_ptr[sb + tl.r1];
        if (e0 == e1) continue;  // uniform over the workgroup
        const int c0 = c * W;
        const int cw = min(W, bi.size - c0);
        __syncthreads();  // previous chunk's gathers are done
        for (int j = threadIdx.x; j < cw; j += NT) lds_sc[j] = sc_in[bi.row0 + c0 + j];
        // row starts of this chunk, in 8-entry vectors relative to the tile's first one
        for (int r = threadIdx.x; r <= nrows; r += NT) bnd[r] = (int)((g.seg_ptr[sb + tl.r0 + r] - e0) >> 3);
        __syncthreads();
        const u32x4 *__restrict__ Lt = reinterpret_cast<const u32x4 *>(g.list + e0);
        if (flat) {
            // rows [ra, rb) occupy the contiguous 8-entry vectors [va, va + nvec) of this chunk
            const int va = __builtin_amdgcn_readfirstlane(bnd[ra]);
            const int nvec = __builtin_amdgcn_readfirstlane(bnd[rb]) - va;
            if (nvec > 0) {
                const u32x4 *__restrict__ L = Lt + va;
                int r = ra;
                int nbnd = __builtin_amdgcn_readfirstlane(bnd[r + 1]) - va;  // first vector after row r
                T as = T(0), ac = T(0);
                // rolling prefetch: four 64-vector spans in flight per wave; loads are issued
                // unconditionally (index clamped) so the in-order wait counts stay exact, and
                // lanes past the end are masked after the gather
                const uint32_t last = (uint32_t)(nvec - 1);
                u32x4 q0 = __builtin_nontemporal_load(L + min((uint32_t)ln, last));
                u32x4 q1 = __builtin_nontemporal_load(L + min((uint32_t)(64 + ln), last));
                u32x4 q2 = __builtin_nontemporal_load(L + min((uint32_t)(128 + ln), last));
                u32x4 q3 = __builtin_nontemporal_load(L + min((uint32_t)(192 + ln), last));
                auto span = [&](const u32x4 q, const int s0) {
                    T ps = T(0), pc = T(0);
                    gather8<T, T2>(lds_sc, q, ps, pc);
                    if (s0 + ln >= nvec) {
                        ps = T(0);
                        pc = T(0);
                    }
                    // rows that end inside (or right at the end of) this span
                    while (nbnd <= s0 + 64 && r < rb) {
                        if (s0 + ln < nbnd) {
                            as += ps;
                            ac += pc;
                            ps = T(0);
                            pc = T(0);
                        }
                        const T ts = wave_sum_dpp(as), tc = wave_sum_dpp(ac);
                        if (ln == 63) {
                            acc_s[r] += sign * ts;
                            acc_c[r] += sign * tc;
                        }
                        as = T(0);
                        ac = T(0);
                        ++r;
                        nbnd = r < rb ? __builtin_amdgcn_readfirstlane(bnd[r + 1]) - va : INT32_MAX;
                    }
                    as += ps;
                    ac += pc;
                };
                for (int s0 = 0; s0 < nvec; s0 += 256) {
                    span(q0, s0);
                    q0 = __builtin_nontemporal_load(L + min((uint32_t)(s0 + 256 + ln), last));
                    span(q1, s0 + 64);
                    q1 = __builtin_nontemporal_load(L + min((uint32_t)(s0 + 320 + ln), last));
                    span(q2, s0 + 128);
                    q2 = __builtin_nontemporal_load(L + min((uint32_t)(s0 + 384 + ln), last));
                    span(q3, s0 + 192);
                    q3 = __builtin_nontemporal_load(L + min((uint32_t)(s0 + 448 + ln), last));
                }
            }
        } else {
            for (int r = grp; r < nrows; r += ngrp) {
                const int v0 = bnd[r];
                const u32x4 *__restrict__ p = Lt + v0;
                const int nv = bnd[r + 1] - v0;
                T xs = T(0), xc = T(0);
                int v = lane;
                for (; v + G < nv; v += 2 * G) {
                    const u32x4 qa = __builtin_nontemporal_load(p + v);
                    const u32x4 qb = __builtin_nontemporal_load(p + v + G);
                    gather8<T, T2>(lds_sc, qa, xs, xc);
                    gather8<T, T2>(lds_sc, qb, xs, xc);
                }
                if (v < nv) gather8<T, T2>(lds_sc, __builtin_nontemporal_load(p + v), xs, xc);
                xs = group_sum_dpp(xs, G);
                xc = group_sum_dpp(xc, G);
                if (lane == G - 1) {
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
        xs = group_sum_dpp(xs, G);
        xc = group_sum_dpp(xc, G);
        if (lane == G - 1) {
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
               (size_t)(threads / 64 + 1) * 2 * elem_bytes + (size_t)(tile_rows + 1) * 4;
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
