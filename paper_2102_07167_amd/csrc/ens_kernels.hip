// ens_kernels.hip -- gfx950 kernels of the shared-graph ensemble path.
//
// With B replicas of one graph, the coupling sums of a row for all replicas at once are the row
// of A X with X = [sin Theta, cos Theta] (n x 2B). For a dense submatrix (a community block, or
// a dense off-diagonal block of two communities) this is a real matrix product A_{a,c} X_c
// (Sec. 3: the block structure and its extension to submatrices; eq.
// KuramotoGraphReformulation: the sine difference expanded into sums of sin and cos). The
// products of one row block's ranges accumulate in one pass along k; k_ens_gemm runs them on the
// matrix cores:
//   * A_b is 0/1 and stored as a bitmask; each lane expands one byte into eight bf16 ones and
//     zeros (exact) by two lookups in a 16-entry nibble table in LDS;
//   * X is split exactly into three bf16 terms x = t0 + t1 + t2 (each the truncated upper half
//     of the remainder: 8 + 8 + 8 significant bits cover the 24 of FP32), so every product is
//     exact and only the FP32 accumulation of the matrix core rounds;
//   * v_mfma_f32_32x32x16_bf16, a 256 x 128 output tile per workgroup (four waves of 64 rows,
//     two 32-row by four 32-column tiles each, so every LDS read of X feeds two products); X is
//     staged in LDS per 32 columns of A, double-buffered, with the next step's X and pattern
//     words loaded into registers while the matrix cores run (512-row tiles, halving the
//     staging per product, measured no faster).
// k_ens_rows then adds the CSR edges (sparse blocks and inter-block edges) by gathering whole
// X rows (all replicas contiguous), and runs the stage epilogue of every replica:
// F = omega + K_e / N ((sum A sin) cos y - (sum A cos) sin y), the RK4 bookkeeping and the next
// stage's (sin, cos).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ens.hpp"
#include "kur_device.hpp"

namespace kur {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_e __attribute__((ext_vector_type(4)));

// bits 0..7 of b as eight bf16 values (bit v -> element v): 1.0 = 0x3F80, 0.0 = 0
// the four bf16 values of a nibble's bits (bit v -> element v), as two words
__device__ __forceinline__ uint2 nibble_bf16(uint32_t n)
{
    uint2 v;
    v.x = ((n >> 0) & 1u) * 0x3F80u | ((n >> 1) & 1u) * 0x3F800000u;
    v.y = ((n >> 2) & 1u) * 0x3F80u | ((n >> 3) & 1u) * 0x3F800000u;
    return v;
}

// bits 8 g .. 8 g + 7 of w as eight bf16 values, from a 16-entry table of nibbles in LDS
__device__ __forceinline__ bf16x8 expand_byte(const uint2 *tab, uint32_t w, int g)
{
    const uint2 lo = tab[(w >> (8 * g)) & 15u], hi = tab[(w >> (8 * g + 4)) & 15u];
    u32x4_e v;
    v.x = lo.x;
    v.y = lo.y;
    v.z = hi.x;
    v.w = hi.y;
    return __builtin_bit_cast(bf16x8, v);
}


// x = t0 + t1 + t2 exactly, each term a bf16 (the upper half of a float): t0 keeps the upper
// half of x (8 significant bits), the remainder x - t0 is exact and has at most 16 significant
// bits, of which t1 keeps the upper 8; the last remainder has at most 8 and is t2 itself. Done
// for two values a, b at once and packed as the B operand wants them: word t holds term t of a
// (low 16 bits) and of b (high 16 bits). v_perm_b32 with selector 0x07060302 takes bytes 2-3 of
// its second operand and bytes 2-3 of its first.
__device__ __forceinline__ void split3_pair(float a, float b, uint32_t &p0, uint32_t &p1, uint32_t &p2)
{
    const uint32_t ua = __float_as_uint(a), ub = __float_as_uint(b);
    const float ra = a - __uint_as_float(ua & 0xFFFF0000u), rb = b - __uint_as_float(ub & 0xFFFF0000u);
    const uint32_t va = __float_as_uint(ra), vb = __float_as_uint(rb);
    const float qa = ra - __uint_as_float(va & 0xFFFF0000u), qb = rb - __uint_as_float(vb & 0xFFFF0000u);
    p0 = __builtin_amdgcn_perm(ub, ua, 0x07060302u);
    p1 = __builtin_amdgcn_perm(vb, va, 0x07060302u);
    p2 = __builtin_amdgcn_perm(__float_as_uint(qb), __float_as_uint(qa), 0x07060302u);
}

// kEnsTileRows / 64 waves, each owning 64 rows; the X staging of a 32-wide k step (4 groups of
// 8 k for 128 columns) is spread over all threads: SGN threads per column, NG groups each
constexpr int kGemmThreads = kEnsTileRows;
constexpr int kStageSGN = kGemmThreads / kEnsTileCols;
constexpr int kStageNG = 4 / kStageSGN;
static_assert(kStageSGN * kStageNG == 4, "staging covers the four 8-wide groups of a step");

__global__ __launch_bounds__(kGemmThreads) void k_ens_gemm(EnsGemmArgs a)
{
    // double buffer of [term][group of 8 k][column]: 8 bf16 of one column, the layout of the B
    // operand; step i is staged into buffer i & 1 while the matrix cores work on the other
    __shared__ u32x4_e xs[2][3][4][kEnsTileCols];
    __shared__ uint2 ntab[16];  // read after the first barrier of the k loop
    if (threadIdx.x < 16) ntab[threadIdx.x] = nibble_bf16(threadIdx.x);
    const EnsItem it = a.items[blockIdx.x];
    const EnsBlk b = a.blk[it.blk];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, half = lane >> 5, l32 = lane & 31;
    // A operand: each wave owns 64 rows as two 32-row tiles; lane holds row l32 of each tile and
    // k = 8 half + v of each 16-wide k step
    const int arow0 = it.r0 + wave * 64 + l32, arow1 = arow0 + 32;
    const bool ok0 = arow0 < b.size, ok1 = arow1 < b.size;
    const uint32_t *ab0 = a.bits + b.bits_off + (int64_t)(ok0 ? arow0 : 0) * b.words;
    const uint32_t *ab1 = a.bits + b.bits_off + (int64_t)(ok1 ? arow1 : 0) * b.words;
    // staging: thread -> one column, k groups sg, sg + SGN, ... of each 32-wide step
    const int sc = tid & (kEnsTileCols - 1), sg = tid >> 7;
    // range of the next load: k only grows and every 32-wide step lies in one range, so the
    // table is read again only where the next range begins
    const EnsRng *rg = a.rng + b.rng0;
    int rl = 0;
    int r_koff = __builtin_amdgcn_readfirstlane(rg[0].koff), r_col0 = __builtin_amdgcn_readfirstlane(rg[0].col0),
        r_len = __builtin_amdgcn_readfirstlane(rg[0].len);
    int next_koff = b.nrng > 1 ? __builtin_amdgcn_readfirstlane(rg[1].koff) : INT32_MAX;
    f32x16 acc[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[rt][c][r] = 0.f;

    const int kend = b.words * 32;
    float v[kStageNG][8];
    // X rows of a step are addressed from a workgroup-uniform base (the range's first row, the
    // tile's first column) with 32-bit per-lane offsets (k J + sc < 2^31 inside one range)
    const uint32_t Ju = (uint32_t)a.J;
    auto load = [&](int k0) {
        if (k0 >= next_koff) {
            ++rl;
            r_koff = __builtin_amdgcn_readfirstlane(rg[rl].koff);
            r_col0 = __builtin_amdgcn_readfirstlane(rg[rl].col0);
            r_len = __builtin_amdgcn_readfirstlane(rg[rl].len);
            next_koff = rl + 1 < b.nrng ? __builtin_amdgcn_readfirstlane(rg[rl + 1].koff) : INT32_MAX;
        }
        const float *xb = reinterpret_cast<const float *>(a.x) + (int64_t)r_col0 * a.J + it.c0;
        const int kl = k0 - r_koff;
        if (kl + 32 <= r_len) {
            // the whole step inside the range: rows kl + 8 (sg + SGN gi) + i, no clamps
#pragma unroll
            for (int gi = 0; gi < kStageNG; ++gi) {
                const uint32_t off = (uint32_t)(kl + 8 * (sg + kStageSGN * gi)) * Ju + (uint32_t)sc;
#pragma unroll
                for (int i = 0; i < 8; ++i) v[gi][i] = xb[off + (uint32_t)i * Ju];
            }
            return;
        }
#pragma unroll
        for (int gi = 0; gi < kStageNG; ++gi)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                // unconditional load of a clamped row (no branch per load), then the mask
                const int k = kl + 8 * (sg + kStageSGN * gi) + i;
                const float t = xb[(uint32_t)(k < r_len ? k : r_len - 1) * Ju + (uint32_t)sc];
                v[gi][i] = k < r_len ? t : 0.f;
            }
    };
    load(0);
    uint32_t w0 = ab0[0], w1 = ab1[0];
    w0 = ok0 ? w0 : 0u;
    w1 = ok1 ? w1 : 0u;
    int buf = 0;
    for (int k0 = 0; k0 < kend; k0 += 32) {
#pragma unroll
        for (int gi = 0; gi < kStageNG; ++gi) {
            uint32_t q0[4], q1[4], q2[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) split3_pair(v[gi][2 * j], v[gi][2 * j + 1], q0[j], q1[j], q2[j]);
            u32x4_e p0, p1, p2;
            p0.x = q0[0]; p0.y = q0[1]; p0.z = q0[2]; p0.w = q0[3];
            p1.x = q1[0]; p1.y = q1[1]; p1.z = q1[2]; p1.w = q1[3];
            p2.x = q2[0]; p2.y = q2[1]; p2.z = q2[2]; p2.w = q2[3];
            const int g = sg + kStageSGN * gi;
            xs[buf][0][g][sc] = p0;
            xs[buf][1][g][sc] = p1;
            xs[buf][2][g][sc] = p2;
        }
        // one barrier per step: a wave past it has finished its reads of the other buffer
        // (step - 1), which the next step overwrites
        __syncthreads();
        const uint32_t c0 = w0, c1 = w1;
        if (k0 + 32 < kend) {
            load(k0 + 32);
            const uint32_t n0 = ab0[(k0 >> 5) + 1], n1 = ab1[(k0 >> 5) + 1];
            w0 = ok0 ? n0 : 0u;
            w1 = ok1 ? n1 : 0u;
        }
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            const int g = 2 * sub + half;
            const bf16x8 av0 = expand_byte(ntab, c0, g);
            const bf16x8 av1 = expand_byte(ntab, c1, g);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct)
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    // one LDS read feeds both row tiles
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, xs[buf][t][g][ct * 32 + l32]);
                    acc[0][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av0, bv, acc[0][ct], 0, 0, 0);
                    acc[1][ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av1, bv, acc[1][ct], 0, 0, 0);
                }
        }
        buf ^= 1;
    }
    // result: lane column l32, register r -> row 8 (r / 4) + 4 half + (r % 4) of the 32-row tile
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = it.r0 + wave * 64 + rt * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
                if (row < b.size)
                    reinterpret_cast<float *>(a.y)[(int64_t)(b.row0 + row) * a.J + it.c0 + ct * 32 + l32] = acc[rt][ct][r];
            }
}

// FP64 products on the FP64 matrix cores with v_mfma_f64_16x16x4f64, whose operands are laid
// out as follows: lane l holds A[l % 16][l / 16] of the 16 x 4 A tile and B[l / 16][l % 16] of
// the 4 x 16 B tile, and register j of lane l holds D[l / 16 + 4 j][l % 16] of the 16 x 16
// result. A workgroup computes a 128 x 64 tile of Y = sum_c A_{a,c} X_c over the row block's
// ranges: four waves of 32 rows, each two 16-row by four 16-column tiles. The 0/1 entries of A
// enter as exact 0.0 and 1.0, so only the FP64 accumulation rounds. X is staged in LDS per 32
// columns of A, double-buffered, with the next step's X and pattern words loaded into
// registers while the matrix cores run; the LDS row pitch puts the k rows read by the two
// halves of a wave on different banks.
constexpr int kF64Pitch = kEnsTileColsF64 + 16;

__global__ __launch_bounds__(256) void k_ens_gemm_f64(EnsGemmArgs a)
{
    typedef double d4 __attribute__((ext_vector_type(4)));
    __shared__ double xs[2][32][kF64Pitch];
    const EnsItem it = a.items[blockIdx.x];
    const EnsBlk b = a.blk[it.blk];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, kq = lane >> 4;
    const int arow0 = it.r0 + wave * 32 + l16, arow1 = arow0 + 16;
    const bool ok0 = arow0 < b.size, ok1 = arow1 < b.size;
    const uint32_t *ab0 = a.bits + b.bits_off + (int64_t)(ok0 ? arow0 : 0) * b.words;
    const uint32_t *ab1 = a.bits + b.bits_off + (int64_t)(ok1 ? arow1 : 0) * b.words;
    // staging: thread -> one column, k rows 8 sg .. 8 sg + 7 of each 32-wide step
    const int sc = tid & (kEnsTileColsF64 - 1), sg = tid >> 6;
    const double *X = reinterpret_cast<const double *>(a.x);
    const EnsRng *rg = a.rng + b.rng0;
    int rl = 0;
    int r_koff = __builtin_amdgcn_readfirstlane(rg[0].koff), r_col0 = __builtin_amdgcn_readfirstlane(rg[0].col0),
        r_len = __builtin_amdgcn_readfirstlane(rg[0].len);
    int next_koff = b.nrng > 1 ? __builtin_amdgcn_readfirstlane(rg[1].koff) : INT32_MAX;
    const uint32_t Ju = (uint32_t)a.J;
    double v[8];
    auto load = [&](int k0) {
        if (k0 >= next_koff) {
            ++rl;
            r_koff = __builtin_amdgcn_readfirstlane(rg[rl].koff);
            r_col0 = __builtin_amdgcn_readfirstlane(rg[rl].col0);
            r_len = __builtin_amdgcn_readfirstlane(rg[rl].len);
            next_koff = rl + 1 < b.nrng ? __builtin_amdgcn_readfirstlane(rg[rl + 1].koff) : INT32_MAX;
        }
        const double *xb = X + (int64_t)r_col0 * a.J + it.c0;
        const int kl = k0 - r_koff + 8 * sg;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            // unconditional load of a clamped row, then the mask
            const int k = kl + i;
            const double t = xb[(uint32_t)(k < r_len ? k : r_len - 1) * Ju + (uint32_t)sc];
            v[i] = k < r_len ? t : 0.0;
        }
    };
    d4 acc[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = d4{0.0, 0.0, 0.0, 0.0};
    const int kend = b.words * 32;
    load(0);
    uint32_t w0 = ab0[0], w1 = ab1[0];
    w0 = ok0 ? w0 : 0u;
    w1 = ok1 ? w1 : 0u;
    int buf = 0;
    for (int k0 = 0; k0 < kend; k0 += 32) {
#pragma unroll
        for (int i = 0; i < 8; ++i) xs[buf][8 * sg + i][sc] = v[i];
        // one barrier per step: a wave past it has finished its reads of the other buffer
        // (step - 1), which the next step overwrites
        __syncthreads();
        const uint32_t c0 = w0, c1 = w1;
        if (k0 + 32 < kend) {
            load(k0 + 32);
            const uint32_t n0 = ab0[(k0 >> 5) + 1], n1 = ab1[(k0 >> 5) + 1];
            w0 = ok0 ? n0 : 0u;
            w1 = ok1 ? n1 : 0u;
        }
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const double a0 = ((c0 >> (4 * kk + kq)) & 1u) ? 1.0 : 0.0;
            const double a1 = ((c1 >> (4 * kk + kq)) & 1u) ? 1.0 : 0.0;
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const double bv = xs[buf][4 * kk + kq][ct * 16 + l16];
                acc[0][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv, acc[0][ct], 0, 0, 0);
                acc[1][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv, acc[1][ct], 0, 0, 0);
            }
        }
        buf ^= 1;
    }
    double *Y = reinterpret_cast<double *>(a.y);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int row = it.r0 + wave * 32 + rt * 16 + kq + 4 * j;
                if (row < b.size) Y[(int64_t)(b.row0 + row) * a.J + it.c0 + ct * 16 + l16] = acc[rt][ct][j];
            }
}

// One wave per row; lane l handles replicas l + 64 q, q < NE. Every load of the row's own data
// (dense-block sums, stage input, omega and the RK4 state) is issued before the CSR gathers, so
// a wave waits on memory about as often as it has groups of CSR entries.
template <typename T, int NE>
__global__ __launch_bounds__(256) void k_ens_rows(EnsRowArgs<T> a)
{
    constexpr int GRP = NE <= 2 ? 8 : 4;  // CSR entries gathered per round
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (m >= a.n) return;
    const int64_t Bp = a.Bp;
    const int64_t J = 2 * Bp;
    const int stage = a.stage;
    // y holds rows of matrix-core blocks only: the branch is uniform over the wave
    const bool dense = __builtin_amdgcn_readfirstlane((int)a.row_gemm[m]) != 0;
    T as[NE], ac[NE], sm[NE], cm[NE], om[NE], th[NE], ks[NE], lo[NE];
    int32_t wd[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        as[q] = T(0);
        ac[q] = T(0);
    }
    if (dense) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            as[q] = a.y[m * J + lane + 64 * q];
            ac[q] = a.y[m * J + Bp + lane + 64 * q];
        }
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int64_t e = lane + 64 * q;
        const int64_t ix = m * Bp + e;
        sm[q] = a.x[m * J + e];
        cm[q] = a.x[m * J + Bp + e];
        om[q] = a.omega[ix];
        th[q] = a.hi[ix];
        ks[q] = stage >= 2 ? a.ksum[ix] : T(0);
        lo[q] = stage == 4 ? a.lo[ix] : T(0);
        wd[q] = stage == 4 ? a.wind[ix] : 0;
    }
    const int64_t p0 = a.csr_ptr[m], p1 = a.csr_ptr[m + 1];
    int64_t p = p0;
    for (; p + GRP <= p1; p += GRP) {
        int64_t col[GRP];
#pragma unroll
        for (int i = 0; i < GRP; ++i) col[i] = a.csr_col[p + i];
        T vs[GRP][NE], vc[GRP][NE];
#pragma unroll
        for (int i = 0; i < GRP; ++i)
#pragma unroll
            for (int q = 0; q < NE; ++q) {
                vs[i][q] = a.x[col[i] * J + lane + 64 * q];
                vc[i][q] = a.x[col[i] * J + Bp + lane + 64 * q];
            }
#pragma unroll
        for (int i = 0; i < GRP; ++i)
#pragma unroll
            for (int q = 0; q < NE; ++q) {
                as[q] += vs[i][q];
                ac[q] += vc[i][q];
            }
    }
    for (; p < p1; ++p) {
        const int64_t col = a.csr_col[p];
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            as[q] += a.x[col * J + lane + 64 * q];
            ac[q] += a.x[col * J + Bp + lane + 64 * q];
        }
    }
#pragma unroll
    for (int q = 0; q < NE; ++q) {
        const int64_t e = lane + 64 * q;
        const int64_t ix = m * Bp + e;
        const T k = om[q] + a.unit[e] * (as[q] * cm[q] - ac[q] * sm[q]);
        if (stage == 0) {
            a.kout[ix] = k;
            continue;
        }
        const T y = rk4_stage<T>(stage, k, a.dt, a.half_dt, a.dt6, a.compensate, &ks[q], &th[q], &lo[q], &wd[q]);
        a.ksum[ix] = ks[q];
        if (stage == 4) {
            a.hi[ix] = th[q];
            a.lo[ix] = lo[q];
            a.wind[ix] = wd[q];
        }
        T sy, cy;
        dev_sincos<T>(y, &sy, &cy);
        a.x_out[m * J + e] = sy;
        a.x_out[m * J + Bp + e] = cy;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_ens_sincos(int64_t n, int32_t Bp, const T *__restrict__ hi, T *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n * Bp) return;
    const int64_t m = i / Bp, e = i - m * Bp;
    T s, c;
    dev_sincos<T>(hi[i], &s, &c);
    x[m * 2 * Bp + e] = s;
    x[m * 2 * Bp + Bp + e] = c;
}

template <typename T>
__global__ __launch_bounds__(256) void k_ens_colsum(int64_t n, int64_t J, const T *__restrict__ x, T *__restrict__ part)
{
    const int64_t r0 = (int64_t)blockIdx.x * 256;
    const int64_t r1 = r0 + 256 < n ? r0 + 256 : n;
    for (int64_t j = threadIdx.x; j < J; j += 256) {
        T s = T(0);
        for (int64_t m = r0; m < r1; ++m) s += x[m * J + j];
        part[(int64_t)blockIdx.x * J + j] = s;
    }
}

template <typename T>
__global__ __launch_bounds__(64) void k_ens_order(int64_t nchunk, int32_t Bp, int32_t B, double inv_n,
                                                  const T *__restrict__ part, double *__restrict__ r,
                                                  double *__restrict__ psi)
{
    const int e = blockIdx.x * 64 + threadIdx.x;
    if (e >= B) return;
    double S = 0.0, C = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) {
        S += (double)part[c * 2 * Bp + e];
        C += (double)part[c * 2 * Bp + Bp + e];
    }
    S *= inv_n;
    C *= inv_n;
    r[e] = sqrt(S * S + C * C);
    psi[e] = atan2(S, C);
}

hipError_t launch_ens_gemm(const EnsGemmArgs &a, int64_t nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ens_gemm, dim3((unsigned)nitems), dim3(kGemmThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_ens_gemm_f64(const EnsGemmArgs &a, int64_t nitems, hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ens_gemm_f64, dim3((unsigned)nitems), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ens_rows(const EnsRowArgs<T> &a, hipStream_t st)
{
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((a.n + 3) / 4)), block(256);
    switch (a.Bp / 64) {
    case 1: hipLaunchKernelGGL((k_ens_rows<T, 1>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_ens_rows<T, 2>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((k_ens_rows<T, 3>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_ens_rows<T, 4>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ens_sincos(int64_t n, int32_t Bp, const T *hi, T *x, hipStream_t st)
{
    const int64_t tot = n * Bp;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ens_sincos<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, Bp, hi, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ens_colsum(int64_t n, int64_t J, const T *x, T *part, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ens_colsum<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, J, x, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ens_order(int64_t n, int32_t Bp, int32_t B, const T *part, double *r, double *psi, hipStream_t st)
{
    if (B <= 0) return hipSuccess;
    const int64_t nchunk = (n + 255) / 256;
    hipLaunchKernelGGL((k_ens_order<T>), dim3((unsigned)((B + 63) / 64)), dim3(64), 0, st, nchunk, Bp, B,
                       1.0 / (double)n, part, r, psi);
    return hipGetLastError();
}

template hipError_t launch_ens_rows<float>(const EnsRowArgs<float> &, hipStream_t);
template hipError_t launch_ens_rows<double>(const EnsRowArgs<double> &, hipStream_t);
template hipError_t launch_ens_sincos<float>(int64_t, int32_t, const float *, float *, hipStream_t);
template hipError_t launch_ens_sincos<double>(int64_t, int32_t, const double *, double *, hipStream_t);
template hipError_t launch_ens_colsum<float>(int64_t, int64_t, const float *, float *, hipStream_t);
template hipError_t launch_ens_colsum<double>(int64_t, int64_t, const double *, double *, hipStream_t);
template hipError_t launch_ens_order<float>(int64_t, int32_t, int32_t, const float *, double *, double *, hipStream_t);
template hipError_t launch_ens_order<double>(int64_t, int32_t, int32_t, const double *, double *, double *, hipStream_t);

}  // namespace kur
