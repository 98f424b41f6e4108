// ens.hpp -- layout and launchers of the shared-graph ensemble path: B replicas of one graph,
// state stored node-major ([n][Bp] per quantity, Bp = B rounded up to 64) so that one row's
// replicas are contiguous.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace kur {

// A row block (community) whose products run on the matrix cores: A_{a,c} X_c for every column
// community c of its ranges (its own block when dense and its dense off-diagonal blocks, in
// block order). The ranges are laid end to end along k, each padded to a multiple of 32 columns.
struct EnsBlk {
    int64_t bits_off;  // first 32-bit word of the block's 0/1 pattern (row-major)
    int32_t row0;      // first block-order row
    int32_t size;      // rows
    int32_t words;     // words per pattern row (k extent / 32); bit (k & 31) of word k / 32 is the
                       // entry at position k along the ranges
    int32_t rng0;      // first range (EnsRng) of this block
    int32_t nrng;      // ranges
    int32_t pad;
};

// One column range of a matrix-core row block: k in [koff, koff + len) are the block-order
// columns col0 .. col0 + len - 1; k up to the next multiple of 32 is padding (pattern bits 0).
struct EnsRng {
    int32_t koff;
    int32_t col0;
    int32_t len;
    int32_t pad;
};

// One workgroup of the dense product: rows [r0, r0 + kEnsTileRows) of block `blk` (block-local) and
// columns [c0, c0 + 128) of X.
struct EnsItem {
    int32_t blk, r0, c0, pad;
};

// output tile of one product workgroup: FP32 (three bf16 terms) and FP64
constexpr int kEnsTileRows = 256;
constexpr int kEnsTileCols = 128;
constexpr int kEnsTileRowsF64 = 128;
constexpr int kEnsTileColsF64 = 64;

struct EnsGemmArgs {
    const EnsBlk *blk;
    const EnsRng *rng;
    const EnsItem *items;
    const uint32_t *bits;
    const void *x;  // [n][J] of the context's reals: sin of every replica, then cos (J = 2 Bp)
    void *y;        // [n][J]: (A sin, A cos) for the rows of matrix-core blocks
    int64_t J;
};

template <typename T>
struct EnsRowArgs {
    int64_t n;
    int32_t Bp;
    int32_t stage;  // 0: derivative only (kout); 1..4: RK4 stage
    int32_t compensate;
    T dt, half_dt, dt6;
    const int64_t *csr_ptr;  // n + 1, block order
    const int32_t *csr_col;  // block-order columns
    const uint8_t *row_gemm; // 1 where y holds the row's matrix-core products
    const T *x;              // [n][J] stage input (sin | cos)
    const T *y;
    T *x_out;                // [n][J] next stage input (sin | cos)
    const T *omega;          // [n][Bp]
    const T *unit;           // [Bp]: K_e / N
    T *hi, *lo;              // [n][Bp] phase and its compensation term
    int32_t *wind;           // [n][Bp]
    T *ksum;                 // [n][Bp]
    T *kout;                 // [n][Bp], stage 0
};

// FP32 products (X split exactly into three bf16 terms) and FP64 products
hipError_t launch_ens_gemm(const EnsGemmArgs &a, int64_t nitems, hipStream_t st);
hipError_t launch_ens_gemm_f64(const EnsGemmArgs &a, int64_t nitems, hipStream_t st);
template <typename T>
hipError_t launch_ens_rows(const EnsRowArgs<T> &a, hipStream_t st);
template <typename T>
hipError_t launch_ens_sincos(int64_t n, int32_t Bp, const T *hi, T *x, hipStream_t st);
// partial column sums of x over chunks of 256 rows: part [ceil(n / 256)][J]
template <typename T>
hipError_t launch_ens_colsum(int64_t n, int64_t J, const T *x, T *part, hipStream_t st);
// r and psi of replicas [0, B) from the partials, written to r[0..B) and psi[0..B)
template <typename T>
hipError_t launch_ens_order(int64_t n, int32_t Bp, int32_t B, const T *part, double *r, double *psi,
                            hipStream_t st);

}  // namespace kur
