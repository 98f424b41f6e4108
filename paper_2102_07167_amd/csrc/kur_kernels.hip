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

#include "kur_device.hpp"
#include "kur_internal.hpp"
#include "kur_kernels.hpp"

namespace kur {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Cache policy of the list stream's buffer loads (bit 0 sc0, bit 1 nt, bit 4 sc1): non-temporal,
// the lists are read once per launch.
#ifndef KUR_LIST_CPOL
#define KUR_LIST_CPOL 2
#endif

// 16-byte vector i of a list segment addressed by a buffer resource (the segment's base and
// byte length; a vector past the end reads as zero).
__device__ __forceinline__ u32x4 list_load(__amdgpu_buffer_rsrc_t r, uint32_t i)
{
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)(i * 16u), 0, KUR_LIST_CPOL);
}

// Buffer resource over the bytes [p, p + bytes), where p and bytes are the same in every lane of
// the wave. Built from readfirstlane copies so that the compiler keeps it in scalar registers;
// from values it cannot prove uniform (loaded from memory) it would otherwise wrap every load in
// a loop over the lanes' distinct resources.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void *p, int64_t bytes)
{
    // readfirstlane returns int: each half goes through uint32_t before widening, or a low half
    // with bit 31 set would sign-extend into the high half
    const uint64_t a = (uint64_t)p;
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint64_t au = ((uint64_t)hi << 32) | (uint64_t)lo;
    return __builtin_amdgcn_make_buffer_rsrc((void *)au, (short)0, __builtin_amdgcn_readfirstlane((int)bytes),
                                             0x00020000);
}


// Sum v over the workgroup in a fixed order and store it to *out (thread 0).
template <typename VT, int NT>
__device__ __forceinline__ void block_sum_store(VT v, VT *red, VT *out)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    const int w = threadIdx.x >> 6;
    __syncthreads();  // red may still be read by other waves
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        VT s = red[0];
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

// ------------------------------------------------------------------------------------------------
// Gather core shared by the right-hand side (per node (sin, cos)) and the Jacobian-transpose
// product (per node (w sin, w cos)): one value pair per list entry.
// ------------------------------------------------------------------------------------------------

template <typename VT> __device__ __forceinline__ VT vzero()
{
    VT v;
    v.x = 0;
    v.y = 0;
    return v;
}

template <typename VT> __device__ __forceinline__ void vacc(VT &a, const VT &b)
{
    a.x += b.x;
    a.y += b.y;
}

template <typename VT, typename S> __device__ __forceinline__ VT vscale(const VT &a, S s)
{
    VT r = a;
    r.x *= s;
    r.y *= s;
    return r;
}

template <typename VT> __device__ __forceinline__ VT vwave_sum_dpp(VT v)
{
    v.x = wave_sum_dpp(v.x);
    v.y = wave_sum_dpp(v.y);
    return v;
}

template <typename VT> __device__ __forceinline__ VT vgroup_sum_dpp(VT v, int G)
{
    v.x = group_sum_dpp(v.x, G);
    v.y = group_sum_dpp(v.y, G);
    return v;
}

template <typename VT> __device__ __forceinline__ VT vwave_sum(VT v)
{
    v.x = wave_sum(v.x);
    v.y = wave_sum(v.y);
    return v;
}

// Accumulate the 8 list entries of one 16-byte vector. Entries are LDS byte offsets of a
// staged value pair.
template <typename VT>
__device__ __forceinline__ void gather8(const VT *lds, const u32x4 q, VT &acc)
{
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
    const char *base = reinterpret_cast<const char *>(lds);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const VT t0 = *reinterpret_cast<const VT *>(base + (w[k] & 0xffffu));
        const VT t1 = *reinterpret_cast<const VT *>(base + (w[k] >> 16));
        vacc(acc, t0);
        vacc(acc, t1);
    }
}

// Slots of the staging area beyond the chunk: slot W is the zero slot of the lists' padding.
constexpr int kXsSlack = 1;

// A 16-byte vector index whose byte offset (0x7FFFFFF0) lies past the end of every bitmask
// segment's buffer resource (at most INT32_MAX bytes, a multiple of 16): such a load returns
// zeros and touches no memory.
constexpr uint32_t kUnitPastEnd = 0x07FFFFFFu;

// The 16 subset sums of four values x0..x3, entry m = sum of x_j over the set bits j of m, stored
// at t[m * P] (P: the table pitch). Each entry is a smaller entry plus one value, in a fixed order:
// t[m] = t[m without its lowest set bit] + x[that bit].
template <typename VT>
__device__ __forceinline__ void subset_sums4(VT *t, int P, const VT x0, const VT x1, const VT x2, const VT x3)
{
    auto add = [](VT a, const VT &b) {
        vacc(a, b);
        return a;
    };
    // stored four at a time, so that few sums are live at once (the row kernel's register budget)
    t[0] = vzero<VT>();
    t[P] = x0;
    t[2 * P] = x1;
    t[3 * P] = add(x1, x0);
    __builtin_amdgcn_sched_barrier(0);
    t[4 * P] = x2;
    t[5 * P] = add(x2, x0);
    const VT v6 = add(x2, x1);
    t[6 * P] = v6;
    t[7 * P] = add(v6, x0);
    __builtin_amdgcn_sched_barrier(0);
    t[8 * P] = x3;
    t[9 * P] = add(x3, x0);
    const VT v10 = add(x3, x1);
    t[10 * P] = v10;
    t[11 * P] = add(v10, x0);
    __builtin_amdgcn_sched_barrier(0);
    const VT v12 = add(x3, x2);
    t[12 * P] = v12;
    t[13 * P] = add(v12, x0);
    const VT v14 = add(v12, x1);
    t[14 * P] = v14;
    t[15 * P] = add(v14, x0);
}

// Pitch of the subset-sum tables of a bitmask sub-chunk: entry m of column group j at
// xs[j * kTabPitch + m]. The lanes of a wave (rows, all at the same group) read distinct
// consecutive entries (distinct banks); the threads that build consecutive groups write at a
// pitch of 17 entries, which spreads them over the banks.
constexpr int kTabPitch = 17;

// Add to acc the row sums of one 128-column bitmask unit, unit SLOT of the sub-chunk: per nibble
// (4 columns, in column order) one read of the subset-sum table of that column group. The
// nibbles of a word are taken times the entry bytes from two masked copies of it (even and odd
// nibbles, one per byte), so that a table read costs one byte extraction; the group's offset
// is a constant of the read.
template <int SLOT, typename VT>
__device__ __forceinline__ void mask_unit(const VT *xs, const u32x4 u, VT &acc)
{
    constexpr int SH = sizeof(VT) == 8 ? 3 : 4;  // log2 of the entry bytes
    constexpr uint32_t M = 0x0F0F0F0Fu << SH;
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
    const char *base = reinterpret_cast<const char *>(xs);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t we = (w[k] << SH) & M;        // nibbles 0, 2, 4, 6 of the word
        uint32_t wo = (w[k] >> (4 - SH)) & M;  // nibbles 1, 3, 5, 7
        // opaque to the compiler, which would otherwise shift and mask every nibble of the word
        asm volatile("" : "+v"(we), "+v"(wo));
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            constexpr int G0 = SLOT * (kMaskUnitCols / 4);
            const int j = G0 + 8 * k + 2 * b;  // group of nibble 2b of word k
            const uint32_t e = (we >> (8 * b)) & 0xFFu, o = (wo >> (8 * b)) & 0xFFu;
            vacc(acc, *reinterpret_cast<const VT *>(base + e + (size_t)j * kTabPitch * sizeof(VT)));
            vacc(acc, *reinterpret_cast<const VT *>(base + o + (size_t)(j + 1) * kTabPitch * sizeof(VT)));
        }
        // an empty statement that no memory access may cross, after every word (measured with it)
        asm volatile("" ::: "memory");
    }
}

// Partial row sums of one bitmask item (see MaskItem) per workgroup, into g.msum at rows
// [out, out + tile rows): over the item's sub-chunks of bitmask segments (see SegD), for a
// segment of ones the sum of x over the row's set bits, for a segment of zeros minus that sum
// (subtracted from the localised order parameters, Sec. 3, eq. KuramotoGraphApproach). Per
// sub-chunk the workgroup builds in LDS the 16 subset sums of every 4 columns (the method of four
// Russians for Boolean matrix-vector products); then thread r mod NT owns row r, keeps four
// 16-byte units of its bits in flight and adds one table entry per nibble. The values of the next
// sub-chunk's tables are fetched into registers while the current one is read, so a table build
// after its barrier only writes LDS. x_in holds the values summed (the tile kernel's staged
// pairs).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_mask(
    DevGraph g, const typename V2<T>::type *__restrict__ x_in)
{
    using VT = typename V2<T>::type;
    // columns per sub-chunk: a multiple of the unit, at most kMaskSubMax <= 4 NT (one column group
    // per thread, at most 8 units; 4 for 16-byte pairs)
    const int S = g.mask_sub;
    // the tables at a fixed LDS address (a table read's offset is then a constant of the read)
    constexpr int kGroups = (sizeof(VT) == 8 ? kMaskSubMax : kMaskSubMax / 2) / 4;
    __shared__ VT xs[kTabPitch * kGroups];
    extern __shared__ __align__(16) unsigned char smem[];
    VT *macc = reinterpret_cast<VT *>(smem);  // tile rows partial sums
    const MaskItem it = g.mitem[blockIdx.x];
    const Tile tl = g.tiles[it.tile];
    const BlkInfo bi = g.blk[tl.block];
    const int nrows = tl.r1 - tl.r0;
    for (int r = threadIdx.x; r < nrows; r += NT) macc[r] = vzero<VT>();
    const int nseg = bi.nchunk;
    // the next bitmask segment at or after c (nseg if none)
    auto next_mask = [&](int c) {
        while (c < nseg && !__builtin_amdgcn_readfirstlane(g.segd[bi.sd0 + c].mask)) ++c;
        return c;
    };
    // this thread's four values of column group j of the sub-chunk starting at column s0 of
    // segment c (zero past the sub-chunk)
    VT f0 = vzero<VT>(), f1 = f0, f2 = f0, f3 = f0;
    auto fetch = [&](int c, int s0) {
        const SegD sd = g.segd[bi.sd0 + c];
        const int ncol = min(S, (int)sd.cw - s0);
        const int ng = (ncol + kMaskUnitCols - 1) / kMaskUnitCols * (kMaskUnitCols / 4);
        const int j = threadIdx.x;
        const int c0 = sd.col0 + s0 + 4 * j, c1 = sd.col0 + s0 + ncol;
        f0 = f1 = f2 = f3 = vzero<VT>();
        if (j < ng) {
            if (c0 < c1) f0 = x_in[c0];
            if (c0 + 1 < c1) f1 = x_in[c0 + 1];
            if (c0 + 2 < c1) f2 = x_in[c0 + 2];
            if (c0 + 3 < c1) f3 = x_in[c0 + 3];
        }
    };
    int c = it.seg, s0 = it.sub * S;
    fetch(c, s0);
    for (int k = 0; k < it.nsub; ++k) {
        const SegD sd = g.segd[bi.sd0 + c];
        const T sign = sd.zeros ? T(-1) : T(1);
        const int cw = __builtin_amdgcn_readfirstlane((int)sd.cw);
        const int nq = (cw + kMaskUnitCols - 1) / kMaskUnitCols;
        const uint32_t ustride = (uint32_t)bi.size;  // units of one row are size apart
        const __amdgpu_buffer_rsrc_t Mt = uniform_rsrc(g.mask + 4 * sd.mbase, (int64_t)bi.size * nq * 16);
        const int ncol = min(S, cw - s0);
        // tables for every group of the units touched (a unit's bits past the segment are zero
        // and read entry 0 of their group, which must exist and be zero)
        const int ng = (ncol + kMaskUnitCols - 1) / kMaskUnitCols * (kMaskUnitCols / 4);
        const int qa = s0 / kMaskUnitCols, qb = (s0 + ncol + kMaskUnitCols - 1) / kMaskUnitCols;
        const int nqs = qb - qa;  // 1 .. 8
        // unit q of row r, or (q past the sub-chunk, or r past the tile) an offset past the end of
        // the buffer, which reads as zero without a memory access: every load is issued
        // unconditionally, so the wave's in-order wait counts stay exact
        auto unit = [&](int q, int r) {
            const bool in = q < qb && r < nrows;
            return list_load(Mt, in ? (uint32_t)q * ustride + (uint32_t)(tl.r0 + r) : kUnitPastEnd);
        };
        // every unit of the thread's first row loads while the tables are built
        u32x4 u0 = unit(qa, threadIdx.x), u1 = unit(qa + 1, threadIdx.x), u2 = unit(qa + 2, threadIdx.x),
              u3 = unit(qa + 3, threadIdx.x), u4 = unit(qa + 4, threadIdx.x), u5 = unit(qa + 5, threadIdx.x),
              u6 = unit(qa + 6, threadIdx.x), u7 = unit(qa + 7, threadIdx.x);
        __syncthreads();  // the previous sub-chunk's readers of the tables are done
        if ((int)threadIdx.x < ng) subset_sums4(xs + kTabPitch * threadIdx.x, 1, f0, f1, f2, f3);
        // the item's next sub-chunk (of this segment or the next bitmask one), whose values are
        // fetched now
        int cn = c, sn = s0 + S;
        if (sn >= cw) {
            cn = next_mask(c + 1);
            sn = 0;
        }
        if (k + 1 < it.nsub) fetch(cn, sn);
        __syncthreads();
        // units in column order, the sub-chunk's eight in flight: once read, each unit's registers
        // receive the same unit of the thread's next row
        for (int r = threadIdx.x; r < nrows; r += NT) {
            VT acc = vzero<VT>();
            mask_unit<0>(xs, u0, acc);
            u0 = unit(qa, r + NT);
            if (nqs > 1) mask_unit<1>(xs, u1, acc);
            u1 = unit(qa + 1, r + NT);
            if (nqs > 2) mask_unit<2>(xs, u2, acc);
            u2 = unit(qa + 2, r + NT);
            if (nqs > 3) mask_unit<3>(xs, u3, acc);
            u3 = unit(qa + 3, r + NT);
            if (nqs > 4) mask_unit<4>(xs, u4, acc);
            u4 = unit(qa + 4, r + NT);
            if (nqs > 5) mask_unit<5>(xs, u5, acc);
            u5 = unit(qa + 5, r + NT);
            if (nqs > 6) mask_unit<6>(xs, u6, acc);
            u6 = unit(qa + 6, r + NT);
            if (nqs > 7) mask_unit<7>(xs, u7, acc);
            u7 = unit(qa + 7, r + NT);
            vacc(macc[r], vscale(acc, sign));  // row r's own thread, in segment order
        }
        c = cn;
        s0 = sn;
    }
    VT *out = reinterpret_cast<VT *>(g.msum) + it.out;
    for (int r = threadIdx.x; r < nrows; r += NT) out[r] = macc[r];
}

// LDS layout of a tile workgroup (bytes are computed by rows_lds_bytes):
//   xs[W + kXsSlack] staged chunk values (slot W all zero while a list is read) | acc[tile_rows] |
//   red[NT/64 + 1] | bnd[tile_rows + 1]
template <typename VT, int NT>
struct TileLds {
    VT *xs;
    VT *acc;
    VT *red;
    int *bnd;
    __device__ TileLds(unsigned char *smem, int W, int tile_rows)
    {
        xs = reinterpret_cast<VT *>(smem);
        acc = xs + W + kXsSlack;
        red = acc + tile_rows;
        bnd = reinterpret_cast<int *>(red + NT / 64 + 1);
    }
};

// For the rows of one tile, accumulate in L.acc[r] the sum over the row's stored lists of x
// (lists of ones added, lists of zeros subtracted) plus the sum over its inter-block columns,
// and fold into L.red[NT/64] the localised order parameters of the row block's column groups,
// sum_q mode_q (sum of x over column block q), from the tile partials of each column block.
// Ends with a barrier; the complete row sum is then (ngrp ? L.red[NT/64] : 0) + acc[r].
// YG: the inter-block gathers read the phase y_l from y_in (half the bytes of a value pair, so
// twice the table fits a cache) and form (sin y_l, cos y_l), which equals x_in[l] bit for bit.
template <typename T, int NT, bool YG = false>
__device__ __forceinline__ void tile_gather(const DevGraph &g, int tile_id, const Tile &tl, const BlkInfo &bi,
                                            const typename V2<T>::type *__restrict__ x_in,
                                            const typename V2<T>::type *__restrict__ part_in,
                                            TileLds<typename V2<T>::type, NT> &L, const T *__restrict__ y_in = nullptr)
{
    using VT = typename V2<T>::type;
    const int W = g.W;
    const int nrows = tl.r1 - tl.r0;
    const int rowbase = bi.row0 + tl.r0;

    // Small tiles are a chain of dependent memory round trips, so the loads that depend only on
    // the tile are issued first: the tile's inter-block range and the first row bound of every
    // thread, and the tile partials of the localised order parameters, which are folded only at
    // the end (one group per wave, at most 64 partials per group).
    const int64_t i0 = g.inter_ptr[rowbase], i1 = g.inter_ptr[rowbase + nrows];
    const int64_t ib0 = (int)threadIdx.x <= nrows ? g.inter_ptr[rowbase + (int)threadIdx.x] : 0;
    const int ngq = bi.ngrp;
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    bool late = false;     // this tile folds at the end (uniform over the workgroup)
    VT pv = vzero<VT>();   // late fold: this lane's partial of the wave's group
    T pmode = T(0);
    if (ngq <= NT / 64) {
        late = true;
        if (wq < ngq) {
            const Grp gq = g.grp[bi.grp0 + wq];
            const int t0 = g.blk[gq.blk].tile0, nt = g.blk[gq.blk].ntiles;
            pmode = (T)gq.mode;
            const int i = threadIdx.x & 63;
            if (nt <= 64) {
                if (i < nt) pv = part_in[t0 + i];
            } else {
                for (int j = i; j < nt; j += 64) vacc(pv, part_in[t0 + j]);
            }
        }
    }

    for (int r = threadIdx.x; r < nrows; r += NT) L.acc[r] = vzero<VT>();
    if (threadIdx.x == 0) L.xs[W] = vzero<VT>();
    if (!late) {
        // more groups than waves: wave w folds the groups w, w + NT/64, ... (each a fixed-order
        // sum of the column block's tile partials, times the group's factor) and thread 0 then
        // adds the waves' results in wave order
        VT sq = vzero<VT>();
        for (int q = wq; q < ngq; q += NT / 64) {
            const Grp gq = g.grp[bi.grp0 + q];
            const int t0 = g.blk[gq.blk].tile0, nt = g.blk[gq.blk].ntiles;
            VT sx = vzero<VT>();
            for (int i = threadIdx.x & 63; i < nt; i += 64) vacc(sx, part_in[t0 + i]);
            sx = vwave_sum(sx);
            vacc(sq, vscale(sx, (T)gq.mode));
        }
        if ((threadIdx.x & 63) == 0) L.red[wq] = sq;
        __syncthreads();
        if (threadIdx.x == 0) {
            // read by the epilogue after the barrier that ends this function
            VT s = L.red[0];
            for (int w = 1; w < NT / 64; ++w) vacc(s, L.red[w]);
            L.red[NT / 64] = s;
        }
    }
    // the accumulators and the pad slot become visible at the first barrier below (every path
    // to a reader passes one)

    // G > 0: G lanes per row (short rows); G == 0: every wave streams a contiguous run of rows;
    // G < 0: no list entries in any chunk (only inter-block entries)
    const bool flat = tl.G == 0;
    const int G = tl.G > 0 ? tl.G : 8;
    const int nchunk = tl.G < 0 ? 0 : bi.nchunk;
    const int lane = threadIdx.x & (G - 1);
    const int grp = threadIdx.x / G;
    const int ngrp = NT / G;
    int staged = -1;  // first column of the chunk held in L.xs (uniform over the workgroup)
    const int ln = threadIdx.x & 63;
    // this wave's rows [ra, rb) in streaming mode (wave-uniform, kept in scalar registers)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ra = (int)(((int64_t)nrows * wv) / (NT / 64));
    const int rb = (int)(((int64_t)nrows * (wv + 1)) / (NT / 64));

    for (int c = 0; c < nchunk; ++c) {
        const SegD sd = g.segd[bi.sd0 + c];
        // a list (or bitmask) of zeros is subtracted from the localised order parameters
        const T sign = sd.zeros ? T(-1) : T(1);
        if (sd.mask) continue;  // summed by k_mask into g.msum, added below
        const int64_t sb = bi.segbase + (int64_t)c * bi.size;
        const int64_t e0 = g.seg_ptr[sb + tl.r0], e1 = g.seg_ptr[sb + tl.r1];
        if (e0 == e1) continue;  // uniform over the workgroup
        __syncthreads();  // previous segment's gathers are done
        if (sd.col0 != staged) {
            for (int j = threadIdx.x; j < sd.cw; j += NT) L.xs[j] = x_in[sd.col0 + j];
            staged = sd.col0;
        }
        // row starts of this chunk, in 8-entry vectors relative to the tile's first one
        for (int r = threadIdx.x; r <= nrows; r += NT) L.bnd[r] = (int)((g.seg_ptr[sb + tl.r0 + r] - e0) >> 3);
        __syncthreads();
        // the tile's list vectors of this chunk, [e0, e1) entries
        const __amdgpu_buffer_rsrc_t Lt = uniform_rsrc(g.list + e0, (e1 - e0) * 2);
        if (flat) {
            // rows [ra, rb) occupy the contiguous 8-entry vectors [va, va + nvec) of this chunk
            const int va = __builtin_amdgcn_readfirstlane(L.bnd[ra]);
            const int nvec = __builtin_amdgcn_readfirstlane(L.bnd[rb]) - va;
            if (nvec > 0) {
                const uint32_t vb = (uint32_t)va;
                int r = ra;
                int nbnd = __builtin_amdgcn_readfirstlane(L.bnd[r + 1]) - va;  // first vector after row r
                VT acc = vzero<VT>();
                // rolling prefetch: four 64-vector spans in flight per wave; loads are issued
                // unconditionally (index clamped) so the in-order wait counts stay exact, and
                // lanes past the end are masked after the gather
                const uint32_t last = (uint32_t)(nvec - 1);
                u32x4 q0 = list_load(Lt, vb + min((uint32_t)ln, last));
                u32x4 q1 = list_load(Lt, vb + min((uint32_t)(64 + ln), last));
                u32x4 q2 = list_load(Lt, vb + min((uint32_t)(128 + ln), last));
                u32x4 q3 = list_load(Lt, vb + min((uint32_t)(192 + ln), last));
                auto span = [&](const u32x4 q, const int s0) {
                    VT p = vzero<VT>();
                    gather8(L.xs, q, p);
                    if (s0 + ln >= nvec) p = vzero<VT>();
                    // rows that end inside (or right at the end of) this span
                    while (nbnd <= s0 + 64 && r < rb) {
                        if (s0 + ln < nbnd) {
                            vacc(acc, p);
                            p = vzero<VT>();
                        }
                        const VT t = vwave_sum_dpp(acc);
                        if (ln == 63) vacc(L.acc[r], vscale(t, sign));
                        acc = vzero<VT>();
                        ++r;
                        nbnd = r < rb ? __builtin_amdgcn_readfirstlane(L.bnd[r + 1]) - va : INT32_MAX;
                    }
                    vacc(acc, p);
                };
                for (int s0 = 0; s0 < nvec; s0 += 256) {
                    span(q0, s0);
                    q0 = list_load(Lt, vb + min((uint32_t)(s0 + 256 + ln), last));
                    span(q1, s0 + 64);
                    q1 = list_load(Lt, vb + min((uint32_t)(s0 + 320 + ln), last));
                    span(q2, s0 + 128);
                    q2 = list_load(Lt, vb + min((uint32_t)(s0 + 384 + ln), last));
                    span(q3, s0 + 192);
                    q3 = list_load(Lt, vb + min((uint32_t)(s0 + 448 + ln), last));
                }
            }
        } else {
            // G lanes per row; the group's first two vectors of its next row load while it sums
            // the current one. Loads past the row are not gathered (past the tile's vectors they
            // read zero without a memory access).
            int r = grp;
            int v0 = r < nrows ? L.bnd[r] : 0;
            u32x4 qa = list_load(Lt, (uint32_t)(v0 + lane)), qb = list_load(Lt, (uint32_t)(v0 + lane + G));
            for (; r < nrows; r += ngrp) {
                const int nv = L.bnd[r + 1] - v0;
                const int rn = r + ngrp;
                const int v0n = rn < nrows ? L.bnd[rn] : v0 + nv;
                const u32x4 na = list_load(Lt, (uint32_t)(v0n + lane)), nb = list_load(Lt, (uint32_t)(v0n + lane + G));
                VT acc = vzero<VT>();
                if (lane < nv) gather8(L.xs, qa, acc);
                if (lane + G < nv) gather8(L.xs, qb, acc);
                for (int v = lane + 2 * G; v < nv; v += 2 * G) {  // rows longer than 2 G vectors
                    const u32x4 ra = list_load(Lt, (uint32_t)(v0 + v));
                    const u32x4 rb2 = list_load(Lt, (uint32_t)(v0 + v + G));
                    gather8(L.xs, ra, acc);
                    if (v + G < nv) gather8(L.xs, rb2, acc);
                }
                acc = vgroup_sum_dpp(acc, G);
                if (lane == G - 1) vacc(L.acc[r], vscale(acc, sign));
                qa = na;
                qb = nb;
                v0 = v0n;
            }
        }
    }

    // the rows' sums over the bitmask segments (the tile's item partial sums, written by k_mask
    // before this launch, in segment order), added by thread r mod NT once the list pass's
    // leaders have finished with acc; the barriers below order them before the epilogue reads acc
    if (g.msum) {  // uniform (a kernel argument)
        const MaskTile mt = g.mtile[tile_id];
        if (mt.cnt > 0) {
            __syncthreads();
            const VT *ms = reinterpret_cast<const VT *>(g.msum) + mt.off;
            for (int r = threadIdx.x; r < nrows; r += NT) {
                VT s = ms[r];
                for (int k = 1; k < mt.cnt; ++k) vacc(s, ms[(int64_t)k * nrows + r]);
                vacc(L.acc[r], s);
            }
        }
    }

    // edges between blocks: straightforward summation from the global table. The tile's rows
    // own the contiguous entries [i0, i1) of the inter CSR; they are gathered in rounds of
    // 4 NT entries (all loads of a round in flight together) into the staging area, which is
    // free now, and each row then adds its entries in order.
    if (i1 > i0) {  // uniform over the workgroup
        const int total = (int)(i1 - i0);
        constexpr int U = 4;
        const int round = min(U * NT, W);  // entries per round: at most the staging area
        __syncthreads();  // the staging area and bnd are no longer read by the list pass
        if ((int)threadIdx.x <= nrows) L.bnd[threadIdx.x] = (int)(ib0 - i0);
        for (int r = threadIdx.x + NT; r <= nrows; r += NT) L.bnd[r] = (int)(g.inter_ptr[rowbase + r] - i0);
        for (int base = 0; base < total; base += round) {
            if (base > 0) __syncthreads();  // the previous round's values are consumed
            const int end = min(total, base + round);
            int col[U];
#pragma unroll
            for (int u = 0; u < U; ++u) col[u] = g.inter_col[i0 + min(base + u * NT + (int)threadIdx.x, end - 1)];
            VT v[U];
            if constexpr (YG) {
                T yv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) yv[u] = y_in[col[u]];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    T sn, cs;
                    dev_sincos<T>(yv[u], &sn, &cs);
                    v[u].x = sn;
                    v[u].y = cs;
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) v[u] = x_in[col[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = base + u * NT + (int)threadIdx.x;
                if (j < end) L.xs[j - base] = v[u];
            }
            __syncthreads();
            for (int r = threadIdx.x; r < nrows; r += NT) {
                const int lo = max(L.bnd[r], base), hi = min(L.bnd[r + 1], end);
                if (lo >= hi) continue;
                VT a = L.xs[lo - base];
                for (int j = lo + 1; j < hi; ++j) vacc(a, L.xs[j - base]);
                vacc(L.acc[r], a);
            }
        }
    }
    if (late) {
        // the late fold: wave w sums its group's partials (fixed order), times the group's factor
        VT sx = vwave_sum(pv);
        if (wq < ngq && (threadIdx.x & 63) == 0) L.red[ngq == 1 ? NT / 64 : wq] = vscale(sx, pmode);
        if (ngq > 1) {
            __syncthreads();
            if (threadIdx.x == 0) {
                VT s = L.red[0];
                for (int w = 1; w < ngq; ++w) vacc(s, L.red[w]);
                L.red[NT / 64] = s;
            }
        }
    }
    __syncthreads();
}

// Right-hand side and classical RK4 stage bookkeeping, one tile per workgroup. Eight waves
// per SIMD in FP32 (64 VGPRs); FP64 gets more registers and no scratch at six.
template <typename T, int NT, bool YG>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4))) void k_rows(DevGraph g, RowArgs<T> a)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    TileLds<T2, NT> L(smem, g.W, g.tile_rows);
    const int tile_id = g.order[blockIdx.x];
    if (tile_id < 0) return;  // empty slot of the XCD-aware launch order
    const Tile tl = g.tiles[tile_id];
    const BlkInfo bi = g.blk[tl.block];
    const int nrows = tl.r1 - tl.r0;
    const int rowbase = bi.row0 + tl.r0;
    const T2 *__restrict__ sc_in = reinterpret_cast<const T2 *>(a.sc_in);

    tile_gather<T, NT, YG>(g, tile_id, tl, bi, sc_in, reinterpret_cast<const T2 *>(a.part_in), L, a.y_in);

    T2 base = vzero<T2>();
    if (bi.ngrp) base = L.red[NT / 64];
    T2 part = vzero<T2>();
    for (int r = threadIdx.x; r < nrows; r += NT) {
        const int m = rowbase + r;
        const T2 scm = sc_in[m];
        const T As = base.x + L.acc[r].x;
        const T Ac = base.y + L.acc[r].y;
        const T scale = a.K * (a.unit ? a.unit[m] : a.inv_n);
        const T k = a.omega[m] + scale * (As * scm.y - Ac * scm.x);
        if (a.stage <= 0) {
            // 0: the derivative; -1: the row's coupling energy cos y (A cos y) + sin y (A sin y).
            // The localised order parameters of a dense block include the row's own node (with
            // the block's factor), whose term cancels in the derivative but adds
            // mode (cos^2 y + sin^2 y) here: it is removed.
            T en = scm.y * Ac + scm.x * As;
            if (bi.mode) en -= (T)bi.mode * (scm.y * scm.y + scm.x * scm.x);
            a.kout[m] = a.stage == 0 ? k : en;
            continue;
        }
        if (a.ac_out) {
            // the adjoint's recompute keeps (A sin y, A cos y) of the stage state; the row's own
            // term in a dense block's sums cancels wherever they are used
            T2 v;
            v.x = As;
            v.y = Ac;
            reinterpret_cast<T2 *>(a.ac_out)[m] = v;
        }
        const T y = rk4_stage<T>(a.stage, k, a.dt, a.half_dt, a.dt6, a.compensate, a.ksum + m, a.hi + m, a.lo + m,
                                 a.wind + m);
        if (YG && a.y_out) a.y_out[m] = y;
        T s, c;
        dev_sincos<T>(y, &s, &c);
        T2 v;
        v.x = s;
        v.y = c;
        reinterpret_cast<T2 *>(a.sc_out)[m] = v;
        part.x += s;
        part.y += c;
    }
    if (a.stage > 0) block_sum_store<T2, NT>(part, L.red, reinterpret_cast<T2 *>(a.part_out) + tile_id);
}

// Maximum over the workgroup of a non-negative value, stored to *out by thread 0.
template <typename T, int NT>
__device__ __forceinline__ void block_max_store(T v, T *red, T *out)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        T m = red[0];
        for (int i = 1; i < NT / 64; ++i) m = fmax(m, red[i]);
        *out = m;
    }
}

// One stage of the embedded Runge-Kutta pair (see EmbArgs); the gathers are those of k_rows.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_rows_emb(DevGraph g, EmbArgs<T> a)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    TileLds<T2, NT> L(smem, g.W, g.tile_rows);
    const int tile_id = g.order[blockIdx.x];
    if (tile_id < 0) return;  // empty slot of the XCD-aware launch order
    const Tile tl = g.tiles[tile_id];
    const BlkInfo bi = g.blk[tl.block];
    const int nrows = tl.r1 - tl.r0;
    const int rowbase = bi.row0 + tl.r0;
    const T2 *__restrict__ sc_in = reinterpret_cast<const T2 *>(a.sc_in);

    tile_gather<T, NT>(g, tile_id, tl, bi, sc_in, reinterpret_cast<const T2 *>(a.part_in), L);

    T2 base = vzero<T2>();
    if (bi.ngrp) base = L.red[NT / 64];
    T2 part = vzero<T2>();
    T emax = T(0);
    const bool last = a.stage == a.nstages;
    for (int r = threadIdx.x; r < nrows; r += NT) {
        const int m = rowbase + r;
        const T2 scm = sc_in[m];
        const T As = base.x + L.acc[r].x;
        const T Ac = base.y + L.acc[r].y;
        const T scale = a.K * (a.unit ? a.unit[m] : a.inv_n);
        const T k = a.omega[m] + scale * (As * scm.y - Ac * scm.x);
        a.kbuf[(int64_t)(a.stage - 1) * a.n + m] = k;
        // sum_{j <= stage} coef[j] k_j in increasing j
        T acc = T(0);
        for (int j = 0; j + 1 < a.stage; ++j) acc += a.coef[j] * a.kbuf[(int64_t)j * a.n + m];
        acc += a.coef[a.stage - 1] * k;
        T y;
        if (!last) {
            y = a.hi[m] + a.dt * acc;
        } else {
            T est = T(0);
            for (int j = 0; j + 1 < a.stage; ++j) est += a.coef2[j] * a.kbuf[(int64_t)j * a.n + m];
            est += a.coef2[a.stage - 1] * k;
            emax = fmax(emax, fabs(a.dt * est));
            y = phase_advance<T>(a.hi[m], a.lo[m], a.wind[m], a.dt * acc, a.compensate, a.hi_new + m, a.lo_new + m,
                                 a.wind_new + m);
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
    block_sum_store<T2, NT>(part, L.red, reinterpret_cast<T2 *>(a.part_out) + tile_id);
    if (last) block_max_store<T, NT>(emax, reinterpret_cast<T *>(&L.red[0]), a.err_part + tile_id);
}

template <typename T>
__global__ __launch_bounds__(256) void k_max_fold(int64_t n, const T *__restrict__ in, T *__restrict__ out)
{
    __shared__ T red[256];
    T m = T(0);
    for (int64_t i = threadIdx.x; i < n; i += 256) m = fmax(m, in[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Discrete adjoint of one classical RK4 stage (reverse order 4, 3, 2, 1). With w = K scale_m l_i
// and x_in holding (w s, w c) at the stage state Y_i, the gathers over the lists of A^T give
// (A^T ws, A^T wc), and
//   (J^T l_i)_m = c_m (A^T wc)_m + s_m (A^T ws)_m - w_m (c_m (A c)_m + s_m (A s)_m)  (= mu_i)
//   dF_m/dK     = scale_m ((A s)_m c_m - (A c)_m s_m),
// obtained by differentiating eq. KuramotoGraph term by term. (s, c) of Y_i come from sc_cur
// and (A s, A c) from ac_rows, both kept by the forward recompute of the stage, so the gathers
// move one value pair per list entry, as in the forward kernel. For symmetric A the layout is
// that of A itself. The epilogue accumulates lam_acc += mu_i, g_omega += l_i, dK += l_i dF/dK,
// and forms l_{i-1} = a dt lam + b dt mu_i and the next stage's x; at stage 1 it stores the
// new lam = lam_acc. Register budget as for k_rows.
template <typename T, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 4))) void k_vjp(DevGraph g, VjpArgs<T> a)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    TileLds<T2, NT> L(smem, g.W, g.tile_rows);
    const int tile_id = g.order[blockIdx.x];
    if (tile_id < 0) return;  // empty slot of the XCD-aware launch order
    const Tile tl = g.tiles[tile_id];
    const BlkInfo bi = g.blk[tl.block];
    const int nrows = tl.r1 - tl.r0;
    const int rowbase = bi.row0 + tl.r0;

    tile_gather<T, NT>(g, tile_id, tl, bi, reinterpret_cast<const T2 *>(a.x_in), reinterpret_cast<const T2 *>(a.part_in), L);

    T2 base = vzero<T2>();
    if (bi.ngrp) base = L.red[NT / 64];
    T2 part = vzero<T2>();
    double gk = 0.0;
    for (int r = threadIdx.x; r < nrows; r += NT) {
        const int m = rowbase + r;
        const T2 scm = reinterpret_cast<const T2 *>(a.sc_cur)[m];
        const T2 ac = reinterpret_cast<const T2 *>(a.ac_rows)[m];
        const T s = scm.x, c = scm.y, As = ac.x, Ac = ac.y;
        const T Aws = base.x + L.acc[r].x, Awc = base.y + L.acc[r].y;
        const T unit = a.unit ? a.unit[m] : a.inv_n;
        const T l = a.lbuf[m];
        const T w = a.K * unit * l;
        const T mu = c * Awc + s * Aws - w * (c * Ac + s * As);
        const T dfdk = unit * (As * c - Ac * s);
        a.g_omega[m] += (double)l;
        gk += (double)l * (double)dfdk;
        const T la = a.lam_acc[m] + mu;
        if (a.stage > 1) {
            a.lam_acc[m] = la;
            const T ln = a.cl * a.lam[m] + a.cm * mu;
            a.lbuf[m] = ln;
            const T wn = a.K * unit * ln;
            const T2 scn = reinterpret_cast<const T2 *>(a.sc_next)[m];
            T2 xn;
            xn.x = wn * scn.x;
            xn.y = wn * scn.y;
            reinterpret_cast<T2 *>(a.x_out)[m] = xn;
            vacc(part, xn);
        } else {
            a.lam[m] = la;
            if (a.sc_next) {
                // the start of the next reverse step, in the arithmetic of k_vjp_init (cl =
                // dt/6): l_4 = cl lam, lam_acc = lam, x = (w s, w c) at that step's Y_4
                const T l4 = a.cl * la;
                a.lbuf[m] = l4;
                a.lam_acc[m] = la;
                const T w4 = a.K * unit * l4;
                const T2 scn = reinterpret_cast<const T2 *>(a.sc_next)[m];
                T2 xn;
                xn.x = w4 * scn.x;
                xn.y = w4 * scn.y;
                reinterpret_cast<T2 *>(a.x_out)[m] = xn;
                vacc(part, xn);
            }
        }
    }
    if (a.stage > 1 || a.sc_next) block_sum_store<T2, NT>(part, L.red, reinterpret_cast<T2 *>(a.part_out) + tile_id);
    // the tile's dK contribution, accumulated over all launches in a fixed order
    __shared__ double gks[NT / 64];
    gk = wave_sum(gk);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) gks[threadIdx.x >> 6] = gk;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = gks[0];
        for (int i = 1; i < NT / 64; ++i) t += gks[i];
        a.gk_part[tile_id] += t;
    }
}

// Start of a reverse RK4 step: l_4 = dt/6 lam, lam_acc = lam, x = (w s, w c) at Y_4.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_vjp_init(const Tile *__restrict__ tiles, const BlkInfo *__restrict__ blk,
                                                 VjpArgs<T> a)
{
    using T2 = typename V2<T>::type;
    __shared__ T2 red[NT / 64];
    const int t = blockIdx.x;
    const Tile tl = tiles[t];
    const int row0 = blk[tl.block].row0 + tl.r0;
    const int nrows = tl.r1 - tl.r0;
    T2 part = vzero<T2>();
    for (int r = threadIdx.x; r < nrows; r += NT) {
        const int m = row0 + r;
        const T lam = a.lam[m];
        const T l4 = a.cl * lam;
        a.lbuf[m] = l4;
        a.lam_acc[m] = lam;
        const T w = a.K * (a.unit ? a.unit[m] : a.inv_n) * l4;
        const T2 sc = reinterpret_cast<const T2 *>(a.sc_next)[m];
        T2 x;
        x.x = w * sc.x;
        x.y = w * sc.y;
        reinterpret_cast<T2 *>(a.x_out)[m] = x;
        vacc(part, x);
    }
    block_sum_store<T2, NT>(part, red, reinterpret_cast<T2 *>(a.part_out) + t);
}

// r e^{i psi} = (1/N) sum_m e^{i theta_m} (Sec. 2, eq. OrderParameter) for every instance of a
// batch (one workgroup each; a single graph is one instance), from the partials of the
// instance's tiles, accumulated in FP64 in a fixed order. The sample index comes from *idx_dev
// when given (graph replay), else from idx.
template <typename T>
__global__ __launch_bounds__(256) void k_order(const typename V2<T>::type *__restrict__ part,
                                               const int64_t *__restrict__ tile_first, const double *__restrict__ inv_n,
                                               int n_inst, double *__restrict__ r_out, double *__restrict__ psi_out,
                                               const int64_t *__restrict__ idx_dev, int64_t idx)
{
    __shared__ double rs[4], rc[4];
    const int inst = blockIdx.x;
    double s = 0.0, c = 0.0;
    for (int64_t t = tile_first[inst] + threadIdx.x; t < tile_first[inst + 1]; t += 256) {
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
        s = (rs[0] + rs[1] + rs[2] + rs[3]) * inv_n[inst];
        c = (rc[0] + rc[1] + rc[2] + rc[3]) * inv_n[inst];
        const int64_t k = (idx_dev ? *idx_dev : idx) * n_inst + inst;
        r_out[k] = sqrt(s * s + c * c);
        psi_out[k] = atan2(s, c);
    }
}

// Streaming read of n 16-byte words (a bandwidth reference for the roofline): every lane
// reads a grid-strided sequence with non-temporal loads and folds it into one word.
__global__ __launch_bounds__(512) void k_stream_read(const u32x4 *__restrict__ p, int64_t n, uint32_t *__restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (; i < n; i += st) {
        const u32x4 v = __builtin_nontemporal_load(p + i);
        acc ^= v.x + v.y + v.z + v.w;
    }
    if (acc == 0x9E3779B9u) out[0] = acc;  // keeps the loads; practically never taken
}

hipError_t launch_stream_read(const void *p, int64_t words, uint32_t *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_stream_read, dim3(2048), dim3(512), 0, st, (const u32x4 *)p, words, out);
    return hipGetLastError();
}

// advance the replayed sample counter
__global__ void k_bump(int64_t *ctr) { *ctr += 1; }

// Partial sums for the diagnostics, one chunk of 256 rows per workgroup, in FP64 and a fixed
// order: the unwrapped phases theta = hi + lo + 2 pi wind, omega, and the potential's row terms
// -omega_m theta_m - K/2 scale_m e_m with e_m the row's coupling energy (Sec. 3, eq.
// ExtendedPotentialConservation; the constant K/2 sum_m scale_m deg_m is added on the host).
template <typename T>
__global__ __launch_bounds__(256) void k_diag(int64_t n, const T *__restrict__ hi, const T *__restrict__ lo,
                                              const int32_t *__restrict__ wind, const T *__restrict__ omega,
                                              const T *__restrict__ unit, const T *__restrict__ e, double K, double inv_n,
                                              double *__restrict__ part)
{
    __shared__ double red[3][256];
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double st = 0.0, so = 0.0, sv = 0.0;
    if (m < n) {
        const double th = (double)hi[m] + (double)lo[m] +
                          (double)wind[m] * ((double)TwoPi<T>::P1 + (double)TwoPi<T>::P2);
        const double om = (double)omega[m];
        const double sc = unit ? (double)unit[m] : inv_n;
        st = th;
        so = om;
        sv = -om * th - 0.5 * K * sc * (double)e[m];
    }
    red[0][threadIdx.x] = st;
    red[1][threadIdx.x] = so;
    red[2][threadIdx.x] = sv;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * (int64_t)blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// Fixed-order fold of the k_diag partials into out[0..3): one workgroup.
__global__ __launch_bounds__(256) void k_diag_fold(int64_t nchunk, const double *__restrict__ part, double *__restrict__ out)
{
    __shared__ double red[3][256];
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t c = threadIdx.x; c < nchunk; c += 256)
        for (int q = 0; q < 3; ++q) a[q] += part[3 * c + q];
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
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

// Calls f(std::integral_constant<int, NT>{}) with NT the workgroup size `threads` of the tile
// kernels: 128, 256, 512 or 1024 (the option checks admit nothing else; anything else takes 512).
template <typename F>
hipError_t with_nt(int threads, F &&f)
{
    switch (threads) {
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    default: return f(std::integral_constant<int, 512>{});
    }
}

// dynamic LDS limit requested for the tile kernels (the rest of the 160 KiB stays for static use)
constexpr int kMaxDynLds = 156 * 1024;

// Raise the dynamic LDS limit of the kernel Fn to Limit bytes (its static LDS plus Limit must fit
// the LDS of a workgroup), once per process (one static per kernel).
template <auto Fn, int Limit = kMaxDynLds>
hipError_t dyn_lds_attr()
{
    static const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void *>(Fn), hipFuncAttributeMaxDynamicSharedMemorySize, Limit);
    return e;
}

template <typename T>
hipError_t launch_sc_init(const DevGraph &g, int ntiles, const T *y, void *sc, void *part, int threads,
                          hipStream_t st)
{
    using T2 = typename V2<T>::type;
    if (ntiles <= 0) return hipSuccess;
    return with_nt(threads, [&](auto nt) -> hipError_t {
        constexpr int NT = decltype(nt)::value;
        hipLaunchKernelGGL((k_sc_init<T, NT>), dim3(ntiles), dim3(NT), 0, st, g.tiles, g.blk, y, (T2 *)sc, (T2 *)part);
        return hipGetLastError();
    });
}

// Bitmask item partial sums into g.msum, before a tile kernel that adds them (no-op for a layout
// without bitmask segments). x_in: the pairs that tile kernel stages. Always 256 threads (the row
// loop covers any tile height), whatever the tile kernel's workgroup size.
template <typename T>
hipError_t launch_mask(const DevGraph &g, const void *x_in, hipStream_t st)
{
    if (!g.msum || g.nmitem <= 0) return hipSuccess;
    constexpr int NT = 256;
    static_assert(kMaskSubMax <= 4 * NT && kMaskSubMax <= 8 * kMaskUnitCols, "one column group per thread, 8 units");
    if (g.mask_sub < kMaskUnitCols || g.mask_sub > (sizeof(T) == 4 ? kMaskSubMax : kMaskSubMax / 2) ||
        g.mask_sub % kMaskUnitCols)
        return hipErrorInvalidValue;
    // the rows' sums beyond the tables' static LDS: at most 4096 rows of 16 bytes
    const size_t lds = (size_t)g.tile_rows * 2 * sizeof(T);
    if (lds > 65536) return hipErrorInvalidValue;
    hipError_t e = dyn_lds_attr<&k_mask<T, NT>, 65536>();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mask<T, NT>), dim3(g.nmitem), dim3(NT), lds, st, g,
                       reinterpret_cast<const typename V2<T>::type *>(x_in));
    return hipGetLastError();
}

size_t rows_lds_bytes(int elem_bytes, int W, int tile_rows, int threads)
{
    const size_t vt = (size_t)2 * elem_bytes;
    size_t b = (size_t)(W + kXsSlack) * vt + (size_t)tile_rows * vt + (size_t)(threads / 64 + 1) * vt +
               (size_t)(tile_rows + 1) * 4;
    return (b + 15) & ~size_t(15);
}

template <typename T>
hipError_t launch_rows(const DevGraph &g, int ntiles, const RowArgs<T> &a, int threads, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    hipError_t em = launch_mask<T>(g, a.sc_in, st);
    if (em != hipSuccess) return em;
    const size_t lds = rows_lds_bytes(sizeof(T), g.W, g.tile_rows, threads);
    const bool yg = a.y_in != nullptr;
    return with_nt(threads, [&](auto nt) -> hipError_t {
        constexpr int NT = decltype(nt)::value;
        hipError_t e = yg ? dyn_lds_attr<&k_rows<T, NT, true>>() : dyn_lds_attr<&k_rows<T, NT, false>>();
        if (e != hipSuccess) return e;
        if (yg)
            hipLaunchKernelGGL((k_rows<T, NT, true>), dim3(g.nlaunch), dim3(NT), lds, st, g, a);
        else
            hipLaunchKernelGGL((k_rows<T, NT, false>), dim3(g.nlaunch), dim3(NT), lds, st, g, a);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_emb(const DevGraph &g, const EmbArgs<T> &a, int threads, hipStream_t st)
{
    if (g.nlaunch <= 0) return hipSuccess;
    hipError_t em = launch_mask<T>(g, a.sc_in, st);
    if (em != hipSuccess) return em;
    const size_t lds = rows_lds_bytes(sizeof(T), g.W, g.tile_rows, threads);
    return with_nt(threads, [&](auto nt) -> hipError_t {
        constexpr int NT = decltype(nt)::value;
        hipError_t e = dyn_lds_attr<&k_rows_emb<T, NT>>();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rows_emb<T, NT>), dim3(g.nlaunch), dim3(NT), lds, st, g, a);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_max_fold(int64_t n, const T *in, T *out, hipStream_t st)
{
    hipLaunchKernelGGL((k_max_fold<T>), dim3(1), dim3(256), 0, st, n, in, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_vjp(const DevGraph &g, int ntiles, const VjpArgs<T> &a, int threads, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    hipError_t em = launch_mask<T>(g, a.x_in, st);
    if (em != hipSuccess) return em;
    const size_t lds = rows_lds_bytes(sizeof(T), g.W, g.tile_rows, threads);
    return with_nt(threads, [&](auto nt) -> hipError_t {
        constexpr int NT = decltype(nt)::value;
        hipError_t e = dyn_lds_attr<&k_vjp<T, NT>>();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_vjp<T, NT>), dim3(g.nlaunch), dim3(NT), lds, st, g, a);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_vjp_init(const DevGraph &g, int ntiles, const VjpArgs<T> &a, int threads, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    return with_nt(threads, [&](auto nt) -> hipError_t {
        constexpr int NT = decltype(nt)::value;
        hipLaunchKernelGGL((k_vjp_init<T, NT>), dim3(ntiles), dim3(NT), 0, st, g.tiles, g.blk, a);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_diag(int64_t n, const void *hi, const void *lo, const int32_t *wind, const void *omega,
                       const void *unit, const void *e, double K, double *part, double *out, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const int64_t nchunk = (n + 255) / 256;
    hipLaunchKernelGGL((k_diag<T>), dim3((unsigned)nchunk), dim3(256), 0, st, n, (const T *)hi, (const T *)lo, wind,
                       (const T *)omega, (const T *)unit, (const T *)e, K, 1.0 / (double)n, part);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL(k_diag_fold, dim3(1), dim3(256), 0, st, nchunk, (const double *)part, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_order(const void *part, const int64_t *tile_first, const double *inv_n, int n_inst, double *r,
                        double *psi, const int64_t *idx_dev, int64_t idx, hipStream_t st)
{
    using T2 = typename V2<T>::type;
    hipLaunchKernelGGL((k_order<T>), dim3(n_inst), dim3(256), 0, st, (const T2 *)part, tile_first, inv_n, n_inst, r,
                       psi, idx_dev, idx);
    return hipGetLastError();
}

hipError_t launch_bump(int64_t *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(1), 0, st, ctr);
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

template hipError_t launch_vjp<float>(const DevGraph &, int, const VjpArgs<float> &, int, hipStream_t);
template hipError_t launch_vjp<double>(const DevGraph &, int, const VjpArgs<double> &, int, hipStream_t);
template hipError_t launch_vjp_init<float>(const DevGraph &, int, const VjpArgs<float> &, int, hipStream_t);
template hipError_t launch_vjp_init<double>(const DevGraph &, int, const VjpArgs<double> &, int, hipStream_t);
template hipError_t launch_emb<float>(const DevGraph &, const EmbArgs<float> &, int, hipStream_t);
template hipError_t launch_emb<double>(const DevGraph &, const EmbArgs<double> &, int, hipStream_t);
template hipError_t launch_max_fold<float>(int64_t, const float *, float *, hipStream_t);
template hipError_t launch_max_fold<double>(int64_t, const double *, double *, hipStream_t);
template hipError_t launch_diag<float>(int64_t, const void *, const void *, const int32_t *, const void *,
                                       const void *, const void *, double, double *, double *, hipStream_t);
template hipError_t launch_diag<double>(int64_t, const void *, const void *, const int32_t *, const void *,
                                        const void *, const void *, double, double *, double *, hipStream_t);
template hipError_t launch_order<float>(const void *, const int64_t *, const double *, int, double *, double *,
                                       const int64_t *, int64_t, hipStream_t);
template hipError_t launch_order<double>(const void *, const int64_t *, const double *, int, double *, double *,
                                        const int64_t *, int64_t, hipStream_t);
template hipError_t launch_phase_out<float>(int64_t, const void *, const void *, const int32_t *, int, void *, hipStream_t);
template hipError_t launch_phase_out<double>(int64_t, const void *, const void *, const int32_t *, int, void *, hipStream_t);

double two_pi_p1(int elem_bytes) { return elem_bytes == 4 ? (double)TwoPi<float>::P1 : TwoPi<double>::P1; }
double two_pi_p2(int elem_bytes) { return elem_bytes == 4 ? (double)TwoPi<float>::P2 : TwoPi<double>::P2; }

}  // namespace kur
