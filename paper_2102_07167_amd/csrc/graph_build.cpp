// graph_build.cpp -- host preprocessing of the graph (untimed set-up work).
//
// 1. Regroup the nodes so that every community is contiguous: a stable counting sort by label,
//    i.e. the permutation P with A~ = P A P^T of the paper (Sec. 3, community detection), done
//    here on given (planted) labels.
// 2. For every diagonal block choose the evaluation: localised order parameters with the list
//    of zero entries when the realised density is at least tau, straightforward summation over
//    the list of one entries otherwise (Sec. 3, eq. KuramotoGraphApproach and the density rule
//    of the introduction).
// 3. Store the lists as 16-bit LDS byte offsets (column relative to a chunk of W columns, times
//    the size of a staged (sin, cos) pair), chunk-major inside a block, every (row, chunk)
//    segment padded to a multiple of 8 entries with the offset of slot W (all zero), so that a
//    kernel reads them with aligned 16-byte loads while the chunk's values sit in LDS.
// 4. All edges between blocks go to a CSR list with block-order columns; then every dense
//    off-diagonal block (a submatrix of two communities whose pairs are mostly nonzero) moves
//    out of that list into lists of zeros against the localised order parameters of its column
//    block (Sec. 3, extension of the approach to submatrices [M1..M2] x [M3..M4]).
// 5. Cut every block into work tiles of similar cost and choose the lanes per row.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "kur_internal.hpp"

namespace kur {

static int host_threads()
{
    const char *e = std::getenv("KUR_THREADS");
    if (!e) e = std::getenv("OMP_NUM_THREADS");
    int t = e ? std::atoi(e) : 0;
    if (t <= 0) t = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
    return std::max(1, std::min(t, 256));
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &f)
{
    if (n <= 0) return;
    int nt = host_threads();
    int64_t per = std::max<int64_t>(1, (n + nt * 8 - 1) / (nt * 8));  // 8 ranges per thread
    std::atomic<int64_t> next{0};
    auto work = [&]() {
        for (;;) {
            int64_t b = next.fetch_add(per);
            if (b >= n) break;
            f(b, std::min(n, b + per));
        }
    };
    if (nt == 1 || n <= per) { work(); return; }
    std::vector<std::thread> th;
    for (int i = 0; i < nt; ++i) th.emplace_back(work);
    for (auto &t : th) t.join();
}

namespace {

struct ErrFlag {
    std::atomic<bool> bad{false};
    std::mutex mu;
    std::string msg;
    void set(const std::string &m)
    {
        std::lock_guard<std::mutex> g(mu);
        if (!bad.load()) { msg = m; bad.store(true); }
    }
};

inline int64_t round8(int64_t x) { return (x + 7) & ~int64_t(7); }

inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Order-dependent hash of a directed pair: the adjacency is symmetric iff the multiset of
// (row, col) pairs equals that of (col, row), which is checked by comparing wrap-around sums.
inline uint64_t pair_hash(uint64_t a, uint64_t b) { return mix64(mix64(a) ^ (b * 0xD6E8FEB86659FD93ull)); }

struct SymHash {
    std::atomic<uint64_t> fwd{0}, bwd{0};
    void add(uint64_t f, uint64_t b)
    {
        fwd.fetch_add(f, std::memory_order_relaxed);
        bwd.fetch_add(b, std::memory_order_relaxed);
    }
};

// Common second half: given the block layout and, for every block-order row, a way to mark
// the row's "listed" block-local columns in a bitmap (for a dense block the ones, which are
// complemented on output; for a sparse block the ones themselves) plus the row's inter
// columns, produce segments, the inter CSR and the tiles.
struct RowSource {
    // mark(m, bits, s): set bit lc for every one entry of row m inside its block (local col);
    // returns the count; must report duplicates through err.
    std::function<int64_t(int64_t, uint64_t *, ErrFlag &)> mark_ones;
    // clear(m, bits): clear what mark_ones set
    std::function<void(int64_t, uint64_t *)> clear;
    // inter(m, out): append block-order inter columns of row m
    std::function<void(int64_t, std::vector<int32_t> &)> inter;
    // number of inter columns of row m
    std::function<int64_t(int64_t)> inter_count;
};

std::string finish(BlockGraph &g, const std::vector<int32_t> &block_of_row, const RowSource &src,
                   const std::vector<uint8_t> *given_mode, const BuildOptions &opt)
{
    const int64_t n = g.n;
    const int32_t W = opt.W;
    g.W = W;
    g.tile_rows = opt.tile_rows;
    g.esz2 = opt.esz2;
    if ((int64_t)W * opt.esz2 > 65535) return "chunk too wide for 16-bit LDS byte offsets";
    int32_t smax = 0;
    for (auto &b : g.blk) smax = std::max(smax, b.size);
    const int64_t words = (smax + 63) / 64 + 1;
    ErrFlag err;

    // per block segment base (chunk-major)
    int64_t tot_segs = 0;
    for (auto &b : g.blk) {
        b.nchunk = (b.size + W - 1) / W;
        b.nlayer = 1;
        b.segbase = tot_segs;
        tot_segs += (int64_t)b.nchunk * b.size;
    }
    std::vector<int32_t> ones_seg(tot_segs, 0);   // one entries per (chunk, row)
    std::vector<int64_t> ones_row(n, 0), inter_row(n, 0);

    // pass A: count ones per chunk
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<uint64_t> bits(words, 0);
        for (int64_t m = lo; m < hi && !err.bad.load(); ++m) {
            const BlkInfo &b = g.blk[block_of_row[m]];
            int64_t cnt = src.mark_ones(m, bits.data(), err);
            int64_t r = m - b.row0;
            for (int32_t c = 0; c < b.nchunk; ++c) {
                int64_t c0 = (int64_t)c * W, c1 = std::min<int64_t>(b.size, c0 + W);
                int64_t k = 0;
                for (int64_t w = c0 / 64; w * 64 < c1; ++w) {
                    uint64_t x = bits[w];
                    int64_t wb = w * 64;
                    if (wb < c0) x &= ~uint64_t(0) << (c0 - wb);
                    if (wb + 64 > c1) x &= (c1 - wb >= 64) ? ~uint64_t(0) : ((uint64_t(1) << (c1 - wb)) - 1);
                    k += __builtin_popcountll(x);
                }
                ones_seg[b.segbase + (int64_t)c * b.size + r] = (int32_t)k;
            }
            ones_row[m] = cnt;
            inter_row[m] = src.inter_count(m);
            src.clear(m, bits.data());
        }
    });
    if (err.bad) return err.msg;

    // density rule per block
    g.n_dense = 0;
    for (int32_t bi = 0; bi < g.nb; ++bi) {
        BlkInfo &b = g.blk[bi];
        if (given_mode) {
            b.mode = (*given_mode)[bi] ? 1 : 0;
        } else {
            int64_t ones = 0;
            for (int64_t m = b.row0; m < b.row0 + b.size; ++m) ones += ones_row[m];
            double pairs = (double)b.size * (double)(b.size - 1);
            double rho = pairs > 0 ? (double)ones / pairs : 0.0;
            b.mode = (b.size >= 2 && rho >= opt.tau) ? 1 : 0;
        }
        g.n_dense += b.mode;
    }
    g.blk_rho.assign(g.nb, 0.0);
    for (int32_t bi = 0; bi < g.nb; ++bi) {
        const BlkInfo &b = g.blk[bi];
        int64_t ones = 0;
        for (int64_t m = b.row0; m < b.row0 + b.size; ++m) ones += ones_row[m];
        const double pairs = (double)b.size * (double)(b.size - 1);
        g.blk_rho[bi] = pairs > 0 ? (double)ones / pairs : 0.0;
    }

    // segment lengths and offsets
    g.seg_ptr.assign(tot_segs + 1, 0);
    g.list_unpadded = 0;
    for (auto &b : g.blk) {
        for (int32_t c = 0; c < b.nchunk; ++c) {
            int64_t c0 = (int64_t)c * W, cw = std::min<int64_t>(b.size, c0 + W) - c0;
            for (int32_t r = 0; r < b.size; ++r) {
                int64_t idx = b.segbase + (int64_t)c * b.size + r;
                int64_t ones = ones_seg[idx];
                int64_t len = ones;
                if (b.mode) {
                    int64_t diag = (r >= c0 && r < c0 + cw) ? 1 : 0;
                    len = cw - ones - diag;
                }
                g.list_unpadded += len;
                g.seg_ptr[idx + 1] = round8(len);
            }
        }
    }
    for (int64_t i = 0; i < tot_segs; ++i) g.seg_ptr[i + 1] += g.seg_ptr[i];
    g.list.assign((size_t)g.seg_ptr[tot_segs], (uint16_t)0);

    g.inter_ptr.assign(n + 1, 0);
    for (int64_t m = 0; m < n; ++m) g.inter_ptr[m + 1] = g.inter_ptr[m] + inter_row[m];
    g.inter_col.assign((size_t)g.inter_ptr[n], 0);
    g.deg.assign(n, 0);

    // pass B: emit the lists and the inter CSR
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<uint64_t> bits(words, 0);
        std::vector<int32_t> tmp;
        for (int64_t m = lo; m < hi && !err.bad.load(); ++m) {
            const BlkInfo &b = g.blk[block_of_row[m]];
            int64_t r = m - b.row0;
            int64_t cnt = src.mark_ones(m, bits.data(), err);
            for (int32_t c = 0; c < b.nchunk; ++c) {
                int64_t c0 = (int64_t)c * W, c1 = std::min<int64_t>(b.size, c0 + W);
                int64_t idx = b.segbase + (int64_t)c * b.size + r;
                uint16_t *out = g.list.data() + g.seg_ptr[idx];
                int64_t k = 0;
                for (int64_t w = c0 / 64; w * 64 < c1; ++w) {
                    uint64_t x = bits[w];
                    if (b.mode) x = ~x;
                    int64_t wb = w * 64;
                    if (wb < c0) x &= ~uint64_t(0) << (c0 - wb);
                    if (wb + 64 > c1) x &= (c1 - wb >= 64) ? ~uint64_t(0) : ((uint64_t(1) << (c1 - wb)) - 1);
                    if (b.mode && r >= wb && r < wb + 64) x &= ~(uint64_t(1) << (r - wb));
                    while (x) {
                        int t = __builtin_ctzll(x);
                        x &= x - 1;
                        out[k++] = (uint16_t)((wb + t - c0) * opt.esz2);
                    }
                }
                int64_t padded = g.seg_ptr[idx + 1] - g.seg_ptr[idx];
                for (; k < padded; ++k) out[k] = (uint16_t)(W * opt.esz2);
            }
            src.clear(m, bits.data());
            tmp.clear();
            src.inter(m, tmp);
            std::sort(tmp.begin(), tmp.end());
            for (size_t i = 1; i < tmp.size(); ++i)
                if (tmp[i] == tmp[i - 1]) { err.set("duplicate column in a row (inter-block entry)"); break; }
            std::copy(tmp.begin(), tmp.end(), g.inter_col.begin() + g.inter_ptr[m]);
            g.deg[m] = (int32_t)std::min<int64_t>(cnt + (int64_t)tmp.size(), INT32_MAX);
        }
    });
    if (err.bad) return err.msg;

    diag_segments(g);
    if (!given_mode) {  // a layout given block by block is used as it is
        std::string msg = add_dense_pairs(g, opt);
        if (!msg.empty()) return msg;
    }
    std::string msg = to_masks(g, opt);
    if (!msg.empty()) return msg;
    make_tiles(g, opt);
    return "";
}

}  // namespace

std::string to_masks(BlockGraph &g, const BuildOptions &opt)
{
    g.mask.clear();
    g.mask_segments = 0;
    if (!(opt.mask_min <= 1.0) || g.W < kMaskMinW || g.seg_ptr.empty()) return "";
    const int64_t n = g.n;
    const uint16_t pad = (uint16_t)(g.W * g.esz2);
    const size_t nsd = g.segd.size();
    // the segments whose stored entries (padded to 8 per row) fill at least mask_min of the cells
    std::vector<int64_t> mbase(nsd, -1);
    int64_t units = 0;
    for (int32_t bi = 0; bi < g.nb; ++bi) {
        const BlkInfo &b = g.blk[bi];
        for (int32_t ch = 0; ch < b.nchunk; ++ch) {
            const SegD &sd = g.segd[b.sd0 + ch];
            const int64_t sb = b.segbase + (int64_t)ch * b.size;
            const double stored = (double)(g.seg_ptr[sb + b.size] - g.seg_ptr[sb]);
            const double cells = (double)b.size * (double)sd.cw;
            if (cells <= 0 || stored <= 0 || stored < opt.mask_min * cells) continue;
            const int64_t seg_units = (int64_t)b.size * ((sd.cw + kMaskUnitCols - 1) / kMaskUnitCols);
            if (seg_units * 16 > INT32_MAX) continue;  // the kernels address a segment with 32-bit offsets
            mbase[b.sd0 + ch] = units;
            units += seg_units;
        }
    }
    if (units == 0) return "";
    if (units > ((int64_t)1 << 40)) return "bitmask layout too large";
    g.mask.assign((size_t)units * 4, 0u);
    std::vector<int32_t> bor(n);
    for (int32_t bi = 0; bi < g.nb; ++bi)
        std::fill(bor.begin() + g.blk[bi].row0, bor.begin() + g.blk[bi].row0 + g.blk[bi].size, bi);
    // fill the bits row by row (each row owns its units) and the new segment lengths
    const int64_t tot = (int64_t)g.seg_ptr.size() - 1;
    std::vector<int64_t> len(tot + 1, 0);
    std::vector<int64_t> moved(n, 0);
    ErrFlag err;
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t m = lo; m < hi && !err.bad.load(); ++m) {
            const BlkInfo &b = g.blk[bor[m]];
            const int64_t r = m - b.row0;
            for (int32_t ch = 0; ch < b.nchunk; ++ch) {
                const int64_t idx = b.segbase + (int64_t)ch * b.size + r;
                const int64_t mb = mbase[b.sd0 + ch];
                if (mb < 0) {
                    len[idx + 1] = g.seg_ptr[idx + 1] - g.seg_ptr[idx];
                    continue;
                }
                for (int64_t e = g.seg_ptr[idx]; e < g.seg_ptr[idx + 1]; ++e) {
                    if (g.list[e] == pad) continue;
                    const int64_t col = g.list[e] / g.esz2;
                    const int64_t q = col / kMaskUnitCols, j = col % kMaskUnitCols;
                    uint32_t &word = g.mask[(size_t)(mb + q * b.size + r) * 4 + (size_t)(j >> 5)];
                    const uint32_t bit = 1u << (j & 31);
                    if (word & bit) {
                        err.set("repeated column in a list segment");
                        break;
                    }
                    word |= bit;
                    ++moved[m];
                }
            }
        }
    });
    if (err.bad) return err.msg;
    // the lists without the bitmask segments
    for (int64_t i = 0; i < tot; ++i) len[i + 1] += len[i];
    std::vector<uint16_t> list((size_t)len[tot]);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t m = lo; m < hi; ++m) {
            const BlkInfo &b = g.blk[bor[m]];
            const int64_t r = m - b.row0;
            for (int32_t ch = 0; ch < b.nchunk; ++ch) {
                const int64_t idx = b.segbase + (int64_t)ch * b.size + r;
                if (mbase[b.sd0 + ch] >= 0) continue;
                std::copy(g.list.begin() + g.seg_ptr[idx], g.list.begin() + g.seg_ptr[idx + 1], list.begin() + len[idx]);
            }
        }
    });
    g.list.swap(list);
    g.seg_ptr.swap(len);
    for (int64_t m = 0; m < n; ++m) g.list_unpadded -= moved[m];
    for (size_t i = 0; i < nsd; ++i) {
        if (mbase[i] < 0) continue;
        g.segd[i].mask = 1;
        g.segd[i].mbase = mbase[i];
        ++g.mask_segments;
    }
    return "";
}

namespace {

// The bitmask sub-chunk width (the option, at most the chunk, in whole units; for 16-byte value
// pairs at most 4 units, so that a table read's constant offset stays below 64 KiB) and item
// size.
void mask_params(BlockGraph &g, const BuildOptions &opt)
{
    const int32_t cap = g.esz2 > 8 ? kMaskSubMax / 2 : kMaskSubMax;
    g.mask_sub = std::max(kMaskUnitCols, std::min({opt.mask_sub, g.W, cap}) / kMaskUnitCols * kMaskUnitCols);
    g.mask_item = opt.mask_item;
}

}  // namespace

void make_tiles(BlockGraph &g, const BuildOptions &opt)
{
    const int64_t n = g.n;
    g.tile_rows = opt.tile_rows;
    g.xcds = opt.xcds;
    mask_params(g, opt);
    // work tiles: consecutive rows of one block with similar cost
    std::vector<int64_t> rowcost(n);
    int64_t total = 0;
    for (auto &b : g.blk) {
        for (int32_t r = 0; r < b.size; ++r) {
            const int64_t m = b.row0 + r;
            int64_t c = 32 + 4 * (g.inter_ptr[m + 1] - g.inter_ptr[m]);
            for (int32_t ch = 0; ch < b.nchunk; ++ch) {
                int64_t idx = b.segbase + (int64_t)ch * b.size + r;
                c += g.seg_ptr[idx + 1] - g.seg_ptr[idx];
                // a bitmask row: cw / 8 bytes and cw / 4 conflict-free table reads
                if (g.segd[b.sd0 + ch].mask) c += (g.segd[b.sd0 + ch].cw + 7) / 8;
            }
            rowcost[m] = c;
            total += c;
        }
    }
    // a tile's list work should amortise its fixed cost (block-sum fold, staging, launch)
    const int64_t target = std::max<int64_t>(opt.tile_min_cost, total / std::max<int64_t>(1, opt.tiles_target));
    g.tiles.clear();
    for (int32_t bi = 0; bi < g.nb; ++bi) {
        BlkInfo &b = g.blk[bi];
        b.tile0 = (int32_t)g.tiles.size();
        int32_t r = 0;
        while (r < b.size) {
            int32_t r1 = r;
            int64_t c = 0;
            while (r1 < b.size && r1 - r < opt.tile_rows && (r1 == r || c + rowcost[b.row0 + r1] <= target)) {
                c += rowcost[b.row0 + r1];
                ++r1;
            }
            // lanes per row: about two 8-entry vectors per lane in a non-empty chunk
            int64_t vec = 0, nonempty = 0, masks = 0;
            for (int32_t ch = 0; ch < b.nchunk; ++ch) {
                int64_t s0 = g.seg_ptr[b.segbase + (int64_t)ch * b.size + r];
                int64_t s1 = g.seg_ptr[b.segbase + (int64_t)ch * b.size + r1];
                vec += (s1 - s0) / 8;
                nonempty += (s1 > s0);
                masks += g.segd[b.sd0 + ch].mask;
            }
            double avg = nonempty ? (double)vec / ((double)(r1 - r) * (double)nonempty) : 0.0;
            int32_t G = 2;
            while (G < 64 && G * 2 < avg) G *= 2;
            if (opt.flat_min_vec > 0 && avg >= opt.flat_min_vec) G = 0;  // wave-streaming mode
            if (nonempty == 0 && masks == 0) G = -1;                      // no list entries at all
            g.tiles.push_back(Tile{bi, r, r1, G});
            r = r1;
        }
        b.ntiles = (int32_t)g.tiles.size() - b.tile0;
    }
    order_tiles(g);
}

namespace {

// The block holding block-order row (or column) r.
int32_t block_at(const BlockGraph &g, int64_t r)
{
    return (int32_t)(std::upper_bound(g.blk.begin(), g.blk.end(), r,
                                      [](int64_t x, const BlkInfo &b) { return x < (int64_t)b.row0; }) -
                     g.blk.begin()) - 1;
}

}  // namespace

void order_tiles(BlockGraph &g)
{
    const size_t nt = g.tiles.size();
    std::vector<int64_t> cost(nt);
    for (size_t t = 0; t < nt; ++t) {
        const Tile &tl = g.tiles[t];
        const BlkInfo &b = g.blk[tl.block];
        int64_t c = 32 * (int64_t)(tl.r1 - tl.r0);
        int64_t staging = 0;  // per nonempty segment the size of its column block
        for (int32_t ch = 0; ch < b.nchunk; ++ch) {
            const int64_t s0 = g.seg_ptr[b.segbase + (int64_t)ch * b.size + tl.r0];
            const int64_t s1 = g.seg_ptr[b.segbase + (int64_t)ch * b.size + tl.r1];
            c += s1 - s0;
            if (s1 > s0) staging += g.blk[block_at(g, g.segd[b.sd0 + ch].col0)].size;
        }
        c += 4 * (g.inter_ptr[b.row0 + tl.r1] - g.inter_ptr[b.row0 + tl.r0]);
        cost[t] = c + staging / 4;
    }
    const int X = std::max(1, g.xcds);
    // units of placement: a block, or for a block costing more than total / (2 X) runs of its
    // consecutive tiles of about that cost each, so that few or uneven blocks still spread over
    // every XCD
    int64_t total = 0;
    for (int64_t c : cost) total += c;
    const int64_t cap = std::max<int64_t>(1, total / (2 * X));
    struct Unit {
        int32_t t0, t1;
        int64_t cost;
    };
    std::vector<Unit> units;
    for (int32_t b = 0; b < g.nb; ++b) {
        const BlkInfo &bi = g.blk[b];
        int32_t t = bi.tile0;
        const int32_t tend = bi.tile0 + bi.ntiles;
        while (t < tend) {
            Unit u{t, t, 0};
            while (u.t1 < tend && (u.t1 == u.t0 || u.cost + cost[u.t1] <= cap)) u.cost += cost[u.t1++];
            units.push_back(u);
            t = u.t1;
        }
    }
    // units to XCDs: largest first, each to the least loaded XCD
    std::stable_sort(units.begin(), units.end(), [](const Unit &a, const Unit &b) { return a.cost > b.cost; });
    std::vector<int64_t> load(X, 0);
    std::vector<int32_t> xcd_of_tile(nt, 0);
    for (const Unit &u : units) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (int32_t t = u.t0; t < u.t1; ++t) xcd_of_tile[t] = x;
        load[x] += u.cost;
    }
    // per XCD, its tiles largest first; then interleave
    std::vector<std::vector<int32_t>> lists(X);
    for (size_t t = 0; t < nt; ++t) lists[xcd_of_tile[t]].push_back((int32_t)t);
    size_t longest = 0;
    for (auto &l : lists) {
        std::stable_sort(l.begin(), l.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
        longest = std::max(longest, l.size());
    }
    g.order.assign(longest * X, -1);
    for (int x = 0; x < X; ++x)
        for (size_t j = 0; j < lists[x].size(); ++j) g.order[j * X + x] = lists[x][j];
    // drop empty slots after the last tile
    while (!g.order.empty() && g.order.back() < 0) g.order.pop_back();
    mask_items(g);
}

void mask_items(BlockGraph &g)
{
    g.mitems.clear();
    g.mtiles.clear();
    g.mask_part_rows = 0;
    if (g.mask_segments == 0) return;
    const int64_t S = g.mask_sub;
    g.mtiles.assign(g.tiles.size(), MaskTile{0, 0, 0});
    std::vector<int64_t> cells;
    for (size_t t = 0; t < g.tiles.size(); ++t) {
        const Tile &tl = g.tiles[t];
        const BlkInfo &b = g.blk[tl.block];
        const int64_t h = tl.r1 - tl.r0;
        MaskTile &mt = g.mtiles[t];
        mt.off = g.mask_part_rows;
        bool open = false;
        for (int32_t ch = 0; ch < b.nchunk; ++ch) {
            const SegD &sd = g.segd[b.sd0 + ch];
            if (!sd.mask) continue;
            for (int64_t s0 = 0; s0 < sd.cw; s0 += S) {
                const int64_t cc = h * std::min<int64_t>(S, sd.cw - s0);
                if (open && cells.back() + cc > g.mask_item) open = false;
                if (!open) {
                    g.mitems.push_back(MaskItem{(int32_t)t, ch, (int32_t)(s0 / S), 0, g.mask_part_rows});
                    cells.push_back(0);
                    g.mask_part_rows += h;
                    ++mt.cnt;
                    open = true;
                }
                ++g.mitems.back().nsub;
                cells.back() += cc;
            }
        }
    }
    // largest first (ties in tile order)
    std::vector<int64_t> idx(g.mitems.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int64_t)i;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return cells[a] > cells[b]; });
    std::vector<MaskItem> sorted(idx.size());
    for (size_t i = 0; i < idx.size(); ++i) sorted[i] = g.mitems[idx[i]];
    g.mitems.swap(sorted);
}

std::string build_complete(int64_t n, const BuildOptions &opt, BlockGraph &g)
{
    if (n < 1 || n > INT32_MAX - 1) return "n must be in [1, 2^31-2]";
    if ((int64_t)opt.W * opt.esz2 > 65535) return "chunk too wide for 16-bit LDS byte offsets";
    g = BlockGraph();
    g.n = n;
    g.nb = 1;
    g.W = opt.W;
    g.tile_rows = opt.tile_rows;
    g.esz2 = opt.esz2;
    g.perm.resize(n);
    std::iota(g.perm.begin(), g.perm.end(), 0);
    BlkInfo b{};
    b.row0 = 0;
    b.size = (int32_t)n;
    b.nchunk = (int32_t)((n + opt.W - 1) / opt.W);
    b.nlayer = 1;
    b.mode = n >= 2 ? 1 : 0;
    b.segbase = 0;
    g.blk.push_back(b);
    g.seg_ptr.assign((size_t)b.nchunk * n + 1, 0);
    g.inter_ptr.assign(n + 1, 0);
    g.deg.assign(n, (int32_t)std::min<int64_t>(n - 1, INT32_MAX));
    g.n_dense = b.mode;
    g.symmetric = true;
    g.blk_rho.assign(1, 1.0);
    diag_segments(g);
    // tiles: only the epilogue works per row (no list entries), so use full-size tiles
    g.blk[0].tile0 = 0;
    for (int64_t r = 0; r < n; r += opt.tile_rows)
        g.tiles.push_back(Tile{0, (int32_t)r, (int32_t)std::min<int64_t>(n, r + opt.tile_rows), -1});
    g.blk[0].ntiles = (int32_t)g.tiles.size();
    g.xcds = opt.xcds;
    mask_params(g, opt);
    order_tiles(g);
    return "";
}

std::string merge_graphs(std::vector<BlockGraph> &parts, BlockGraph &g, std::vector<int64_t> &row_first,
                         std::vector<int64_t> &tile_first)
{
    if (parts.empty()) return "no instances";
    g = BlockGraph();
    g.W = parts[0].W;
    g.tile_rows = parts[0].tile_rows;
    g.esz2 = parts[0].esz2;
    g.xcds = parts[0].xcds;
    g.mask_sub = parts[0].mask_sub;
    g.mask_item = parts[0].mask_item;
    g.symmetric = true;
    int64_t n = 0, nb = 0, segs = 0, entries = 0, inter = 0, tiles = 0;
    for (const BlockGraph &p : parts) {
        if (p.W != g.W || p.tile_rows != g.tile_rows || p.esz2 != g.esz2 || p.mask_sub != g.mask_sub ||
            p.mask_item != g.mask_item)
            return "instances built with different layouts";
        n += p.n;
        nb += p.nb;
        segs += (int64_t)p.seg_ptr.size() - 1;
        entries += (int64_t)p.list.size();
        inter += (int64_t)p.inter_col.size();
        tiles += (int64_t)p.tiles.size();
    }
    if (n > INT32_MAX - 1 || nb > INT32_MAX || tiles > INT32_MAX) return "batch too large";
    g.n = n;
    g.nb = (int32_t)nb;
    g.perm.reserve(n);
    g.blk.reserve(nb);
    g.seg_ptr.reserve(segs + 1);
    g.list.reserve(entries);
    g.inter_ptr.reserve(n + 1);
    g.inter_col.reserve(inter);
    g.tiles.reserve(tiles);
    g.deg.reserve(n);
    row_first.assign(1, 0);
    tile_first.assign(1, 0);
    g.inter_ptr.push_back(0);
    int64_t roff = 0, segoff = 0, loff = 0, toff = 0, boff = 0;
    for (BlockGraph &p : parts) {
        for (int32_t v : p.perm) g.perm.push_back((int32_t)(v + roff));
        const int32_t sdoff = (int32_t)g.segd.size(), goff = (int32_t)g.grp.size();
        for (BlkInfo b : p.blk) {
            b.row0 += (int32_t)roff;
            b.segbase += segoff;
            b.tile0 += (int32_t)toff;
            b.sd0 += sdoff;
            b.grp0 += goff;
            g.blk.push_back(b);
        }
        const int64_t moff = (int64_t)g.mask.size() / 4;  // mask units before this part
        for (SegD d : p.segd) {
            d.col0 += (int32_t)roff;
            if (d.mask) d.mbase += moff;
            g.segd.push_back(d);
        }
        g.mask.insert(g.mask.end(), p.mask.begin(), p.mask.end());
        g.mask_segments += p.mask_segments;
        for (Grp q : p.grp) {
            q.blk += (int32_t)boff;
            g.grp.push_back(q);
        }
        g.blk_rho.insert(g.blk_rho.end(), p.blk_rho.begin(), p.blk_rho.end());
        g.pair_rho.insert(g.pair_rho.end(), p.pair_rho.begin(), p.pair_rho.end());
        g.n_pairs += p.n_pairs;
        for (size_t i = 0; i + 1 < p.seg_ptr.size(); ++i) g.seg_ptr.push_back(p.seg_ptr[i] + loff);
        g.list.insert(g.list.end(), p.list.begin(), p.list.end());
        for (int64_t m = 0; m < p.n; ++m) g.inter_ptr.push_back(p.inter_ptr[m + 1] + (g.inter_ptr.size() > 0 ? g.inter_ptr[roff] : 0));
        for (int32_t v : p.inter_col) g.inter_col.push_back((int32_t)(v + roff));
        for (Tile t : p.tiles) {
            t.block += (int32_t)boff;
            g.tiles.push_back(t);
        }
        g.deg.insert(g.deg.end(), p.deg.begin(), p.deg.end());
        g.list_unpadded += p.list_unpadded;
        g.n_dense += p.n_dense;
        g.symmetric = g.symmetric && p.symmetric;
        roff += p.n;
        segoff += (int64_t)p.seg_ptr.size() - 1;
        loff += (int64_t)p.list.size();
        toff += (int64_t)p.tiles.size();
        boff += p.nb;
        row_first.push_back(roff);
        tile_first.push_back(toff);
        p = BlockGraph();  // release the part
    }
    g.seg_ptr.push_back(loff);
    order_tiles(g);
    return "";
}

std::string validate_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels)
{
    if (n < 1 || n > INT32_MAX - 1) return "n must be in [1, 2^31-2]";
    if (!row_ptr || !labels) return "row_ptr and labels must not be NULL";
    if (row_ptr[0] != 0) return "row_ptr[0] must be 0";
    for (int64_t m = 0; m < n; ++m)
        if (row_ptr[m + 1] < row_ptr[m]) return "row_ptr must be non-decreasing";
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && !col) return "col must not be NULL";
    {
        std::atomic<bool> bad{false};
        parallel_for(nnz, [&](int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; ++e)
                if (col[e] < 0 || col[e] >= n) { bad = true; return; }
        });
        if (bad) return "column index out of range";
    }
    for (int64_t u = 0; u < n; ++u)
        if (labels[u] < 0) return "labels must be >= 0";
    return "";
}

bool csr_symmetric(int64_t n, const int64_t *row_ptr, const int32_t *col)
{
    // the sums of a 64-bit hash over the (row, col) pairs and over the (col, row) pairs agree
    // for a symmetric pattern (diagonal entries ignored)
    SymHash sym;
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        uint64_t f = 0, b = 0;
        for (int64_t u = lo; u < hi; ++u)
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                if (col[e] == u) continue;
                f += pair_hash((uint64_t)u, (uint64_t)col[e]);
                b += pair_hash((uint64_t)col[e], (uint64_t)u);
            }
        sym.add(f, b);
    });
    return sym.fwd.load() == sym.bwd.load();
}

int32_t regroup_by_labels(int64_t n, const int32_t *labels, std::vector<int32_t> &perm, std::vector<int32_t> &node_at,
                          std::vector<int32_t> &block_of_row, std::vector<int64_t> &block_ptr)
{
    // communities ordered by label value; stable counting sort of the nodes
    std::vector<int32_t> uniq(labels, labels + n);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
    const int32_t nb = (int32_t)uniq.size();
    std::vector<int32_t> comm(n);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t u = lo; u < hi; ++u)
            comm[u] = (int32_t)(std::lower_bound(uniq.begin(), uniq.end(), labels[u]) - uniq.begin());
    });
    block_ptr.assign(nb + 1, 0);
    for (int64_t u = 0; u < n; ++u) block_ptr[comm[u] + 1]++;
    for (int32_t b = 0; b < nb; ++b) block_ptr[b + 1] += block_ptr[b];
    perm.resize(n);
    node_at.resize(n);
    block_of_row.resize(n);
    std::vector<int64_t> fill(block_ptr.begin(), block_ptr.end() - 1);
    for (int64_t u = 0; u < n; ++u) {
        const int64_t m = fill[comm[u]]++;
        perm[u] = (int32_t)m;
        node_at[m] = (int32_t)u;
        block_of_row[m] = comm[u];
    }
    return nb;
}

std::string build_from_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels,
                           const BuildOptions &opt, BlockGraph &g)
{
    std::string msg = validate_csr(n, row_ptr, col, labels);
    if (!msg.empty()) return msg;
    const bool symmetric = csr_symmetric(n, row_ptr, col);
    g = BlockGraph();
    g.n = n;
    std::vector<int32_t> node_at, block_of_row;
    std::vector<int64_t> bptr;
    g.nb = regroup_by_labels(n, labels, g.perm, node_at, block_of_row, bptr);
    const int32_t nb = g.nb;
    g.blk.resize(nb);
    for (int32_t b = 0; b < nb; ++b) {
        g.blk[b] = BlkInfo{};
        g.blk[b].row0 = (int32_t)bptr[b];
        g.blk[b].size = (int32_t)(bptr[b + 1] - bptr[b]);
    }
    const int32_t *perm = g.perm.data();
    RowSource src;
    src.mark_ones = [&](int64_t m, uint64_t *bits, ErrFlag &err) -> int64_t {
        int64_t u = node_at[m];
        const BlkInfo &b = g.blk[block_of_row[m]];
        int64_t k = 0;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t pv = perm[col[e]];
            if (pv == m || pv < b.row0 || pv >= b.row0 + b.size) continue;
            int64_t lc = pv - b.row0;
            uint64_t bit = uint64_t(1) << (lc & 63);
            if (bits[lc >> 6] & bit) { err.set("duplicate column in a row"); continue; }
            bits[lc >> 6] |= bit;
            ++k;
        }
        return k;
    };
    src.clear = [&](int64_t m, uint64_t *bits) {
        int64_t u = node_at[m];
        const BlkInfo &b = g.blk[block_of_row[m]];
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t pv = perm[col[e]];
            if (pv < b.row0 || pv >= b.row0 + b.size) continue;
            int64_t lc = pv - b.row0;
            bits[lc >> 6] = 0;
        }
    };
    src.inter_count = [&](int64_t m) -> int64_t {
        int64_t u = node_at[m];
        const BlkInfo &b = g.blk[block_of_row[m]];
        int64_t k = 0;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t pv = perm[col[e]];
            k += (pv < b.row0 || pv >= b.row0 + b.size);
        }
        return k;
    };
    src.inter = [&](int64_t m, std::vector<int32_t> &out) {
        int64_t u = node_at[m];
        const BlkInfo &b = g.blk[block_of_row[m]];
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            int64_t pv = perm[col[e]];
            if (pv < b.row0 || pv >= b.row0 + b.size) out.push_back((int32_t)pv);
        }
    };
    msg = finish(g, block_of_row, src, nullptr, opt);
    g.symmetric = symmetric;
    return msg;
}

std::string build_from_csr_w(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                             const int32_t *labels, const BuildOptions &opt, BlockGraph &g)
{
    std::string msg = validate_csr(n, row_ptr, col, labels);
    if (!msg.empty()) return msg;
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && !weight) return "weight must not be NULL";
    for (int64_t e = 0; e < nnz; ++e)
        if (weight[e] < 0 || weight[e] > kMaxWeight) return "weights must be in [0, 255]";
    const int32_t W = opt.W;
    if ((int64_t)W * opt.esz2 > 65535) return "chunk too wide for 16-bit LDS byte offsets";
    // symmetry of the weighted pattern (diagonal and zero weights ignored)
    SymHash sym;
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        uint64_t f = 0, b = 0;
        for (int64_t u = lo; u < hi; ++u)
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                if (col[e] == u || weight[e] == 0) continue;
                f += pair_hash((uint64_t)u, (uint64_t)col[e]) * (uint64_t)weight[e];
                b += pair_hash((uint64_t)col[e], (uint64_t)u) * (uint64_t)weight[e];
            }
        sym.add(f, b);
    });
    g = BlockGraph();
    g.n = n;
    g.W = W;
    g.tile_rows = opt.tile_rows;
    g.esz2 = opt.esz2;
    std::vector<int32_t> node_at, block_of_row;
    std::vector<int64_t> bptr;
    g.nb = regroup_by_labels(n, labels, g.perm, node_at, block_of_row, bptr);
    const int32_t nb = g.nb;
    g.blk.resize(nb);
    int32_t smax = 0;
    for (int32_t b = 0; b < nb; ++b) {
        g.blk[b] = BlkInfo{};
        g.blk[b].row0 = (int32_t)bptr[b];
        g.blk[b].size = (int32_t)(bptr[b + 1] - bptr[b]);
        smax = std::max(smax, g.blk[b].size);
    }
    // per block: histogram of the weights of its off-diagonal pairs (duplicates rejected)
    ErrFlag err;
    std::vector<std::vector<int64_t>> hist(nb, std::vector<int64_t>(kMaxWeight + 1, 0));
    std::vector<std::mutex> hist_mu(nb);
    std::vector<int64_t> inter_row(n, 0), wdeg(n, 0);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<uint8_t> val((size_t)smax + 1, 0);
        std::vector<int64_t> h(kMaxWeight + 1, 0);
        for (int64_t m = lo; m < hi && !err.bad.load(); ++m) {
            const int32_t b = block_of_row[m];
            const int64_t r0 = g.blk[b].row0, s = g.blk[b].size, u = node_at[m];
            std::fill(h.begin(), h.end(), 0);
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                const int64_t pv = g.perm[col[e]];
                const int32_t w = weight[e];
                if (pv == m || w == 0) continue;
                wdeg[m] += w;
                if (pv < r0 || pv >= r0 + s) {
                    inter_row[m] += w;  // listed once per unit of weight
                    continue;
                }
                if (val[pv - r0]) err.set("duplicate column in a row");
                val[pv - r0] = (uint8_t)w;
                h[w]++;
            }
            for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                const int64_t pv = g.perm[col[e]];
                if (pv >= r0 && pv < r0 + s) val[pv - r0] = 0;
            }
            std::lock_guard<std::mutex> lk(hist_mu[b]);
            for (int v = 1; v <= kMaxWeight; ++v) hist[b][v] += h[v];
        }
    });
    if (err.bad) return err.msg;
    // prevalent value (ties: the smaller) and layers per block
    int64_t tot_segs = 0;
    g.n_dense = 0;
    for (int32_t b = 0; b < nb; ++b) {
        BlkInfo &bi = g.blk[b];
        const int64_t s = bi.size;
        int64_t nz = 0;
        int32_t jmax = 0;
        for (int v = 1; v <= kMaxWeight; ++v)
            if (hist[b][v]) {
                nz += hist[b][v];
                jmax = v;
            }
        hist[b][0] = s * (s - 1) - nz;
        int32_t vb = 0;
        for (int v = 1; v <= jmax; ++v)
            if (hist[b][v] > hist[b][vb]) vb = v;
        bi.mode = s >= 2 ? vb : 0;
        bi.nlayer = std::max(1, jmax);
        bi.nchunk = (int32_t)((s + W - 1) / W) * bi.nlayer;
        bi.segbase = tot_segs;
        tot_segs += (int64_t)bi.nchunk * s;
        g.n_dense += bi.mode > 0;
    }
    // per segment (column chunk, layer) list lengths: layer t <= mode lists the columns (not the
    // row itself) with weight < t, layer t > mode those with weight >= t
    g.seg_ptr.assign(tot_segs + 1, 0);
    std::vector<int64_t> unpadded(n, 0);
    auto row_pass = [&](bool emit) {
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            std::vector<uint8_t> val((size_t)smax + 1, 0);
            std::vector<int32_t> tmp;
            for (int64_t m = lo; m < hi; ++m) {
                const BlkInfo &bi = g.blk[block_of_row[m]];
                const int64_t r0 = bi.row0, s = bi.size, u = node_at[m], r = m - r0;
                for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    const int64_t pv = g.perm[col[e]];
                    if (pv != m && weight[e] > 0 && pv >= r0 && pv < r0 + s) val[pv - r0] = (uint8_t)weight[e];
                }
                const int32_t ncc = bi.nchunk / bi.nlayer;
                int64_t total = 0;
                for (int32_t cc = 0; cc < ncc; ++cc) {
                    const int64_t c0 = (int64_t)cc * W, c1 = std::min<int64_t>(s, c0 + W);
                    for (int32_t t = 1; t <= bi.nlayer; ++t) {
                        const int64_t idx = bi.segbase + (int64_t)((int64_t)cc * bi.nlayer + t - 1) * s + r;
                        const bool zeros = t <= bi.mode;
                        uint16_t *out = emit ? g.list.data() + g.seg_ptr[idx] : nullptr;
                        int64_t k = 0;
                        for (int64_t lc = c0; lc < c1; ++lc) {
                            const bool listed = zeros ? (lc != r && val[lc] < t) : (val[lc] >= t);
                            if (!listed) continue;
                            if (emit) out[k] = (uint16_t)((lc - c0) * opt.esz2);
                            ++k;
                        }
                        if (emit) {
                            const int64_t padded = g.seg_ptr[idx + 1] - g.seg_ptr[idx];
                            for (; k < padded; ++k) out[k] = (uint16_t)(W * opt.esz2);
                        } else {
                            g.seg_ptr[idx + 1] = round8(k);
                            total += k;
                        }
                    }
                }
                if (!emit) unpadded[m] = total;
                for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    const int64_t pv = g.perm[col[e]];
                    if (pv >= r0 && pv < r0 + s) val[pv - r0] = 0;
                }
                if (emit) {
                    tmp.clear();
                    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                        const int64_t pv = g.perm[col[e]];
                        if (pv != m && weight[e] > 0 && (pv < r0 || pv >= r0 + s))
                            for (int32_t k = 0; k < weight[e]; ++k) tmp.push_back((int32_t)pv);
                    }
                    std::sort(tmp.begin(), tmp.end());
                    std::copy(tmp.begin(), tmp.end(), g.inter_col.begin() + g.inter_ptr[m]);
                }
            }
        });
    };
    row_pass(false);
    for (int64_t i = 0; i < tot_segs; ++i) g.seg_ptr[i + 1] += g.seg_ptr[i];
    g.list.assign((size_t)g.seg_ptr[tot_segs], (uint16_t)0);
    g.list_unpadded = 0;
    for (int64_t m = 0; m < n; ++m) g.list_unpadded += unpadded[m];
    g.inter_ptr.assign(n + 1, 0);
    for (int64_t m = 0; m < n; ++m) g.inter_ptr[m + 1] = g.inter_ptr[m] + inter_row[m];
    g.inter_col.assign((size_t)g.inter_ptr[n], 0);
    row_pass(true);
    g.deg.assign(n, 0);
    for (int64_t m = 0; m < n; ++m) g.deg[m] = (int32_t)std::min<int64_t>(wdeg[m], INT32_MAX);
    g.symmetric = sym.fwd.load() == sym.bwd.load();
    g.weighted = true;
    g.blk_rho.assign(nb, 0.0);
    for (int32_t b = 0; b < nb; ++b) {
        const double s = g.blk[b].size, pairs = s * (s - 1);
        g.blk_rho[b] = pairs > 0 ? (pairs - (double)hist[b][0]) / pairs : 0.0;
    }
    diag_segments(g);
    msg = add_dense_pairs(g, opt);
    if (!msg.empty()) return msg;
    msg = to_masks(g, opt);
    if (!msg.empty()) return msg;
    make_tiles(g, opt);
    return "";
}

std::string build_from_blocks(int64_t n, int32_t nb, const int64_t *block_ptr, const uint8_t *mode,
                              const int64_t *list_ptr, const uint16_t *list_col, const int64_t *inter_ptr,
                              const int32_t *inter_col, const int32_t *perm, const BuildOptions &opt,
                              BlockGraph &g)
{
    if (n < 1 || n > INT32_MAX - 1) return "n must be in [1, 2^31-2]";
    if (nb < 1 || nb > n) return "nb must be in [1, n]";
    if (!block_ptr || !mode || !list_ptr || !inter_ptr) return "block_ptr, mode, list_ptr, inter_ptr must not be NULL";
    if (block_ptr[0] != 0 || block_ptr[nb] != n) return "block_ptr must start at 0 and end at n";
    for (int32_t b = 0; b < nb; ++b) {
        if (block_ptr[b + 1] <= block_ptr[b]) return "block_ptr must be strictly increasing";
        if (block_ptr[b + 1] - block_ptr[b] > 65535) return "block sizes must be <= 65535";
    }
    if (list_ptr[0] != 0 || inter_ptr[0] != 0) return "list_ptr[0] and inter_ptr[0] must be 0";
    for (int64_t m = 0; m < n; ++m)
        if (list_ptr[m + 1] < list_ptr[m] || inter_ptr[m + 1] < inter_ptr[m])
            return "list_ptr and inter_ptr must be non-decreasing";
    if (list_ptr[n] > 0 && !list_col) return "list_col must not be NULL";
    if (inter_ptr[n] > 0 && !inter_col) return "inter_col must not be NULL";
    g = BlockGraph();
    g.n = n;
    g.nb = nb;
    std::vector<int32_t> block_of_row(n);
    g.blk.resize(nb);
    for (int32_t b = 0; b < nb; ++b) {
        g.blk[b] = BlkInfo{};
        g.blk[b].row0 = (int32_t)block_ptr[b];
        g.blk[b].size = (int32_t)(block_ptr[b + 1] - block_ptr[b]);
        for (int64_t m = block_ptr[b]; m < block_ptr[b + 1]; ++m) block_of_row[m] = b;
    }
    for (int64_t m = 0; m < n; ++m) {
        const BlkInfo &b = g.blk[block_of_row[m]];
        int64_t r = m - b.row0;
        for (int64_t e = list_ptr[m]; e < list_ptr[m + 1]; ++e)
            if (list_col[e] >= b.size || list_col[e] == r) return "list_col out of range or on the diagonal";
        for (int64_t e = inter_ptr[m]; e < inter_ptr[m + 1]; ++e)
            if (inter_col[e] < 0 || inter_col[e] >= n || (inter_col[e] >= b.row0 && inter_col[e] < b.row0 + b.size))
                return "inter_col out of range or inside the row's own block";
    }
    g.perm.resize(n);
    if (perm) {
        std::vector<uint8_t> seen(n, 0);
        for (int64_t u = 0; u < n; ++u) {
            if (perm[u] < 0 || perm[u] >= n || seen[perm[u]]) return "perm is not a permutation";
            seen[perm[u]] = 1;
            g.perm[u] = perm[u];
        }
    } else {
        std::iota(g.perm.begin(), g.perm.end(), 0);
    }
    std::vector<uint8_t> modes(mode, mode + nb);
    for (int32_t b = 0; b < nb; ++b) g.blk[b].mode = modes[b] ? 1 : 0;
    // symmetry: the list of a block (zeros or ones, in block-order coordinates) and the inter
    // entries must each be symmetric
    SymHash sym;
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        uint64_t f = 0, b = 0;
        for (int64_t m = lo; m < hi; ++m) {
            const int64_t r0 = g.blk[block_of_row[m]].row0;
            for (int64_t e = list_ptr[m]; e < list_ptr[m + 1]; ++e) {
                const uint64_t v = (uint64_t)(r0 + list_col[e]);
                f += pair_hash((uint64_t)m, v);
                b += pair_hash(v, (uint64_t)m);
            }
            for (int64_t e = inter_ptr[m]; e < inter_ptr[m + 1]; ++e) {
                const uint64_t v = (uint64_t)inter_col[e];
                f += pair_hash((uint64_t)m, v);
                b += pair_hash(v, (uint64_t)m);
            }
        }
        sym.add(f, b);
    });
    // finish() marks the one entries of a row and complements them for a dense block; a dense
    // block's given list holds the zeros, so its ones are everything else except the diagonal.
    RowSource src;
    src.mark_ones = [&](int64_t m, uint64_t *bits, ErrFlag &err) -> int64_t {
        const BlkInfo &b = g.blk[block_of_row[m]];
        const int64_t r = m - b.row0, s = b.size;
        if (!b.mode) {
            int64_t k = 0;
            for (int64_t e = list_ptr[m]; e < list_ptr[m + 1]; ++e) {
                int64_t lc = list_col[e];
                uint64_t bit = uint64_t(1) << (lc & 63);
                if (bits[lc >> 6] & bit) { err.set("duplicate column in a row"); continue; }
                bits[lc >> 6] |= bit;
                ++k;
            }
            return k;
        }
        for (int64_t w = 0; w * 64 < s; ++w)
            bits[w] = (s - w * 64 >= 64) ? ~uint64_t(0) : ((uint64_t(1) << (s - w * 64)) - 1);
        bits[r >> 6] &= ~(uint64_t(1) << (r & 63));
        int64_t k = s - 1;
        for (int64_t e = list_ptr[m]; e < list_ptr[m + 1]; ++e) {
            int64_t lc = list_col[e];
            uint64_t bit = uint64_t(1) << (lc & 63);
            if (!(bits[lc >> 6] & bit)) { err.set("duplicate column in a row"); continue; }
            bits[lc >> 6] &= ~bit;
            --k;
        }
        return k;
    };
    src.clear = [&](int64_t m, uint64_t *bits) {
        const BlkInfo &b = g.blk[block_of_row[m]];
        if (!b.mode) {
            for (int64_t e = list_ptr[m]; e < list_ptr[m + 1]; ++e) bits[list_col[e] >> 6] = 0;
        } else {
            std::memset(bits, 0, sizeof(uint64_t) * (size_t)((b.size + 63) / 64));
        }
    };
    src.inter_count = [&](int64_t m) -> int64_t { return inter_ptr[m + 1] - inter_ptr[m]; };
    src.inter = [&](int64_t m, std::vector<int32_t> &out) {
        for (int64_t e = inter_ptr[m]; e < inter_ptr[m + 1]; ++e) out.push_back(inter_col[e]);
    };
    std::string msg = finish(g, block_of_row, src, &modes, opt);
    g.symmetric = sym.fwd.load() == sym.bwd.load();
    return msg;
}

void diag_segments(BlockGraph &g)
{
    const int32_t W = g.W;
    g.segd.clear();
    g.grp.clear();
    for (int32_t bi = 0; bi < g.nb; ++bi) {
        BlkInfo &b = g.blk[bi];
        b.sd0 = (int32_t)g.segd.size();
        const int32_t ncc = (b.size + W - 1) / W;
        for (int32_t cc = 0; cc < ncc; ++cc)
            for (int32_t t = 1; t <= b.nlayer; ++t)
                g.segd.push_back(SegD{b.row0 + cc * W, (int16_t)std::min(W, b.size - cc * W), (int8_t)(t <= b.mode), 0, 0});
        b.grp0 = (int32_t)g.grp.size();
        b.ngrp = b.mode > 0 ? 1 : 0;
        if (b.mode > 0) g.grp.push_back(Grp{bi, b.mode});
    }
}

std::string add_dense_pairs(BlockGraph &g, const BuildOptions &opt)
{
    g.n_pairs = 0;
    g.pair_rho.clear();
    if (!opt.pairs || g.nb < 2 || g.inter_col.empty()) return "";
    const int64_t n = g.n;
    const int32_t nb = g.nb, W = g.W;
    const int64_t pmin = std::max<int32_t>(1, opt.pair_min);
    std::vector<int32_t> bor(n);
    for (int32_t b = 0; b < nb; ++b)
        std::fill(bor.begin() + g.blk[b].row0, bor.begin() + g.blk[b].row0 + g.blk[b].size, b);

    // per row block, the distinct nonzero entries towards every other block (the inter list of
    // a row is sorted and holds a column once per unit of weight), and for a weighted graph the
    // value histogram of the blocks that can have a positive prevalent value
    struct Pair {
        int32_t c;
        int32_t mode;
        int32_t nlayer;
    };
    std::vector<std::vector<Pair>> dense(nb);
    std::vector<std::vector<double>> rho_of(nb);
    parallel_for(nb, [&](int64_t lo, int64_t hi) {
        std::unordered_map<int32_t, int64_t> cnt;
        std::unordered_map<int32_t, std::vector<int64_t>> hist;
        for (int64_t a = lo; a < hi; ++a) {
            const BlkInfo &ba = g.blk[a];
            if (ba.size < pmin) continue;
            cnt.clear();
            for (int64_t m = ba.row0; m < ba.row0 + ba.size; ++m)
                for (int64_t e = g.inter_ptr[m]; e < g.inter_ptr[m + 1]; ++e)
                    if (e == g.inter_ptr[m] || g.inter_col[e] != g.inter_col[e - 1]) ++cnt[bor[g.inter_col[e]]];
            std::vector<std::pair<int32_t, int64_t>> cand;
            for (const auto &kv : cnt)
                if (g.blk[kv.first].size >= pmin) cand.push_back(kv);
            std::sort(cand.begin(), cand.end());
            hist.clear();
            for (const auto &cv : cand) {
                const double cells = (double)ba.size * (double)g.blk[cv.first].size;
                const double rho = (double)cv.second / cells;
                if (!g.weighted) {
                    rho_of[a].push_back(rho);
                    if (rho >= opt.tau) dense[a].push_back(Pair{cv.first, 1, 1});
                } else if (2.0 * (double)cv.second >= cells) {
                    hist[cv.first].assign(kMaxWeight + 1, 0);
                }
            }
            if (hist.empty()) continue;
            for (int64_t m = ba.row0; m < ba.row0 + ba.size; ++m) {
                const int64_t e1 = g.inter_ptr[m + 1];
                for (int64_t e = g.inter_ptr[m]; e < e1;) {
                    int64_t f = e + 1;
                    while (f < e1 && g.inter_col[f] == g.inter_col[e]) ++f;
                    auto it = hist.find(bor[g.inter_col[e]]);
                    if (it != hist.end()) it->second[std::min<int64_t>(f - e, kMaxWeight)]++;
                    e = f;
                }
            }
            for (const auto &cv : cand) {
                auto it = hist.find(cv.first);
                if (it == hist.end()) continue;
                std::vector<int64_t> &h = it->second;
                h[0] = (int64_t)ba.size * g.blk[cv.first].size - cv.second;
                int32_t vb = 0, jmax = 0;
                for (int v = 1; v <= kMaxWeight; ++v) {
                    if (h[v]) jmax = v;
                    if (h[v] > h[vb]) vb = v;
                }
                if (vb > 0) dense[a].push_back(Pair{cv.first, vb, jmax});
            }
        }
    });
    for (int32_t a = 0; a < nb; ++a) {
        g.pair_rho.insert(g.pair_rho.end(), rho_of[a].begin(), rho_of[a].end());
        g.n_pairs += (int64_t)dense[a].size();
    }
    if (g.n_pairs == 0) return "";

    // new segment descriptors and groups: a row block keeps its own segments and appends, per
    // dense partner, the partner's column chunks, each in layers
    std::vector<SegD> segd;
    std::vector<Grp> grp;
    std::vector<int32_t> nseg_old(nb);
    std::vector<int64_t> segbase_old(nb);
    int64_t tot = 0;
    for (int32_t a = 0; a < nb; ++a) {
        BlkInfo &b = g.blk[a];
        nseg_old[a] = b.nchunk;
        segbase_old[a] = b.segbase;
        const int32_t sd0 = (int32_t)segd.size();
        segd.insert(segd.end(), g.segd.begin() + b.sd0, g.segd.begin() + b.sd0 + b.nchunk);
        const int32_t grp0 = (int32_t)grp.size();
        grp.insert(grp.end(), g.grp.begin() + b.grp0, g.grp.begin() + b.grp0 + b.ngrp);
        int64_t nseg = b.nchunk;
        for (const Pair &p : dense[a]) {
            const BlkInfo &bc = g.blk[p.c];
            const int32_t ncc = (bc.size + W - 1) / W;
            for (int32_t cc = 0; cc < ncc; ++cc)
                for (int32_t t = 1; t <= p.nlayer; ++t)
                    segd.push_back(SegD{bc.row0 + cc * W, (int16_t)std::min(W, bc.size - cc * W), (int8_t)(t <= p.mode), 0, 0});
            nseg += (int64_t)ncc * p.nlayer;
            grp.push_back(Grp{p.c, p.mode});
        }
        if (nseg > INT32_MAX) return "too many segments in a block";
        b.sd0 = sd0;
        b.grp0 = grp0;
        b.ngrp += (int32_t)dense[a].size();
        b.nchunk = (int32_t)nseg;
        b.segbase = tot;
        tot += nseg * b.size;
    }

    // per row: its old segments as they are, then the partner segments (layer t <= mode lists
    // the columns with a value below t, the others the columns with a value of at least t), and
    // the inter entries of the other blocks
    std::vector<int64_t> seg_ptr(tot + 1, 0);
    std::vector<uint16_t> list;
    std::vector<int64_t> inter_ptr(n + 1, 0);
    std::vector<int32_t> inter_col;
    std::vector<int64_t> unpadded(n, 0);
    int32_t smax = 0;
    for (const BlkInfo &b : g.blk) smax = std::max(smax, b.size);
    auto row_pass = [&](bool emit) {
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            std::vector<uint8_t> val((size_t)smax, 0);
            for (int64_t m = lo; m < hi; ++m) {
                const int32_t a = bor[m];
                const BlkInfo &b = g.blk[a];
                const int64_t r = m - b.row0;
                for (int32_t ch = 0; ch < nseg_old[a]; ++ch) {
                    const int64_t io = segbase_old[a] + (int64_t)ch * b.size + r;
                    const int64_t in = b.segbase + (int64_t)ch * b.size + r;
                    const int64_t len = g.seg_ptr[io + 1] - g.seg_ptr[io];
                    if (emit)
                        std::copy(g.list.begin() + g.seg_ptr[io], g.list.begin() + g.seg_ptr[io + 1],
                                  list.begin() + seg_ptr[in]);
                    else
                        seg_ptr[in + 1] = len;
                }
                const int64_t e0 = g.inter_ptr[m], e1 = g.inter_ptr[m + 1];
                int32_t ch = nseg_old[a];
                int64_t kept = 0, added = 0;
                int64_t prev = e0;  // entries before the next partner are kept
                for (const Pair &p : dense[a]) {
                    const BlkInfo &bc = g.blk[p.c];
                    const int32_t *ic = g.inter_col.data();
                    const int64_t f0 = std::lower_bound(ic + prev, ic + e1, bc.row0) - ic;
                    const int64_t f1 = std::lower_bound(ic + f0, ic + e1, bc.row0 + bc.size) - ic;
                    if (emit) std::copy(ic + prev, ic + f0, inter_col.begin() + inter_ptr[m] + kept);
                    kept += f0 - prev;
                    prev = f1;
                    for (int64_t e = f0; e < f1; ++e) val[ic[e] - bc.row0]++;
                    const int32_t ncc = (bc.size + W - 1) / W;
                    for (int32_t cc = 0; cc < ncc; ++cc) {
                        const int64_t c0 = (int64_t)cc * W, c1 = std::min<int64_t>(bc.size, c0 + W);
                        for (int32_t t = 1; t <= p.nlayer; ++t, ++ch) {
                            const int64_t idx = b.segbase + (int64_t)ch * b.size + r;
                            const bool zeros = t <= p.mode;
                            uint16_t *out = emit ? list.data() + seg_ptr[idx] : nullptr;
                            int64_t k = 0;
                            for (int64_t lc = c0; lc < c1; ++lc) {
                                if (zeros ? val[lc] >= t : val[lc] < t) continue;
                                if (emit) out[k] = (uint16_t)((lc - c0) * g.esz2);
                                ++k;
                            }
                            if (emit) {
                                for (const int64_t padded = seg_ptr[idx + 1] - seg_ptr[idx]; k < padded; ++k)
                                    out[k] = (uint16_t)(W * g.esz2);
                            } else {
                                seg_ptr[idx + 1] = round8(k);
                                added += k;
                            }
                        }
                    }
                    for (int64_t e = f0; e < f1; ++e) val[ic[e] - bc.row0] = 0;
                }
                if (emit) std::copy(g.inter_col.begin() + prev, g.inter_col.begin() + e1,
                                    inter_col.begin() + inter_ptr[m] + kept);
                kept += e1 - prev;
                if (!emit) {
                    inter_ptr[m + 1] = kept;
                    unpadded[m] = added;
                }
            }
        });
    };
    row_pass(false);
    for (int64_t i = 0; i < tot; ++i) seg_ptr[i + 1] += seg_ptr[i];
    for (int64_t m = 0; m < n; ++m) inter_ptr[m + 1] += inter_ptr[m];
    list.assign((size_t)seg_ptr[tot], (uint16_t)0);
    inter_col.assign((size_t)inter_ptr[n], 0);
    row_pass(true);
    for (int64_t m = 0; m < n; ++m) g.list_unpadded += unpadded[m];
    g.seg_ptr.swap(seg_ptr);
    g.list.swap(list);
    g.inter_ptr.swap(inter_ptr);
    g.inter_col.swap(inter_col);
    g.segd.swap(segd);
    g.grp.swap(grp);
    return "";
}

}  // namespace kur
