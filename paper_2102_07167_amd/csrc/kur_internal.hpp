// kur_internal.hpp -- internal data layout shared by the host preprocessing and the HIP code.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace kur {

// One diagonal block (a community after regrouping) as the kernels see it: the row block of its
// rows. A weighted block is handled as a sum of 0/1 layers A = sum_{t >= 1} [A >= t]: layers
// t <= mode are mostly ones and store their zeros (subtracted from the localised order
// parameters), layers t > mode store their ones. A 0/1 block has one layer and mode 0 or 1.
// The row block's segments run over column groups: first its own columns, then every dense
// off-diagonal block of its rows (a partner column block whose pairs are mostly nonzero), each
// in column chunks of width W and, inside a chunk, in layers.
struct BlkInfo {
    int32_t row0;     // first block-order row
    int32_t size;     // rows (= columns) of the block
    int32_t nchunk;   // segments per row (over all column groups), described by segd[sd0 ..]
    int32_t mode;     // layers of the diagonal block stored as lists of zeros (its prevalent
                      // value); 0 for a sparse diagonal block
    int64_t segbase;  // index into seg_ptr of (segment 0, local row 0); segment c, row r at
                      // segbase + c * size + r
    int32_t tile0;    // first tile of this block (tiles of a block are contiguous)
    int32_t ntiles;
    int32_t nlayer;   // 0/1 layers of the diagonal block (1 for a 0/1 block)
    int32_t ngrp;     // column groups whose localised order parameters enter the rows: grp[grp0 ..]
    int32_t grp0;
    int32_t sd0;      // first segment descriptor of this block
};

// One segment of a row block: the columns [col0, col0 + cw) (block order), whether its entries
// are zeros (subtracted from the localised order parameters) or ones (added), and how they are
// stored. mask == 0: a 16-bit list per row (seg_ptr, list), read against the chunk staged in LDS.
// mask == 1: a bitmask of kMaskUnitCols-column units, unit q of local row r at
// mask[mbase + q * size + r] (size = rows of the row block); bit j of 32-bit word w of unit q is
// column kMaskUnitCols * q + 32 w + j of the segment. Such a segment's list is empty.
struct SegD {
    int32_t col0;
    int16_t cw;
    int8_t zeros;
    int8_t mask;
    int64_t mbase;
};

// Columns of one bitmask unit (four 32-bit words, one 16-byte load).
constexpr int32_t kMaskUnitCols = 128;
// Least chunk width for bitmask segments.
constexpr int32_t kMaskMinW = 4 * kMaskUnitCols;
// Most columns of one sub-chunk of a bitmask segment (one set of subset-sum tables in LDS, built
// by one thread per four columns of the 256 threads of the bitmask kernel).
constexpr int32_t kMaskSubMax = 1024;

// The bitmask work of a layout is cut into items: consecutive sub-chunks (of mask_sub columns,
// the last one of a segment shorter) of the bitmask segments of one tile, in segment order,
// starting at sub-chunk sub of segment seg (an index into the block's segd). One workgroup of
// the bitmask kernel sums an item over the tile's rows into the partial sums at rows
// [out, out + tile rows) of the item buffer; the tile kernel adds its tile's partial sums.
struct MaskItem {
    int32_t tile;
    int32_t seg;
    int32_t sub;
    int32_t nsub;
    int64_t out;
};

// Per tile: its items' partial sums, cnt runs of (tile rows) pairs from row off of the item
// buffer, in segment order.
struct MaskTile {
    int64_t off;
    int32_t cnt;
    int32_t pad;
};

// A column block whose localised order parameters enter every row of a row block with factor
// mode (the prevalent value of that submatrix): the diagonal block when dense, and every dense
// off-diagonal block.
struct Grp {
    int32_t blk;
    int32_t mode;
};

// One unit of work: rows [r0, r1) (block-local) of one block, G lanes per row (G == 0: each
// wave streams a contiguous run of the tile's rows; G == -1: the rows store no list entries).
struct Tile {
    int32_t block;
    int32_t r0;
    int32_t r1;
    int32_t G;
};

struct BuildOptions {
    double tau = 0.5;        // dense if realised density >= tau
    int32_t W = 8192;        // chunk width (columns staged in LDS at a time)
    int32_t tile_rows = 1024;
    int64_t tiles_target = 4096;
    int64_t tile_min_cost = 16384;  // least work per tile, in list-entry equivalents
    double flat_min_vec = 8.0;  // rows averaging at least this many 8-entry vectors: wave streaming
    int32_t esz2 = 8;           // bytes of one staged (sin, cos) pair; list entries are LDS byte
                                // offsets col * esz2, so W * esz2 must stay below 65536
    int32_t xcds = 1;           // launch order for this many round-robin XCDs (1: plain largest first)
    bool pairs = true;          // dense off-diagonal blocks use localised order parameters
    int32_t pair_min = 32;      // least rows and columns of such a block
    double mask_min = 2.0;      // a segment holding at least this many list entries per cell is
                                // stored as a bitmask (needs W >= kMaskMinW); above 1: never
    int32_t mask_sub = 1024;    // columns of a bitmask sub-chunk (a multiple of kMaskUnitCols,
                                // at most kMaskSubMax)
    int64_t mask_item = 1 << 15;  // cells (rows x columns) of a bitmask work item, at most (an
                                  // item holds at least one sub-chunk)
};

// The graph in block order, ready for upload.
struct BlockGraph {
    int64_t n = 0;
    int32_t nb = 0;
    int32_t W = 0;
    int32_t tile_rows = 0;
    int32_t esz2 = 8;
    std::vector<int32_t> perm;        // user node -> block-order row
    std::vector<BlkInfo> blk;
    std::vector<SegD> segd;           // segment descriptors (every block's from blk[].sd0)
    std::vector<Grp> grp;             // column groups with localised order parameters
    std::vector<int64_t> seg_ptr;     // total segments + 1 (segment-major inside every block)
    std::vector<uint16_t> list;       // chunk-relative LDS byte offset (col * esz2), segments
                                      // padded to 8 entries with W * esz2 (the zero slot)
    std::vector<uint32_t> mask;       // bitmask segments, 4 words per unit (see SegD)
    int64_t mask_segments = 0;        // segment descriptors stored as bitmasks
    std::vector<int64_t> inter_ptr;   // n + 1, block order
    std::vector<int32_t> inter_col;   // block-order columns
    std::vector<Tile> tiles;
    std::vector<int32_t> order;       // launch order of tiles; -1 marks an empty slot (see order_tiles)
    int32_t mask_sub = 1024;          // columns of a bitmask sub-chunk (see MaskItem)
    int64_t mask_item = 1 << 15;      // most cells of a bitmask item beyond its first sub-chunk
    std::vector<MaskItem> mitems;     // bitmask items in launch order (largest first)
    std::vector<MaskTile> mtiles;     // per tile its items' partial sums (empty without bitmasks)
    int64_t mask_part_rows = 0;       // rows of the item buffer
    int32_t xcds = 1;
    std::vector<int32_t> deg;         // row degree (ones of the row), block order
    int64_t list_unpadded = 0;
    int64_t n_dense = 0;
    int64_t n_pairs = 0;              // dense off-diagonal blocks
    bool symmetric = false;           // A equals its transpose (checked by a 64-bit hash)
    // the density tests of the build (for the tuner: two thresholds with equal outcomes build
    // equal layouts): per block its realised density; per nonzero off-diagonal block with at
    // least pair_min rows and columns its density (0/1 graphs)
    std::vector<double> blk_rho;
    std::vector<double> pair_rho;
    bool weighted = false;            // built from integer weights (prevalent-value rule)
};

// Host preprocessing entry points; return "" on success or an error message.
std::string build_from_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels,
                           const BuildOptions &opt, BlockGraph &out);
std::string build_from_blocks(int64_t n, int32_t nb, const int64_t *block_ptr, const uint8_t *mode,
                              const int64_t *list_ptr, const uint16_t *list_col, const int64_t *inter_ptr,
                              const int32_t *inter_col, const int32_t *perm, const BuildOptions &opt,
                              BlockGraph &out);

// Pieces of build_from_csr shared with the ensemble builder: argument validation ("" if valid),
// the symmetry test of the pattern (diagonal ignored), and the regroup of the nodes by label
// value (stable counting sort; perm: user -> block order, node_at: block order -> user,
// block_ptr: nb + 1 block boundaries). Returns the number of blocks.
std::string validate_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels);
bool csr_symmetric(int64_t n, const int64_t *row_ptr, const int32_t *col);
int32_t regroup_by_labels(int64_t n, const int32_t *labels, std::vector<int32_t> &perm, std::vector<int32_t> &node_at,
                          std::vector<int32_t> &block_of_row, std::vector<int64_t> &block_ptr);

// Weighted adjacency: col as in build_from_csr, weight[e] in [0, kMaxWeight] the integer value
// A_ml of entry e (0: absent). Every block is split into 0/1 layers A = sum_t [A >= t]; its
// prevalent value (the most frequent value of its off-diagonal pairs, zeros included) is the
// number of layers stored as zeros; edges between blocks are listed once per unit of weight.
// deg holds the weighted row sums.
constexpr int32_t kMaxWeight = 255;
std::string build_from_csr_w(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                             const int32_t *labels, const BuildOptions &opt, BlockGraph &out);

// Segment descriptors and column groups of the diagonal blocks alone (every builder ends with
// this before add_dense_pairs): per block, for every column chunk its layers.
void diag_segments(BlockGraph &g);

// Moves every dense off-diagonal block (row block a, column block c) out of the inter-block
// CSR into a column group of a: dense when a and c have at least pair_min nodes each and, for
// a 0/1 graph, the realised density is at least tau, for a weighted graph the prevalent value
// of its pairs (zeros included) is positive. Its layers are stored like those of a diagonal
// block. Rebuilds seg_ptr, list, segd, grp, the inter CSR and the tiles; a no-op when
// opt.pairs is false or no block is dense.
std::string add_dense_pairs(BlockGraph &g, const BuildOptions &opt);

// Stores every segment whose list (entries padded to 8 per row) fills at least opt.mask_min of
// its cells as a bitmask (see SegD) and removes it from the lists; a no-op when mask_min is
// above 1 or W < kMaskMinW. Runs after the segments are final, before the tiles are cut. The
// kernels sum a bitmask segment's row through subset-sum tables of four columns (the method of
// four Russians for Boolean matrix-vector products): one table read per four cells.
std::string to_masks(BlockGraph &g, const BuildOptions &opt);

// The complete graph on n nodes: one dense block whose list of zeros is empty.
std::string build_complete(int64_t n, const BuildOptions &opt, BlockGraph &out);

// Block-diagonal union of independent graphs (no edges between parts), part i occupying the
// user nodes and block-order rows that follow those of parts 0..i-1. row_first[i] and
// tile_first[i] (size parts+1) receive the row and tile ranges of every part.
std::string merge_graphs(std::vector<BlockGraph> &parts, BlockGraph &out, std::vector<int64_t> &row_first,
                         std::vector<int64_t> &tile_first);

// Work tiles from the segment and inter-block offsets alone (the lists are not read): rows of one
// block grouped until a tile carries max(tile_min_cost, total / tiles_target) of estimated work
// or tile_rows rows; sets blk[].tile0/ntiles, tiles, tile_rows and the launch order.
void make_tiles(BlockGraph &g, const BuildOptions &opt);

// Launch order of tiles. Workgroup i of a launch runs on XCD i mod g.xcds (round-robin
// dispatch) and every XCD has its own L2, so the blocks are first spread over the XCDs by
// estimated cost (largest to the least loaded XCD), and all tiles of a block run on its XCD:
// the block's staged (sin, cos) chunks are then read from HBM once and hit that L2 for the
// other tiles. A block costing more than total / (2 xcds) is placed as runs of consecutive
// tiles of about that cost, so that few or uneven blocks still use every XCD. Within an XCD the
// tiles run largest first; slot j * xcds + x holds the j-th tile of XCD x, and -1 where XCD x
// has fewer tiles. xcds = 1 gives the plain largest-first order.
void order_tiles(BlockGraph &g);

// The bitmask items of the tiles (see MaskItem), rebuilt with every tiling: per tile its bitmask
// sub-chunks in segment order, cut into items of at most g.mask_item cells (rows x columns, at
// least one sub-chunk each); partial-sum rows assigned tile by tile; the launch order is the
// largest item first, so that the last workgroups to start are the shortest. Called by
// order_tiles.
void mask_items(BlockGraph &g);

// Runs f(i) for i in [0, n) on the host threads (static contiguous ranges).
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &f);

}  // namespace kur
