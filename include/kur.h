/*
 * kur.h -- C ABI of the MI355X (gfx950) library for the Kuramoto model on graphs.
 *
 * Problem (Boehle, Kuehn, Thalhammer, arXiv 2102.07167, Sec. 3, eq. KuramotoGraph):
 *     theta_m'(t) = omega_m + K / Mscale_m * sum_l A_ml sin(theta_l(t) - theta_m(t)),  A_ml in {0,1}
 * with uniform scaling Mscale_m = N (default) or non-uniform scaling Mscale_m = sum_l A_ml
 * (option "scaling" = 1; a zero row then gives theta_m' = omega_m). Row m receives from column l.
 *
 * Method (Sec. 3, eq. KuramotoGraphApproach and the remark after it): after the nodes are
 * regrouped so that every community is contiguous (Sec. 3, community detection: the
 * permutation P A P^T), every diagonal block is evaluated either
 *   - "dense": with the localised order parameters S_b = sum_{l in b} sin theta_l and
 *     C_b = sum_{l in b} cos theta_l, minus the few entries with A_ml = 0 (list of zeros), or
 *   - "sparse": by straightforward summation over the entries with A_ml = 1 (list of ones),
 * and all edges between communities by straightforward summation over a CSR list. The sine of a
 * difference is expanded by the addition theorem (Sec. 2, eq. KuramotoReformulation), so every
 * list entry costs one gather of (sin theta_l, cos theta_l).
 * Time integration: classical fourth-order Runge-Kutta with a fixed step. Order parameter:
 * r e^{i psi} = (1/N) sum_m e^{i theta_m} (Sec. 2, eq. OrderParameter).
 *
 * Conventions
 *   - Every call returns kur_status; nothing throws or aborts across the ABI. On failure,
 *     kur_last_error(ctx) describes the problem (valid until the next call on ctx).
 *   - Host arrays passed in are borrowed for the duration of the call and copied; the library
 *     owns every device buffer it allocates. Host arrays are double precision for both
 *     dtypes; a KUR_F32 context rounds them to float on upload.
 *   - Arrays in "user order" are indexed by the caller's node numbering; the library keeps its
 *     own block order internally and applies the permutation on the way in and out.
 *   - Argument validation (shapes, ranges, finiteness, graph consistency) happens on the host
 *     before any device work, and a rejected call leaves the context unchanged.
 *   - A context drives one device and one stream; it is not thread safe.
 *   - *_dev variants take device pointers, enqueue on the context stream and do not
 *     synchronise; the pointers must stay valid until that stream work completes.
 */
#ifndef KUR_H
#define KUR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kur_ctx kur_ctx;

typedef enum {
    KUR_OK = 0,
    KUR_EINVAL = 1,     /* invalid argument; nothing was changed */
    KUR_ENOMEM = 2,     /* host or device allocation failed */
    KUR_EDEVICE = 3,    /* HIP runtime error, or no device (host-only context) */
    KUR_ESTATE = 4,     /* call out of order (e.g. stepping before a graph was set) */
    KUR_ENONFINITE = 5  /* a non-finite phase was detected */
} kur_status;

typedef enum { KUR_F32 = 1, KUR_F64 = 2 } kur_dtype;

/* Library version as 10000*major + 100*minor + patch. */
int kur_version(void);

/*
 * Create a context computing in dtype on HIP device `device`. hip_stream is a hipStream_t to
 * enqueue on (NULL: the context creates its own stream at default priority).
 * device = -1 creates a host-only context: graph preprocessing and validation work, every
 * call that needs the GPU returns KUR_EDEVICE.
 */
kur_status kur_create(kur_ctx **out, kur_dtype dtype, int device, void *hip_stream);

/* Release every resource of ctx (NULL is accepted). Waits for the context stream. */
void kur_destroy(kur_ctx *ctx);

/* Human-readable description of the last failure on ctx ("" if none; ctx may be NULL). */
const char *kur_last_error(const kur_ctx *ctx);

/*
 * Set a tuning or model option; takes effect at the next kur_set_graph* call unless noted.
 *   "tau"         density threshold: a diagonal block whose realised density is >= tau is
 *                 evaluated with localised order parameters (list of zeros), otherwise with its
 *                 list of ones. Default 0.5 (Sec. 3: precompute when ones outnumber zeros).
 *                 With "pairs" on, the same test applies to every off-diagonal block (the
 *                 submatrix of two communities) of a 0/1 graph.
 *   "pairs"       1 (default): a dense off-diagonal block (both communities at least "pair_min"
 *                 nodes; density >= tau for a 0/1 graph, positive prevalent value for an integer-
 *                 weighted one) is evaluated with the localised order parameters of its column
 *                 community minus its list of zeros (Sec. 3, extension to submatrices
 *                 [M1..M2] x [M3..M4], eq. KuramotoGraphApproach) instead of through the
 *                 inter-block list; 0: every edge between communities is listed. Graphs given
 *                 block by block (kur_set_graph) keep the given layout.
 *   "pair_min"    least nodes of both communities of such a block (1..65536). Default 32.
 *   "mask_min"    a segment (one column chunk of a block, one layer) whose stored list holds at
 *                 least this many entries per cell (0..1e9; above 1: never) is stored instead as
 *                 a bitmask, 1 bit per cell, in units of 128 columns per row. The kernels sum a
 *                 bitmask row through tables of the 16 subset sums of every 4 columns, built in
 *                 LDS per chunk (the method of four Russians for Boolean matrix-vector
 *                 products): one table read per 4 cells instead of one staged-value read per
 *                 list entry. Needs a chunk of at least 512 columns. The same sums in another
 *                 order. Takes effect at the next graph set. Default 2 (off).
 *   "mask_sub"    columns of one set of those tables (a multiple of 128 in [128, 1024], at most
 *                 the chunk; in FP64 at most 512). Default 1024.
 *   "mask_item"   the bitmask work is cut into items of consecutive tables' worth of one tile's
 *                 bitmask rows, each of at most this many cells (rows x columns; at least one
 *                 set of tables), summed by one workgroup each, largest first, into partial
 *                 sums that the tile adds in segment order (1..1e12). Default 32768. Both take
 *                 effect at the next graph set or re-tiling.
 *   "transpose"   1: kur_set_graph_csr / kur_set_graph_csr_w on a device context also build and
 *                 keep the layout of A^T when A is asymmetric (same block order; about the
 *                 memory of A's layout again), which the adjoint of an asymmetric A needs.
 *                 0 (default): not kept.
 *   "chunk"       columns of a diagonal block staged in LDS at a time: a multiple of 64, at
 *                 most 8128 (FP32) or 4032 (FP64). Default 4096 (FP32), 4032 (FP64).
 *   "tile_rows"   maximal rows per work tile (64..4096). Default 256.
 *   "threads"     threads per workgroup of the tile kernels: 128, 256, 512 or 1024. Default 512.
 *                 Smaller workgroups let a compute unit hold more tiles at once, which pays
 *                 where tiles carry little work each. The staged chunk, tile_rows and the
 *                 threads must fit the LDS of one workgroup (else KUR_EINVAL).
 *   "tiles"       target number of work tiles (>= 1). Default 4096.
 *   "tile_min_cost" least work per tile in list-entry equivalents (a row costs its stored list
 *                 entries + 4 per inter-block entry + 32). Default 16384.
 *   "xcds"        launch order of the tiles for this many XCDs dispatched round-robin: the tiles
 *                 of a block all run on one XCD, whose L2 then serves the block's re-staged
 *                 (sin, cos) chunks; 1: plain largest-first order (default; the tuner tries
 *                 8, the XCD count of MI355X).
 *   "inter_gather" 1: the row kernel's inter-block gathers read the 4-byte stage phase and form
 *                 (sin, cos) (half the cache footprint of the pairs; the same values bit for bit);
 *                 0: they read the (sin, cos) pair. Default 1 in FP32, 0 in FP64; the tuner tries
 *                 both. Immediate.
 *   "flat_min_vec" rows of a tile averaging at least this many 8-entry list vectors per chunk
 *                 are streamed one contiguous run per wavefront; shorter rows get a group of
 *                 lanes each. 0 disables streaming. Default 8.
 *   "scaling"     0: K/N (uniform, default); 1: K/deg_m (non-uniform). Immediate.
 *   "compensate"  1: compensated phase update with winding (default); 0: plain update. Immediate.
 *   "timing"      1: time every launch of the row kernel with HIP events (see kur_kernel_time).
 *                 Immediate; disables graph replay and the one-workgroup run ("persistent")
 *                 while on.
 *   "checkpoint_every" C > 0: kur_step_rk4 keeps the phases every C steps for
 *                 kur_adjoint_rk4_recorded (and launches without graph replay); 0 (default) off.
 *                 Immediate.
 *   "adjoint_keep" 1 (default): the adjoint calls keep their work buffers (about
 *                 (16 ckpt_every + 16) n reals) in the context for the next call; 0: release
 *                 them now and after every adjoint call. Immediate.
 *   "record_stages" 1: such a recording run also keeps (sin, cos) and the row sums
 *                 (A sin, A cos) of every stage state, 16 n reals per step (KUR_ENOMEM if the
 *                 device cannot hold them), so that kur_adjoint_rk4_recorded recomputes nothing;
 *                 0 (default): checkpoints only. Immediate.
 *   "graph"       1 (default): kur_step_rk4 captures one sampling period (r_every steps, else
 *                 "graph_steps" steps) into a HIP graph and replays it; 0: plain launches.
 *   "graph_steps" steps per replayed graph when no order parameter is sampled (default 16).
 *   "persistent"  1 (default): kur_step_rk4 on a complete graph (kur_set_graph_complete) of at
 *                 most 1024 nodes, without checkpoints or "timing", runs the call in one
 *                 workgroup that keeps the state in registers (Sec. 2: the classical model
 *                 through its order parameter): launches of whole sampling periods of at most
 *                 about 65536 steps, instead of four launches per step; 0: the row kernel as
 *                 for any graph. Equal results up to the order of the sums.
 *   "ens_tau"     shared-graph ensembles: blocks (and off-diagonal blocks, see below) at least
 *                 this dense form their products on the matrix cores (0..2, above 1: none).
 *                 Default 0.5. Takes effect at the next kur_ens_set_graph_csr.
 * Unknown keys and out-of-range values return KUR_EINVAL.
 */
kur_status kur_set_option(kur_ctx *ctx, const char *key, double value);

/*
 * Set the graph from a CSR adjacency in user order plus a community label per node (the 0/1
 * adjacency A of Sec. 3, eq. KuramotoGraph; the labels are the planted communities of Sec. 3,
 * community detection in graphs); the library does the host preprocessing: a stable counting
 * sort of the nodes by label (the permutation P A P^T to block structure), the per-block
 * dense/sparse choice at "tau" (Sec. 3, eq. KuramotoGraphApproach: list of zeros or list of
 * ones), the list build and the work decomposition. Synchronous; KUR_EINVAL on any
 * inconsistency (nothing installed), KUR_ENOMEM if host or device memory runs out.
 *   n           number of oscillators (1 <= n < 2^31)
 *   row_ptr     n+1 offsets, row_ptr[0] = 0, non-decreasing
 *   col         row_ptr[n] column indices in [0, n); row m lists the l with A_ml = 1, in any
 *               order, without duplicates. Diagonal entries are ignored (sin 0 = 0).
 *   labels      n community labels >= 0 (any values; communities are ordered by label)
 * The adjacency may be asymmetric.
 */
kur_status kur_set_graph_csr(kur_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const int32_t *labels);

/*
 * Integer-weighted graph (Introduction, generalisations: coefficients in a finite set {0..J},
 * one value prevalent per block): as kur_set_graph_csr, with weight[e] in [0, 255] the value
 * A_ml of entry e (0: absent). Every community block is split into 0/1 layers
 * A = sum_{t >= 1} [A >= t]; its prevalent value v (the most frequent value among its
 * off-diagonal pairs, zeros included) is the number of layers evaluated with the localised
 * order parameters (lists of zeros, eq. KuramotoGraphApproach); the layers above v store their
 * ones. An entry with value a != v thus costs |a - v| list entries. Edges between blocks are
 * summed straightforwardly, listed once per unit of weight. Non-uniform scaling uses the
 * weighted row sums. As for kur_set_graph_csr, the adjoint of an asymmetric A needs the option
 * "transpose".
 */
kur_status kur_set_graph_csr_w(kur_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                               const int32_t *weight, const int32_t *labels);

/*
 * Set the graph already in block form (the expert path; no community search is done): the
 * regrouped adjacency of Sec. 3, eq. KuramotoGraphApproach, given block by block as the lists
 * that equation evaluates (zeros of a dense diagonal block, ones of a sparse one, and the
 * straightforwardly summed entries between blocks). Arrays are borrowed for the call and
 * copied; KUR_EINVAL on any inconsistency listed below.
 *   n, nb        nodes and diagonal blocks; block b owns block-order rows
 *                [block_ptr[b], block_ptr[b+1]), block sizes 1..65535
 *   block_ptr    nb+1 offsets, block_ptr[0] = 0, strictly increasing, block_ptr[nb] = n
 *   mode         nb flags: 1 = the block list holds the ZERO entries (l != m) of the block,
 *                0 = it holds the ONE entries
 *   list_ptr     n+1 offsets into list_col (block order)
 *   list_col     block-local column indices (0 <= c < block size, c != row's own local index),
 *                no duplicates
 *   inter_ptr    n+1 offsets into inter_col (block order)
 *   inter_col    block-order column indices outside the row's own block, no duplicates
 *   perm         n entries: perm[u] = block-order index of user node u (NULL = identity);
 *                must be a permutation
 */
kur_status kur_set_graph(kur_ctx *ctx, int64_t n, int32_t nb, const int64_t *block_ptr,
                         const uint8_t *mode, const int64_t *list_ptr, const uint16_t *list_col,
                         const int64_t *inter_ptr, const int32_t *inter_col, const int32_t *perm);

/* The complete graph on n nodes (the classical all-to-all model of Sec. 2, eq. Kuramoto): one
 * dense block with an empty list of zeros, so F = omega + K (S cos theta - C sin theta) with the
 * global order parameters (Sec. 2, eq. KuramotoReformulation). */
kur_status kur_set_graph_complete(kur_ctx *ctx, int64_t n);

/*
 * Batches of independent instances integrated together (ensembles, K sweeps): the instances
 * form one block-diagonal graph, every row carries its instance's factor K_i / N_i, and the
 * order parameter is sampled per instance.
 *   kur_batch_begin   starts a new batch (drops instances added earlier)
 *   kur_batch_add     appends one instance: n oscillators, complete != 0 for all-to-all
 *                     (row_ptr, col, labels ignored) or a CSR in the instance's own numbering with
 *                     labels as for kur_set_graph_csr; its K, omega (n) and theta0 (n). The
 *                     instance's preprocessing runs here, so the caller may free its arrays.
 *   kur_batch_commit  installs the union as the context's graph, with the instances' omega and
 *                     theta0 in user order (instance 0 first) and K = 1 as a global factor.
 *   kur_batch_info    number of instances and their first user node (n_inst + 1 entries).
 *   kur_batch_step    like kur_step_rk4; r_out/psi_out receive (nsteps/r_every + 1) x n_inst
 *                     values, sample-major.
 * The adjoint is not available for a batch.
 */
kur_status kur_batch_begin(kur_ctx *ctx);
kur_status kur_batch_add(kur_ctx *ctx, int64_t n, int complete, const int64_t *row_ptr, const int32_t *col,
                         const int32_t *labels, double K, const double *omega, const double *theta0);
kur_status kur_batch_commit(kur_ctx *ctx);
kur_status kur_batch_info(const kur_ctx *ctx, int32_t *n_inst, int64_t *row_first);
kur_status kur_batch_step(kur_ctx *ctx, double dt, int64_t nsteps, int64_t r_every, double *r_out, double *psi_out);

/* Graph statistics after kur_set_graph*: out[0..9] = n, nb, dense blocks, list entries
 * (unpadded), list entries (padded, as stored), inter entries, tiles, chunk width, 1 if the
 * adjacency is symmetric, largest block size. */
kur_status kur_graph_info(const kur_ctx *ctx, int64_t out[10]);

/* Bitmask segments of the installed layout (option "mask_min"): out[0] = segments stored as
 * bitmasks, out[1] = their bytes. KUR_ESTATE without a graph. */
kur_status kur_graph_masks(const kur_ctx *ctx, int64_t out[2]);

/* Bitmask work items of a host-only context's layout (options "mask_sub" and "mask_item"):
 * *count receives their number. If items is not NULL it receives 9 values per item, in launch
 * order: tile, block, first segment (block-local index), first sub-chunk of that segment,
 * sub-chunks, tile rows, 128-column units per row, cells (rows x columns) and the first row of
 * its partial sums in the item buffer. Caller-owned, 9 * count entries. KUR_ESTATE without a
 * graph or on a device context. For the tests of the item cut. */
kur_status kur_graph_mask_items(const kur_ctx *ctx, int64_t *count, int64_t *items);

/* Permutation in use: perm[u] = block-order index of user node u (n entries). */
kur_status kur_get_perm(const kur_ctx *ctx, int32_t *perm);

/*
 * Introspection of the host preprocessing, for host-only contexts (device = -1), which keep
 * the built layout in host memory. kur_get_blocks: block_ptr (nb+1) and mode (nb; the number of
 * 0/1 layers stored as lists of zeros: 1 = list of zeros for a 0/1 block). kur_get_row_lists:
 * for block-order row `row`, the block-local columns stored in the list of its own block
 * (ascending; zeros for a dense block, ones for a sparse one) and its inter-block columns
 * (block order, ascending; without the dense off-diagonal blocks, see kur_get_row_layers).
 * Pass NULL arrays to query the counts; otherwise the arrays must hold *nlist and *ninter
 * entries (the counts are written back). Device contexts return KUR_ESTATE.
 */
kur_status kur_get_blocks(const kur_ctx *ctx, int64_t *block_ptr, uint8_t *mode);
kur_status kur_get_row_lists(const kur_ctx *ctx, int64_t row, int32_t *list, int64_t *nlist, int32_t *inter,
                             int64_t *ninter);
/* Host-only contexts: every stored list entry of block-order row `row` (its own block and its
 * dense off-diagonal blocks) with its 0/1 layer: cols receives block-order columns, layer the
 * 1-based layer inside the column community's group; a layer up to the group's mode (see
 * kur_get_block_groups; 0 for a community without a group) holds zeros, the others ones. cols
 * and layer hold *count entries on entry (both NULL: count only); *count receives the count.
 * Row m of A is then: mode_q on every column of every group q (but not m itself), minus one per
 * zero entry, plus one per one entry, plus one per inter-block entry. */
kur_status kur_get_row_layers(const kur_ctx *ctx, int64_t row, int32_t *cols, int32_t *layer, int64_t *count);
/* Column groups of block `block` (any context with a graph): the communities whose localised
 * order parameters enter every row of the block, with their factor (the prevalent value of that
 * submatrix): the block itself when dense, then its dense off-diagonal blocks in block order.
 * blk and mode hold *count entries on entry (both NULL: count only); *count receives the count. */
kur_status kur_get_block_groups(const kur_ctx *ctx, int32_t block, int32_t *blk, int32_t *mode, int32_t *count);
/* Number of dense off-diagonal blocks of the installed graph (ordered pairs of communities). */
kur_status kur_graph_pairs(const kur_ctx *ctx, int64_t *n_pairs);

/* Intrinsic frequencies omega_m and coupling constant K of Sec. 3, eq. KuramotoGraph (Sec. 2,
 * eq. Kuramoto for the complete graph): omega has n entries in user order, finite; K finite.
 * Copied to the device (rounded to float in a KUR_F32 context). KUR_ESTATE before a graph is
 * set; KUR_EINVAL (nothing changed) on a NULL or non-finite argument. */
kur_status kur_set_params(kur_ctx *ctx, const double *omega, double K);

/* Phases theta_m (n, user order, finite, |theta| <= 1e9, any real value) of the state of
 * Sec. 3, eq. KuramotoGraph, phases on the circle S^1 (Sec. 2): stored as a wrapped value in
 * [-pi, pi] plus a compensation term and an int32 winding count, so that kur_get_phases can
 * return the unwrapped trajectory. KUR_ESTATE before a graph; KUR_EINVAL (nothing changed) on a
 * NULL or out-of-range argument. */
kur_status kur_set_phases(kur_ctx *ctx, const double *theta);

/*
 * Evaluate the right-hand side F_m(theta) = omega_m + K/Mscale_m sum_l A_ml sin(theta_l -
 * theta_m) of Sec. 3, eq. KuramotoGraph, by the block method of eq. KuramotoGraphApproach
 * (localised order parameters minus zeros for dense blocks, straightforward sums elsewhere), at
 * theta (n, user order, finite; NULL = the current phases), into dtheta (n, user order).
 * Synchronous. KUR_ESTATE without graph, omega/K or (theta NULL) phases; KUR_EINVAL on NULL
 * dtheta or non-finite theta.
 */
kur_status kur_eval_rhs(kur_ctx *ctx, const double *theta, double *dtheta);

/*
 * Advance the current phases by nsteps classical RK4 steps of size dt (finite, nonzero) of
 * the system of Sec. 3, eq. KuramotoGraph (the explicit fourth-order Runge-Kutta method of Sec. 2,
 * numerical integration, here with a fixed step): y_{n+1} = y_n + dt/6 (k1 + 2 k2 + 2 k3 + k4).
 * If r_every > 0 the order parameter is sampled at steps 0, r_every, 2 r_every, ...,
 * floor(nsteps/r_every) r_every, i.e. nsteps/r_every + 1 values, written to r_out and psi_out
 * (either may be NULL). With r_out == psi_out == NULL the call only enqueues work.
 * Returns KUR_ENONFINITE if a sampled order parameter is not finite.
 */
kur_status kur_step_rk4(kur_ctx *ctx, double dt, int64_t nsteps, int64_t r_every, double *r_out,
                        double *psi_out);

/* Current phases theta_m (n, user order; Sec. 3, eq. KuramotoGraph): wrapped != 0 gives values
 * in [-pi, pi), wrapped == 0 the unwrapped phases (wrapped value plus 2 pi times the winding
 * count). Synchronous. KUR_ESTATE without phases; KUR_EINVAL on NULL theta. */
kur_status kur_get_phases(kur_ctx *ctx, double *theta, int wrapped);

/* Order parameter r e^{i psi} = (1/N) sum_m e^{i theta_m} of the current phases (Sec. 2, eq.
 * OrderParameter): r in [0, 1], psi = atan2 of the mean sine and cosine. Synchronous.
 * KUR_ESTATE without phases; KUR_EINVAL on NULL r or psi. */
kur_status kur_order_parameter(kur_ctx *ctx, double *r, double *psi);

/*
 * Save / restore the phase state (wrapped phases, compensation terms and winding counts, block
 * order) so that a run can be resumed bit for bit. With blob == NULL, *bytes receives the size.
 */
kur_status kur_get_state(kur_ctx *ctx, void *blob, size_t *bytes);
kur_status kur_set_state(kur_ctx *ctx, const void *blob, size_t bytes);

/*
 * Gradients of a loss L(theta(T)) through nsteps classical RK4 steps of size dt started at
 * theta0: the discrete adjoint of exactly the computed RK4 trajectory (not the continuous
 * adjoint equation). With l_i = dL/dk_i and lam = dL/dtheta at the end of a step, one step
 * back reads l4 = dt/6 lam, l3 = dt/3 lam + dt J(Y4)^T l4, l2 = dt/3 lam + dt/2 J(Y3)^T l3,
 * l1 = dt/6 lam + dt/2 J(Y2)^T l2, lam <- lam + sum_i J(Y_i)^T l_i, dL/domega += sum_i l_i,
 * dL/dK += sum_i <l_i, dF/dK(Y_i)>, where J is the Jacobian of eq. KuramotoGraph.
 * The forward pass keeps the phases every ckpt_every steps and each segment is recomputed
 * before its reverse sweep. The context's own phase state is not touched.
 *   theta0      n, user order (NULL: the current phases)
 *   dl_dthetaT  n, user order: dL/dtheta(T)
 *   g_theta0, g_omega (n, user order) and g_K (scalar) receive the gradients (any may be NULL)
 * J^T l needs the columns of A: for a symmetric adjacency the lists of A serve; an asymmetric
 * one needs the layout of A^T, built by kur_set_graph_csr / kur_set_graph_csr_w when the option
 * "transpose" is 1 (KUR_EINVAL otherwise). The recompute of a segment keeps (sin, cos) and the
 * row sums (A sin, A cos) of every stage state. Uses device memory of about
 * (16 ckpt_every + 16) n reals plus 2 n reals per checkpoint, kept for the next call unless
 * the option "adjoint_keep" is 0. Synchronous. KUR_ENOMEM (with the failing allocation in
 * kur_last_error) if the device cannot hold them.
 */
kur_status kur_adjoint_rk4(kur_ctx *ctx, const double *theta0, double dt, int64_t nsteps, int64_t ckpt_every,
                           const double *dl_dthetaT, double *g_theta0, double *g_omega, double *g_K);

/*
 * The same gradients for the run of the last kur_step_rk4 call made with the option
 * "checkpoint_every" = C > 0, which kept the phases every C steps: the forward pass is not
 * repeated. If that run had "record_stages" = 1, the segments are not recomputed either: the
 * reverse sweep reads the recorded stage states. Returns KUR_ESTATE if no such run is recorded or the graph, omega, K or an option
 * changed since. Synchronous.
 */
kur_status kur_adjoint_rk4_recorded(kur_ctx *ctx, const double *dl_dthetaT, double *g_theta0, double *g_omega,
                                    double *g_K);

/* The recorded run kur_adjoint_rk4_recorded would use: a serial number that grows with every
 * recording (0 if none is usable), its dt and its number of steps (either may be NULL). */
kur_status kur_recorded_run(const kur_ctx *ctx, int64_t *serial, double *dt, int64_t *nsteps);

/*
 * Advance nsteps steps of size dt with the implicit midpoint rule, the second-order symmetric
 * (geometric) integrator theta_{n+1} = theta_n + dt F((theta_n + theta_{n+1}) / 2) (Sec. 2,
 * numerical integration: a second-order geometric integrator beside the explicit RK4). The
 * implicit equation is solved by `iters` fixed-point iterations on the midpoint Y, each one
 * evaluation of F: Y_0 = theta_n, Y_i = theta_n + dt/2 F(Y_{i-1}) (i < iters), and
 * theta_{n+1} = theta_n + dt F(Y_{iters-1}). iters = 1 is explicit Euler, iters = 2 the explicit
 * midpoint rule; the error of the fixed point shrinks by about dt/2 |dF| per iteration. The
 * phase update is compensated and wrapped as for kur_step_rk4; r_every, r_out and psi_out as
 * there. Plain launches (no graph replay, no checkpoint recording). iters in [1, 64].
 */
kur_status kur_step_midpoint(kur_ctx *ctx, double dt, int64_t nsteps, int32_t iters, int64_t r_every, double *r_out,
                             double *psi_out);

/*
 * Integrate from the current state over the time t_end > 0 with a variable step size: the
 * explicit embedded Runge-Kutta pair of orders 4 and 5 of Fehlberg (six evaluations of F per
 * attempted step), propagating the fourth-order solution (Sec. 2, numerical integration: a
 * variable stepsize fourth-order explicit Runge-Kutta method). The local error estimate of a
 * step of size h is e = max_m |h sum_j (b5_j - b4_j) k_{j,m}|; the step is accepted when
 * e <= atol (an absolute tolerance on the phases), and the next size is
 * h min(4, max(0.2, 0.9 (e / atol)^(-1/5))) (4 when e = 0); the last step is shortened to end
 * at t_end. dt0 is the first trial size; at most max_steps steps are attempted. The phase
 * update is compensated and wrapped as for kur_step_rk4. out[4] receives the time reached, the
 * proposed next step size, the accepted and the rejected steps. In FP32 choose atol above the
 * FP32 noise of the estimate (about 1e-6 h |F|). Synchronises once per attempted step.
 */
kur_status kur_step_adaptive(kur_ctx *ctx, double t_end, double dt0, double atol, int64_t max_steps, double *out);

/*
 * Diagnostics of the current state (single systems; a batch returns KUR_ESTATE), computed on
 * the device with FP64 sums in a fixed order:
 *   out[0]  the potential V(theta) = -omega^T theta + K/2 sum_{m,l} At_ml (1 - cos(theta_l -
 *           theta_m)), At_ml = A_ml / Mscale_m (Sec. 3, eq. ExtendedPotentialConservation; Sec. 2,
 *           eq. Potential for the complete graph), with theta the unwrapped phases. For a
 *           symmetric A with uniform scaling the dynamics is its gradient flow, so V does not
 *           increase along a trajectory;
 *   out[1]  the mean of the unwrapped phases, (1/N) sum_m theta_m;
 *   out[2]  the mean of omega.
 * The mean deviation of eq. Means is out[1](t) - out[1](0) - t out[2]; it vanishes for a
 * symmetric A with uniform scaling (eq. KuramotoGraphConservation). Synchronous.
 */
kur_status kur_diagnostics(kur_ctx *ctx, double *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * or monitoring loops, harnesses that forbid hipMalloc): kur_diagnostics with the same out[3],
 * computed by the same kernels in the same order (equal bit for bit), but with its FP64 partial
 * sums in a fixed scratch array of 1.5 MiB that every GPU the library runs on holds until the
 * process ends, instead of memory allocated per call. It calls no hipMalloc or hipFree; the
 * inputs and outputs are the context's own buffers and out. The scratch serves n <= 2^24
 * (16777216) nodes: a larger graph returns KUR_EINVAL (use kur_diagnostics). All calls on one
 * GPU share its scratch and it keeps the last call's contents (nothing in it has to start at
 * zero); calls that overlap in time on one GPU race on it and must be serialised by the caller.
 * The energy evaluation is not timed even with option "timing" (timing allocates events).
 * Synchronous; KUR_EDEVICE if the scratch's device address could not be found.
 */
kur_status kur_diagnostics_noalloc(kur_ctx *ctx, double *out);

/* Wait for all work enqueued on the context stream. */
kur_status kur_sync(kur_ctx *ctx);

/*
 * Row-kernel timing (option "timing" = 1): number of timed launches and their total duration
 * in milliseconds since the option was last enabled. Synchronises the stream.
 */
kur_status kur_kernel_time(kur_ctx *ctx, int64_t *launches, double *total_ms);

/* Reference for the roofline: achieved bandwidth (GB/s) of a plain streaming read of `bytes`
 * (1 MiB .. 64 GiB, temporary device buffer) with 16-byte non-temporal loads, repeated
 * `repeats` times. Synchronous. */
kur_status kur_read_bandwidth(kur_ctx *ctx, int64_t bytes, int32_t repeats, double *gbps);

/*
 * Layout autotuning. The density threshold tau that decides whether a block stores its zeros
 * (localised order parameters) or its ones (straightforward summation) follows the
 * Introduction and Sec. 3: precomputed sums pay off once ones outnumber zeros, so tau = 1/2
 * minimises the stored bytes. The tuner times whole RK4 steps of the row kernel with HIP events
 * for candidate values of tau, the chunk width ("chunk") and the tile options ("tile_rows",
 * "tile_min_cost", "flat_min_vec", "threads", "xcds", "inter_gather"), by coordinate descent from the options in
 * force; a candidate wins only when it is at least 1 % faster. Results do not change with the
 * layout beyond rounding order.
 *
 * report (may be NULL) receives 14 doubles: tau, chunk, threads, tile_rows, tile_min_cost,
 * flat_min_vec, ms per RK4 step of the chosen layout, ms per step of the starting layout (NaN
 * when taken from the cache), candidates timed, cache status (1: loaded from the cache, 0:
 * tuned and stored or no cache given, -1: tuned but the cache file could not be written), list
 * builds, seconds spent, xcds, inter_gather (-1: a cache line that leaves the dtype's
 * default). Synchronous; effort 0, 1 or 2 widens the candidate sets.
 *
 * kur_autotune_csr: takes the arguments of kur_set_graph_csr and ends with that graph installed
 * in the chosen layout, as kur_set_graph_csr would (omega, K and phases unset); the options
 * chosen stay in force for later builds. cache_path (NULL: none) is a text file with one line
 * per graph signature (dtype, device, n, edge count and a sampled hash of row offsets and
 * labels); a matching line skips the timing, also on a host-only context. Without a match a
 * host-only context returns KUR_EDEVICE. The lists are rebuilt once per timed tau or chunk.
 *
 * kur_tune_tiles: tile options only, on the installed graph or batch (no list rebuild; the
 * lists, omega, K and phases stay as they are). Device contexts only.
 *
 * kur_tune_key: the cache signature of a graph for this context (NUL-terminated, at most 255
 * characters) in buf of len bytes.
 */
kur_status kur_autotune_csr(kur_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                            const int32_t *labels, int32_t effort, const char *cache_path, double *report);
kur_status kur_tune_tiles(kur_ctx *ctx, int32_t effort, double *report);
kur_status kur_tune_key(kur_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *labels, char *buf,
                        size_t len);

/*
 * Shared-graph ensembles: B replicas (1..256) of one graph, each with its own omega, K and
 * phases, integrated together with classical RK4. The replicas' coupling sums of a row are the
 * row of A X with X = [sin Theta, cos Theta] (n x 2B), the sums of eq.
 * KuramotoGraphReformulation for all replicas at once. For every community block whose realised
 * density is at least the option "ens_tau" (default 0.5; above 1: none), and every off-diagonal
 * block of two communities of at least 32 nodes whose density is at least max(ens_tau, 0.01),
 * this is a dense matrix product A_{a,c} X_c, run on the matrix cores (0/1 pattern stored as a
 * bitmask; FP32 contexts split X exactly into three bf16 terms with FP32 accumulation, FP64
 * contexts multiply FP64 X by exact 0.0/1.0 entries with FP64 accumulation; the products of one
 * row community accumulate in one pass); all other edges are summed as CSR rows (Sec. 3: block
 * structure with dense and sparse parts, and its extension to submatrices). Replica e follows
 * d theta_m / dt = omega_{e,m} + (K_e / N) sum_l A_ml sin(theta_l - theta_m).
 * FP32 and FP64 contexts (the context's reals throughout). Independent of the single-system
 * graph and state.
 *
 * kur_ens_set_graph_csr  CSR with planted labels, as kur_set_graph_csr; host-only contexts keep
 *                        the layout for inspection (kur_ens_row_pattern); params and phases unset
 * kur_ens_set_params     K (B) and omega (B x n, replica-major, user order); copied. KUR_EINVAL
 *                        when a matrix-core community's rows times 2 Bp reach 2^31 (the products
 *                        address one community's X rows with 32-bit offsets: 4.19 M nodes at
 *                        B = 256)
 * kur_ens_set_phases     theta (B x n, replica-major, user order, |theta| <= 1e9)
 * kur_ens_eval_rhs       dtheta (B x n) at the current phases
 * kur_ens_step           nsteps RK4 steps of size dt; with r_every > 0, r_out and psi_out (each
 *                        (nsteps / r_every + 1) x B, sample-major, may be NULL) receive the order
 *                        parameter of every replica at step 0 and every r_every steps
 * kur_ens_get_phases     theta (B x n), wrapped to [-pi, pi) or unwrapped (winding counts)
 * kur_ens_info           out[12]: n, blocks, matrix-core row blocks, their rows, cells of their
 *                        products (sum of rows x columns), CSR entries, B, B padded to 64,
 *                        matrix-product work items, symmetric, off-diagonal blocks on the matrix
 *                        cores, cells the product tiles issue (rows padded to the tile
 *                        height, 256 in FP32 and 128 in FP64; columns of every range to 32)
 * kur_ens_block_modes    per block (either may be NULL): 1 if its own block is on the matrix
 *                        cores, realised density of its own block
 * kur_ens_get_perm       user node -> block-order row (n)
 * kur_ens_row_pattern    host-only contexts: block-order row m's CSR columns (block order) into
 *                        csr_cols, which holds *ncsr entries on entry (NULL: count only; too few:
 *                        KUR_EINVAL); *ncsr receives the count. dense (n bytes, block order,
 *                        may be NULL) receives the row's 0/1 pattern on the columns of its
 *                        matrix-core products and 0 elsewhere
 * kur_ens_kernel_time    with option "timing" = 1: out[4] = matrix-product launches, their total
 *                        ms, row-kernel launches, their total ms, since the previous call
 * kur_ens_autotune_csr   times RK4 steps of B replicas (synthetic values) for candidate
 *                        thresholds, installs the graph with the fastest, sets "ens_tau";
 *                        report (may be NULL) receives 6 doubles: threshold, ms per step, ms with
 *                        every block on the matrix cores, ms with none (NaN if not timed),
 *                        candidates timed, seconds
 */
kur_status kur_ens_set_graph_csr(kur_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                                 const int32_t *labels);
kur_status kur_ens_set_params(kur_ctx *ctx, int32_t B, const double *K, const double *omega);
kur_status kur_ens_set_phases(kur_ctx *ctx, const double *theta);
kur_status kur_ens_eval_rhs(kur_ctx *ctx, double *dtheta);
kur_status kur_ens_step(kur_ctx *ctx, double dt, int64_t nsteps, int64_t r_every, double *r_out, double *psi_out);
kur_status kur_ens_get_phases(kur_ctx *ctx, double *theta, int wrapped);
kur_status kur_ens_info(kur_ctx *ctx, int64_t *out);
kur_status kur_ens_block_modes(kur_ctx *ctx, uint8_t *gemm, double *density);
kur_status kur_ens_get_perm(kur_ctx *ctx, int32_t *perm);
kur_status kur_ens_row_pattern(kur_ctx *ctx, int64_t m, int32_t *csr_cols, int64_t *ncsr, uint8_t *dense);
kur_status kur_ens_kernel_time(kur_ctx *ctx, double *out);
kur_status kur_ens_autotune_csr(kur_ctx *ctx, int64_t n, const int64_t *row_ptr, const int32_t *col,
                                const int32_t *labels, int32_t B, int32_t effort, double *report);

/*
 * Device-pointer variants, for callers whose data already lives on the device (torch tensors:
 * data_ptr()). Every array is a device array on the context's device, in USER order, of the
 * context dtype (float for KUR_F32, double for KUR_F64), n entries unless stated. The calls
 * enqueue on the context stream (kur_stream) and return without synchronising; the pointers
 * are borrowed and must stay valid until that stream work completes, and the caller orders its
 * own streams against the context stream. Device arrays are not read on the host, so their
 * values are not validated: non-finite inputs propagate (a sampled order parameter then reports
 * KUR_ENONFINITE). Host-side checks (NULL pointers, call order) return as for the host calls.
 *
 * kur_stream                    the hipStream_t the context enqueues on
 * kur_set_params_dev            omega_dev (Sec. 3, eq. KuramotoGraph) and K (host value, finite),
 *                               as kur_set_params
 * kur_set_phases_dev            theta_dev, as kur_set_phases (the same split into wrapped value,
 *                               compensation term and winding count, computed in FP64 on the
 *                               device; |theta| must stay below 1e9)
 * kur_eval_rhs_dev              F(theta) into dtheta_dev, as kur_eval_rhs (theta_dev NULL: the
 *                               current phases)
 * kur_get_phases_dev            the current phases into theta_dev, wrapped or unwrapped, as
 *                               kur_get_phases
 * kur_order_parameter_dev       rpsi_dev[0] = r, rpsi_dev[1] = psi of theta_dev (NULL: the current
 *                               phases), Sec. 2 eq. OrderParameter, with FP64 sums in a fixed order
 * kur_order_parameter_vjp_dev   the vector-Jacobian product of that map: with (r, psi) = rpsi_dev
 *                               and (g_r, g_psi) = grad_dev, dtheta_dev[m] (accumulate = 1: +=)
 *                               g_r sin(psi - theta_m) / N + g_psi cos(psi - theta_m) / (N r),
 *                               the derivative of r = |(1/N) sum e^{i theta}| and of its angle;
 *                               both terms are 0 when r = 0 (a loss on r(T) differentiates to
 *                               dL/dtheta(T) on the device)
 * kur_adjoint_rk4_dev           as kur_adjoint_rk4 with theta0_dev (NULL: the current phases),
 *                               dl_dthetaT_dev and the gradients g_theta0_dev, g_omega_dev (n) and
 *                               g_K_dev (one value) on the device (any output may be NULL)
 * kur_adjoint_rk4_recorded_dev  as kur_adjoint_rk4_recorded, device seed and gradients
 * The adjoint calls keep their work buffers in the context for the next call (option
 * "adjoint_keep" = 0 releases them after every call, which then synchronises).
 */
kur_status kur_stream(const kur_ctx *ctx, void **hip_stream);
kur_status kur_set_params_dev(kur_ctx *ctx, const void *omega_dev, double K);
kur_status kur_set_phases_dev(kur_ctx *ctx, const void *theta_dev);
kur_status kur_eval_rhs_dev(kur_ctx *ctx, const void *theta_dev, void *dtheta_dev);
kur_status kur_get_phases_dev(kur_ctx *ctx, void *theta_dev, int wrapped);
kur_status kur_order_parameter_dev(kur_ctx *ctx, const void *theta_dev, void *rpsi_dev);
kur_status kur_order_parameter_vjp_dev(kur_ctx *ctx, const void *theta_dev, const void *rpsi_dev, const void *grad_dev,
                                       void *dtheta_dev, int accumulate);
kur_status kur_adjoint_rk4_dev(kur_ctx *ctx, const void *theta0_dev, double dt, int64_t nsteps, int64_t ckpt_every,
                               const void *dl_dthetaT_dev, void *g_theta0_dev, void *g_omega_dev, void *g_K_dev);
kur_status kur_adjoint_rk4_recorded_dev(kur_ctx *ctx, const void *dl_dthetaT_dev, void *g_theta0_dev,
                                        void *g_omega_dev, void *g_K_dev);

#ifdef __cplusplus
}
#endif
#endif /* KUR_H */
