// kur_api.cpp -- the C ABI declared in include/kur.h: context, validation, device buffers,
// permutation handling and the RK4 driver loop. Every numerical step runs in the HIP kernels
// of kur_kernels.hip; this file only moves data and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/kur.h"
#include "kur_internal.hpp"
#include "kur_io.hpp"
#include "kur_kernels.hpp"
#include "kur_noalloc.hpp"
#include "kur_tune.hpp"

using namespace kur;

static constexpr double kPi = 3.14159265358979323846;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Work buffers of the adjoint, kept by the context between calls (option "adjoint_keep").
struct AdjBufs {
    DevBuf hi, lo, wind, ksum, ck, slots, acs, fpart[2], x[2], xpart[2], lam, lam_acc, lbuf, gom, gk;
};

}  // namespace

struct kur_ctx {
    kur_dtype dtype = KUR_F32;
    int esz = 4;  // bytes per real
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    BuildOptions bopt;
    int threads = 512;
    int scaling = 0;
    int compensate = 1;
    int timing = 0;

    // graph (host metadata)
    bool has_graph = false;
    int64_t n = 0;
    int32_t nb = 0;
    int32_t ntiles = 0;
    int32_t nlaunch = 0;  // workgroups of a tile launch (tiles plus empty slots of the launch order)
    int32_t W = 0, tile_rows = 0;
    std::vector<int32_t> perm;
    std::vector<int32_t> deg;
    int64_t info[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int64_t mask_info[2] = {0, 0};  // bitmask segments, their bytes
    bool symmetric = false;
    BlockGraph host_graph;  // full layout, kept by host-only contexts for introspection
    BlockGraph skel;        // device contexts: blocks, segment and inter offsets (no lists), for re-tiling
    TileParams tiles_installed;  // tile options of the installed layout
    EnsState *ens = nullptr;     // shared-graph ensembles (ensemble.cpp)
    double ens_tau = 0.5;        // ensembles: blocks at least this dense use the matrix cores

    // device graph
    DevBuf d_blk, d_segd, d_grp, d_tiles, d_order, d_seg, d_list, d_iptr, d_icol, d_mask;
    DevBuf d_msum;              // bitmask item partial sums (k_mask), when a layout has any
    DevBuf d_mitem, d_mtile, d_mitemT, d_mtileT;  // bitmask items and per-tile item runs (A, A^T)
    int32_t nmitem = 0, nmitemT = 0, mask_sub = 1024, mask_subT = 1024;
    bool masks = false, masksT = false;  // the layout (of A, of A^T) has bitmask segments
    // layout of A^T for the adjoint of an asymmetric A (option "transpose")
    int transpose = 0;
    bool has_T = false;
    int32_t ntT = 0, nlaunchT = 0, tile_rowsT = 0;
    DevBuf d_blkT, d_segdT, d_grpT, d_tilesT, d_orderT, d_segT, d_listT, d_iptrT, d_icolT, d_maskT;
    // device state
    DevBuf d_omega, d_unit, d_hi, d_lo, d_wind, d_ksum, d_sc[2], d_part[2], d_sce, d_parte, d_kout, d_y;
    DevBuf d_r, d_psi;
    DevBuf d_yb[2];  // stage inputs y of RK4 stages 2..4 (option "inter_gather" = 1)
    int inter_gather = 1;  // 1: inter-block gathers read the phase and form (sin, cos); 0: the pair
                           // (default 1 for FP32, 0 for FP64)
    DevBuf d_perm;   // user node -> block-order row, for the device-pointer calls
    DevBuf d_opart;  // FP64 partials of the order parameter of a device phase vector
    AdjBufs adj;     // adjoint work buffers
    int adjoint_keep = 1;
    int cur = 0;
    bool sc_valid = false;
    bool complete_graph = false;  // the installed graph came from kur_set_graph_complete
    int persistent = 1;           // complete graphs of at most 1024 nodes: one-workgroup RK4 runs
    bool has_params = false, has_phases = false;
    double K = 0.0;

    // instances: a single graph is one instance; a batch is a block-diagonal union
    int32_t n_inst = 0;
    bool batch = false;
    std::vector<int64_t> inst_row_first, inst_tile_first;
    DevBuf d_tile_first, d_inv_n, d_ctr;
    // batch under construction
    std::vector<BlockGraph> pend_graph;
    std::vector<double> pend_omega, pend_theta, pend_unit;
    std::vector<double> pend_K;
    bool pend_open = false;

    // checkpoints recorded by kur_step_rk4 (option "checkpoint_every") for the adjoint
    int64_t ckpt_every = 0;
    DevBuf d_ck;
    bool rec_valid = false;
    // option "record_stages": the recording run also keeps (sin, cos) and (A sin, A cos) of every
    // stage state, so that the recorded adjoint needs no recompute
    int record_stages = 0;
    bool rec_stages = false;
    DevBuf d_rsc, d_rac;
    double rec_dt = 0.0;
    int64_t rec_nsteps = 0, rec_C = 0;
    uint64_t rec_gen = 0;
    int64_t rec_serial = 0;

    // replayed step graph
    int use_graph = 1;
    int64_t graph_steps = 16;
    hipGraphExec_t gexec = nullptr;
    // every value baked into a captured graph: a change of any forces a new capture
    struct GraphKey {
        uint64_t gen;
        double dt;
        int64_t period;
        int sample;
        int cur;
        const void *r;    // sample buffers written by the captured order-parameter kernel
        const void *psi;
        const void *ctr;
        bool operator==(const GraphKey &o) const
        {
            return gen == o.gen && dt == o.dt && period == o.period && sample == o.sample && cur == o.cur &&
                   r == o.r && psi == o.psi && ctr == o.ctr;
        }
    } gkey{0, 0.0, 0, 0, 0, nullptr, nullptr, nullptr};
    uint64_t gen = 1;  // bumped whenever launch arguments may change

    // timing of the row kernel
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    int64_t t_launches = 0;
    double t_ms = 0.0;
};

namespace {

kur_status fail(kur_ctx *c, kur_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

kur_status hip_fail(kur_ctx *c, hipError_t e, const char *what)
{
    return fail(c, e == hipErrorOutOfMemory ? KUR_ENOMEM : KUR_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr, what)                          \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_fail(ctx, _e, what); \
    } while (0)

void dfree(DevBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

hipError_t dalloc(DevBuf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes && bytes > 0) return hipSuccess;
    dfree(b);
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return e;
    }
    b.bytes = bytes;
    return hipSuccess;
}

hipError_t upload(DevBuf &b, const void *src, size_t bytes, hipStream_t st)
{
    hipError_t e = dalloc(b, bytes);
    if (e != hipSuccess || bytes == 0) return e;
    e = hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

// The bitmask items and per-tile item runs of a layout, and room for their partial sums (T:
// bytes of the dtype); nothing for a layout without bitmask segments.
hipError_t upload_mask_items(DevBuf &items, DevBuf &tiles, DevBuf &sums, const BlockGraph &g, size_t T,
                             hipStream_t st)
{
    if (g.mitems.empty()) return hipSuccess;
    hipError_t e;
    if ((e = upload(items, g.mitems.data(), sizeof(MaskItem) * g.mitems.size(), st)) != hipSuccess ||
        (e = upload(tiles, g.mtiles.data(), sizeof(MaskTile) * g.mtiles.size(), st)) != hipSuccess)
        return e;
    return dalloc(sums, 2 * T * (size_t)g.mask_part_rows);
}

void free_adj(AdjBufs &B)
{
    DevBuf *b[] = {&B.hi, &B.lo, &B.wind, &B.ksum, &B.ck, &B.slots, &B.acs, &B.fpart[0], &B.fpart[1], &B.x[0], &B.x[1],
                   &B.xpart[0], &B.xpart[1], &B.lam, &B.lam_acc, &B.lbuf, &B.gom, &B.gk};
    for (DevBuf *p : b) dfree(*p);
}

void free_all(kur_ctx *c)
{
    DevBuf *bufs[] = {&c->d_blk, &c->d_segd, &c->d_grp, &c->d_tiles, &c->d_order, &c->d_seg, &c->d_list, &c->d_iptr, &c->d_icol,
                      &c->d_omega, &c->d_unit, &c->d_hi, &c->d_lo, &c->d_wind, &c->d_ksum, &c->d_sc[0],
                      &c->d_sc[1], &c->d_part[0], &c->d_part[1], &c->d_sce, &c->d_parte, &c->d_kout, &c->d_y,
                      &c->d_r, &c->d_psi, &c->d_tile_first, &c->d_inv_n, &c->d_ctr, &c->d_ck,
                      &c->d_blkT, &c->d_segdT, &c->d_grpT, &c->d_tilesT, &c->d_orderT, &c->d_segT,
                      &c->d_listT, &c->d_iptrT, &c->d_icolT, &c->d_rsc, &c->d_rac, &c->d_perm, &c->d_opart,
                      &c->d_yb[0], &c->d_yb[1], &c->d_mask, &c->d_maskT, &c->d_msum,
                      &c->d_mitem, &c->d_mtile, &c->d_mitemT, &c->d_mtileT};
    for (DevBuf *b : bufs) dfree(*b);
    free_adj(c->adj);
    c->has_T = false;
    c->masks = c->masksT = false;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
}

bool finite_arr(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

DevGraph devgraph(const kur_ctx *c)
{
    DevGraph g;
    g.blk = (const BlkInfo *)c->d_blk.p;
    g.segd = (const SegD *)c->d_segd.p;
    g.grp = (const Grp *)c->d_grp.p;
    g.tiles = (const Tile *)c->d_tiles.p;
    g.order = (const int32_t *)c->d_order.p;
    g.seg_ptr = (const int64_t *)c->d_seg.p;
    g.list = (const uint16_t *)c->d_list.p;
    g.mask = (const uint32_t *)c->d_mask.p;
    g.inter_ptr = (const int64_t *)c->d_iptr.p;
    g.inter_col = (const int32_t *)c->d_icol.p;
    g.W = c->W;
    g.tile_rows = c->tile_rows;
    g.nlaunch = c->nlaunch;
    g.msum = c->masks ? c->d_msum.p : nullptr;
    g.mitem = (const MaskItem *)c->d_mitem.p;
    g.mtile = (const MaskTile *)c->d_mtile.p;
    g.nmitem = c->nmitem;
    g.mask_sub = c->mask_sub;
    return g;
}

// The layout of A^T (same block order and chunk width; its own segments and tiles).
DevGraph devgraph_t(const kur_ctx *c)
{
    DevGraph g;
    g.blk = (const BlkInfo *)c->d_blkT.p;
    g.segd = (const SegD *)c->d_segdT.p;
    g.grp = (const Grp *)c->d_grpT.p;
    g.tiles = (const Tile *)c->d_tilesT.p;
    g.order = (const int32_t *)c->d_orderT.p;
    g.seg_ptr = (const int64_t *)c->d_segT.p;
    g.list = (const uint16_t *)c->d_listT.p;
    g.mask = (const uint32_t *)c->d_maskT.p;
    g.msum = c->masksT ? c->d_msum.p : nullptr;
    g.mitem = (const MaskItem *)c->d_mitemT.p;
    g.mtile = (const MaskTile *)c->d_mtileT.p;
    g.nmitem = c->nmitemT;
    g.mask_sub = c->mask_subT;
    g.inter_ptr = (const int64_t *)c->d_iptrT.p;
    g.inter_col = (const int32_t *)c->d_icolT.p;
    g.W = c->W;
    g.tile_rows = c->tile_rowsT;
    g.nlaunch = c->nlaunchT;
    return g;
}

// host double array (user order) -> device T array (block order)
hipError_t upload_perm(kur_ctx *c, DevBuf &b, const double *src)
{
    const int64_t n = c->n;
    hipError_t e;
    if (c->esz == 4) {
        std::vector<float> t(n);
        for (int64_t u = 0; u < n; ++u) t[c->perm[u]] = (float)src[u];
        e = upload(b, t.data(), sizeof(float) * n, c->stream);
    } else {
        std::vector<double> t(n);
        for (int64_t u = 0; u < n; ++u) t[c->perm[u]] = src[u];
        e = upload(b, t.data(), sizeof(double) * n, c->stream);
    }
    return e;
}

// device T array (block order) -> host double (user order)
hipError_t download_perm(kur_ctx *c, const void *dsrc, double *dst)
{
    const int64_t n = c->n;
    if (c->esz == 4) {
        std::vector<float> t(n);
        hipError_t e = hipMemcpyAsync(t.data(), dsrc, sizeof(float) * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return e;
        for (int64_t u = 0; u < n; ++u) dst[u] = (double)t[c->perm[u]];
    } else {
        std::vector<double> t(n);
        hipError_t e = hipMemcpyAsync(t.data(), dsrc, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return e;
        for (int64_t u = 0; u < n; ++u) dst[u] = t[c->perm[u]];
    }
    return hipSuccess;
}

kur_status need_device(kur_ctx *c)
{
    if (!c) return KUR_EINVAL;
    if (c->host_only) return fail(c, KUR_EDEVICE, "host-only context (device = -1)");
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    return KUR_OK;
}

kur_status need_ready(kur_ctx *c, bool params, bool phases)
{
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    if (params && !c->has_params) return fail(c, KUR_ESTATE, "omega and K not set");
    if (phases && !c->has_phases) return fail(c, KUR_ESTATE, "phases not set");
    return KUR_OK;
}

// per-row unit scale 1/deg_m for non-uniform scaling (zero rows: 0, so theta' = omega)
kur_status set_unit(kur_ctx *c)
{
    c->gen++;
    if (c->batch) return KUR_OK;  // a batch carries its own per-row factors K_i / N_i
    if (c->scaling == 0) {
        dfree(c->d_unit);
        return KUR_OK;
    }
    const int64_t n = c->n;
    hipError_t e;
    if (c->esz == 4) {
        std::vector<float> t(n);
        for (int64_t m = 0; m < n; ++m) t[m] = c->deg[m] > 0 ? (float)(1.0 / (double)c->deg[m]) : 0.0f;
        e = upload(c->d_unit, t.data(), sizeof(float) * n, c->stream);
    } else {
        std::vector<double> t(n);
        for (int64_t m = 0; m < n; ++m) t[m] = c->deg[m] > 0 ? 1.0 / (double)c->deg[m] : 0.0;
        e = upload(c->d_unit, t.data(), sizeof(double) * n, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "row scale upload");
    return KUR_OK;
}

template <typename T>
RowArgs<T> row_args(kur_ctx *c, int stage, double dt)
{
    RowArgs<T> a;
    a.stage = stage;
    a.compensate = c->compensate;
    a.dt = (T)dt;
    a.half_dt = (T)(0.5 * dt);
    a.dt6 = (T)(dt / 6.0);
    a.K = (T)c->K;
    a.inv_n = (T)(1.0 / (double)c->n);
    a.unit = (const T *)c->d_unit.p;
    a.omega = (const T *)c->d_omega.p;
    a.hi = (T *)c->d_hi.p;
    a.lo = (T *)c->d_lo.p;
    a.wind = (int32_t *)c->d_wind.p;
    a.ksum = (T *)c->d_ksum.p;
    a.kout = (T *)c->d_kout.p;
    a.sc_in = c->d_sc[c->cur].p;
    a.part_in = c->d_part[c->cur].p;
    a.sc_out = c->d_sc[c->cur ^ 1].p;
    a.part_out = c->d_part[c->cur ^ 1].p;
    a.ac_out = nullptr;
    a.y_in = nullptr;
    a.y_out = nullptr;
    return a;
}

hipError_t timed_rows(kur_ctx *c, const DevGraph &g, const void *args)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
                c->ev.push_back(e);
            }
        }
        e0 = c->ev[c->ev_used];
        e1 = c->ev[c->ev_used + 1];
        c->ev_used += 2;
        hipError_t r = hipEventRecord(e0, c->stream);
        if (r != hipSuccess) return r;
    }
    hipError_t r;
    if (c->esz == 4)
        r = launch_rows<float>(g, c->ntiles, *(const RowArgs<float> *)args, c->threads, c->stream);
    else
        r = launch_rows<double>(g, c->ntiles, *(const RowArgs<double> *)args, c->threads, c->stream);
    if (r != hipSuccess) return r;
    if (c->timing) {
        r = hipEventRecord(e1, c->stream);
        if (r != hipSuccess) return r;
        c->t_launches += 1;
    }
    return hipSuccess;
}

// fold recorded event pairs into the totals (synchronises)
hipError_t harvest_events(kur_ctx *c)
{
    if (c->ev_used == 0) return hipSuccess;
    hipError_t r = hipStreamSynchronize(c->stream);
    if (r != hipSuccess) return r;
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        r = hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
        if (r != hipSuccess) return r;
        c->t_ms += ms;
    }
    c->ev_used = 0;
    return hipSuccess;
}

kur_status sc_init(kur_ctx *c, const void *y, DevBuf &sc, DevBuf &part)
{
    DevGraph g = devgraph(c);
    hipError_t e;
    if (c->esz == 4)
        e = launch_sc_init<float>(g, c->ntiles, (const float *)y, sc.p, part.p, c->threads, c->stream);
    else
        e = launch_sc_init<double>(g, c->ntiles, (const double *)y, sc.p, part.p, c->threads, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "sc_init launch");
    return KUR_OK;
}

kur_status upload_instances(kur_ctx *c)
{
    std::vector<double> inv(c->n_inst);
    for (int32_t i = 0; i < c->n_inst; ++i) inv[i] = 1.0 / (double)(c->inst_row_first[i + 1] - c->inst_row_first[i]);
    hipError_t e;
    if ((e = upload(c->d_tile_first, c->inst_tile_first.data(), 8 * c->inst_tile_first.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_inv_n, inv.data(), 8 * inv.size(), c->stream)) != hipSuccess ||
        (e = dalloc(c->d_ctr, 64)) != hipSuccess)
        return hip_fail(c, e, "instance tables");
    return KUR_OK;
}

kur_status install_graph(kur_ctx *c, BlockGraph &g)
{
    c->complete_graph = false;  // set again by kur_set_graph_complete after a successful install
    const size_t lds = rows_lds_bytes(c->esz, g.W, g.tile_rows, c->threads);
    if (lds > 156 * 1024) return fail(c, KUR_EINVAL, "chunk/tile_rows/threads exceed the LDS of a workgroup");
    if (g.tiles.size() > (size_t)INT32_MAX) return fail(c, KUR_EINVAL, "too many tiles");
    if (!c->host_only) {
        HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
        free_all(c);
        hipError_t e;
        const int64_t n = g.n;
        const size_t T = (size_t)c->esz;
        if ((e = upload(c->d_blk, g.blk.data(), sizeof(BlkInfo) * g.blk.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_segd, g.segd.data(), sizeof(SegD) * g.segd.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_grp, g.grp.data(), sizeof(Grp) * g.grp.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_tiles, g.tiles.data(), sizeof(Tile) * g.tiles.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_order, g.order.data(), sizeof(int32_t) * g.order.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_seg, g.seg_ptr.data(), sizeof(int64_t) * g.seg_ptr.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_list, g.list.data(), sizeof(uint16_t) * g.list.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_mask, g.mask.data(), sizeof(uint32_t) * g.mask.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_iptr, g.inter_ptr.data(), sizeof(int64_t) * g.inter_ptr.size(), c->stream)) != hipSuccess ||
            (e = upload(c->d_icol, g.inter_col.data(), sizeof(int32_t) * g.inter_col.size(), c->stream)) != hipSuccess ||
            (e = dalloc(c->d_omega, T * n)) != hipSuccess || (e = dalloc(c->d_hi, T * n)) != hipSuccess ||
            (e = dalloc(c->d_lo, T * n)) != hipSuccess || (e = dalloc(c->d_wind, 4 * n)) != hipSuccess ||
            (e = dalloc(c->d_ksum, T * n)) != hipSuccess || (e = dalloc(c->d_sc[0], 2 * T * n)) != hipSuccess ||
            (e = dalloc(c->d_sc[1], 2 * T * n)) != hipSuccess || (e = dalloc(c->d_sce, 2 * T * n)) != hipSuccess ||
            (e = dalloc(c->d_part[0], 2 * T * g.tiles.size())) != hipSuccess ||
            (e = dalloc(c->d_part[1], 2 * T * g.tiles.size())) != hipSuccess ||
            (e = dalloc(c->d_parte, 2 * T * g.tiles.size())) != hipSuccess ||
            (e = dalloc(c->d_kout, T * n)) != hipSuccess || (e = dalloc(c->d_y, T * n)) != hipSuccess ||
            (e = upload(c->d_perm, g.perm.data(), sizeof(int32_t) * n, c->stream)) != hipSuccess ||
            (e = dalloc(c->d_yb[0], T * n)) != hipSuccess || (e = dalloc(c->d_yb[1], T * n)) != hipSuccess ||
            (e = upload_mask_items(c->d_mitem, c->d_mtile, c->d_msum, g, T, c->stream)) != hipSuccess) {
            free_all(c);
            c->has_graph = false;
            return hip_fail(c, e, "graph upload");
        }
    }
    c->n = g.n;
    c->nb = g.nb;
    c->ntiles = (int32_t)g.tiles.size();
    c->nlaunch = (int32_t)g.order.size();
    c->W = g.W;
    c->tile_rows = g.tile_rows;
    c->perm.swap(g.perm);
    c->deg.swap(g.deg);
    c->info[0] = g.n;
    c->info[1] = g.nb;
    c->info[2] = g.n_dense;
    c->info[3] = g.list_unpadded;
    c->info[4] = (int64_t)g.list.size();
    c->info[5] = (int64_t)g.inter_col.size();
    c->info[6] = (int64_t)g.tiles.size();
    c->info[7] = g.W;
    c->info[8] = g.symmetric ? 1 : 0;
    int64_t smax = 0;
    for (const BlkInfo &b : g.blk) smax = std::max<int64_t>(smax, b.size);
    c->info[9] = smax;
    c->mask_info[0] = g.mask_segments;
    c->mask_info[1] = (int64_t)g.mask.size() * 4;
    c->masks = g.mask_segments > 0;
    c->nmitem = (int32_t)g.mitems.size();
    c->mask_sub = g.mask_sub;
    c->masksT = false;
    c->symmetric = g.symmetric;
    c->tiles_installed.threads = c->threads;
    c->tiles_installed.tile_rows = g.tile_rows;
    c->tiles_installed.tile_min_cost = c->bopt.tile_min_cost;
    c->tiles_installed.flat_min_vec = c->bopt.flat_min_vec;
    c->tiles_installed.xcds = c->bopt.xcds;
    c->tiles_installed.inter_gather = c->inter_gather;
    if (c->host_only) {
        c->host_graph = std::move(g);
    } else {
        c->skel = BlockGraph();
        c->skel.n = g.n;
        c->skel.nb = g.nb;
        c->skel.W = g.W;
        c->skel.tile_rows = g.tile_rows;
        c->skel.esz2 = g.esz2;
        c->skel.blk.swap(g.blk);
        c->skel.segd.swap(g.segd);
        c->skel.grp.swap(g.grp);
        c->skel.seg_ptr.swap(g.seg_ptr);
        c->skel.blk_rho.swap(g.blk_rho);
        c->skel.pair_rho.swap(g.pair_rho);
        c->skel.n_pairs = g.n_pairs;
        c->skel.weighted = g.weighted;
        c->skel.mask_segments = g.mask_segments;
        c->skel.inter_ptr.swap(g.inter_ptr);
    }
    c->has_graph = true;
    c->has_params = false;
    c->has_phases = false;
    c->sc_valid = false;
    c->cur = 0;
    c->gen++;
    c->batch = false;
    c->n_inst = 1;
    c->inst_row_first = {0, c->n};
    c->inst_tile_first = {0, (int64_t)c->ntiles};
    if (!c->host_only) {
        kur_status s = upload_instances(c);
        if (s != KUR_OK) return s;
        return set_unit(c);
    }
    return KUR_OK;
}

// CSR of A^T in user order (columns ascending), with the weights when given.
void transpose_csr(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                   std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<int32_t> &wt)
{
    const int64_t nnz = row_ptr[n];
    rp.assign(n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) rp[col[e] + 1]++;
    for (int64_t u = 0; u < n; ++u) rp[u + 1] += rp[u];
    ci.resize(nnz);
    if (weight) wt.resize(nnz);
    std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
    for (int64_t u = 0; u < n; ++u)
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int64_t f = fill[col[e]]++;
            ci[f] = (int32_t)u;
            if (weight) wt[f] = weight[e];
        }
}

// After install_graph of an asymmetric A on a device context with option "transpose": build
// the layout of A^T with the same labels and options (hence the same block order) and upload it.
kur_status install_transpose(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const int32_t *weight, const int32_t *labels)
{
    c->has_T = false;
    c->masksT = false;
    if (c->host_only || c->symmetric || !c->transpose) return KUR_OK;
    BlockGraph t;
    std::string msg;
    try {
        std::vector<int64_t> rp;
        std::vector<int32_t> ci, wt;
        transpose_csr(n, row_ptr, col, weight, rp, ci, wt);
        msg = weight ? build_from_csr_w(n, rp.data(), ci.data(), wt.data(), labels, c->bopt, t)
                     : build_from_csr(n, rp.data(), ci.data(), labels, c->bopt, t);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed building the transposed layout");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, "transposed layout: " + msg);
    if (t.perm != c->perm || t.W != c->W) return fail(c, KUR_EINVAL, "transposed layout differs in block order");
    if (t.tiles.size() > (size_t)INT32_MAX) return fail(c, KUR_EINVAL, "too many tiles");
    hipError_t e;
    if ((e = upload(c->d_blkT, t.blk.data(), sizeof(BlkInfo) * t.blk.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_segdT, t.segd.data(), sizeof(SegD) * t.segd.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_grpT, t.grp.data(), sizeof(Grp) * t.grp.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_tilesT, t.tiles.data(), sizeof(Tile) * t.tiles.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_orderT, t.order.data(), sizeof(int32_t) * t.order.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_segT, t.seg_ptr.data(), sizeof(int64_t) * t.seg_ptr.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_listT, t.list.data(), sizeof(uint16_t) * t.list.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_maskT, t.mask.data(), sizeof(uint32_t) * t.mask.size(), c->stream)) != hipSuccess ||
        (e = upload_mask_items(c->d_mitemT, c->d_mtileT, c->d_msum, t, (size_t)c->esz, c->stream)) != hipSuccess ||
        (e = upload(c->d_iptrT, t.inter_ptr.data(), sizeof(int64_t) * t.inter_ptr.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_icolT, t.inter_col.data(), sizeof(int32_t) * t.inter_col.size(), c->stream)) != hipSuccess)
        return hip_fail(c, e, "transposed layout upload");
    c->ntT = (int32_t)t.tiles.size();
    c->nlaunchT = (int32_t)t.order.size();
    c->masksT = t.mask_segments > 0;
    c->nmitemT = (int32_t)t.mitems.size();
    c->mask_subT = t.mask_sub;
    c->tile_rowsT = t.tile_rows;
    c->has_T = true;
    return KUR_OK;
}

// The run of a small complete graph in one workgroup (k_persist_complete), in launches of at
// most about 65536 steps (whole sampling periods) so that no launch holds the device for long;
// leaves the (sin, cos) of the state to be rebuilt by the next call that needs them. ck (null:
// none) receives (hi, lo) before every step that is a multiple of ck_every.
template <typename T>
hipError_t run_persistent(kur_ctx *c, double dt, int64_t nsteps, int64_t r_every, T *ck = nullptr,
                          int64_t ck_every = 1)
{
    PersistArgs<T> a;
    a.n = c->n;
    a.r_every = r_every;
    a.compensate = c->compensate;
    a.dt = (T)dt;
    a.half_dt = (T)(0.5 * dt);
    a.dt6 = (T)(dt / 6.0);
    a.K = (T)c->K;
    a.inv_n = (T)(1.0 / (double)c->n);
    a.unit = (const T *)c->d_unit.p;
    a.omega = (const T *)c->d_omega.p;
    a.hi = (T *)c->d_hi.p;
    a.lo = (T *)c->d_lo.p;
    a.wind = (int32_t *)c->d_wind.p;
    a.ck = ck;
    a.ck_every = ck_every;
    const int64_t chunk = r_every > 0 ? std::max<int64_t>(1, 65536 / r_every) * r_every : 65536;
    int64_t done = 0;
    do {
        a.step0 = done;
        a.nsteps = std::min(chunk, nsteps - done);
        a.final_sample = done + a.nsteps == nsteps;  // else the next launch's step 0 is that sample
        a.r_out = (double *)c->d_r.p + (r_every > 0 ? done / r_every : 0);
        a.psi_out = (double *)c->d_psi.p + (r_every > 0 ? done / r_every : 0);
        const hipError_t e = launch_persist_complete<T>(a, c->stream);
        if (e != hipSuccess) return e;
        done += a.nsteps;
    } while (done < nsteps);
    return hipSuccess;
}

}  // namespace

extern "C" {

int kur_version(void) { return 100; }

kur_status kur_create(kur_ctx **out, kur_dtype dtype, int device, void *hip_stream)
{
    if (!out) return KUR_EINVAL;
    *out = nullptr;
    if (dtype != KUR_F32 && dtype != KUR_F64) return KUR_EINVAL;
    if (device < -1) return KUR_EINVAL;
    kur_ctx *c = new (std::nothrow) kur_ctx();
    if (!c) return KUR_ENOMEM;
    c->dtype = dtype;
    c->esz = dtype == KUR_F32 ? 4 : 8;
    c->bopt.W = 4096;
    c->bopt.tile_rows = 256;
    c->bopt.esz2 = 8;
    if (dtype == KUR_F64) {
        // the widest chunk whose 16-byte pairs (and the zero slot) keep 16-bit LDS offsets:
        // measured 5.8 % faster than 2048 at N = 2^20 and equal on 1024-node blocks
        c->bopt.esz2 = 16;
        c->bopt.W = (int32_t)((65535 / c->bopt.esz2) / 64 * 64);
    }
    // FP32: the inter-block gathers read 4-byte phases (half the cache footprint of the pairs);
    // FP64 keeps the pair gathers (its sin/cos would cost occupancy)
    c->inter_gather = dtype == KUR_F32 ? 1 : 0;
    c->device = device;
    c->host_only = device < 0;
    if (!c->host_only) {
        int cnt = 0;
        if (hipGetDeviceCount(&cnt) != hipSuccess || device >= cnt) {
            (void)hipGetLastError();
            delete c;
            return KUR_EDEVICE;
        }
        if (hipSetDevice(device) != hipSuccess) {
            delete c;
            return KUR_EDEVICE;
        }
        // the device address of the fixed scratch of kur_diagnostics_noalloc (once per device;
        // a failure shows up as KUR_EDEVICE from that call only)
        (void)noalloc_scratch_init(device);
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
                delete c;
                return KUR_EDEVICE;
            }
            c->own_stream = true;
        }
    }
    *out = c;
    return KUR_OK;
}

void kur_destroy(kur_ctx *c)
{
    if (!c) return;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        free_all(c);
        ens_free(c->ens);
        c->ens = nullptr;
        for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    }
    ens_free(c->ens);
    delete c;
}

const char *kur_last_error(const kur_ctx *c) { return c ? c->err.c_str() : ""; }

kur_status kur_set_option(kur_ctx *c, const char *key, double v)
{
    if (!c || !key) return KUR_EINVAL;
    c->err.clear();
    std::string k(key);
    if (!std::isfinite(v)) return fail(c, KUR_EINVAL, "option value must be finite");
    if (k == "tau") {
        if (v < 0.0 || v > 1.0 + 1e-12) return fail(c, KUR_EINVAL, "tau must be in [0, 1]");
        c->bopt.tau = v;
    } else if (k == "chunk") {
        int64_t w = (int64_t)v;
        if ((double)w != v || w < 64 || w % 64 || w * c->bopt.esz2 > 65535)
            return fail(c, KUR_EINVAL, "chunk must be a multiple of 64 in [64, 65535 / pair bytes] (8128 FP32, 4032 FP64)");
        c->bopt.W = (int32_t)w;
    } else if (k == "tile_rows") {
        int64_t t = (int64_t)v;
        if ((double)t != v || t < 64 || t > 4096) return fail(c, KUR_EINVAL, "tile_rows must be an integer in [64, 4096]");
        c->bopt.tile_rows = (int32_t)t;
    } else if (k == "tiles") {
        int64_t t = (int64_t)v;
        if ((double)t != v || t < 1 || t > (int64_t)1 << 24) return fail(c, KUR_EINVAL, "tiles must be an integer in [1, 2^24]");
        c->bopt.tiles_target = t;
    } else if (k == "tile_min_cost") {
        if (v != (int64_t)v || v < 1 || v > 1e9) return fail(c, KUR_EINVAL, "tile_min_cost must be an integer in [1, 1e9]");
        c->bopt.tile_min_cost = (int64_t)v;
    } else if (k == "flat_min_vec") {
        if (v < 0.0 || v > 1e6) return fail(c, KUR_EINVAL, "flat_min_vec must be in [0, 1e6]");
        c->bopt.flat_min_vec = v;
    } else if (k == "xcds") {
        if (v != (int64_t)v || v < 1 || v > 64) return fail(c, KUR_EINVAL, "xcds must be an integer in [1, 64]");
        c->bopt.xcds = (int32_t)v;
    } else if (k == "transpose") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "transpose must be 0 or 1");
        c->transpose = (int)v;
    } else if (k == "pairs") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "pairs must be 0 or 1");
        c->bopt.pairs = v != 0;
    } else if (k == "mask_min") {
        if (!(v >= 0.0) || v > 1e9) return fail(c, KUR_EINVAL, "mask_min must be in [0, 1e9]");
        c->bopt.mask_min = v;
    } else if (k == "mask_sub") {
        if (v != (int64_t)v || v < kMaskUnitCols || v > kMaskSubMax || (int64_t)v % kMaskUnitCols)
            return fail(c, KUR_EINVAL, "mask_sub must be a multiple of 128 in [128, 1024]");
        c->bopt.mask_sub = (int32_t)v;
    } else if (k == "mask_item") {
        if (v != (int64_t)v || v < 1 || v > 1e12) return fail(c, KUR_EINVAL, "mask_item must be an integer in [1, 1e12]");
        c->bopt.mask_item = (int64_t)v;
    } else if (k == "pair_min") {
        if (v != (int64_t)v || v < 1 || v > 65536) return fail(c, KUR_EINVAL, "pair_min must be an integer in [1, 65536]");
        c->bopt.pair_min = (int32_t)v;
    } else if (k == "threads") {
        if (v != 128 && v != 256 && v != 512 && v != 1024)
            return fail(c, KUR_EINVAL, "threads must be 128, 256, 512 or 1024");
        if (c->has_graph && rows_lds_bytes(c->esz, c->W, c->tile_rows, (int)v) > 156 * 1024)
            return fail(c, KUR_EINVAL, "threads exceed the LDS budget of the current graph layout");
        c->threads = (int)v;
        c->gen++;
    } else if (k == "scaling") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "scaling must be 0 or 1");
        c->scaling = (int)v;
        if (c->has_graph && !c->host_only) return set_unit(c);
    } else if (k == "compensate") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "compensate must be 0 or 1");
        c->compensate = (int)v;
        c->gen++;
    } else if (k == "inter_gather") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "inter_gather must be 0 or 1");
        c->inter_gather = (int)v;
        c->tiles_installed.inter_gather = c->inter_gather;
        c->gen++;
    } else if (k == "adjoint_keep") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "adjoint_keep must be 0 or 1");
        c->adjoint_keep = (int)v;
        if (!v && !c->host_only) {
            HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
            HIPCHK(c, hipStreamSynchronize(c->stream), "adjoint buffers");
            free_adj(c->adj);
        }
    } else if (k == "record_stages") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "record_stages must be 0 or 1");
        c->record_stages = (int)v;
    } else if (k == "checkpoint_every") {
        if (v != (int64_t)v || v < 0 || v > 1e9) return fail(c, KUR_EINVAL, "checkpoint_every must be an integer >= 0");
        c->ckpt_every = (int64_t)v;
    } else if (k == "graph") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "graph must be 0 or 1");
        c->use_graph = (int)v;
    } else if (k == "persistent") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "persistent must be 0 or 1");
        c->persistent = (int)v;
    } else if (k == "ens_tau") {
        if (v < 0.0 || v > 2.0) return fail(c, KUR_EINVAL, "ens_tau must be in [0, 2] (above 1: no block on the matrix cores)");
        c->ens_tau = v;
    } else if (k == "graph_steps") {
        if (v != (int64_t)v || v < 1 || v > 4096) return fail(c, KUR_EINVAL, "graph_steps must be an integer in [1, 4096]");
        c->graph_steps = (int64_t)v;
    } else if (k == "timing") {
        if (v != 0 && v != 1) return fail(c, KUR_EINVAL, "timing must be 0 or 1");
        if (!c->host_only) {
            hipError_t e = harvest_events(c);
            if (e != hipSuccess) return hip_fail(c, e, "timing");
        }
        c->timing = (int)v;
        c->t_launches = 0;
        c->t_ms = 0.0;
    } else {
        return fail(c, KUR_EINVAL, "unknown option '" + k + "'");
    }
    return KUR_OK;
}

kur_status kur_set_graph_csr(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const int32_t *labels)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    BlockGraph g;
    std::string msg;
    try {
        msg = build_from_csr(n, row_ptr, col, labels, c->bopt, g);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in graph preprocessing");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, msg);
    kur_status s = install_graph(c, g);
    if (s != KUR_OK) return s;
    return install_transpose(c, n, row_ptr, col, nullptr, labels);
}

kur_status kur_set_graph_csr_w(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *weight,
                               const int32_t *labels)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    BlockGraph g;
    std::string msg;
    try {
        msg = build_from_csr_w(n, row_ptr, col, weight, labels, c->bopt, g);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in graph preprocessing");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, msg);
    kur_status s = install_graph(c, g);
    if (s != KUR_OK) return s;
    return install_transpose(c, n, row_ptr, col, weight, labels);
}

kur_status kur_set_graph(kur_ctx *c, int64_t n, int32_t nb, const int64_t *block_ptr, const uint8_t *mode,
                         const int64_t *list_ptr, const uint16_t *list_col, const int64_t *inter_ptr,
                         const int32_t *inter_col, const int32_t *perm)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    BlockGraph g;
    std::string msg;
    try {
        msg = build_from_blocks(n, nb, block_ptr, mode, list_ptr, list_col, inter_ptr, inter_col, perm, c->bopt, g);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in graph preprocessing");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, msg);
    return install_graph(c, g);
}

kur_status kur_graph_info(const kur_ctx *c, int64_t out[10])
{
    if (!c || !out) return KUR_EINVAL;
    if (!c->has_graph) return KUR_ESTATE;
    std::memcpy(out, c->info, sizeof(c->info));
    return KUR_OK;
}

kur_status kur_graph_masks(const kur_ctx *c, int64_t out[2])
{
    if (!c || !out) return KUR_EINVAL;
    if (!c->has_graph) return KUR_ESTATE;
    out[0] = c->mask_info[0];
    out[1] = c->mask_info[1];
    return KUR_OK;
}

kur_status kur_graph_mask_items(const kur_ctx *c, int64_t *count, int64_t *items)
{
    if (!c || !count) return KUR_EINVAL;
    if (!c->has_graph || !c->host_only) return KUR_ESTATE;
    const BlockGraph &g = c->host_graph;
    *count = (int64_t)g.mitems.size();
    if (!items) return KUR_OK;
    const int64_t S = g.mask_sub;
    for (size_t i = 0; i < g.mitems.size(); ++i) {
        const MaskItem &it = g.mitems[i];
        const Tile &tl = g.tiles[it.tile];
        const BlkInfo &b = g.blk[tl.block];
        const int64_t h = tl.r1 - tl.r0;
        // the item's sub-chunks, in the order the kernel visits them
        int64_t units = 0, cells = 0;
        int32_t ch = it.seg;
        int64_t s0 = (int64_t)it.sub * S;
        for (int32_t k = 0; k < it.nsub && ch < b.nchunk; ++k) {
            const int64_t w = std::min<int64_t>(S, g.segd[b.sd0 + ch].cw - s0);
            units += (w + kMaskUnitCols - 1) / kMaskUnitCols;
            cells += h * w;
            s0 += S;
            if (s0 >= g.segd[b.sd0 + ch].cw) {
                s0 = 0;
                do ++ch;
                while (ch < b.nchunk && !g.segd[b.sd0 + ch].mask);
            }
        }
        int64_t *o = items + 9 * i;
        o[0] = it.tile;
        o[1] = tl.block;
        o[2] = it.seg;
        o[3] = it.sub;
        o[4] = it.nsub;
        o[5] = h;
        o[6] = units;
        o[7] = cells;
        o[8] = it.out;
    }
    return KUR_OK;
}

kur_status kur_get_perm(const kur_ctx *c, int32_t *perm)
{
    if (!c || !perm) return KUR_EINVAL;
    if (!c->has_graph) return KUR_ESTATE;
    std::memcpy(perm, c->perm.data(), sizeof(int32_t) * c->n);
    return KUR_OK;
}

kur_status kur_get_blocks(const kur_ctx *c, int64_t *block_ptr, uint8_t *mode)
{
    if (!c || !block_ptr || !mode) return KUR_EINVAL;
    if (!c->has_graph || !c->host_only) return KUR_ESTATE;
    const BlockGraph &g = c->host_graph;
    for (int32_t b = 0; b < g.nb; ++b) {
        block_ptr[b] = g.blk[b].row0;
        mode[b] = (uint8_t)g.blk[b].mode;
    }
    block_ptr[g.nb] = g.n;
    return KUR_OK;
}

// The chunk-relative columns of segment ch of block-local row r, ascending, from its list or its
// bitmask; f(col) returns false to stop (then so does this call).
extern "C++" template <typename F>
bool seg_row_cols(const BlockGraph &g, const BlkInfo &bi, int32_t ch, int64_t r, F &&f)
{
    const SegD &sd = g.segd[bi.sd0 + ch];
    if (sd.mask) {
        const int64_t nq = (sd.cw + kMaskUnitCols - 1) / kMaskUnitCols;
        for (int64_t q = 0; q < nq; ++q)
            for (int w = 0; w < 4; ++w) {
                uint32_t x = g.mask[(size_t)(sd.mbase + q * bi.size + r) * 4 + w];
                while (x) {
                    const int t = __builtin_ctz(x);
                    x &= x - 1;
                    if (!f((int32_t)(q * kMaskUnitCols + 32 * w + t))) return false;
                }
            }
        return true;
    }
    const int64_t idx = bi.segbase + (int64_t)ch * bi.size + r;
    for (int64_t e = g.seg_ptr[idx]; e < g.seg_ptr[idx + 1]; ++e) {
        if (g.list[e] == (uint16_t)(g.W * g.esz2)) continue;  // padding
        if (!f((int32_t)(g.list[e] / g.esz2))) return false;
    }
    return true;
}

kur_status kur_get_row_lists(const kur_ctx *c, int64_t row, int32_t *list, int64_t *nlist, int32_t *inter,
                             int64_t *ninter)
{
    if (!c || !nlist || !ninter) return KUR_EINVAL;
    if (!c->has_graph || !c->host_only) return KUR_ESTATE;
    const BlockGraph &g = c->host_graph;
    if (row < 0 || row >= g.n) return KUR_EINVAL;
    int32_t b = (int32_t)(std::upper_bound(g.blk.begin(), g.blk.end(), (int32_t)row,
                                           [](int32_t r, const BlkInfo &x) { return r < x.row0; }) - g.blk.begin()) - 1;
    const BlkInfo &bi = g.blk[b];
    const int64_t r = row - bi.row0;
    int64_t k = 0;
    for (int32_t ch = 0; ch < bi.nchunk; ++ch) {
        const SegD &sd = g.segd[bi.sd0 + ch];
        if (sd.col0 < bi.row0 || sd.col0 >= bi.row0 + bi.size) continue;  // a dense off-diagonal block
        const bool ok = seg_row_cols(g, bi, ch, r, [&](int32_t col) {
            if (list) {
                if (k >= *nlist) return false;
                list[k] = sd.col0 - bi.row0 + col;
            }
            ++k;
            return true;
        });
        if (!ok) return KUR_EINVAL;
    }
    const int64_t ni = g.inter_ptr[row + 1] - g.inter_ptr[row];
    if (inter) {
        if (ni > *ninter) return KUR_EINVAL;
        std::memcpy(inter, g.inter_col.data() + g.inter_ptr[row], sizeof(int32_t) * ni);
    }
    *nlist = k;
    *ninter = ni;
    return KUR_OK;
}

kur_status kur_get_row_layers(const kur_ctx *c, int64_t row, int32_t *cols, int32_t *layer, int64_t *count)
{
    if (!c || !count) return KUR_EINVAL;
    if (!c->has_graph || !c->host_only) return KUR_ESTATE;
    const BlockGraph &g = c->host_graph;
    if (row < 0 || row >= g.n) return KUR_EINVAL;
    const int32_t b = (int32_t)(std::upper_bound(g.blk.begin(), g.blk.end(), (int32_t)row,
                                                 [](int32_t r, const BlkInfo &x) { return r < x.row0; }) - g.blk.begin()) - 1;
    const BlkInfo &bi = g.blk[b];
    const int64_t r = row - bi.row0;
    int64_t k = 0;
    int32_t layer_no = 0, last_col0 = -1;
    for (int32_t ch = 0; ch < bi.nchunk; ++ch) {
        const SegD &sd = g.segd[bi.sd0 + ch];
        // the layers of one column chunk are consecutive segments
        layer_no = sd.col0 == last_col0 ? layer_no + 1 : 1;
        last_col0 = sd.col0;
        const bool ok = seg_row_cols(g, bi, ch, r, [&](int32_t col) {
            if (cols || layer) {
                if (k >= *count) return false;
                if (cols) cols[k] = sd.col0 + col;
                if (layer) layer[k] = layer_no;
            }
            ++k;
            return true;
        });
        if (!ok) return KUR_EINVAL;
    }
    *count = k;
    return KUR_OK;
}

kur_status kur_get_block_groups(const kur_ctx *c, int32_t block, int32_t *blk, int32_t *mode, int32_t *count)
{
    if (!c || !count) return KUR_EINVAL;
    if (!c->has_graph) return KUR_ESTATE;
    const BlockGraph &g = c->host_only ? c->host_graph : c->skel;
    if (block < 0 || block >= g.nb) return KUR_EINVAL;
    const BlkInfo &bi = g.blk[block];
    if ((blk || mode) && *count < bi.ngrp) return KUR_EINVAL;
    for (int32_t q = 0; q < bi.ngrp; ++q) {
        if (blk) blk[q] = g.grp[bi.grp0 + q].blk;
        if (mode) mode[q] = g.grp[bi.grp0 + q].mode;
    }
    *count = bi.ngrp;
    return KUR_OK;
}

kur_status kur_graph_pairs(const kur_ctx *c, int64_t *n_pairs)
{
    if (!c || !n_pairs) return KUR_EINVAL;
    if (!c->has_graph) return KUR_ESTATE;
    *n_pairs = (c->host_only ? c->host_graph : c->skel).n_pairs;
    return KUR_OK;
}

kur_status kur_set_params(kur_ctx *c, const double *omega, double K)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    if (!omega) return fail(c, KUR_EINVAL, "omega must not be NULL");
    if (!std::isfinite(K)) return fail(c, KUR_EINVAL, "K must be finite");
    if (!finite_arr(omega, c->n)) return fail(c, KUR_EINVAL, "omega must be finite");
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    hipError_t e = upload_perm(c, c->d_omega, omega);
    if (e != hipSuccess) return hip_fail(c, e, "omega upload");
    c->K = K;
    c->has_params = true;
    c->gen++;
    return KUR_OK;
}

kur_status kur_set_phases(kur_ctx *c, const double *theta)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    if (!theta) return fail(c, KUR_EINVAL, "theta must not be NULL");
    for (int64_t u = 0; u < c->n; ++u)
        if (!std::isfinite(theta[u]) || std::fabs(theta[u]) > 1e9)
            return fail(c, KUR_EINVAL, "theta must be finite with |theta| <= 1e9");
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    const int64_t n = c->n;
    const double P1 = two_pi_p1(c->esz), P2 = two_pi_p2(c->esz);
    std::vector<int32_t> wind(n);
    std::vector<double> red(n);
    for (int64_t u = 0; u < n; ++u) {
        double q = std::nearbyint(theta[u] / (2.0 * kPi));
        wind[c->perm[u]] = (int32_t)q;
        red[c->perm[u]] = (theta[u] - q * P1) - q * P2;
    }
    hipError_t e;
    if (c->esz == 4) {
        std::vector<float> hi(n), lo(n);
        for (int64_t m = 0; m < n; ++m) {
            hi[m] = (float)red[m];
            lo[m] = (float)(red[m] - (double)hi[m]);
        }
        if ((e = upload(c->d_hi, hi.data(), 4 * n, c->stream)) != hipSuccess ||
            (e = upload(c->d_lo, lo.data(), 4 * n, c->stream)) != hipSuccess)
            return hip_fail(c, e, "phase upload");
    } else {
        std::vector<double> lo(n, 0.0);
        if ((e = upload(c->d_hi, red.data(), 8 * n, c->stream)) != hipSuccess ||
            (e = upload(c->d_lo, lo.data(), 8 * n, c->stream)) != hipSuccess)
            return hip_fail(c, e, "phase upload");
    }
    if ((e = upload(c->d_wind, wind.data(), 4 * n, c->stream)) != hipSuccess) return hip_fail(c, e, "phase upload");
    c->has_phases = true;
    c->sc_valid = false;
    return KUR_OK;
}

static kur_status eval_common(kur_ctx *c, const void *y_dev, void *out_dev, int stage = 0, bool timed = true)
{
    kur_status s = sc_init(c, y_dev, c->d_sce, c->d_parte);
    if (s != KUR_OK) return s;
    DevGraph g = devgraph(c);
    hipError_t e;
    if (c->esz == 4) {
        RowArgs<float> a = row_args<float>(c, stage, 0.0);
        a.sc_in = c->d_sce.p;
        a.part_in = c->d_parte.p;
        a.kout = (float *)out_dev;
        if (c->inter_gather) a.y_in = (const float *)y_dev;
        e = timed ? timed_rows(c, g, &a) : launch_rows<float>(g, c->ntiles, a, c->threads, c->stream);
    } else {
        RowArgs<double> a = row_args<double>(c, stage, 0.0);
        a.sc_in = c->d_sce.p;
        a.part_in = c->d_parte.p;
        a.kout = (double *)out_dev;
        if (c->inter_gather) a.y_in = (const double *)y_dev;
        e = timed ? timed_rows(c, g, &a) : launch_rows<double>(g, c->ntiles, a, c->threads, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "rhs launch");
    return KUR_OK;
}

kur_status kur_eval_rhs(kur_ctx *c, const double *theta, double *dtheta)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!dtheta) return fail(c, KUR_EINVAL, "dtheta must not be NULL");
    kur_status s = need_ready(c, true, theta == nullptr);
    if (s != KUR_OK) return s;
    const void *y;
    if (theta) {
        for (int64_t u = 0; u < c->n; ++u)
            if (!std::isfinite(theta[u])) return fail(c, KUR_EINVAL, "theta must be finite");
        // reduce to [-pi, pi] in double before rounding to the context type
        std::vector<double> red(c->n);
        for (int64_t u = 0; u < c->n; ++u) red[u] = std::remainder(theta[u], 2.0 * kPi);
        hipError_t e = upload_perm(c, c->d_y, red.data());
        if (e != hipSuccess) return hip_fail(c, e, "theta upload");
        y = c->d_y.p;
    } else {
        y = c->d_hi.p;
    }
    s = eval_common(c, y, c->d_kout.p);
    if (s != KUR_OK) return s;
    hipError_t e = download_perm(c, c->d_kout.p, dtheta);
    if (e != hipSuccess) return hip_fail(c, e, "rhs download");
    return KUR_OK;
}

kur_status kur_eval_rhs_dev(kur_ctx *c, const void *theta_dev, void *dtheta_dev)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!dtheta_dev) return fail(c, KUR_EINVAL, "dtheta_dev must not be NULL");
    kur_status s = need_ready(c, true, theta_dev == nullptr);
    if (s != KUR_OK) return s;
    const int32_t *perm = (const int32_t *)c->d_perm.p;
    const void *y = c->d_hi.p;
    if (theta_dev) {
        hipError_t e = c->esz == 4 ? launch_reduce_in<float>(c->n, perm, theta_dev, c->d_y.p, c->stream)
                                   : launch_reduce_in<double>(c->n, perm, theta_dev, c->d_y.p, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "theta scatter");
        y = c->d_y.p;
    }
    s = eval_common(c, y, c->d_kout.p);
    if (s != KUR_OK) return s;
    hipError_t e = c->esz == 4 ? launch_gather_out<float, float>(c->n, perm, c->d_kout.p, dtheta_dev, c->stream)
                               : launch_gather_out<double, double>(c->n, perm, c->d_kout.p, dtheta_dev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "rhs gather");
    return KUR_OK;
}

kur_status kur_set_params_dev(kur_ctx *c, const void *omega_dev, double K)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    if (!omega_dev) return fail(c, KUR_EINVAL, "omega_dev must not be NULL");
    if (!std::isfinite(K)) return fail(c, KUR_EINVAL, "K must be finite");
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    const int32_t *perm = (const int32_t *)c->d_perm.p;
    hipError_t e = c->esz == 4 ? launch_scatter_in<float>(c->n, perm, omega_dev, c->d_omega.p, c->stream)
                               : launch_scatter_in<double>(c->n, perm, omega_dev, c->d_omega.p, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "omega scatter");
    c->K = K;
    c->has_params = true;
    c->gen++;
    return KUR_OK;
}

kur_status kur_set_phases_dev(kur_ctx *c, const void *theta_dev)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    if (!theta_dev) return fail(c, KUR_EINVAL, "theta_dev must not be NULL");
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    const int32_t *perm = (const int32_t *)c->d_perm.p;
    const double P1 = two_pi_p1(c->esz), P2 = two_pi_p2(c->esz);
    hipError_t e = c->esz == 4
                       ? launch_phase_in<float>(c->n, perm, theta_dev, P1, P2, c->d_hi.p, c->d_lo.p, (int32_t *)c->d_wind.p, c->stream)
                       : launch_phase_in<double>(c->n, perm, theta_dev, P1, P2, c->d_hi.p, c->d_lo.p, (int32_t *)c->d_wind.p, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "phase split");
    c->has_phases = true;
    c->sc_valid = false;
    return KUR_OK;
}

kur_status kur_order_parameter_dev(kur_ctx *c, const void *theta_dev, void *rpsi_dev)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!rpsi_dev) return fail(c, KUR_EINVAL, "rpsi_dev must not be NULL");
    kur_status s = need_ready(c, false, theta_dev == nullptr);
    if (s != KUR_OK) return s;
    hipError_t e;
    if ((e = dalloc(c->d_opart, 2 * sizeof(double) * kOpParts)) != hipSuccess) return hip_fail(c, e, "partials");
    const void *th = theta_dev;
    if (!th) {  // the current phases (wrapped; any order)
        e = c->esz == 4 ? launch_phase_out<float>(c->n, c->d_hi.p, c->d_lo.p, (const int32_t *)c->d_wind.p, 0, c->d_y.p, c->stream)
                        : launch_phase_out<double>(c->n, c->d_hi.p, c->d_lo.p, (const int32_t *)c->d_wind.p, 0, c->d_y.p, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "phase launch");
        th = c->d_y.p;
    }
    e = c->esz == 4 ? launch_order_param<float>(c->n, th, (double *)c->d_opart.p, rpsi_dev, c->stream)
                    : launch_order_param<double>(c->n, th, (double *)c->d_opart.p, rpsi_dev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "order parameter launch");
    return KUR_OK;
}

kur_status kur_order_parameter_vjp_dev(kur_ctx *c, const void *theta_dev, const void *rpsi_dev, const void *grad_dev,
                                       void *dtheta_dev, int accumulate)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!theta_dev || !rpsi_dev || !grad_dev || !dtheta_dev)
        return fail(c, KUR_EINVAL, "device pointers must not be NULL");
    if (accumulate != 0 && accumulate != 1) return fail(c, KUR_EINVAL, "accumulate must be 0 or 1");
    kur_status s = need_ready(c, false, false);
    if (s != KUR_OK) return s;
    hipError_t e = c->esz == 4 ? launch_order_param_vjp<float>(c->n, theta_dev, rpsi_dev, grad_dev, accumulate, dtheta_dev, c->stream)
                               : launch_order_param_vjp<double>(c->n, theta_dev, rpsi_dev, grad_dev, accumulate, dtheta_dev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "order parameter vjp launch");
    return KUR_OK;
}

kur_status kur_stream(const kur_ctx *c, void **hip_stream)
{
    if (!c || !hip_stream) return KUR_EINVAL;
    *hip_stream = (void *)c->stream;
    return KUR_OK;
}

// The diagnostics into out[0..3) with part (3 ceil(n / 256) doubles) and res (3 doubles) of
// device scratch; timed: the energy evaluation is timed like other row-kernel launches.
static kur_status diag_impl(kur_ctx *c, double *out, double *part, double *res, bool timed)
{
    const int64_t n = c->n;
    kur_status s = eval_common(c, c->d_hi.p, c->d_kout.p, -1, timed);
    if (s != KUR_OK) return s;
    hipError_t e = c->esz == 4 ? launch_diag<float>(n, c->d_hi.p, c->d_lo.p, (const int32_t *)c->d_wind.p, c->d_omega.p,
                                                    c->d_unit.p, c->d_kout.p, c->K, part, res, c->stream)
                               : launch_diag<double>(n, c->d_hi.p, c->d_lo.p, (const int32_t *)c->d_wind.p, c->d_omega.p,
                                                     c->d_unit.p, c->d_kout.p, c->K, part, res, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "diagnostics launch");
    double h[3];
    if ((e = hipMemcpyAsync(h, res, 24, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "diagnostics download");
    // the constant of the potential, K/2 sum_m scale_m deg_m, from the host degrees
    double cst = 0.0;
    for (int64_t m = 0; m < n; ++m) cst += c->scaling ? (c->deg[m] > 0 ? 1.0 : 0.0) : (double)c->deg[m] / (double)n;
    out[0] = h[2] + 0.5 * c->K * cst;
    out[1] = h[0] / (double)n;
    out[2] = h[1] / (double)n;
    return KUR_OK;
}

kur_status kur_diagnostics(kur_ctx *c, double *out)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!out) return fail(c, KUR_EINVAL, "out must not be NULL");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    if (c->batch) return fail(c, KUR_ESTATE, "diagnostics are defined per system, not for a batch");
    DevBuf part, res;
    hipError_t e;
    const int64_t nchunk = (c->n + 255) / 256;
    if ((e = dalloc(part, 24 * (size_t)nchunk)) != hipSuccess || (e = dalloc(res, 24)) != hipSuccess)
        return hip_fail(c, e, "diagnostics buffers");
    struct Release {
        DevBuf *a, *b;
        ~Release()
        {
            dfree(*a);
            dfree(*b);
        }
    } rel{&part, &res};
    return diag_impl(c, out, (double *)part.p, (double *)res.p, true);
}

kur_status kur_diagnostics_noalloc(kur_ctx *c, double *out)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!out) return fail(c, KUR_EINVAL, "out must not be NULL");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    if (c->batch) return fail(c, KUR_ESTATE, "diagnostics are defined per system, not for a batch");
    if (c->n > kNoAllocMaxN)
        return fail(c, KUR_EINVAL, "kur_diagnostics_noalloc: n = " + std::to_string(c->n) +
                                       " exceeds its fixed scratch (at most " + std::to_string(kNoAllocMaxN) +
                                       " nodes); use kur_diagnostics");
    double *scr = (double *)noalloc_scratch(c->device);
    if (!scr) return fail(c, KUR_EDEVICE, "the fixed scratch of this device could not be located");
    return diag_impl(c, out, scr, scr + noalloc_totals_offset(), false);
}

static hipError_t launch_sample(kur_ctx *c, const int64_t *idx_dev, int64_t idx)
{
    return c->esz == 4
               ? launch_order<float>(c->d_part[c->cur].p, (const int64_t *)c->d_tile_first.p, (const double *)c->d_inv_n.p,
                                     c->n_inst, (double *)c->d_r.p, (double *)c->d_psi.p, idx_dev, idx, c->stream)
               : launch_order<double>(c->d_part[c->cur].p, (const int64_t *)c->d_tile_first.p, (const double *)c->d_inv_n.p,
                                      c->n_inst, (double *)c->d_r.p, (double *)c->d_psi.p, idx_dev, idx, c->stream);
}

// One RK4 step. With rsc/rac (a recording run with option "record_stages"), the stage inputs'
// (sin, cos) are read from and written to rsc[4 s + i - 1] (step s, stage i) instead of the
// context's double buffer, and their row sums go to rac[4 s + i - 1].
static hipError_t launch_step(kur_ctx *c, const DevGraph &g, double dt, char *rsc = nullptr, char *rac = nullptr,
                              int64_t step = 0)
{
    const size_t P = 2 * (size_t)c->esz * (size_t)c->n;
    // stage inputs for the phase gathers: theta (hi), then y2, y3, y4 alternating in two buffers
    void *yin[4] = {c->d_hi.p, c->d_yb[0].p, c->d_yb[1].p, c->d_yb[0].p};
    void *yout[4] = {c->d_yb[0].p, c->d_yb[1].p, c->d_yb[0].p, nullptr};
    for (int stage = 1; stage <= 4; ++stage) {
        hipError_t e;
        const int64_t i = 4 * step + stage;
        if (c->esz == 4) {
            RowArgs<float> a = row_args<float>(c, stage, dt);
            if (rsc) {
                a.sc_in = rsc + (size_t)(i - 1) * P;
                a.sc_out = rsc + (size_t)i * P;
                a.ac_out = rac + (size_t)(i - 1) * P;
            }
            if (c->inter_gather) {
                a.y_in = (const float *)yin[stage - 1];
                a.y_out = (float *)yout[stage - 1];
            }
            e = timed_rows(c, g, &a);
        } else {
            RowArgs<double> a = row_args<double>(c, stage, dt);
            if (rsc) {
                a.sc_in = rsc + (size_t)(i - 1) * P;
                a.sc_out = rsc + (size_t)i * P;
                a.ac_out = rac + (size_t)(i - 1) * P;
            }
            if (c->inter_gather) {
                a.y_in = (const double *)yin[stage - 1];
                a.y_out = (double *)yout[stage - 1];
            }
            e = timed_rows(c, g, &a);
        }
        if (e != hipSuccess) return e;
        c->cur ^= 1;
    }
    if (c->timing && c->ev_used + 16 > 4096) return harvest_events(c);
    return hipSuccess;
}

// Device buffers for nsamp order-parameter samples of every instance: room for at least 256
// samples, grown by powers of two. The captured step graph names these buffers, so runs of
// different lengths keep one graph.
static hipError_t sample_alloc(kur_ctx *c, int64_t nsamp)
{
    int64_t cap = 256;
    while (cap < nsamp) cap *= 2;
    const size_t bytes = sizeof(double) * (size_t)cap * (size_t)c->n_inst;
    hipError_t e = dalloc(c->d_r, bytes);
    if (e == hipSuccess) e = dalloc(c->d_psi, bytes);
    return e;
}

// Capture `period` steps (and, when sampling, the order-parameter kernel with a device-side
// sample index) into one executable graph, reusing the cached one when nothing changed.
static hipError_t step_graph(kur_ctx *c, const DevGraph &g, double dt, int64_t period, bool sample)
{
    kur_ctx::GraphKey key{c->gen, dt, period, sample ? 1 : 0, c->cur, c->d_r.p, c->d_psi.p, c->d_ctr.p};
    if (c->gexec && c->gkey == key) return hipSuccess;
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const int cur0 = c->cur;
    hipError_t le = hipSuccess;
    for (int64_t s = 0; s < period && le == hipSuccess; ++s) le = launch_step(c, g, dt);
    if (le == hipSuccess && sample) {
        le = launch_sample(c, (const int64_t *)c->d_ctr.p, 0);
        if (le == hipSuccess) le = launch_bump((int64_t *)c->d_ctr.p, c->stream);
    }
    c->cur = cur0;  // the capture did not run anything
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->stream, &graph);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->gexec = nullptr;
        return e;
    }
    c->gkey = key;
    return hipSuccess;
}

// Enqueue nsteps RK4 steps with order-parameter samples every r_every steps (all instances).
static kur_status run_steps(kur_ctx *c, double dt, int64_t nsteps, int64_t r_every)
{
    const int64_t nsamp = r_every > 0 ? nsteps / r_every + 1 : 0;
    hipError_t e;
    if (nsamp > 0 && (e = sample_alloc(c, nsamp)) != hipSuccess) return hip_fail(c, e, "r buffer");
    // a small complete graph without kernel timing or a stage record: one launch for the whole
    // run (checkpoints for the adjoint written by the same launch)
    if (c->complete_graph && c->persistent && !c->batch && !(c->ckpt_every > 0 && c->record_stages) && !c->timing &&
        c->n <= (int64_t)kPersistThreads * kPersistMaxRows) {
        const int64_t C = c->ckpt_every;
        void *ck = nullptr;
        if (C > 0) {
            const int64_t nseg = nsteps > 0 ? (nsteps + C - 1) / C : 0;
            c->rec_valid = false;
            c->rec_stages = false;
            if ((e = dalloc(c->d_ck, 2 * (size_t)c->esz * (size_t)c->n * (size_t)std::max<int64_t>(nseg, 1))) !=
                hipSuccess)
                return hip_fail(c, e, "checkpoints");
            dfree(c->d_rsc);  // a previous stage record
            dfree(c->d_rac);
            ck = c->d_ck.p;
        }
        if (nsteps > 0 || r_every > 0) {
            e = c->esz == 4 ? run_persistent<float>(c, dt, nsteps, r_every, (float *)ck, C > 0 ? C : 1)
                            : run_persistent<double>(c, dt, nsteps, r_every, (double *)ck, C > 0 ? C : 1);
            if (e != hipSuccess) return hip_fail(c, e, "persistent rk4 launch");
            c->sc_valid = false;
        }
        if (C > 0) {
            c->rec_valid = true;
            c->rec_stages = false;
            c->rec_dt = dt;
            c->rec_nsteps = nsteps;
            c->rec_C = C;
            c->rec_gen = c->gen;
            c->rec_serial++;
        }
        return KUR_OK;
    }
    if (!c->sc_valid) {
        kur_status s = sc_init(c, c->d_hi.p, c->d_sc[c->cur], c->d_part[c->cur]);
        if (s != KUR_OK) return s;
        c->sc_valid = true;
    }
    const DevGraph g = devgraph(c);
    int64_t done = 0, k = 0;
    if (r_every > 0) {
        if ((e = launch_sample(c, nullptr, 0)) != hipSuccess) return hip_fail(c, e, "order parameter launch");
        k = 1;
    }
    const int64_t period = r_every > 0 ? r_every : std::max<int64_t>(1, c->graph_steps);
    const int64_t reps = nsteps / period;
    const int64_t C = c->batch ? 0 : c->ckpt_every;  // record checkpoints: plain launches
    const bool stages = C > 0 && c->record_stages;
    const size_t P = 2 * (size_t)c->esz * (size_t)c->n;  // bytes of one (sin, cos) or row-sum slot
    if (C > 0) {
        const size_t TN = (size_t)c->esz * (size_t)c->n;
        const int64_t nseg = nsteps > 0 ? (nsteps + C - 1) / C : 0;
        c->rec_valid = false;
        c->rec_stages = false;
        if ((e = dalloc(c->d_ck, 2 * TN * (size_t)std::max<int64_t>(nseg, 1))) != hipSuccess) return hip_fail(c, e, "checkpoints");
        if (!stages) {
            dfree(c->d_rsc);  // a previous stage record
            dfree(c->d_rac);
        } else {
            if ((e = dalloc(c->d_rsc, P * (size_t)(4 * nsteps + 1))) != hipSuccess ||
                (e = dalloc(c->d_rac, P * (size_t)std::max<int64_t>(4 * nsteps, 1))) != hipSuccess) {
                dfree(c->d_rsc);
                dfree(c->d_rac);
                return fail(c, KUR_ENOMEM, "device memory for the stage record (" +
                                               std::to_string((double)P * (8.0 * nsteps + 1) / 1e9) +
                                               " GB): lower nsteps or set record_stages to 0");
            }
            if ((e = hipMemcpyAsync(c->d_rsc.p, c->d_sc[c->cur].p, P, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
                return hip_fail(c, e, "stage record");
        }
    }
    if (C == 0 && c->use_graph && !c->timing && reps >= 2) {
        if (r_every > 0) {
            const int64_t one = 1;
            if ((e = hipMemcpyAsync(c->d_ctr.p, &one, sizeof(one), hipMemcpyHostToDevice, c->stream)) != hipSuccess ||
                (e = hipStreamSynchronize(c->stream)) != hipSuccess)
                return hip_fail(c, e, "sample counter");
        }
        if ((e = step_graph(c, g, dt, period, r_every > 0)) != hipSuccess) return hip_fail(c, e, "step graph");
        for (int64_t i = 0; i < reps; ++i)
            if ((e = hipGraphLaunch(c->gexec, c->stream)) != hipSuccess) return hip_fail(c, e, "step graph launch");
        done = reps * period;  // four stage swaps per step: c->cur is unchanged
        if (r_every > 0) k += reps;
    }
    for (int64_t step = done; step < nsteps; ++step) {
        if (C > 0 && step % C == 0) {
            const size_t TN = (size_t)c->esz * (size_t)c->n;
            char *ck = (char *)c->d_ck.p + (size_t)(step / C) * 2 * TN;
            if ((e = hipMemcpyAsync(ck, c->d_hi.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
                (e = hipMemcpyAsync(ck + TN, c->d_lo.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
                return hip_fail(c, e, "checkpoint copy");
        }
        if ((e = stages ? launch_step(c, g, dt, (char *)c->d_rsc.p, (char *)c->d_rac.p, step) : launch_step(c, g, dt)) !=
            hipSuccess)
            return hip_fail(c, e, "rk4 stage launch");
        if (r_every > 0 && (step + 1) % r_every == 0) {
            if ((e = launch_sample(c, nullptr, k)) != hipSuccess) return hip_fail(c, e, "order parameter launch");
            ++k;
        }
    }
    if (stages && (e = hipMemcpyAsync(c->d_sc[c->cur].p, (char *)c->d_rsc.p + (size_t)(4 * nsteps) * P, P,
                                      hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
        return hip_fail(c, e, "stage record");
    if (C > 0) {
        c->rec_valid = true;
        c->rec_stages = stages;
        c->rec_dt = dt;
        c->rec_nsteps = nsteps;
        c->rec_C = C;
        c->rec_gen = c->gen;
        c->rec_serial++;
    }
    return KUR_OK;
}

static kur_status fetch_samples(kur_ctx *c, int64_t count, double *r_out, double *psi_out)
{
    if (count <= 0 || (!r_out && !psi_out)) return KUR_OK;
    std::vector<double> r(count), p(count);
    hipError_t e = hipMemcpyAsync(r.data(), c->d_r.p, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(p.data(), c->d_psi.p, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "r download");
    if (r_out) std::memcpy(r_out, r.data(), sizeof(double) * count);
    if (psi_out) std::memcpy(psi_out, p.data(), sizeof(double) * count);
    for (int64_t i = 0; i < count; ++i)
        if (!std::isfinite(r[i])) return fail(c, KUR_ENONFINITE, "non-finite order parameter (phases are not finite)");
    return KUR_OK;
}

kur_status kur_step_rk4(kur_ctx *c, double dt, int64_t nsteps, int64_t r_every, double *r_out, double *psi_out)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!std::isfinite(dt) || dt == 0.0) return fail(c, KUR_EINVAL, "dt must be finite and nonzero");
    if (nsteps < 0 || r_every < 0) return fail(c, KUR_EINVAL, "nsteps and r_every must be >= 0");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    if (c->batch && r_every > 0 && (r_out || psi_out))
        return fail(c, KUR_EINVAL, "a batch samples per instance: use kur_batch_step");
    s = run_steps(c, dt, nsteps, r_every);
    if (s != KUR_OK) return s;
    return fetch_samples(c, r_every > 0 ? nsteps / r_every + 1 : 0, r_out, psi_out);
}

// Implicit midpoint rule by fixed-point iteration on the midpoint Y: Y_0 = theta_n,
// Y_i = theta_n + dt/2 F(Y_{i-1}) for i < iters, theta_{n+1} = theta_n + dt F(Y_{iters-1}).
// One row-kernel launch per iteration (stage 5, the last one stage 6).
static kur_status run_midpoint(kur_ctx *c, double dt, int64_t nsteps, int32_t iters, int64_t r_every)
{
    const int64_t nsamp = r_every > 0 ? nsteps / r_every + 1 : 0;
    hipError_t e;
    if (nsamp > 0 && (e = sample_alloc(c, nsamp)) != hipSuccess) return hip_fail(c, e, "r buffer");
    if (!c->sc_valid) {
        kur_status s = sc_init(c, c->d_hi.p, c->d_sc[c->cur], c->d_part[c->cur]);
        if (s != KUR_OK) return s;
        c->sc_valid = true;
    }
    const DevGraph g = devgraph(c);
    int64_t k = 0;
    if (r_every > 0 && (e = launch_sample(c, nullptr, k++)) != hipSuccess) return hip_fail(c, e, "order parameter launch");
    for (int64_t step = 0; step < nsteps; ++step) {
        for (int32_t it = 1; it <= iters; ++it) {
            const int stage = it < iters ? 5 : 6;
            if (c->esz == 4) {
                RowArgs<float> a = row_args<float>(c, stage, dt);
                e = timed_rows(c, g, &a);
            } else {
                RowArgs<double> a = row_args<double>(c, stage, dt);
                e = timed_rows(c, g, &a);
            }
            if (e != hipSuccess) return hip_fail(c, e, "midpoint launch");
            c->cur ^= 1;
        }
        if (c->timing && c->ev_used + 2 * (size_t)iters > 4096 && (e = harvest_events(c)) != hipSuccess)
            return hip_fail(c, e, "timing");
        if (r_every > 0 && (step + 1) % r_every == 0 && (e = launch_sample(c, nullptr, k++)) != hipSuccess)
            return hip_fail(c, e, "order parameter launch");
    }
    return KUR_OK;
}

kur_status kur_step_midpoint(kur_ctx *c, double dt, int64_t nsteps, int32_t iters, int64_t r_every, double *r_out,
                             double *psi_out)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!std::isfinite(dt) || dt == 0.0) return fail(c, KUR_EINVAL, "dt must be finite and nonzero");
    if (nsteps < 0 || r_every < 0) return fail(c, KUR_EINVAL, "nsteps and r_every must be >= 0");
    if (iters < 1 || iters > 64) return fail(c, KUR_EINVAL, "iters must be in [1, 64]");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    if (c->batch && r_every > 0 && (r_out || psi_out))
        return fail(c, KUR_EINVAL, "a batch samples per instance: use kur_batch_step");
    s = run_midpoint(c, dt, nsteps, iters, r_every);
    if (s != KUR_OK) return s;
    return fetch_samples(c, r_every > 0 ? nsteps / r_every + 1 : 0, r_out, psi_out);
}

}  // extern "C"

// Fehlberg's embedded Runge-Kutta pair of orders 4 and 5 (E. Fehlberg, NASA TR R-315, 1969):
// stage inputs Y_{i+1} = theta + dt sum_j kAemb[i][j] k_j, the order-4 weights propagate the
// solution and the order-5 weights estimate its local error.
static const double kAemb[5][5] = {
    {1.0 / 4.0, 0, 0, 0, 0},
    {3.0 / 32.0, 9.0 / 32.0, 0, 0, 0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0, 0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0},
};
static const double kB4emb[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0, -1.0 / 5.0, 0.0};
static const double kB5emb[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0, -9.0 / 50.0, 2.0 / 55.0};

template <typename T>
static kur_status adaptive_impl(kur_ctx *c, double t_end, double dt0, double atol, int64_t max_steps, double *out)
{
    const int64_t n = c->n;
    const size_t TN = sizeof(T) * (size_t)n;
    DevBuf kbuf, hi2, lo2, wind2, errp, errv;
    struct Release {
        DevBuf *b[6];
        ~Release()
        {
            for (DevBuf *x : b) dfree(*x);
        }
    } rel{{&kbuf, &hi2, &lo2, &wind2, &errp, &errv}};
    hipError_t e;
    if ((e = dalloc(kbuf, 6 * TN)) != hipSuccess || (e = dalloc(hi2, TN)) != hipSuccess ||
        (e = dalloc(lo2, TN)) != hipSuccess || (e = dalloc(wind2, 4 * (size_t)n)) != hipSuccess ||
        (e = dalloc(errp, sizeof(T) * (size_t)std::max(1, c->ntiles))) != hipSuccess ||
        (e = dalloc(errv, sizeof(T))) != hipSuccess)
        return hip_fail(c, e, "adaptive buffers");
    const DevGraph g = devgraph(c);
    double t = 0.0, dt = std::min(dt0, t_end);
    int64_t acc = 0, rej = 0;
    while (t < t_end && acc + rej < max_steps) {
        const double h = std::min(dt, t_end - t);
        if (!c->sc_valid) {
            kur_status s = sc_init(c, c->d_hi.p, c->d_sc[c->cur], c->d_part[c->cur]);
            if (s != KUR_OK) return s;
            c->sc_valid = true;
        }
        for (int stage = 1; stage <= 6; ++stage) {
            EmbArgs<T> a{};
            a.stage = stage;
            a.nstages = 6;
            a.compensate = c->compensate;
            a.dt = (T)h;
            a.K = (T)c->K;
            a.inv_n = (T)(1.0 / (double)n);
            a.unit = (const T *)c->d_unit.p;
            a.omega = (const T *)c->d_omega.p;
            a.hi = (const T *)c->d_hi.p;
            a.lo = (const T *)c->d_lo.p;
            a.wind = (const int32_t *)c->d_wind.p;
            a.hi_new = (T *)hi2.p;
            a.lo_new = (T *)lo2.p;
            a.wind_new = (int32_t *)wind2.p;
            a.kbuf = (T *)kbuf.p;
            a.n = n;
            for (int j = 0; j < 6; ++j) {
                a.coef[j] = (T)(stage < 6 ? (j < 5 ? kAemb[stage - 1][j] : 0.0) : kB4emb[j]);
                a.coef2[j] = (T)(kB5emb[j] - kB4emb[j]);
            }
            a.err_part = (T *)errp.p;
            a.sc_in = c->d_sc[c->cur].p;
            a.part_in = c->d_part[c->cur].p;
            a.sc_out = c->d_sc[c->cur ^ 1].p;
            a.part_out = c->d_part[c->cur ^ 1].p;
            if ((e = launch_emb<T>(g, a, c->threads, c->stream)) != hipSuccess) return hip_fail(c, e, "adaptive stage launch");
            c->cur ^= 1;
        }
        T err_dev;
        if ((e = launch_max_fold<T>(std::max(1, c->ntiles), (const T *)errp.p, (T *)errv.p, c->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(&err_dev, errv.p, sizeof(T), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess)
            return hip_fail(c, e, "adaptive error estimate");
        const double errn = (double)err_dev / atol;
        if (!std::isfinite(errn)) {
            c->sc_valid = false;
            return fail(c, KUR_ENONFINITE, "non-finite local error estimate");
        }
        if (errn <= 1.0) {
            // accept: the candidate becomes the state; sc of the current parity already holds
            // its (sin, cos) and block partials
            if ((e = hipMemcpyAsync(c->d_hi.p, hi2.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
                (e = hipMemcpyAsync(c->d_lo.p, lo2.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
                (e = hipMemcpyAsync(c->d_wind.p, wind2.p, 4 * (size_t)n, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
                return hip_fail(c, e, "adaptive accept");
            t = h == t_end - t ? t_end : t + h;  // a step clamped to the end lands on it
            ++acc;
        } else {
            ++rej;
            c->sc_valid = false;  // the stages overwrote the (sin, cos) of the state
        }
        const double fac = errn == 0.0 ? 4.0 : std::min(4.0, std::max(0.2, 0.9 * std::pow(errn, -0.2)));
        dt = h * fac;
    }
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_fail(c, e, "adaptive sync");
    out[0] = t;
    out[1] = dt;
    out[2] = (double)acc;
    out[3] = (double)rej;
    return KUR_OK;
}

extern "C" {

kur_status kur_step_adaptive(kur_ctx *c, double t_end, double dt0, double atol, int64_t max_steps, double *out)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!out) return fail(c, KUR_EINVAL, "out must not be NULL");
    if (!(std::isfinite(t_end) && t_end > 0.0) || !(std::isfinite(dt0) && dt0 > 0.0) || !(std::isfinite(atol) && atol > 0.0))
        return fail(c, KUR_EINVAL, "t_end, dt0 and atol must be finite and positive");
    if (max_steps < 1) return fail(c, KUR_EINVAL, "max_steps must be >= 1");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    return c->esz == 4 ? adaptive_impl<float>(c, t_end, dt0, atol, max_steps, out)
                       : adaptive_impl<double>(c, t_end, dt0, atol, max_steps, out);
}

kur_status kur_get_phases(kur_ctx *c, double *theta, int wrapped)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!theta) return fail(c, KUR_EINVAL, "theta must not be NULL");
    kur_status s = need_ready(c, false, true);
    if (s != KUR_OK) return s;
    const int64_t n = c->n;
    std::vector<int32_t> wind(n);
    std::vector<double> hi(n), lo(n);
    hipError_t e;
    if (c->esz == 4) {
        std::vector<float> h(n), l(n);
        e = hipMemcpyAsync(h.data(), c->d_hi.p, 4 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(l.data(), c->d_lo.p, 4 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(wind.data(), c->d_wind.p, 4 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        for (int64_t m = 0; m < n; ++m) {
            hi[m] = h[m];
            lo[m] = l[m];
        }
    } else {
        e = hipMemcpyAsync(hi.data(), c->d_hi.p, 8 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(lo.data(), c->d_lo.p, 8 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(wind.data(), c->d_wind.p, 4 * n, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "phase download");
    const double P1 = two_pi_p1(c->esz), P2 = two_pi_p2(c->esz);
    for (int64_t u = 0; u < n; ++u) {
        const int64_t m = c->perm[u];
        double x = hi[m] + lo[m];
        if (wrapped) {
            x = std::remainder(x, 2.0 * kPi);
            if (x >= kPi) x -= 2.0 * kPi;
        } else {
            x += (double)wind[m] * P1 + (double)wind[m] * P2;
        }
        theta[u] = x;
    }
    return KUR_OK;
}

kur_status kur_get_phases_dev(kur_ctx *c, void *theta_dev, int wrapped)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!theta_dev) return fail(c, KUR_EINVAL, "theta_dev must not be NULL");
    kur_status s = need_ready(c, false, true);
    if (s != KUR_OK) return s;
    const int32_t *perm = (const int32_t *)c->d_perm.p;
    const double P1 = two_pi_p1(c->esz), P2 = two_pi_p2(c->esz);
    const int w = wrapped ? 1 : 0;
    hipError_t e = c->esz == 4 ? launch_phase_out_user<float>(c->n, perm, c->d_hi.p, c->d_lo.p, (const int32_t *)c->d_wind.p, w, P1, P2, theta_dev, c->stream)
                               : launch_phase_out_user<double>(c->n, perm, c->d_hi.p, c->d_lo.p, (const int32_t *)c->d_wind.p, w, P1, P2, theta_dev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "phase launch");
    return KUR_OK;
}

kur_status kur_order_parameter(kur_ctx *c, double *r, double *psi)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!r || !psi) return fail(c, KUR_EINVAL, "r and psi must not be NULL");
    kur_status s = need_ready(c, false, true);
    if (s != KUR_OK) return s;
    if (!c->sc_valid) {
        s = sc_init(c, c->d_hi.p, c->d_sc[c->cur], c->d_part[c->cur]);
        if (s != KUR_OK) return s;
        c->sc_valid = true;
    }
    hipError_t e;
    const size_t need = sizeof(double) * (size_t)c->n_inst;
    if ((e = dalloc(c->d_r, std::max(need, c->d_r.bytes))) != hipSuccess ||
        (e = dalloc(c->d_psi, std::max(need, c->d_psi.bytes))) != hipSuccess)
        return hip_fail(c, e, "r buffer");
    if ((e = launch_sample(c, nullptr, 0)) != hipSuccess) return hip_fail(c, e, "order parameter launch");
    std::vector<double> rv(c->n_inst), pv(c->n_inst);
    s = fetch_samples(c, c->n_inst, rv.data(), pv.data());
    *r = rv[0];
    *psi = pv[0];
    return s;
}

struct StateHeader {
    char magic[4];
    int32_t version;
    int32_t esz;
    int32_t pad;
    int64_t n;
};

kur_status kur_get_state(kur_ctx *c, void *blob, size_t *bytes)
{
    if (!c || !bytes) return KUR_EINVAL;
    c->err.clear();
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    const size_t need = sizeof(StateHeader) + (size_t)c->n * (2 * c->esz + 4);
    if (!blob) {
        *bytes = need;
        return KUR_OK;
    }
    if (*bytes < need) return fail(c, KUR_EINVAL, "state buffer too small");
    kur_status s = need_ready(c, false, true);
    if (s != KUR_OK) return s;
    StateHeader h = {{'K', 'U', 'R', 'S'}, 1, c->esz, 0, c->n};
    char *p = (char *)blob;
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    hipError_t e = hipMemcpyAsync(p, c->d_hi.p, (size_t)c->n * c->esz, hipMemcpyDeviceToHost, c->stream);
    p += (size_t)c->n * c->esz;
    if (e == hipSuccess) e = hipMemcpyAsync(p, c->d_lo.p, (size_t)c->n * c->esz, hipMemcpyDeviceToHost, c->stream);
    p += (size_t)c->n * c->esz;
    if (e == hipSuccess) e = hipMemcpyAsync(p, c->d_wind.p, (size_t)c->n * 4, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state download");
    *bytes = need;
    return KUR_OK;
}

kur_status kur_set_state(kur_ctx *c, const void *blob, size_t bytes)
{
    if (!c || !blob) return KUR_EINVAL;
    c->err.clear();
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    const size_t need = sizeof(StateHeader) + (size_t)c->n * (2 * c->esz + 4);
    StateHeader h;
    if (bytes < sizeof(h)) return fail(c, KUR_EINVAL, "state blob too small");
    std::memcpy(&h, blob, sizeof(h));
    if (std::memcmp(h.magic, "KURS", 4) != 0 || h.version != 1 || h.esz != c->esz || h.n != c->n || bytes != need)
        return fail(c, KUR_EINVAL, "state blob does not match this context (dtype, n or format)");
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    const char *p = (const char *)blob + sizeof(h);
    hipError_t e;
    if ((e = upload(c->d_hi, p, (size_t)c->n * c->esz, c->stream)) != hipSuccess ||
        (e = upload(c->d_lo, p + (size_t)c->n * c->esz, (size_t)c->n * c->esz, c->stream)) != hipSuccess ||
        (e = upload(c->d_wind, p + (size_t)2 * c->n * c->esz, (size_t)c->n * 4, c->stream)) != hipSuccess)
        return hip_fail(c, e, "state upload");
    c->has_phases = true;
    c->sc_valid = false;
    return KUR_OK;
}

kur_status kur_sync(kur_ctx *c)
{
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    return KUR_OK;
}

kur_status kur_kernel_time(kur_ctx *c, int64_t *launches, double *total_ms)
{
    if (!c || !launches || !total_ms) return KUR_EINVAL;
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    hipError_t e = harvest_events(c);
    if (e != hipSuccess) return hip_fail(c, e, "timing");
    *launches = c->t_launches;
    *total_ms = c->t_ms;
    return KUR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------------
// Discrete adjoint of kur_step_rk4 with checkpointing
// ------------------------------------------------------------------------------------------------

namespace {


// Inputs and outputs of one adjoint call, all in user order: host FP64 arrays, or (dev) device
// arrays of the context type.
struct AdjIO {
    bool dev = false;
    const double *theta0_host = nullptr;  // start of the forward run (host calls)
    const void *theta0_dev = nullptr;     // start of the forward run (device calls)
    const double *seed_host = nullptr;    // dL/dtheta(T)
    const void *seed_dev = nullptr;
    double *gt_host = nullptr, *gw_host = nullptr, *gk_host = nullptr;
    void *gt_dev = nullptr, *gw_dev = nullptr, *gk_dev = nullptr;
};

// The forward run starts at io's theta0, or at the context's current phases when neither is
// given; ck_ext: device checkpoints recorded by kur_step_rk4 instead (then the forward pass is
// not run here and theta0 is unused).
// rec_sc, rec_ac: the stage record of that run (option "record_stages"), or null: then no
// segment is recomputed and the reverse sweep reads the recorded stage states.
template <typename T>
kur_status adjoint_impl(kur_ctx *c, const AdjIO &io, const void *ck_ext, double dt, int64_t nsteps, int64_t C,
                        const void *rec_sc = nullptr, const void *rec_ac = nullptr)
{
    using std::vector;
    const int64_t n = c->n;
    const int nt = c->ntiles;
    const size_t TN = sizeof(T) * (size_t)n;
    hipStream_t st = c->stream;
    const bool stored = rec_sc != nullptr;
    if (stored) C = std::max<int64_t>(nsteps, 1);  // one segment: the whole recorded run
    const int64_t nseg = nsteps > 0 ? (nsteps + C - 1) / C : 0;
    const int64_t nslot = stored ? 1 : 4 * std::min<int64_t>(C, std::max<int64_t>(nsteps, 1)) + 1;
    // asymmetric A: the Jacobian-transpose gathers run over the layout of A^T (its own tiles)
    const bool asym = !c->symmetric;
    const int ntv = asym ? c->ntT : nt;
    // small complete graphs: the whole adjoint in one workgroup per launch (k_persist_adjoint),
    // with the forward pass in the one-workgroup RK4 run; dK partials per thread of it
    const bool pers = c->complete_graph && c->persistent && n <= (int64_t)kPersistThreads * kPersistMaxRows && !stored;
    const int ngk = pers ? kPersistThreads : ntv;
    AdjBufs &B = c->adj;
    hipError_t e;
    if ((e = dalloc(B.hi, TN)) != hipSuccess || (e = dalloc(B.lo, TN)) != hipSuccess ||
        (e = dalloc(B.wind, 4 * (size_t)n)) != hipSuccess || (e = dalloc(B.ksum, TN)) != hipSuccess ||
        (!ck_ext && (e = dalloc(B.ck, 2 * TN * (size_t)std::max<int64_t>(nseg, 1))) != hipSuccess) ||
        (e = dalloc(B.slots, 2 * TN * (size_t)nslot)) != hipSuccess ||
        (e = dalloc(B.acs, 2 * TN * (size_t)(nslot - 1))) != hipSuccess ||
        (e = dalloc(B.fpart[0], 2 * sizeof(T) * nt)) != hipSuccess || (e = dalloc(B.fpart[1], 2 * sizeof(T) * nt)) != hipSuccess ||
        (e = dalloc(B.x[0], 2 * TN)) != hipSuccess || (e = dalloc(B.x[1], 2 * TN)) != hipSuccess ||
        (e = dalloc(B.xpart[0], 2 * sizeof(T) * ntv)) != hipSuccess || (e = dalloc(B.xpart[1], 2 * sizeof(T) * ntv)) != hipSuccess ||
        (e = dalloc(B.lam, TN)) != hipSuccess || (e = dalloc(B.lam_acc, TN)) != hipSuccess ||
        (e = dalloc(B.lbuf, TN)) != hipSuccess || (e = dalloc(B.gom, 8 * (size_t)n)) != hipSuccess ||
        (e = dalloc(B.gk, 8 * (size_t)ngk)) != hipSuccess)
        return hip_fail(c, e, "adjoint buffers");

    // initial phases (block order), split as in kur_set_phases; the seed dL/dtheta(T)
    {
        const double P1 = two_pi_p1(c->esz), P2 = two_pi_p2(c->esz);
        const bool from_state = !ck_ext && !io.theta0_host && !io.theta0_dev;
        if (from_state &&
            ((e = hipMemcpyAsync(B.hi.p, c->d_hi.p, TN, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
             (e = hipMemcpyAsync(B.lo.p, c->d_lo.p, TN, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
             (e = hipMemcpyAsync(B.wind.p, c->d_wind.p, 4 * n, hipMemcpyDeviceToDevice, st)) != hipSuccess))
            return hip_fail(c, e, "adjoint start state");
        if (io.dev) {
            if (!ck_ext && io.theta0_dev &&
                (e = launch_phase_in<T>(n, (const int32_t *)c->d_perm.p, io.theta0_dev, P1, P2, B.hi.p, B.lo.p,
                                        (int32_t *)B.wind.p, st)) != hipSuccess)
                return hip_fail(c, e, "adjoint start phases");
            if ((e = launch_scatter_in<T>(n, (const int32_t *)c->d_perm.p, io.seed_dev, B.lam.p, st)) != hipSuccess)
                return hip_fail(c, e, "adjoint seed");
        } else {
            const bool up = !ck_ext && io.theta0_host;
            vector<T> hi(up ? n : 0), lo(up ? n : 0), lam(n);
            vector<int32_t> wind(up ? n : 0);
            for (int64_t u = 0; u < n; ++u) {
                const int64_t m = c->perm[u];
                lam[m] = (T)io.seed_host[u];
                if (!up) continue;
                const double th = io.theta0_host[u];
                const double q = std::nearbyint(th / (2.0 * kPi));
                const double red = (th - q * P1) - q * P2;
                hi[m] = (T)red;
                lo[m] = (T)(red - (double)hi[m]);
                wind[m] = (int32_t)q;
            }
            if ((up && ((e = hipMemcpyAsync(B.hi.p, hi.data(), TN, hipMemcpyHostToDevice, st)) != hipSuccess ||
                        (e = hipMemcpyAsync(B.lo.p, lo.data(), TN, hipMemcpyHostToDevice, st)) != hipSuccess ||
                        (e = hipMemcpyAsync(B.wind.p, wind.data(), 4 * n, hipMemcpyHostToDevice, st)) != hipSuccess)) ||
                (e = hipMemcpyAsync(B.lam.p, lam.data(), TN, hipMemcpyHostToDevice, st)) != hipSuccess ||
                (e = hipStreamSynchronize(st)) != hipSuccess)
                return hip_fail(c, e, "adjoint upload");
        }
        // a recompute from recorded checkpoints restores (hi, lo) only: its winding counts start at 0
        if ((ck_ext && (e = hipMemsetAsync(B.wind.p, 0, 4 * (size_t)n, st)) != hipSuccess) ||
            (e = hipMemsetAsync(B.gom.p, 0, 8 * (size_t)n, st)) != hipSuccess ||
            (e = hipMemsetAsync(B.gk.p, 0, 8 * (size_t)ngk, st)) != hipSuccess)
            return hip_fail(c, e, "adjoint clear");
    }
    if (pers && nsteps > 0) {
        // forward: launches of at most about 65536 steps, checkpoints every C steps
        if (!ck_ext) {
            PersistArgs<T> a;
            a.n = n;
            a.r_every = 0;
            a.final_sample = 0;
            a.compensate = c->compensate;
            a.dt = (T)dt;
            a.half_dt = (T)(0.5 * dt);
            a.dt6 = (T)(dt / 6.0);
            a.K = (T)c->K;
            a.inv_n = (T)(1.0 / (double)n);
            a.unit = (const T *)c->d_unit.p;
            a.omega = (const T *)c->d_omega.p;
            a.hi = (T *)B.hi.p;
            a.lo = (T *)B.lo.p;
            a.wind = (int32_t *)B.wind.p;
            a.r_out = a.psi_out = nullptr;
            a.ck = (T *)B.ck.p;
            a.ck_every = C;
            const int64_t chunk = std::max<int64_t>(1, 65536 / C) * C;
            for (int64_t done = 0; done < nsteps; done += chunk) {
                a.step0 = done;
                a.nsteps = std::min(chunk, nsteps - done);
                if ((e = launch_persist_complete<T>(a, st)) != hipSuccess) return hip_fail(c, e, "adjoint forward");
            }
        }
        // reverse: launches of whole segments, at most about 65536 steps each
        PersistAdjArgs<T> v;
        v.n = n;
        v.nsteps = nsteps;
        v.ck_every = C;
        v.compensate = c->compensate;
        v.dt = (T)dt;
        v.half_dt = (T)(0.5 * dt);
        v.dt6 = (T)(dt / 6.0);
        v.dt3 = (T)(dt / 3.0);
        v.K = (T)c->K;
        v.inv_n = (T)(1.0 / (double)n);
        v.unit = (const T *)c->d_unit.p;
        v.omega = (const T *)c->d_omega.p;
        v.ck = ck_ext ? (const T *)ck_ext : (const T *)B.ck.p;
        v.ystore = (T *)B.slots.p;
        v.lam = (T *)B.lam.p;
        v.g_omega = (double *)B.gom.p;
        v.gk_part = (double *)B.gk.p;
        const int64_t per = std::max<int64_t>(1, 65536 / C);
        for (int64_t hi = nseg - 1; hi >= 0; hi -= per) {
            v.seg_hi = hi;
            v.seg_lo = std::max<int64_t>(0, hi - per + 1);
            if ((e = launch_persist_adjoint<T>(v, st)) != hipSuccess) return hip_fail(c, e, "adjoint reverse");
        }
    }
    const DevGraph g = devgraph(c);
    const DevGraph gv = asym ? devgraph_t(c) : g;  // layout of the Jacobian-transpose gathers
    auto rows = [&](int stage, const void *sc_in, const void *p_in, void *sc_out, void *p_out,
                    void *ac_out) -> hipError_t {
        RowArgs<T> a = row_args<T>(c, stage, dt);
        a.hi = (T *)B.hi.p;
        a.lo = (T *)B.lo.p;
        a.wind = (int32_t *)B.wind.p;
        a.ksum = (T *)B.ksum.p;
        a.sc_in = sc_in;
        a.part_in = p_in;
        a.sc_out = sc_out;
        a.part_out = p_out;
        a.ac_out = ac_out;
        return launch_rows<T>(g, nt, a, c->threads, st);
    };
    auto slot = [&](int64_t i) -> void * {
        return (stored ? (char *)rec_sc : (char *)B.slots.p) + (size_t)i * 2 * TN;
    };
    auto acslot = [&](int64_t i) -> void * {
        return (stored ? (char *)rec_ac : (char *)B.acs.p) + (size_t)i * 2 * TN;
    };

    const char *ckbase = ck_ext ? (const char *)ck_ext : (const char *)B.ck.p;
    // forward pass, keeping (hi, lo) every C steps (unless recorded by the caller's run)
    if (nsteps > 0 && !ck_ext && !pers) {
        int cur = 0;
        if ((e = launch_sc_init<T>(g, nt, (const T *)B.hi.p, slot(0), B.fpart[0].p, c->threads, st)) != hipSuccess)
            return hip_fail(c, e, "adjoint forward");
        void *fsc[2] = {slot(0), slot(1)};
        for (int64_t step = 0; step < nsteps; ++step) {
            if (step % C == 0) {
                char *ck = (char *)B.ck.p + (size_t)(step / C) * 2 * TN;
                if ((e = hipMemcpyAsync(ck, B.hi.p, TN, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
                    (e = hipMemcpyAsync(ck + TN, B.lo.p, TN, hipMemcpyDeviceToDevice, st)) != hipSuccess)
                    return hip_fail(c, e, "adjoint checkpoint");
            }
            for (int stage = 1; stage <= 4; ++stage) {
                if ((e = rows(stage, fsc[cur], B.fpart[cur].p, fsc[cur ^ 1], B.fpart[cur ^ 1].p, nullptr)) != hipSuccess)
                    return hip_fail(c, e, "adjoint forward");
                cur ^= 1;
            }
        }
    }

    // reverse sweep, segment by segment
    const T tdt = (T)dt;
    // recompute a segment of len steps from (hi, lo), keeping (sin, cos) of every stage state and
    // its row sums (A sin, A cos): Y_i of step k at slot 4k+i-1
    auto recompute = [&](int64_t len) -> hipError_t {
        hipError_t r = launch_sc_init<T>(g, nt, (const T *)B.hi.p, slot(0), B.fpart[0].p, c->threads, st);
        int cur = 0;
        for (int64_t k = 0; k < len && r == hipSuccess; ++k)
            for (int stage = 1; stage <= 4 && r == hipSuccess; ++stage) {
                const int64_t i = 4 * k + stage;
                r = rows(stage, slot(i - 1), B.fpart[cur].p, slot(i), B.fpart[cur ^ 1].p, acslot(i - 1));
                cur ^= 1;
            }
        return r;
    };
    // the reverse steps len-1 .. 0 of a segment (slots as above)
    auto sweep = [&](int64_t len) -> hipError_t {
        hipError_t r = hipSuccess;
        for (int64_t k = len - 1; k >= 0 && r == hipSuccess; --k) {
            VjpArgs<T> v;
            v.K = (T)c->K;
            v.inv_n = (T)(1.0 / (double)n);
            v.unit = (const T *)c->d_unit.p;
            v.lam = (T *)B.lam.p;
            v.lam_acc = (T *)B.lam_acc.p;
            v.lbuf = (T *)B.lbuf.p;
            v.g_omega = (double *)B.gom.p;
            v.gk_part = (double *)B.gk.p;
            int xc = 0;
            v.stage = 4;
            v.cl = (T)(dt / 6.0);
            v.cm = T(0);
            v.sc_next = slot(4 * k + 3);
            v.sc_cur = nullptr;
            v.ac_rows = nullptr;
            v.x_in = nullptr;
            v.part_in = nullptr;
            v.x_out = B.x[0].p;
            v.part_out = B.xpart[0].p;
            // the first step of the segment starts here; every later one was started by the
            // stage-1 launch of the step before it (same arithmetic, one launch less per step)
            if (k == len - 1) r = launch_vjp_init<T>(gv, ntv, v, c->threads, st);
            for (int i = 4; i >= 1 && r == hipSuccess; --i) {
                v.stage = i;
                // l_{i-1} = cl lam + cm mu_i: (dt/3, dt), (dt/3, dt/2), (dt/6, dt/2)
                v.cl = i == 4 ? (T)(dt / 3.0) : i == 3 ? (T)(dt / 3.0) : (T)(dt / 6.0);
                v.cm = i == 4 ? tdt : (T)(0.5 * dt);
                v.sc_cur = slot(4 * k + i - 1);
                v.ac_rows = acslot(4 * k + i - 1);
                v.sc_next = i > 1 ? slot(4 * k + i - 2) : k > 0 ? slot(4 * (k - 1) + 3) : nullptr;
                v.x_in = B.x[xc].p;
                v.part_in = B.xpart[xc].p;
                v.x_out = B.x[xc ^ 1].p;
                v.part_out = B.xpart[xc ^ 1].p;
                r = launch_vjp<T>(gv, ntv, v, c->threads, st);
                xc ^= 1;
            }
        }
        return r;
    };
    for (int64_t seg = pers ? -1 : nseg - 1; seg >= 0; --seg) {
        const int64_t s0 = seg * C, len = std::min<int64_t>(C, nsteps - s0);
        if (!stored) {
            const char *ck = ckbase + (size_t)seg * 2 * TN;
            if ((e = hipMemcpyAsync(B.hi.p, ck, TN, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
                (e = hipMemcpyAsync(B.lo.p, ck + TN, TN, hipMemcpyDeviceToDevice, st)) != hipSuccess)
                return hip_fail(c, e, "adjoint restore");
            if ((e = recompute(len)) != hipSuccess) return hip_fail(c, e, "adjoint recompute");
        }
        if ((e = sweep(len)) != hipSuccess) return hip_fail(c, e, "adjoint stage");
    }

    // results
    if (io.dev) {
        const int32_t *perm = (const int32_t *)c->d_perm.p;
        if ((io.gt_dev && (e = launch_gather_out<T, T>(n, perm, B.lam.p, io.gt_dev, st)) != hipSuccess) ||
            (io.gw_dev && (e = launch_gather_out<double, T>(n, perm, B.gom.p, io.gw_dev, st)) != hipSuccess) ||
            (io.gk_dev && (e = launch_fold_sum<T>(ngk, (const double *)B.gk.p, io.gk_dev, st)) != hipSuccess))
            return hip_fail(c, e, "adjoint results");
    } else {
        vector<T> lam(n);
        vector<double> gom(n), gk(ngk);
        if ((e = hipMemcpyAsync(lam.data(), B.lam.p, TN, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(gom.data(), B.gom.p, 8 * (size_t)n, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipMemcpyAsync(gk.data(), B.gk.p, 8 * (size_t)ngk, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(c, e, "adjoint download");
        for (int64_t u = 0; u < n; ++u) {
            if (io.gt_host) io.gt_host[u] = (double)lam[c->perm[u]];
            if (io.gw_host) io.gw_host[u] = gom[c->perm[u]];
        }
        if (io.gk_host) {
            double t = 0.0;
            for (int i = 0; i < ngk; ++i) t += gk[i];
            *io.gk_host = t;
        }
    }
    if (!c->adjoint_keep) {
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(c, e, "adjoint");
        free_adj(B);
    }
    return KUR_OK;
}

// Validation shared by the adjoint calls (host-side; nothing is enqueued).
kur_status adjoint_check(kur_ctx *c)
{
    if (!c->symmetric && !c->has_T)
        return fail(c, KUR_EINVAL, "the adjoint of an asymmetric adjacency needs its transposed layout: set option "
                                   "\"transpose\" to 1 before kur_set_graph_csr / kur_set_graph_csr_w");
    if (c->batch) return fail(c, KUR_EINVAL, "the adjoint of a batch is not supported");
    if (rows_lds_bytes(c->esz, c->W, c->symmetric ? c->tile_rows : c->tile_rowsT, c->threads) > 156 * 1024)
        return fail(c, KUR_EINVAL, "chunk/tile_rows of the transposed layout exceed the LDS of a workgroup");
    return KUR_OK;
}

kur_status adjoint_run(kur_ctx *c, const AdjIO &io, double dt, int64_t nsteps, int64_t ckpt_every)
{
    const int64_t C = std::min<int64_t>(ckpt_every, std::max<int64_t>(nsteps, 1));
    try {
        return c->esz == 4 ? adjoint_impl<float>(c, io, nullptr, dt, nsteps, C)
                           : adjoint_impl<double>(c, io, nullptr, dt, nsteps, C);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in the adjoint");
    }
}

kur_status adjoint_run_recorded(kur_ctx *c, const AdjIO &io)
{
    if (!c->rec_valid || c->rec_gen != c->gen)
        return fail(c, KUR_ESTATE, "no checkpoints recorded by kur_step_rk4 for the current graph, omega and K");
    try {
        const void *rsc = c->rec_stages ? c->d_rsc.p : nullptr, *rac = c->rec_stages ? c->d_rac.p : nullptr;
        return c->esz == 4 ? adjoint_impl<float>(c, io, c->d_ck.p, c->rec_dt, c->rec_nsteps, c->rec_C, rsc, rac)
                           : adjoint_impl<double>(c, io, c->d_ck.p, c->rec_dt, c->rec_nsteps, c->rec_C, rsc, rac);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in the adjoint");
    }
}

}  // namespace

extern "C" kur_status kur_adjoint_rk4(kur_ctx *c, const double *theta0, double dt, int64_t nsteps, int64_t ckpt_every,
                                      const double *dl_dthetaT, double *g_theta0, double *g_omega, double *g_K)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!std::isfinite(dt) || dt == 0.0) return fail(c, KUR_EINVAL, "dt must be finite and nonzero");
    if (nsteps < 0 || ckpt_every < 1) return fail(c, KUR_EINVAL, "nsteps must be >= 0 and ckpt_every >= 1");
    if (!dl_dthetaT) return fail(c, KUR_EINVAL, "dl_dthetaT must not be NULL");
    kur_status s = need_ready(c, true, theta0 == nullptr);
    if (s != KUR_OK) return s;
    if ((s = adjoint_check(c)) != KUR_OK) return s;
    for (int64_t u = 0; u < c->n; ++u)
        if ((theta0 && (!std::isfinite(theta0[u]) || std::fabs(theta0[u]) > 1e9)) || !std::isfinite(dl_dthetaT[u]))
            return fail(c, KUR_EINVAL, "theta0 and dl_dthetaT must be finite (|theta0| <= 1e9)");
    AdjIO io;
    io.theta0_host = theta0;
    io.seed_host = dl_dthetaT;
    io.gt_host = g_theta0;
    io.gw_host = g_omega;
    io.gk_host = g_K;
    return adjoint_run(c, io, dt, nsteps, ckpt_every);
}

extern "C" kur_status kur_adjoint_rk4_dev(kur_ctx *c, const void *theta0_dev, double dt, int64_t nsteps,
                                          int64_t ckpt_every, const void *dl_dthetaT_dev, void *g_theta0_dev,
                                          void *g_omega_dev, void *g_K_dev)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!std::isfinite(dt) || dt == 0.0) return fail(c, KUR_EINVAL, "dt must be finite and nonzero");
    if (nsteps < 0 || ckpt_every < 1) return fail(c, KUR_EINVAL, "nsteps must be >= 0 and ckpt_every >= 1");
    if (!dl_dthetaT_dev) return fail(c, KUR_EINVAL, "dl_dthetaT_dev must not be NULL");
    kur_status s = need_ready(c, true, theta0_dev == nullptr);
    if (s != KUR_OK) return s;
    if ((s = adjoint_check(c)) != KUR_OK) return s;
    AdjIO io;
    io.dev = true;
    io.theta0_dev = theta0_dev;
    io.seed_dev = dl_dthetaT_dev;
    io.gt_dev = g_theta0_dev;
    io.gw_dev = g_omega_dev;
    io.gk_dev = g_K_dev;
    return adjoint_run(c, io, dt, nsteps, ckpt_every);
}

// ------------------------------------------------------------------------------------------------
// complete graph and batches of independent instances
// ------------------------------------------------------------------------------------------------

extern "C" kur_status kur_set_graph_complete(kur_ctx *c, int64_t n)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    BlockGraph g;
    std::string msg;
    try {
        msg = build_complete(n, c->bopt, g);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in graph preprocessing");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, msg);
    kur_status s = install_graph(c, g);
    if (s == KUR_OK) c->complete_graph = true;
    return s;
}

extern "C" kur_status kur_batch_begin(kur_ctx *c)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    c->pend_graph.clear();
    c->pend_omega.clear();
    c->pend_theta.clear();
    c->pend_K.clear();
    c->pend_open = true;
    return KUR_OK;
}

extern "C" kur_status kur_batch_add(kur_ctx *c, int64_t n, int complete, const int64_t *row_ptr, const int32_t *col,
                                    const int32_t *labels, double K, const double *omega, const double *theta0)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!c->pend_open) return fail(c, KUR_ESTATE, "kur_batch_begin was not called");
    if (n < 1) return fail(c, KUR_EINVAL, "n must be >= 1");
    if (!omega || !theta0) return fail(c, KUR_EINVAL, "omega and theta0 must not be NULL");
    if (!std::isfinite(K)) return fail(c, KUR_EINVAL, "K must be finite");
    for (int64_t u = 0; u < n; ++u)
        if (!std::isfinite(omega[u]) || !std::isfinite(theta0[u]) || std::fabs(theta0[u]) > 1e9)
            return fail(c, KUR_EINVAL, "omega and theta0 must be finite (|theta0| <= 1e9)");
    BlockGraph g;
    std::string msg;
    try {
        msg = complete ? build_complete(n, c->bopt, g) : build_from_csr(n, row_ptr, col, labels, c->bopt, g);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed in graph preprocessing");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, msg);
    c->pend_graph.push_back(std::move(g));
    c->pend_omega.insert(c->pend_omega.end(), omega, omega + n);
    c->pend_theta.insert(c->pend_theta.end(), theta0, theta0 + n);
    c->pend_K.push_back(K);
    return KUR_OK;
}

extern "C" kur_status kur_batch_commit(kur_ctx *c)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!c->pend_open || c->pend_graph.empty()) return fail(c, KUR_ESTATE, "no instances added");
    const int64_t ninst = (int64_t)c->pend_graph.size();
    if (ninst > 65535) return fail(c, KUR_EINVAL, "at most 65535 instances");
    std::vector<int64_t> nrow(ninst);
    for (int64_t i = 0; i < ninst; ++i) nrow[i] = c->pend_graph[i].n;
    BlockGraph g;
    std::vector<int64_t> row_first, tile_first;
    std::string msg;
    try {
        msg = merge_graphs(c->pend_graph, g, row_first, tile_first);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed while merging the batch");
    }
    if (!msg.empty()) return fail(c, KUR_EINVAL, msg);
    std::vector<double> omega, theta, K;
    omega.swap(c->pend_omega);
    theta.swap(c->pend_theta);
    K.swap(c->pend_K);
    c->pend_graph.clear();
    c->pend_open = false;
    kur_status s = install_graph(c, g);
    if (s != KUR_OK) return s;
    c->batch = true;
    c->n_inst = (int32_t)ninst;
    c->inst_row_first = row_first;
    c->inst_tile_first = tile_first;
    if (c->host_only) return KUR_OK;
    if ((s = upload_instances(c)) != KUR_OK) return s;
    // per-row coupling K_i / N_i with a global factor K = 1 (block order = user order per instance)
    std::vector<double> unit(c->n);
    for (int64_t i = 0; i < ninst; ++i)
        for (int64_t m = row_first[i]; m < row_first[i + 1]; ++m) unit[m] = K[i] / (double)nrow[i];
    hipError_t e;
    if (c->esz == 4) {
        std::vector<float> tb(c->n);
        for (int64_t u = 0; u < c->n; ++u) tb[c->perm[u]] = (float)unit[u];
        e = upload(c->d_unit, tb.data(), 4 * c->n, c->stream);
    } else {
        std::vector<double> tb(c->n);
        for (int64_t u = 0; u < c->n; ++u) tb[c->perm[u]] = unit[u];
        e = upload(c->d_unit, tb.data(), 8 * c->n, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "batch coupling upload");
    if ((s = kur_set_params(c, omega.data(), 1.0)) != KUR_OK) return s;
    return kur_set_phases(c, theta.data());
}

extern "C" kur_status kur_batch_info(const kur_ctx *c, int32_t *n_inst, int64_t *row_first)
{
    if (!c || !n_inst) return KUR_EINVAL;
    if (!c->has_graph) return KUR_ESTATE;
    *n_inst = c->n_inst;
    if (row_first) std::memcpy(row_first, c->inst_row_first.data(), sizeof(int64_t) * (c->n_inst + 1));
    return KUR_OK;
}

extern "C" kur_status kur_batch_step(kur_ctx *c, double dt, int64_t nsteps, int64_t r_every, double *r_out,
                                     double *psi_out)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!std::isfinite(dt) || dt == 0.0) return fail(c, KUR_EINVAL, "dt must be finite and nonzero");
    if (nsteps < 0 || r_every < 0) return fail(c, KUR_EINVAL, "nsteps and r_every must be >= 0");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    s = run_steps(c, dt, nsteps, r_every);
    if (s != KUR_OK) return s;
    return fetch_samples(c, r_every > 0 ? (nsteps / r_every + 1) * c->n_inst : 0, r_out, psi_out);
}

extern "C" kur_status kur_read_bandwidth(kur_ctx *c, int64_t bytes, int32_t repeats, double *gbps)
{
    if (!c || !gbps) return KUR_EINVAL;
    c->err.clear();
    if (bytes < (1 << 20) || bytes > ((int64_t)64 << 30) || repeats < 1 || repeats > 1000)
        return fail(c, KUR_EINVAL, "bytes must be in [1 MiB, 64 GiB] and repeats in [1, 1000]");
    kur_status s = need_device(c);
    if (s != KUR_OK) return s;
    const int64_t words = bytes / 16;
    DevBuf buf, out;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    float ms = 0.f;
    if ((e = dalloc(buf, (size_t)words * 16)) != hipSuccess || (e = dalloc(out, 64)) != hipSuccess ||
        (e = hipMemsetAsync(buf.p, 1, (size_t)words * 16, c->stream)) != hipSuccess ||
        (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
        (e = launch_stream_read(buf.p, words, (uint32_t *)out.p, c->stream)) != hipSuccess ||
        (e = hipEventRecord(e0, c->stream)) != hipSuccess)
        goto done;
    for (int32_t r = 0; r < repeats && e == hipSuccess; ++r) e = launch_stream_read(buf.p, words, (uint32_t *)out.p, c->stream);
    if (e == hipSuccess && (e = hipEventRecord(e1, c->stream)) == hipSuccess && (e = hipEventSynchronize(e1)) == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dfree(buf);
    dfree(out);
    if (e != hipSuccess) return hip_fail(c, e, "read bandwidth");
    *gbps = (double)words * 16.0 * repeats / ((double)ms * 1e-3) / 1e9;
    return KUR_OK;
}

extern "C" kur_status kur_adjoint_rk4_recorded(kur_ctx *c, const double *dl_dthetaT, double *g_theta0, double *g_omega,
                                               double *g_K)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!dl_dthetaT) return fail(c, KUR_EINVAL, "dl_dthetaT must not be NULL");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    if ((s = adjoint_check(c)) != KUR_OK) return s;
    for (int64_t u = 0; u < c->n; ++u)
        if (!std::isfinite(dl_dthetaT[u])) return fail(c, KUR_EINVAL, "dl_dthetaT must be finite");
    AdjIO io;
    io.seed_host = dl_dthetaT;
    io.gt_host = g_theta0;
    io.gw_host = g_omega;
    io.gk_host = g_K;
    return adjoint_run_recorded(c, io);
}

extern "C" kur_status kur_adjoint_rk4_recorded_dev(kur_ctx *c, const void *dl_dthetaT_dev, void *g_theta0_dev,
                                                   void *g_omega_dev, void *g_K_dev)
{
    if (!c) return KUR_EINVAL;
    c->err.clear();
    if (!dl_dthetaT_dev) return fail(c, KUR_EINVAL, "dl_dthetaT_dev must not be NULL");
    kur_status s = need_ready(c, true, true);
    if (s != KUR_OK) return s;
    if ((s = adjoint_check(c)) != KUR_OK) return s;
    AdjIO io;
    io.dev = true;
    io.seed_dev = dl_dthetaT_dev;
    io.gt_dev = g_theta0_dev;
    io.gw_dev = g_omega_dev;
    io.gk_dev = g_K_dev;
    return adjoint_run_recorded(c, io);
}

extern "C" kur_status kur_recorded_run(const kur_ctx *c, int64_t *serial, double *dt, int64_t *nsteps)
{
    if (!c || !serial) return KUR_EINVAL;
    const bool ok = c->rec_valid && c->rec_gen == c->gen;
    *serial = ok ? c->rec_serial : 0;
    if (dt) *dt = ok ? c->rec_dt : 0.0;
    if (nsteps) *nsteps = ok ? c->rec_nsteps : 0;
    return KUR_OK;
}

// ---------------------------------------------------------------------------------------------
// Hooks of the layout autotuner (kur_tune.hpp).

namespace kur {

EnsState *&ctx_ens_slot(kur_ctx *c) { return c->ens; }
int ctx_device(const kur_ctx *c) { return c->device; }
hipStream_t ctx_stream(const kur_ctx *c) { return c->stream; }
int ctx_timing(const kur_ctx *c) { return c->timing; }
int ctx_compensate(const kur_ctx *c) { return c->compensate; }
double ctx_ens_tau(const kur_ctx *c) { return c->ens_tau; }
void ctx_set_ens_tau(kur_ctx *c, double tau) { c->ens_tau = tau; }

bool ctx_is_device(const kur_ctx *c) { return c && !c->host_only; }
bool ctx_has_graph(const kur_ctx *c) { return c && c->has_graph; }
int ctx_esz(const kur_ctx *c) { return c->esz; }
kur_status ctx_fail(kur_ctx *c, kur_status s, const std::string &msg) { return fail(c, s, msg); }
int32_t ctx_max_chunk(const kur_ctx *c) { return (int32_t)((65535 / c->bopt.esz2) / 64 * 64); }

std::string ctx_arch(const kur_ctx *c)
{
    if (c->host_only) return "host";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return "unknown";
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

TileParams ctx_tile_params(const kur_ctx *c) { return c->tiles_installed; }

bool ctx_layout_fits(const kur_ctx *c, int32_t chunk, const TileParams &t)
{
    // the row kernel (the adjoint kernel stages the same width)
    return rows_lds_bytes(c->esz, chunk > 0 ? chunk : c->W, t.tile_rows, t.threads) <= 156 * 1024;
}

LayoutParams ctx_layout_params(const kur_ctx *c)
{
    LayoutParams l;
    l.tau = c->bopt.tau;
    l.chunk = c->bopt.W;
    l.mask_min = c->bopt.mask_min;
    return l;
}

kur_status ctx_set_build_options(kur_ctx *c, const LayoutParams &l, const TileParams &t)
{
    if (!(l.tau >= 0.0 && l.tau <= 1.0) || l.chunk < 64 || l.chunk % 64 || l.chunk > ctx_max_chunk(c) ||
        !(l.mask_min >= 0.0 && l.mask_min <= 1e9) ||
        t.tile_rows < 64 || t.tile_rows > 4096 || t.tile_min_cost < 1 || !(t.flat_min_vec >= 0.0) ||
        (t.threads != 128 && t.threads != 256 && t.threads != 512 && t.threads != 1024) || t.xcds < 1 || t.xcds > 64 ||
        t.inter_gather < -1 || t.inter_gather > 1)
        return fail(c, KUR_EINVAL, "layout options out of range");
    if (t.inter_gather >= 0) c->inter_gather = t.inter_gather;
    c->bopt.tau = l.tau;
    c->bopt.W = l.chunk;
    c->bopt.mask_min = l.mask_min;
    c->bopt.tile_rows = t.tile_rows;
    c->bopt.tile_min_cost = t.tile_min_cost;
    c->bopt.flat_min_vec = t.flat_min_vec;
    c->bopt.xcds = t.xcds;
    c->threads = t.threads;
    c->gen++;
    return KUR_OK;
}

kur_status ctx_retile(kur_ctx *c, const TileParams &t)
{
    if (!c->has_graph) return fail(c, KUR_ESTATE, "no graph set");
    if (t.tile_rows < 64 || t.tile_rows > 4096 || t.tile_min_cost < 1 || !(t.flat_min_vec >= 0.0) ||
        (t.threads != 128 && t.threads != 256 && t.threads != 512 && t.threads != 1024) || t.xcds < 1 || t.xcds > 64 ||
        t.inter_gather < -1 || t.inter_gather > 1)
        return fail(c, KUR_EINVAL, "tile options out of range");
    if (t.inter_gather >= 0) c->inter_gather = t.inter_gather;
    if (!ctx_layout_fits(c, c->W, t)) return fail(c, KUR_EINVAL, "chunk/tile_rows/threads exceed the LDS of a workgroup");
    BlockGraph &L = c->host_only ? c->host_graph : c->skel;
    BuildOptions o = c->bopt;
    o.tile_rows = t.tile_rows;
    o.tile_min_cost = t.tile_min_cost;
    o.flat_min_vec = t.flat_min_vec;
    o.xcds = t.xcds;
    try {
        make_tiles(L, o);
    } catch (const std::bad_alloc &) {
        return fail(c, KUR_ENOMEM, "host allocation failed while re-tiling");
    }
    if (L.order.size() > (size_t)INT32_MAX) return fail(c, KUR_EINVAL, "too many tiles");
    c->ntiles = (int32_t)L.tiles.size();
    c->nlaunch = (int32_t)L.order.size();
    c->tile_rows = t.tile_rows;
    c->threads = t.threads;
    c->info[6] = c->ntiles;
    c->bopt.tile_rows = t.tile_rows;
    c->bopt.tile_min_cost = t.tile_min_cost;
    c->bopt.flat_min_vec = t.flat_min_vec;
    c->bopt.xcds = t.xcds;
    c->tiles_installed = t;
    c->tiles_installed.inter_gather = c->inter_gather;
    // tiles never span blocks and an instance is a run of whole blocks: its first tile is the
    // first tile of the first block at or after its first row
    c->inst_tile_first.assign(c->n_inst + 1, (int64_t)c->ntiles);
    for (int32_t i = 0; i < c->n_inst; ++i) {
        const int64_t r = c->inst_row_first[i];
        auto it = std::lower_bound(L.blk.begin(), L.blk.end(), r,
                                   [](const BlkInfo &b, int64_t row) { return (int64_t)b.row0 < row; });
        if (it != L.blk.end()) c->inst_tile_first[i] = it->tile0;
    }
    c->sc_valid = false;
    c->gen++;
    if (c->host_only) return KUR_OK;
    HIPCHK(c, hipSetDevice(c->device), "hipSetDevice");
    hipError_t e;
    const size_t T = (size_t)c->esz;
    if ((e = upload(c->d_blk, L.blk.data(), sizeof(BlkInfo) * L.blk.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_tiles, L.tiles.data(), sizeof(Tile) * L.tiles.size(), c->stream)) != hipSuccess ||
        (e = upload(c->d_order, L.order.data(), sizeof(int32_t) * L.order.size(), c->stream)) != hipSuccess ||
        (e = dalloc(c->d_part[0], 2 * T * L.tiles.size())) != hipSuccess ||
        (e = dalloc(c->d_part[1], 2 * T * L.tiles.size())) != hipSuccess ||
        (e = dalloc(c->d_parte, 2 * T * L.tiles.size())) != hipSuccess ||
        (e = upload_mask_items(c->d_mitem, c->d_mtile, c->d_msum, L, T, c->stream)) != hipSuccess) {
        c->has_graph = false;  // partially replaced device layout: unusable until the next set_graph
        return hip_fail(c, e, "re-tiled layout upload");
    }
    c->nmitem = (int32_t)L.mitems.size();
    c->mask_sub = L.mask_sub;
    L.tiles.clear();
    L.tiles.shrink_to_fit();
    L.order.clear();
    L.order.shrink_to_fit();
    L.mitems = std::vector<MaskItem>();
    L.mtiles = std::vector<MaskTile>();
    return upload_instances(c);
}

kur_status ctx_time_steps(kur_ctx *c, int trials, double *ms_per_step)
{
    kur_status s = need_ready(c, false, false);
    if (s != KUR_OK) return s;
    const bool synth = !(c->has_params && c->has_phases);
    const int64_t n = c->n;
    const size_t TN = (size_t)c->esz * (size_t)n;
    DevBuf sv_hi, sv_lo, sv_wind;
    hipError_t e = hipSuccess;
    struct Release {
        DevBuf *b[3];
        ~Release()
        {
            for (DevBuf *x : b) dfree(*x);
        }
    } rel{{&sv_hi, &sv_lo, &sv_wind}};
    if (synth) {
        // omega = 0, K = 1 and phases spread by the golden ratio: the timed work does not
        // depend on the values
        std::vector<double> om(n, 0.0), th(n);
        for (int64_t u = 0; u < n; ++u) th[u] = 2.0 * kPi * std::fmod(0.6180339887498949 * (double)u, 1.0);
        if ((s = kur_set_params(c, om.data(), 1.0)) != KUR_OK || (s = kur_set_phases(c, th.data())) != KUR_OK)
            return s;
    } else {
        if ((e = dalloc(sv_hi, TN)) != hipSuccess || (e = dalloc(sv_lo, TN)) != hipSuccess ||
            (e = dalloc(sv_wind, 4 * (size_t)n)) != hipSuccess ||
            (e = hipMemcpyAsync(sv_hi.p, c->d_hi.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(sv_lo.p, c->d_lo.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(sv_wind.p, c->d_wind.p, 4 * (size_t)n, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
            return hip_fail(c, e, "state save");
    }
    const int cur0 = c->cur;
    const int timing0 = c->timing;
    c->timing = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e300;
    if ((e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess) {
        if (!c->sc_valid) {
            s = sc_init(c, c->d_hi.p, c->d_sc[c->cur], c->d_part[c->cur]);
            c->sc_valid = s == KUR_OK;
        }
        const DevGraph g = devgraph(c);
        const double dt = 1e-3;
        int64_t steps = 1;
        for (int t = -1; t < trials && s == KUR_OK && e == hipSuccess; ++t) {
            // t = -1: warm-up step, then one step to size the trials to about 4 ms each
            if (t == -1 && (e = launch_step(c, g, dt)) != hipSuccess) break;
            if ((e = hipEventRecord(e0, c->stream)) != hipSuccess) break;
            for (int64_t k = 0; k < steps && e == hipSuccess; ++k) e = launch_step(c, g, dt);
            if (e != hipSuccess || (e = hipEventRecord(e1, c->stream)) != hipSuccess ||
                (e = hipEventSynchronize(e1)) != hipSuccess)
                break;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
            if (t == -1)
                steps = std::min<int64_t>(256, std::max<int64_t>(2, (int64_t)std::ceil(4.0 / std::max(1e-3, (double)ms))));
            else
                best = std::min(best, (double)ms / (double)steps);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->timing = timing0;
    c->cur = cur0;
    c->sc_valid = false;
    if (s != KUR_OK) return s;
    if (e != hipSuccess) return hip_fail(c, e, "timed steps");
    if (synth) {
        c->has_params = false;
        c->has_phases = false;
    } else {
        if ((e = hipMemcpyAsync(c->d_hi.p, sv_hi.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(c->d_lo.p, sv_lo.p, TN, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(c->d_wind.p, sv_wind.p, 4 * (size_t)n, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(c->stream)) != hipSuccess)
            return hip_fail(c, e, "state restore");
    }
    *ms_per_step = best;
    return KUR_OK;
}

void ctx_block_stats(const kur_ctx *c, std::vector<double> &density, std::vector<int32_t> &size,
                     std::vector<double> &pair_density)
{
    const BlockGraph &L = c->host_only ? c->host_graph : c->skel;
    density = L.blk_rho;
    density.resize(L.blk.size(), 0.0);
    size.assign(L.blk.size(), 0);
    for (size_t b = 0; b < L.blk.size(); ++b) size[b] = L.blk[b].size;
    pair_density = L.pair_rho;
}

}  // namespace kur
