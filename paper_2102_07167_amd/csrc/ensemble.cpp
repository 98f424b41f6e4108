// ensemble.cpp -- the shared-graph ensemble path of the C ABI (kur_ens_*): B replicas of one
// graph with their own omega, K and phases, integrated together so that every dense block's
// coupling sums for all replicas form one matrix product on the matrix cores.
//
// Host layout (block order, the same regroup by planted label as the single-system path):
//   * blocks whose realised density is at least the option "ens_tau" store their 0/1 pattern as
//     a row-major bitmask (product A_b X_b in k_ens_gemm);
//   * every other edge (the ones of the remaining blocks and all inter-block edges) goes into
//     one CSR over block-order columns, gathered by k_ens_rows.
// Device state is node-major, [n][Bp] per quantity (Bp = B rounded up to 64; the padding
// replicas have omega = 0, K = 0 and phase 0 and are never reported).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/kur.h"
#include "ens.hpp"
#include "kur_internal.hpp"
#include "kur_kernels.hpp"
#include "kur_tune.hpp"

using namespace kur;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int32_t kMaxReplicas = 256;

struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n)
    {
        if (n <= bytes && p) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, std::max<size_t>(n, 256));
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        bytes = std::max<size_t>(n, 256);
        return hipSuccess;
    }
    template <typename T> T *as() const { return (T *)p; }
};

hipError_t put(DBuf &b, const void *src, size_t n, hipStream_t st)
{
    hipError_t e = b.ensure(n);
    if (e != hipSuccess || n == 0) return e;
    e = hipMemcpyAsync(b.p, src, n, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

struct EnsLayout {
    int64_t n = 0;
    int32_t nb = 0;
    bool symmetric = false;
    std::vector<int32_t> perm;        // user node -> block-order row
    std::vector<int64_t> block_ptr;   // nb + 1
    std::vector<double> density;      // realised density per block
    std::vector<uint8_t> gemm;        // per block: its own (diagonal) block on the matrix cores
    std::vector<EnsBlk> gblk;         // matrix-core row blocks, largest k extent first
    std::vector<EnsRng> rng;          // their column ranges
    std::vector<double> pair_density; // densities of the off-diagonal blocks that a threshold can
                                      // put on the matrix cores (both sides >= kPairMin, >= kPairFloor)
    int64_t n_pair_ranges = 0;        // dense off-diagonal blocks on the matrix cores
    std::vector<uint32_t> bits;
    std::vector<int64_t> csr_ptr;     // n + 1
    std::vector<int32_t> csr_col;
    std::vector<uint8_t> row_gemm;    // n
    int64_t gemm_rows = 0, gemm_pairs = 0;
};

// Off-diagonal blocks go on the matrix cores only with both communities of at least kPairMin
// nodes and a density of at least max(threshold, kPairFloor): below about 1 % the CSR rows are
// cheaper (a matrix-core cell costs about 1/100 of a gathered entry at B = 128), and the floor
// bounds the pattern memory by the edge count.
constexpr int64_t kPairMin = 32;
constexpr double kPairFloor = 0.01;

// Builds the ensemble layout; "" on success. Duplicate columns in a row are an error, diagonal
// entries are ignored (A_mm = 0), as in the single-system builder. A community's own block and
// its off-diagonal blocks with density >= tau (see kPairMin, kPairFloor) become column ranges of
// its matrix-core row block; every other edge goes to the CSR rows.
std::string build_layout(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels, double tau,
                         EnsLayout &L)
{
    std::string msg = validate_csr(n, row_ptr, col, labels);
    if (!msg.empty()) return msg;
    L = EnsLayout();
    L.n = n;
    L.symmetric = csr_symmetric(n, row_ptr, col);
    std::vector<int32_t> node_at, block_of_row;
    L.nb = regroup_by_labels(n, labels, L.perm, node_at, block_of_row, L.block_ptr);
    const int32_t nb = L.nb;
    auto bsize = [&](int32_t b) { return L.block_ptr[b + 1] - L.block_ptr[b]; };

    // pass 1 (per row block): entries towards every column block; duplicates are found in pass 2
    std::vector<std::vector<std::pair<int32_t, int64_t>>> cnt(nb);
    parallel_for(nb, [&](int64_t lo, int64_t hi) {
        std::unordered_map<int32_t, int64_t> h;
        for (int64_t a = lo; a < hi; ++a) {
            h.clear();
            for (int64_t m = L.block_ptr[a]; m < L.block_ptr[a + 1]; ++m) {
                const int64_t u = node_at[m];
                for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    const int64_t pv = L.perm[col[e]];
                    if (pv != m) ++h[block_of_row[pv]];
                }
            }
            cnt[a].assign(h.begin(), h.end());
            std::sort(cnt[a].begin(), cnt[a].end());
        }
    });

    // column ranges of every row block, in block order: its own block when dense and its dense
    // partners (pass 2 walks the ranges and the sorted columns of a row together)
    L.density.assign(nb, 0.0);
    L.gemm.assign(nb, 0);
    std::vector<std::vector<int32_t>> ranges(nb);
    for (int32_t a = 0; a < nb; ++a) {
        const int64_t s = bsize(a);
        for (const auto &kv : cnt[a]) {
            const int32_t c = kv.first;
            if (c == a) {
                const double pairs = (double)s * (double)(s - 1);
                L.density[a] = pairs > 0 ? (double)kv.second / pairs : 0.0;
                continue;
            }
            if (s < kPairMin || bsize(c) < kPairMin) continue;
            const double rho = (double)kv.second / ((double)s * (double)bsize(c));
            if (rho < kPairFloor) continue;
            L.pair_density.push_back(rho);
            if (rho >= tau) ranges[a].push_back(c);
        }
        L.gemm[a] = (s >= 2 && L.density[a] >= tau) ? 1 : 0;
        L.n_pair_ranges += (int64_t)ranges[a].size();
        if (L.gemm[a]) ranges[a].insert(std::lower_bound(ranges[a].begin(), ranges[a].end(), a), a);  // block order
    }
    // matrix-core row blocks and their ranges; bit position of (row block a, column block c)
    std::vector<int32_t> gidx(nb, -1);
    int64_t words_total = 0;
    for (int32_t a = 0; a < nb; ++a) {
        if (ranges[a].empty()) continue;
        EnsBlk e{};
        e.row0 = (int32_t)L.block_ptr[a];
        e.size = (int32_t)bsize(a);
        e.rng0 = (int32_t)L.rng.size();
        e.nrng = (int32_t)ranges[a].size();
        int64_t koff = 0;
        for (int32_t c : ranges[a]) {
            L.rng.push_back(EnsRng{(int32_t)koff, (int32_t)L.block_ptr[c], (int32_t)bsize(c), 0});
            koff += (bsize(c) + 31) / 32 * 32;
            L.gemm_pairs += (int64_t)e.size * bsize(c);
        }
        if (koff / 32 > INT32_MAX) return "matrix-core row block too wide";
        e.words = (int32_t)(koff / 32);
        e.bits_off = words_total;
        words_total += (int64_t)e.size * e.words;
        L.gemm_rows += e.size;
        gidx[a] = (int32_t)L.gblk.size();
        L.gblk.push_back(e);
    }
    L.row_gemm.assign(n, 0);
    for (int64_t m = 0; m < n; ++m) L.row_gemm[m] = gidx[block_of_row[m]] >= 0 ? 1 : 0;
    L.bits.assign((size_t)words_total, 0u);

    // pass 2: per row, its columns sorted; those inside a range set pattern bits, the others
    // form the CSR row (counted first, then emitted)
    std::vector<int64_t> csr_cnt(n, 0);
    std::atomic<bool> dup{false};
    auto row_pass = [&](bool emit) {
        parallel_for(n, [&](int64_t lo, int64_t hi) {
            std::vector<int32_t> cols;
            for (int64_t m = lo; m < hi; ++m) {
                const int32_t a = block_of_row[m];
                const int64_t u = node_at[m];
                cols.clear();
                for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
                    const int64_t pv = L.perm[col[e]];
                    if (pv != m) cols.push_back((int32_t)pv);
                }
                std::sort(cols.begin(), cols.end());
                if (!emit) {
                    for (size_t i = 1; i < cols.size(); ++i)
                        if (cols[i] == cols[i - 1]) dup = true;
                }
                const EnsBlk *g = gidx[a] >= 0 ? &L.gblk[gidx[a]] : nullptr;
                uint32_t *bits = g && emit ? L.bits.data() + g->bits_off + (m - g->row0) * (int64_t)g->words : nullptr;
                int32_t *dst = emit ? L.csr_col.data() + L.csr_ptr[m] : nullptr;
                int64_t k = 0;
                int32_t r = 0;  // ranges are in block order, as are the sorted columns
                for (int32_t v : cols) {
                    while (g && r < g->nrng && v >= L.rng[g->rng0 + r].col0 + L.rng[g->rng0 + r].len) ++r;
                    if (g && r < g->nrng && v >= L.rng[g->rng0 + r].col0) {
                        const EnsRng &R = L.rng[g->rng0 + r];
                        if (bits) {
                            const int64_t pos = R.koff + (v - R.col0);
                            bits[pos >> 5] |= 1u << (pos & 31);
                        }
                        continue;
                    }
                    if (dst) dst[k] = v;
                    ++k;
                }
                if (!emit) csr_cnt[m] = k;
            }
        });
    };
    row_pass(false);
    if (dup) return "duplicate column in a row";
    L.csr_ptr.assign(n + 1, 0);
    for (int64_t m = 0; m < n; ++m) L.csr_ptr[m + 1] = L.csr_ptr[m] + csr_cnt[m];
    L.csr_col.assign((size_t)L.csr_ptr[n], 0);
    row_pass(true);

    // longest work items launch first
    std::vector<size_t> ord(L.gblk.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
        return (int64_t)L.gblk[x].size * L.gblk[x].words > (int64_t)L.gblk[y].size * L.gblk[y].words;
    });
    std::vector<EnsBlk> sorted;
    for (size_t i : ord) sorted.push_back(L.gblk[i]);
    L.gblk.swap(sorted);
    return "";
}

}  // namespace

namespace kur {

struct EnsState {
    EnsLayout L;
    bool has_graph = false;
    // device layout
    DBuf d_gblk, d_rng, d_bits, d_csr_ptr, d_csr_col, d_row_gemm, d_items;
    int64_t nitems = 0;
    int64_t items_J = -1;
    // replicas
    int32_t B = 0, Bp = 0;
    bool has_params = false, has_phases = false, x_valid = false;
    DBuf d_omega, d_unit, d_hi, d_lo, d_wind, d_ksum, d_x[2], d_y, d_kout, d_part, d_r, d_psi;
    int cur = 0;
    // timing of the two stage kernels
    std::vector<hipEvent_t> ev;  // pairs
    std::vector<int> ev_kind;    // 0: matrix product, 1: rows
    size_t ev_used = 0;
    int64_t t_n[2] = {0, 0};
    double t_ms[2] = {0.0, 0.0};
    ~EnsState()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

void ens_free(EnsState *s) { delete s; }

}  // namespace kur

namespace {

EnsState *state(kur_ctx *c)
{
    EnsState *&s = ctx_ens_slot(c);
    if (!s) s = new (std::nothrow) EnsState();
    return s;
}

kur_status hipfail(kur_ctx *c, hipError_t e, const char *what)
{
    return ctx_fail(c, e == hipErrorOutOfMemory ? KUR_ENOMEM : KUR_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

kur_status need_real(kur_ctx *c)
{
    if (ctx_esz(c) != 4 && ctx_esz(c) != 8) return ctx_fail(c, KUR_EINVAL, "ensembles run in FP32 or FP64");
    return KUR_OK;
}

// output tile of the dense products for the context's reals
int tile_rows(kur_ctx *c) { return ctx_esz(c) == 8 ? kEnsTileRowsF64 : kEnsTileRows; }
int tile_cols(kur_ctx *c) { return ctx_esz(c) == 8 ? kEnsTileColsF64 : kEnsTileCols; }

// items of the dense products for J columns
hipError_t upload_items(kur_ctx *c, EnsState &S)
{
    const int64_t J = 2 * (int64_t)S.Bp;
    if (S.items_J == J) return hipSuccess;
    const int TR = tile_rows(c), TC = tile_cols(c);
    std::vector<EnsItem> items;
    for (size_t g = 0; g < S.L.gblk.size(); ++g)
        for (int32_t r0 = 0; r0 < S.L.gblk[g].size; r0 += TR)
            for (int64_t c0 = 0; c0 < J; c0 += TC) items.push_back(EnsItem{(int32_t)g, r0, (int32_t)c0, 0});
    S.nitems = (int64_t)items.size();
    S.items_J = J;
    return put(S.d_items, items.data(), sizeof(EnsItem) * items.size(), ctx_stream(c));
}

hipError_t record(kur_ctx *c, EnsState &S, int kind, bool end)
{
    if (!ctx_timing(c)) return hipSuccess;
    if (!end && S.ev_used + 2 > S.ev.size()) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            S.ev.push_back(e);
            S.ev_kind.push_back(0);
        }
    }
    if (!end) {
        S.ev_kind[S.ev_used] = kind;
        return hipEventRecord(S.ev[S.ev_used], ctx_stream(c));
    }
    hipError_t r = hipEventRecord(S.ev[S.ev_used + 1], ctx_stream(c));
    S.ev_used += 2;
    return r;
}

hipError_t harvest(kur_ctx *c, EnsState &S)
{
    if (S.ev_used == 0) return hipSuccess;
    hipError_t r = hipStreamSynchronize(ctx_stream(c));
    if (r != hipSuccess) return r;
    for (size_t i = 0; i + 1 < S.ev_used; i += 2) {
        float ms = 0.f;
        if ((r = hipEventElapsedTime(&ms, S.ev[i], S.ev[i + 1])) != hipSuccess) return r;
        S.t_ms[S.ev_kind[i]] += ms;
        S.t_n[S.ev_kind[i]] += 1;
    }
    S.ev_used = 0;
    return hipSuccess;
}

// one stage: dense products, then rows (CSR gathers + epilogue) from x[cur] into x[cur ^ 1]
template <typename T>
hipError_t launch_stage_t(kur_ctx *c, EnsState &S, int stage, double dt)
{
    const hipStream_t st = ctx_stream(c);
    const int64_t J = 2 * (int64_t)S.Bp;
    hipError_t e;
    if (S.nitems > 0) {
        EnsGemmArgs g;
        g.blk = S.d_gblk.as<EnsBlk>();
        g.rng = S.d_rng.as<EnsRng>();
        g.items = S.d_items.as<EnsItem>();
        g.bits = S.d_bits.as<uint32_t>();
        g.x = S.d_x[S.cur].p;
        g.y = S.d_y.p;
        g.J = J;
        if ((e = record(c, S, 0, false)) != hipSuccess ||
            (e = sizeof(T) == 8 ? launch_ens_gemm_f64(g, S.nitems, st) : launch_ens_gemm(g, S.nitems, st)) != hipSuccess ||
            (e = record(c, S, 0, true)) != hipSuccess)
            return e;
    }
    EnsRowArgs<T> a;
    a.n = S.L.n;
    a.Bp = S.Bp;
    a.stage = stage;
    a.compensate = ctx_compensate(c);
    a.dt = (T)dt;
    a.half_dt = (T)(0.5 * dt);
    a.dt6 = (T)(dt / 6.0);
    a.csr_ptr = S.d_csr_ptr.as<int64_t>();
    a.csr_col = S.d_csr_col.as<int32_t>();
    a.row_gemm = S.d_row_gemm.as<uint8_t>();
    a.x = S.d_x[S.cur].as<T>();
    a.y = S.d_y.as<T>();
    a.x_out = S.d_x[S.cur ^ 1].as<T>();
    a.omega = S.d_omega.as<T>();
    a.unit = S.d_unit.as<T>();
    a.hi = S.d_hi.as<T>();
    a.lo = S.d_lo.as<T>();
    a.wind = S.d_wind.as<int32_t>();
    a.ksum = S.d_ksum.as<T>();
    a.kout = S.d_kout.as<T>();
    if ((e = record(c, S, 1, false)) != hipSuccess || (e = launch_ens_rows<T>(a, st)) != hipSuccess ||
        (e = record(c, S, 1, true)) != hipSuccess)
        return e;
    if (stage != 0) S.cur ^= 1;
    if (ctx_timing(c) && S.ev_used + 8 > 4096) return harvest(c, S);
    return hipSuccess;
}

hipError_t launch_stage(kur_ctx *c, EnsState &S, int stage, double dt)
{
    return ctx_esz(c) == 8 ? launch_stage_t<double>(c, S, stage, dt) : launch_stage_t<float>(c, S, stage, dt);
}

hipError_t ensure_x(kur_ctx *c, EnsState &S)
{
    if (S.x_valid) return hipSuccess;
    hipError_t e = ctx_esz(c) == 8
                       ? launch_ens_sincos<double>(S.L.n, S.Bp, S.d_hi.as<double>(), S.d_x[S.cur].as<double>(), ctx_stream(c))
                       : launch_ens_sincos<float>(S.L.n, S.Bp, S.d_hi.as<float>(), S.d_x[S.cur].as<float>(), ctx_stream(c));
    if (e == hipSuccess) S.x_valid = true;
    return e;
}

hipError_t sample(kur_ctx *c, EnsState &S, int64_t k)
{
    const hipStream_t st = ctx_stream(c);
    double *r = S.d_r.as<double>() + k * S.B, *psi = S.d_psi.as<double>() + k * S.B;
    if (ctx_esz(c) == 8) {
        hipError_t e = launch_ens_colsum<double>(S.L.n, 2 * (int64_t)S.Bp, S.d_x[S.cur].as<double>(), S.d_part.as<double>(), st);
        return e != hipSuccess ? e : launch_ens_order<double>(S.L.n, S.Bp, S.B, S.d_part.as<double>(), r, psi, st);
    }
    hipError_t e = launch_ens_colsum<float>(S.L.n, 2 * (int64_t)S.Bp, S.d_x[S.cur].as<float>(), S.d_part.as<float>(), st);
    return e != hipSuccess ? e : launch_ens_order<float>(S.L.n, S.Bp, S.B, S.d_part.as<float>(), r, psi, st);
}

kur_status install_layout(kur_ctx *c, EnsState &S, EnsLayout &L)
{
    S.has_graph = false;
    S.has_params = S.has_phases = S.x_valid = false;
    S.B = S.Bp = 0;
    S.items_J = -1;
    S.nitems = 0;
    S.L = std::move(L);
    if (ctx_is_device(c)) {
        const hipStream_t st = ctx_stream(c);
        hipError_t e;
        if ((e = hipSetDevice(ctx_device(c))) != hipSuccess ||
            (e = put(S.d_gblk, S.L.gblk.data(), sizeof(EnsBlk) * S.L.gblk.size(), st)) != hipSuccess ||
            (e = put(S.d_rng, S.L.rng.data(), sizeof(EnsRng) * S.L.rng.size(), st)) != hipSuccess ||
            (e = put(S.d_bits, S.L.bits.data(), 4 * S.L.bits.size(), st)) != hipSuccess ||
            (e = put(S.d_csr_ptr, S.L.csr_ptr.data(), 8 * S.L.csr_ptr.size(), st)) != hipSuccess ||
            (e = put(S.d_csr_col, S.L.csr_col.data(), 4 * S.L.csr_col.size(), st)) != hipSuccess ||
            (e = put(S.d_row_gemm, S.L.row_gemm.data(), S.L.row_gemm.size(), st)) != hipSuccess)
            return hipfail(c, e, "ensemble layout upload");
        // the host copies of the large arrays are not needed any more
        std::vector<uint32_t>().swap(S.L.bits);
        std::vector<int32_t>().swap(S.L.csr_col);
    }
    S.has_graph = true;
    return KUR_OK;
}

kur_status ens_ready(kur_ctx *c, EnsState *&S, bool phases)
{
    if (!c) return KUR_EINVAL;
    kur_status s = need_real(c);
    if (s != KUR_OK) return s;
    if (!ctx_is_device(c)) return ctx_fail(c, KUR_EDEVICE, "host-only context (device = -1)");
    S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (!S->has_graph) return ctx_fail(c, KUR_ESTATE, "no ensemble graph set");
    if (!S->has_params) return ctx_fail(c, KUR_ESTATE, "ensemble omega and K not set");
    if (phases && !S->has_phases) return ctx_fail(c, KUR_ESTATE, "ensemble phases not set");
    hipError_t e = hipSetDevice(ctx_device(c));
    if (e != hipSuccess) return hipfail(c, e, "hipSetDevice");
    return KUR_OK;
}

template <typename T>
kur_status set_params_t(kur_ctx *c, EnsState &S, int32_t B, const double *K, const double *omega)
{
    const int64_t n = S.L.n;
    const int32_t Bp = (B + 63) / 64 * 64;
    const size_t z = sizeof(T);
    std::vector<T> om((size_t)n * Bp, T(0)), unit(Bp, T(0));
    for (int32_t e = 0; e < B; ++e) {
        unit[e] = (T)(K[e] / (double)n);
        for (int64_t u = 0; u < n; ++u) om[(size_t)S.L.perm[u] * Bp + e] = (T)omega[(size_t)e * n + u];
    }
    const hipStream_t st = ctx_stream(c);
    const size_t NB = (size_t)n * Bp;
    const int64_t nchunk = (n + 255) / 256;
    hipError_t err;
    if ((err = put(S.d_omega, om.data(), z * NB, st)) != hipSuccess || (err = put(S.d_unit, unit.data(), z * Bp, st)) != hipSuccess ||
        (err = S.d_hi.ensure(z * NB)) != hipSuccess || (err = S.d_lo.ensure(z * NB)) != hipSuccess ||
        (err = S.d_wind.ensure(4 * NB)) != hipSuccess || (err = S.d_ksum.ensure(z * NB)) != hipSuccess ||
        (err = S.d_x[0].ensure(2 * z * NB)) != hipSuccess || (err = S.d_x[1].ensure(2 * z * NB)) != hipSuccess ||
        (err = S.d_y.ensure(2 * z * NB)) != hipSuccess || (err = S.d_kout.ensure(z * NB)) != hipSuccess ||
        (err = S.d_part.ensure(2 * z * (size_t)nchunk * Bp)) != hipSuccess)
        return hipfail(c, err, "ensemble buffers");
    if (Bp != S.Bp) S.has_phases = false;
    S.B = B;
    S.Bp = Bp;
    if ((err = upload_items(c, S)) != hipSuccess) return hipfail(c, err, "ensemble work items");
    S.has_params = true;
    return KUR_OK;
}

kur_status set_params_impl(kur_ctx *c, EnsState &S, int32_t B, const double *K, const double *omega)
{
    return ctx_esz(c) == 8 ? set_params_t<double>(c, S, B, K, omega) : set_params_t<float>(c, S, B, K, omega);
}

template <typename T>
kur_status set_phases_t(kur_ctx *c, EnsState &S, const double *theta)
{
    const int64_t n = S.L.n;
    const int32_t B = S.B, Bp = S.Bp;
    const size_t NB = (size_t)n * Bp;
    std::vector<T> hi(NB, T(0)), lo(NB, T(0));
    std::vector<int32_t> wind(NB, 0);
    const double P1 = two_pi_p1(sizeof(T)), P2 = two_pi_p2(sizeof(T));
    for (int32_t e = 0; e < B; ++e)
        for (int64_t u = 0; u < n; ++u) {
            const double t = theta[(size_t)e * n + u];
            const double q = std::nearbyint(t / (2.0 * kPi));
            const double red = (t - q * P1) - q * P2;
            const size_t ix = (size_t)S.L.perm[u] * Bp + e;
            hi[ix] = (T)red;
            lo[ix] = (T)(red - (double)hi[ix]);
            wind[ix] = (int32_t)q;
        }
    const hipStream_t st = ctx_stream(c);
    hipError_t err;
    if ((err = put(S.d_hi, hi.data(), sizeof(T) * NB, st)) != hipSuccess || (err = put(S.d_lo, lo.data(), sizeof(T) * NB, st)) != hipSuccess ||
        (err = put(S.d_wind, wind.data(), 4 * NB, st)) != hipSuccess)
        return hipfail(c, err, "ensemble phase upload");
    S.has_phases = true;
    S.x_valid = false;
    S.cur = 0;
    return KUR_OK;
}

kur_status set_phases_impl(kur_ctx *c, EnsState &S, const double *theta)
{
    return ctx_esz(c) == 8 ? set_phases_t<double>(c, S, theta) : set_phases_t<float>(c, S, theta);
}

bool finite_all(const double *a, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

// best of `trials` timings of whole RK4 steps, ms per step (phases restored afterwards)
kur_status time_steps(kur_ctx *c, EnsState &S, int trials, double *ms_per_step)
{
    const hipStream_t st = ctx_stream(c);
    const size_t NB = (size_t)S.L.n * S.Bp, z = (size_t)ctx_esz(c);
    DBuf sh, sl, sw;
    hipError_t e;
    if ((e = sh.ensure(z * NB)) != hipSuccess || (e = sl.ensure(z * NB)) != hipSuccess || (e = sw.ensure(4 * NB)) != hipSuccess ||
        (e = hipMemcpyAsync(sh.p, S.d_hi.p, z * NB, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(sl.p, S.d_lo.p, z * NB, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(sw.p, S.d_wind.p, 4 * NB, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return hipfail(c, e, "ensemble state save");
    const int cur0 = S.cur;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best = 1e300;
    int64_t steps = 1;
    if ((e = hipEventCreate(&e0)) == hipSuccess && (e = hipEventCreate(&e1)) == hipSuccess && (e = ensure_x(c, S)) == hipSuccess) {
        for (int t = -1; t < trials && e == hipSuccess; ++t) {
            for (int st4 = 1; t == -1 && st4 <= 4 && e == hipSuccess; ++st4) e = launch_stage(c, S, st4, 1e-3);
            if (e != hipSuccess || (e = hipEventRecord(e0, st)) != hipSuccess) break;
            for (int64_t k = 0; k < steps && e == hipSuccess; ++k)
                for (int st4 = 1; st4 <= 4 && e == hipSuccess; ++st4) e = launch_stage(c, S, st4, 1e-3);
            if (e != hipSuccess || (e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) break;
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
    if (e == hipSuccess) {
        if ((e = hipMemcpyAsync(S.d_hi.p, sh.p, z * NB, hipMemcpyDeviceToDevice, st)) == hipSuccess &&
            (e = hipMemcpyAsync(S.d_lo.p, sl.p, z * NB, hipMemcpyDeviceToDevice, st)) == hipSuccess &&
            (e = hipMemcpyAsync(S.d_wind.p, sw.p, 4 * NB, hipMemcpyDeviceToDevice, st)) == hipSuccess)
            e = hipStreamSynchronize(st);
    }
    S.cur = cur0;
    S.x_valid = false;
    if (e != hipSuccess) return hipfail(c, e, "ensemble timing");
    *ms_per_step = best;
    return KUR_OK;
}

}  // namespace

extern "C" {

kur_status kur_ens_set_graph_csr(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels)
{
    if (!c) return KUR_EINVAL;
    kur_status s = need_real(c);
    if (s != KUR_OK) return s;
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    EnsLayout L;
    std::string msg;
    try {
        msg = build_layout(n, row_ptr, col, labels, ctx_ens_tau(c), L);
    } catch (const std::bad_alloc &) {
        return ctx_fail(c, KUR_ENOMEM, "host allocation failed while building the ensemble layout");
    }
    if (!msg.empty()) return ctx_fail(c, KUR_EINVAL, msg);
    return install_layout(c, *S, L);
}

kur_status kur_ens_info(kur_ctx *c, int64_t *out)
{
    if (!c || !out) return KUR_EINVAL;
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (!S->has_graph) return ctx_fail(c, KUR_ESTATE, "no ensemble graph set");
    const EnsLayout &L = S->L;
    out[0] = L.n;
    out[1] = L.nb;
    out[2] = (int64_t)L.gblk.size();
    out[3] = L.gemm_rows;
    out[4] = L.gemm_pairs;
    out[5] = L.csr_ptr.empty() ? 0 : L.csr_ptr.back();
    out[6] = S->B;
    out[7] = S->Bp;
    out[8] = S->nitems;
    out[9] = L.symmetric ? 1 : 0;
    out[10] = L.n_pair_ranges;
    int64_t padded = 0;  // cells the product tiles issue: rows to the tile height, k extent to 32
    const int64_t TR = tile_rows(c);
    for (const EnsBlk &g : L.gblk) padded += (int64_t)((g.size + TR - 1) / TR) * TR * g.words * 32;
    out[11] = padded;
    return KUR_OK;
}

kur_status kur_ens_block_modes(kur_ctx *c, uint8_t *gemm, double *density)
{
    if (!c) return KUR_EINVAL;
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (!S->has_graph) return ctx_fail(c, KUR_ESTATE, "no ensemble graph set");
    if (gemm) std::memcpy(gemm, S->L.gemm.data(), S->L.gemm.size());
    if (density) std::memcpy(density, S->L.density.data(), 8 * S->L.density.size());
    return KUR_OK;
}

kur_status kur_ens_get_perm(kur_ctx *c, int32_t *perm)
{
    if (!c || !perm) return KUR_EINVAL;
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (!S->has_graph) return ctx_fail(c, KUR_ESTATE, "no ensemble graph set");
    std::memcpy(perm, S->L.perm.data(), 4 * S->L.perm.size());
    return KUR_OK;
}

kur_status kur_ens_row_pattern(kur_ctx *c, int64_t m, int32_t *csr_cols, int64_t *ncsr, uint8_t *dense)
{
    if (!c || !ncsr) return KUR_EINVAL;
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (!S->has_graph) return ctx_fail(c, KUR_ESTATE, "no ensemble graph set");
    if (ctx_is_device(c)) return ctx_fail(c, KUR_ESTATE, "row patterns are kept by host-only contexts only");
    const EnsLayout &L = S->L;
    if (m < 0 || m >= L.n) return ctx_fail(c, KUR_EINVAL, "row out of range");
    const int64_t cnt = L.csr_ptr[m + 1] - L.csr_ptr[m];
    const int64_t cap = *ncsr;
    *ncsr = cnt;
    if (csr_cols) {
        if (cap < cnt) return ctx_fail(c, KUR_EINVAL, "csr_cols holds fewer entries than the row");
        std::memcpy(csr_cols, L.csr_col.data() + L.csr_ptr[m], 4 * (size_t)cnt);
    }
    if (dense) {
        std::memset(dense, 0, (size_t)L.n);
        if (L.row_gemm[m]) {
            const int32_t b = (int32_t)(std::upper_bound(L.block_ptr.begin(), L.block_ptr.end(), m) - L.block_ptr.begin()) - 1;
            const int64_t r0 = L.block_ptr[b];
            for (const EnsBlk &g : L.gblk)
                if (g.row0 == r0) {
                    const uint32_t *row = L.bits.data() + g.bits_off + (m - r0) * g.words;
                    for (int32_t q = 0; q < g.nrng; ++q) {
                        const EnsRng &R = L.rng[g.rng0 + q];
                        for (int64_t j = 0; j < R.len; ++j) {
                            const int64_t k = R.koff + j;
                            dense[R.col0 + j] = (row[k >> 5] >> (k & 31)) & 1u;
                        }
                    }
                }
        }
    }
    return KUR_OK;
}

kur_status kur_ens_set_params(kur_ctx *c, int32_t B, const double *K, const double *omega)
{
    if (!c) return KUR_EINVAL;
    kur_status s = need_real(c);
    if (s != KUR_OK) return s;
    if (!ctx_is_device(c)) return ctx_fail(c, KUR_EDEVICE, "host-only context (device = -1)");
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (!S->has_graph) return ctx_fail(c, KUR_ESTATE, "no ensemble graph set");
    if (B < 1 || B > kMaxReplicas) return ctx_fail(c, KUR_EINVAL, "B must be in [1, 256]");
    if (!K || !omega) return ctx_fail(c, KUR_EINVAL, "K and omega must not be NULL");
    if (!finite_all(K, B) || !finite_all(omega, (size_t)B * S->L.n)) return ctx_fail(c, KUR_EINVAL, "K and omega must be finite");
    {
        // the matrix-product kernels address the X rows of one range with 32-bit offsets k J + c
        const int64_t J = 2 * (int64_t)((B + 63) / 64 * 64);
        int64_t maxlen = 0;
        for (const EnsRng &R : S->L.rng) maxlen = std::max<int64_t>(maxlen, R.len);
        if (maxlen * J >= ((int64_t)1 << 31))
            return ctx_fail(c, KUR_EINVAL, "a matrix-core community of " + std::to_string(maxlen) + " nodes is too large for " +
                                               std::to_string(B) + " replicas (its rows x 2 Bp must stay below 2^31)");
    }
    hipError_t e = hipSetDevice(ctx_device(c));
    if (e != hipSuccess) return hipfail(c, e, "hipSetDevice");
    return set_params_impl(c, *S, B, K, omega);
}

kur_status kur_ens_set_phases(kur_ctx *c, const double *theta)
{
    EnsState *S = nullptr;
    kur_status s = ens_ready(c, S, false);
    if (s != KUR_OK) return s;
    if (!theta) return ctx_fail(c, KUR_EINVAL, "theta must not be NULL");
    const size_t cnt = (size_t)S->B * S->L.n;
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(theta[i]) || std::fabs(theta[i]) > 1e9) return ctx_fail(c, KUR_EINVAL, "theta must be finite with |theta| <= 1e9");
    return set_phases_impl(c, *S, theta);
}

kur_status kur_ens_eval_rhs(kur_ctx *c, double *dtheta)
{
    EnsState *S = nullptr;
    kur_status s = ens_ready(c, S, true);
    if (s != KUR_OK) return s;
    if (!dtheta) return ctx_fail(c, KUR_EINVAL, "dtheta must not be NULL");
    hipError_t e;
    if ((e = ensure_x(c, *S)) != hipSuccess || (e = launch_stage(c, *S, 0, 0.0)) != hipSuccess) return hipfail(c, e, "ensemble rhs");
    const int64_t n = S->L.n;
    const size_t NB = (size_t)n * S->Bp;
    if (ctx_esz(c) == 8) {
        std::vector<double> k(NB);
        if ((e = hipMemcpyAsync(k.data(), S->d_kout.p, 8 * NB, hipMemcpyDeviceToHost, ctx_stream(c))) != hipSuccess ||
            (e = hipStreamSynchronize(ctx_stream(c))) != hipSuccess)
            return hipfail(c, e, "ensemble rhs download");
        for (int32_t r = 0; r < S->B; ++r)
            for (int64_t u = 0; u < n; ++u) dtheta[(size_t)r * n + u] = k[(size_t)S->L.perm[u] * S->Bp + r];
        return KUR_OK;
    }
    std::vector<float> k(NB);
    if ((e = hipMemcpyAsync(k.data(), S->d_kout.p, 4 * NB, hipMemcpyDeviceToHost, ctx_stream(c))) != hipSuccess ||
        (e = hipStreamSynchronize(ctx_stream(c))) != hipSuccess)
        return hipfail(c, e, "ensemble rhs download");
    for (int32_t r = 0; r < S->B; ++r)
        for (int64_t u = 0; u < n; ++u) dtheta[(size_t)r * n + u] = k[(size_t)S->L.perm[u] * S->Bp + r];
    return KUR_OK;
}

kur_status kur_ens_step(kur_ctx *c, double dt, int64_t nsteps, int64_t r_every, double *r_out, double *psi_out)
{
    EnsState *S = nullptr;
    kur_status s = ens_ready(c, S, true);
    if (s != KUR_OK) return s;
    if (!std::isfinite(dt) || dt == 0.0) return ctx_fail(c, KUR_EINVAL, "dt must be finite and nonzero");
    if (nsteps < 0 || r_every < 0) return ctx_fail(c, KUR_EINVAL, "nsteps and r_every must be >= 0");
    const int64_t nsamp = r_every > 0 ? nsteps / r_every + 1 : 0;
    hipError_t e;
    if (nsamp > 0 && ((e = S->d_r.ensure(8 * (size_t)nsamp * S->B)) != hipSuccess ||
                      (e = S->d_psi.ensure(8 * (size_t)nsamp * S->B)) != hipSuccess))
        return hipfail(c, e, "sample buffers");
    if ((e = ensure_x(c, *S)) != hipSuccess) return hipfail(c, e, "ensemble sincos");
    int64_t k = 0;
    if (nsamp > 0 && (e = sample(c, *S, k++)) != hipSuccess) return hipfail(c, e, "ensemble sample");
    for (int64_t step = 0; step < nsteps; ++step) {
        for (int st4 = 1; st4 <= 4; ++st4)
            if ((e = launch_stage(c, *S, st4, dt)) != hipSuccess) return hipfail(c, e, "ensemble stage");
        if (r_every > 0 && (step + 1) % r_every == 0 && (e = sample(c, *S, k++)) != hipSuccess)
            return hipfail(c, e, "ensemble sample");
    }
    if (nsamp > 0 && (r_out || psi_out)) {
        std::vector<double> r((size_t)nsamp * S->B), p((size_t)nsamp * S->B);
        if ((e = hipMemcpyAsync(r.data(), S->d_r.p, 8 * r.size(), hipMemcpyDeviceToHost, ctx_stream(c))) != hipSuccess ||
            (e = hipMemcpyAsync(p.data(), S->d_psi.p, 8 * p.size(), hipMemcpyDeviceToHost, ctx_stream(c))) != hipSuccess ||
            (e = hipStreamSynchronize(ctx_stream(c))) != hipSuccess)
            return hipfail(c, e, "sample download");
        if (r_out) std::memcpy(r_out, r.data(), 8 * r.size());
        if (psi_out) std::memcpy(psi_out, p.data(), 8 * p.size());
    }
    return KUR_OK;
}

kur_status kur_ens_get_phases(kur_ctx *c, double *theta, int wrapped)
{
    EnsState *S = nullptr;
    kur_status s = ens_ready(c, S, true);
    if (s != KUR_OK) return s;
    if (!theta) return ctx_fail(c, KUR_EINVAL, "theta must not be NULL");
    const int64_t n = S->L.n;
    const size_t NB = (size_t)n * S->Bp, z = (size_t)ctx_esz(c);
    // the phase and its compensation term as stored (FP32 or FP64), widened to double below
    std::vector<unsigned char> hi(z * NB), lo(z * NB);
    std::vector<int32_t> wind(NB);
    const hipStream_t st = ctx_stream(c);
    hipError_t e;
    if ((e = hipMemcpyAsync(hi.data(), S->d_hi.p, z * NB, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(lo.data(), S->d_lo.p, z * NB, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync(wind.data(), S->d_wind.p, 4 * NB, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hipfail(c, e, "ensemble phase download");
    auto real_at = [&](const std::vector<unsigned char> &v, size_t i) {
        if (z == 8) {
            double d;
            std::memcpy(&d, v.data() + 8 * i, 8);
            return d;
        }
        float f;
        std::memcpy(&f, v.data() + 4 * i, 4);
        return (double)f;
    };
    const double P1 = two_pi_p1((int)z), P2 = two_pi_p2((int)z);
    for (int32_t r = 0; r < S->B; ++r)
        for (int64_t u = 0; u < n; ++u) {
            const size_t ix = (size_t)S->L.perm[u] * S->Bp + r;
            double x = real_at(hi, ix) + real_at(lo, ix);
            if (wrapped) {
                x = std::remainder(x, 2.0 * kPi);
                if (x >= kPi) x -= 2.0 * kPi;
            } else {
                x += (double)wind[ix] * P1 + (double)wind[ix] * P2;
            }
            theta[(size_t)r * n + u] = x;
        }
    return KUR_OK;
}

kur_status kur_ens_kernel_time(kur_ctx *c, double *out)
{
    if (!c || !out) return KUR_EINVAL;
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    if (ctx_is_device(c)) {
        hipError_t e = harvest(c, *S);
        if (e != hipSuccess) return hipfail(c, e, "ensemble timing");
    }
    out[0] = (double)S->t_n[0];
    out[1] = S->t_ms[0];
    out[2] = (double)S->t_n[1];
    out[3] = S->t_ms[1];
    S->t_n[0] = S->t_n[1] = 0;
    S->t_ms[0] = S->t_ms[1] = 0.0;
    return KUR_OK;
}

kur_status kur_ens_autotune_csr(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *labels,
                                int32_t B, int32_t effort, double *report)
{
    if (!c) return KUR_EINVAL;
    kur_status s = need_real(c);
    if (s != KUR_OK) return s;
    if (!ctx_is_device(c)) return ctx_fail(c, KUR_EDEVICE, "tuning needs a device context");
    if (effort < 0 || effort > 2) return ctx_fail(c, KUR_EINVAL, "effort must be 0, 1 or 2");
    if (B < 1 || B > kMaxReplicas) return ctx_fail(c, KUR_EINVAL, "B must be in [1, 256]");
    EnsState *S = state(c);
    if (!S) return ctx_fail(c, KUR_ENOMEM, "host allocation failed");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> taus = {0.0, 0.5, 2.0};
    if (effort >= 1) taus = {0.0, 0.25, 0.5, 0.75, 0.9, 2.0};
    if (effort >= 2) taus = {0.0, 0.1, 0.25, 0.4, 0.5, 0.6, 0.75, 0.85, 0.9, 0.95, 2.0};
    std::vector<std::vector<uint8_t>> seen;
    std::vector<double> seen_ms;
    double best_tau = ctx_ens_tau(c), best_ms = 1e300;
    int timed = 0;
    std::vector<double> density, pair_density;
    std::vector<int64_t> bsize;
    // which blocks and off-diagonal blocks a threshold puts on the matrix cores
    auto selection = [&](double tau) {
        std::vector<uint8_t> m(density.size() + pair_density.size());
        for (size_t b = 0; b < density.size(); ++b) m[b] = (bsize[b] >= 2 && density[b] >= tau) ? 1 : 0;
        for (size_t q = 0; q < pair_density.size(); ++q) m[density.size() + q] = pair_density[q] >= tau ? 1 : 0;
        return m;
    };
    for (double tau : taus) {
        if (!density.empty() && std::find(seen.begin(), seen.end(), selection(tau)) != seen.end()) continue;
        EnsLayout L;
        std::string msg;
        try {
            msg = build_layout(n, row_ptr, col, labels, tau, L);
        } catch (const std::bad_alloc &) {
            return ctx_fail(c, KUR_ENOMEM, "host allocation failed while building the ensemble layout");
        }
        if (!msg.empty()) return ctx_fail(c, KUR_EINVAL, msg);
        if (density.empty()) {
            density = L.density;
            pair_density = L.pair_density;
            for (int32_t b = 0; b < L.nb; ++b) bsize.push_back(L.block_ptr[b + 1] - L.block_ptr[b]);
        }
        seen.push_back(selection(tau));
        if ((s = install_layout(c, *S, L)) != KUR_OK) return s;
        std::vector<double> K(B, 1.0), om((size_t)B * n, 0.0), th((size_t)B * n);
        for (size_t i = 0; i < th.size(); ++i) th[i] = 2.0 * kPi * std::fmod(0.6180339887498949 * (double)i, 1.0);
        if ((s = set_params_impl(c, *S, B, K.data(), om.data())) != KUR_OK || (s = set_phases_impl(c, *S, th.data())) != KUR_OK)
            return s;
        double ms = 0.0;
        if ((s = time_steps(c, *S, 3, &ms)) != KUR_OK) return s;
        ++timed;
        seen_ms.push_back(ms);
        if (ms < best_ms) {
            best_ms = ms;
            best_tau = tau;
        }
    }
    // the two extremes: every block on the matrix cores (first candidate, tau = 0) and none
    double ms_none = NAN;
    for (size_t i = 0; i < seen.size(); ++i)
        if (std::find(seen[i].begin(), seen[i].end(), (uint8_t)1) == seen[i].end()) ms_none = seen_ms[i];
    ctx_set_ens_tau(c, best_tau);
    if ((s = kur_ens_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
    if (report) {
        report[0] = best_tau;
        report[1] = best_ms;
        report[2] = seen_ms.empty() ? NAN : seen_ms[0];
        report[3] = ms_none;
        report[4] = timed;
        report[5] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return KUR_OK;
}

}  // extern "C"
