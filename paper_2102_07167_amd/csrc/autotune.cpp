// autotune.cpp -- picks the layout options of the row kernel by timing whole RK4 steps on the
// device: the tile shape (rows per tile, least work per tile, lanes-per-row versus wave
// streaming, threads per workgroup), the chunk width of the LDS-staged (sin, cos) columns, and
// the density threshold tau above which a block stores its zeros (localised order parameters)
// rather than its ones (Introduction and Sec. 3: precomputed block sums pay off once a block
// holds more ones than zeros, which makes tau = 1/2 the byte-minimal threshold; the timing
// decides whether another value runs faster on this device), and whether segments dense in list
// entries are stored as bitmasks (option mask_min).
//
// The search is a coordinate descent: each option in turn is set to every candidate value while
// the others keep their best values so far, and a candidate replaces the incumbent only when it
// is at least 1 % faster. Tile options re-group the installed rows (no list rebuild); tau, the
// chunk width and the bitmask threshold rebuild the lists from the adjacency. Results are kept in a plain-text cache,
// one line per graph signature, so a graph of the same shape on the same device is configured
// without timing.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/kur.h"
#include "kur_internal.hpp"
#include "kur_tune.hpp"

using namespace kur;

namespace {

constexpr double kGain = 0.99;  // a candidate must take at most 99 % of the incumbent's time

uint64_t mix(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Signature of a graph's shape: dtype, device, n, edge count and a hash of row offsets and
// labels sampled at about 4096 rows. Equal signatures are taken to want equal layouts; a
// collision can only cost speed, never correctness.
std::string graph_key(const kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *labels)
{
    uint64_t h = mix((uint64_t)n) ^ mix((uint64_t)row_ptr[n] + 0x51ull);
    const int64_t stride = std::max<int64_t>(1, n / 4096);
    for (int64_t i = 0; i < n; i += stride) {
        h = mix(h ^ (uint64_t)row_ptr[i + 1]);
        h = mix(h ^ (uint64_t)(uint32_t)labels[i]);
    }
    char buf[256];
    std::snprintf(buf, sizeof(buf), "kur2 %s %s n=%lld nnz=%lld h=%016llx", ctx_esz(c) == 4 ? "f32" : "f64",
                  ctx_arch(c).c_str(), (long long)n, (long long)row_ptr[n], (unsigned long long)h);
    return buf;
}

struct Choice {
    LayoutParams l;
    TileParams t;
    double ms = 1e300;
};

// Cache lines: "<key>\t<tau> <chunk> <threads> <tile_rows> <tile_min_cost> <flat_min_vec> <xcds> <ms>
// [<inter_gather> [<mask_min>]]" (without the inter_gather field the dtype's default gathers,
// without mask_min no bitmask segments). The last line with a matching key wins; malformed lines
// are skipped.
bool cache_lookup(const char *path, const std::string &key, Choice &out)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        char *tab = std::strchr(line, '\t');
        if (!tab || (size_t)(tab - line) != key.size() || std::strncmp(line, key.c_str(), key.size()) != 0) continue;
        Choice ch;
        int chunk = 0, threads = 0, rows = 0, xcds = 0, ig = -1;
        long long cost = 0;
        double mm = 2.0;
        const int got = std::sscanf(tab + 1, "%lf %d %d %d %lld %lf %d %lf %d %lf", &ch.l.tau, &chunk, &threads,
                                    &rows, &cost, &ch.t.flat_min_vec, &xcds, &ch.ms, &ig, &mm);
        if (got < 8 || got > 10) continue;
        if (got >= 9 && ig != 0 && ig != 1) continue;
        if (got == 10 && !(mm >= 0.0 && mm <= 1e9)) continue;
        ch.t.inter_gather = got >= 9 ? ig : -1;
        ch.l.mask_min = got == 10 ? mm : 2.0;
        ch.t.xcds = xcds;
        ch.l.chunk = chunk;
        ch.t.threads = threads;
        ch.t.tile_rows = rows;
        ch.t.tile_min_cost = cost;
        out = ch;
        found = true;
    }
    std::fclose(f);
    return found;
}

bool cache_store(const char *path, const std::string &key, const Choice &ch)
{
    if (!path) return true;
    FILE *f = std::fopen(path, "a");
    if (!f) return false;
    const int r = std::fprintf(f, "%s\t%.17g %d %d %d %lld %.17g %d %.6g %d %.17g\n", key.c_str(), ch.l.tau,
                               ch.l.chunk, ch.t.threads, ch.t.tile_rows, (long long)ch.t.tile_min_cost,
                               ch.t.flat_min_vec, ch.t.xcds, ch.ms, ch.t.inter_gather, ch.l.mask_min);
    return std::fclose(f) == 0 && r > 0;
}

struct Search {
    kur_ctx *c;
    int effort;
    int timed = 0;
    int builds = 0;
};

std::vector<int64_t> cost_values(int effort)
{
    if (effort == 0) return {8192, 32768};
    if (effort == 1) return {4096, 8192, 32768, 65536};
    return {2048, 4096, 8192, 32768, 65536, 131072, 262144};
}

std::vector<int32_t> row_values(int effort)
{
    if (effort == 0) return {128, 512};
    if (effort == 1) return {64, 128, 512, 1024};
    return {64, 128, 512, 1024, 2048, 4096};
}

std::vector<double> flat_values(int effort)
{
    // 0 turns wave streaming off (every tile uses lanes per row)
    if (effort == 0) return {4, 16};
    if (effort == 1) return {0, 2, 4, 16};
    return {0, 1, 2, 4, 16, 32};
}

// Coordinate descent over the tile options of the installed graph, starting from `best` (the
// installed options, already timed). Leaves the best tile layout installed.
kur_status search_tiles(Search &S, Choice &best)
{
    const int sweeps = S.effort >= 2 ? 2 : 1;
    for (int sweep = 0; sweep < sweeps; ++sweep) {
        for (int dim = 0; dim < 6; ++dim) {
            std::vector<TileParams> cands;
            if (dim == 0)
                for (int64_t v : cost_values(S.effort)) { TileParams t = best.t; t.tile_min_cost = v; cands.push_back(t); }
            if (dim == 1)
                for (int32_t v : {128, 256, 512, 1024}) { TileParams t = best.t; t.threads = v; cands.push_back(t); }
            if (dim == 2)
                for (int32_t v : row_values(S.effort)) { TileParams t = best.t; t.tile_rows = v; cands.push_back(t); }
            if (dim == 3)
                for (double v : flat_values(S.effort)) { TileParams t = best.t; t.flat_min_vec = v; cands.push_back(t); }
            if (dim == 4)  // XCD-aware launch order on or off
                for (int32_t v : {1, 8}) { TileParams t = best.t; t.xcds = v; cands.push_back(t); }
            if (dim == 5)  // inter-block gathers of phases or of (sin, cos) pairs
                for (int32_t v : {0, 1}) { TileParams t = best.t; t.inter_gather = v; cands.push_back(t); }
            const TileParams incumbent = best.t;
            for (const TileParams &t : cands) {
                if (t == incumbent || t == best.t || !ctx_layout_fits(S.c, 0, t)) continue;
                kur_status s = ctx_retile(S.c, t);
                if (s != KUR_OK) return s;
                double ms = 0.0;
                if ((s = ctx_time_steps(S.c, 3, &ms)) != KUR_OK) return s;
                ++S.timed;
                if (ms < best.ms * kGain) {
                    best.t = t;
                    best.ms = ms;
                }
            }
        }
    }
    if (ctx_tile_params(S.c) != best.t) return ctx_retile(S.c, best.t);
    return KUR_OK;
}

// Which blocks and off-diagonal blocks a threshold makes dense; two thresholds with equal
// patterns build equal layouts.
std::vector<uint8_t> modes_for(const std::vector<double> &rho, const std::vector<int32_t> &size,
                               const std::vector<double> &pair_rho, double tau)
{
    std::vector<uint8_t> m(rho.size() + pair_rho.size());
    for (size_t b = 0; b < rho.size(); ++b) m[b] = (size[b] >= 2 && rho[b] >= tau) ? 1 : 0;
    for (size_t p = 0; p < pair_rho.size(); ++p) m[rho.size() + p] = pair_rho[p] >= tau ? 1 : 0;
    return m;
}

void fill_report(double *report, const Choice &best, double ms_default, const Search &S, double from_cache,
                 double seconds)
{
    if (!report) return;
    report[0] = best.l.tau;
    report[1] = best.l.chunk;
    report[2] = best.t.threads;
    report[3] = best.t.tile_rows;
    report[4] = (double)best.t.tile_min_cost;
    report[5] = best.t.flat_min_vec;
    report[6] = best.ms;
    report[7] = ms_default;
    report[8] = S.timed;
    report[9] = from_cache;
    report[10] = S.builds;
    report[11] = seconds;
    report[12] = best.t.xcds;
    report[13] = best.t.inter_gather;
}

}  // namespace

extern "C" kur_status kur_tune_key(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *labels, char *buf,
                                   size_t len)
{
    if (!c || !buf || len == 0) return KUR_EINVAL;
    if (n < 1 || n > INT32_MAX - 1 || !row_ptr || !labels) return ctx_fail(c, KUR_EINVAL, "invalid graph arguments");
    const std::string key = graph_key(c, n, row_ptr, labels);
    if (key.size() + 1 > len) return ctx_fail(c, KUR_EINVAL, "key buffer too small");
    std::memcpy(buf, key.c_str(), key.size() + 1);
    return KUR_OK;
}

extern "C" kur_status kur_tune_tiles(kur_ctx *c, int32_t effort, double *report)
{
    if (!c) return KUR_EINVAL;
    if (effort < 0 || effort > 2) return ctx_fail(c, KUR_EINVAL, "effort must be 0, 1 or 2");
    if (!ctx_is_device(c)) return ctx_fail(c, KUR_EDEVICE, "tuning needs a device context");
    if (!ctx_has_graph(c)) return ctx_fail(c, KUR_ESTATE, "no graph set");
    const auto t0 = std::chrono::steady_clock::now();
    Search S{c, effort};
    Choice best;
    best.l = ctx_layout_params(c);
    best.t = ctx_tile_params(c);
    kur_status s = ctx_time_steps(c, 3, &best.ms);
    if (s != KUR_OK) return s;
    ++S.timed;
    const double ms_default = best.ms;
    if ((s = search_tiles(S, best)) != KUR_OK) return s;
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    fill_report(report, best, ms_default, S, 0.0, sec);
    return KUR_OK;
}

extern "C" kur_status kur_autotune_csr(kur_ctx *c, int64_t n, const int64_t *row_ptr, const int32_t *col,
                                       const int32_t *labels, int32_t effort, const char *cache_path, double *report)
{
    if (!c) return KUR_EINVAL;
    if (effort < 0 || effort > 2) return ctx_fail(c, KUR_EINVAL, "effort must be 0, 1 or 2");
    if (n < 1 || n > INT32_MAX - 1 || !row_ptr || !labels) return ctx_fail(c, KUR_EINVAL, "invalid graph arguments");
    const auto t0 = std::chrono::steady_clock::now();
    auto seconds = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    const std::string key = graph_key(c, n, row_ptr, labels);
    Search S{c, effort};
    Choice best;
    kur_status s;
    if (cache_lookup(cache_path, key, best)) {
        if ((s = ctx_set_build_options(c, best.l, best.t)) != KUR_OK) return s;
        if ((s = kur_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
        S.builds = 1;
        fill_report(report, best, NAN, S, 1.0, seconds());
        return KUR_OK;
    }
    if (!ctx_is_device(c)) return ctx_fail(c, KUR_EDEVICE, "tuning needs a device context (no cached entry for this graph)");

    // the options in force are the starting point
    best.l = ctx_layout_params(c);
    if ((s = kur_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
    S.builds = 1;
    best.t = ctx_tile_params(c);
    if ((s = ctx_time_steps(c, 3, &best.ms)) != KUR_OK) return s;
    ++S.timed;
    const double ms_default = best.ms;
    const LayoutParams l0 = best.l;
    if ((s = search_tiles(S, best)) != KUR_OK) return s;

    std::vector<double> rho, pair_rho;
    std::vector<int32_t> size;
    ctx_block_stats(c, rho, size, pair_rho);
    int32_t max_block = 0;
    for (int32_t v : size) max_block = std::max(max_block, v);
    Choice installed = best;

    // density threshold
    std::vector<double> taus;
    if (effort == 1) taus = {0.4, 0.6};
    if (effort >= 2) taus = {0.3, 0.4, 0.45, 0.55, 0.6, 0.7};
    std::vector<std::vector<uint8_t>> seen = {modes_for(rho, size, pair_rho, best.l.tau)};
    for (double tau : taus) {
        const std::vector<uint8_t> m = modes_for(rho, size, pair_rho, tau);
        if (std::find(seen.begin(), seen.end(), m) != seen.end()) continue;  // same layout as one timed
        seen.push_back(m);
        Choice cand = best;
        cand.l.tau = tau;
        if ((s = ctx_set_build_options(c, cand.l, cand.t)) != KUR_OK) return s;
        if ((s = kur_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
        ++S.builds;
        if ((s = ctx_time_steps(c, 3, &cand.ms)) != KUR_OK) return s;
        ++S.timed;
        installed = cand;
        if (cand.ms < best.ms * kGain) best = cand;
    }

    // chunk width: the largest block rounded up to 64 columns (least LDS when every block fits
    // one chunk), then half and the maximum
    std::vector<int32_t> chunks;
    const int32_t wmax = ctx_max_chunk(c);
    const int32_t fit = std::min(wmax, std::max<int32_t>(64, (max_block + 63) / 64 * 64));
    if (fit < best.l.chunk) chunks.push_back(fit);
    if (effort >= 1) {
        chunks.push_back(std::max<int32_t>(64, best.l.chunk / 2 / 64 * 64));
        chunks.push_back(wmax);
    }
    if (effort >= 2) chunks.push_back(std::max<int32_t>(64, best.l.chunk / 4 / 64 * 64));
    std::vector<int32_t> tried = {best.l.chunk};
    for (int32_t w : chunks) {
        if (std::find(tried.begin(), tried.end(), w) != tried.end()) continue;
        if (w > fit && best.l.chunk >= fit) continue;  // every block already fits one chunk
        if (!ctx_layout_fits(c, w, best.t)) continue;
        tried.push_back(w);
        Choice cand = best;
        cand.l.chunk = w;
        if ((s = ctx_set_build_options(c, cand.l, cand.t)) != KUR_OK) return s;
        if ((s = kur_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
        ++S.builds;
        if ((s = ctx_time_steps(c, 3, &cand.ms)) != KUR_OK) return s;
        ++S.timed;
        installed = cand;
        if (cand.ms < best.ms * kGain) best = cand;
    }

    // bitmask segments (needs a chunk of at least kMaskMinW): off, or from a list density
    std::vector<double> mask_mins;
    if (best.l.chunk >= kMaskMinW) {
        if (effort == 1) mask_mins = {0.2, 0.3};
        if (effort >= 2) mask_mins = {0.2, 0.3, 0.4};
        if (best.l.mask_min <= 1.0) mask_mins.push_back(2.0);
    }
    for (double mm : mask_mins) {
        if (mm == best.l.mask_min) continue;
        Choice cand = best;
        cand.l.mask_min = mm;
        if ((s = ctx_set_build_options(c, cand.l, cand.t)) != KUR_OK) return s;
        if ((s = kur_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
        ++S.builds;
        if ((s = ctx_time_steps(c, 3, &cand.ms)) != KUR_OK) return s;
        ++S.timed;
        installed = cand;
        if (cand.ms < best.ms * kGain) best = cand;
    }

    // install the winner, and re-tune its tiles if the lists changed
    if (installed.l != best.l || installed.t != best.t) {
        if ((s = ctx_set_build_options(c, best.l, best.t)) != KUR_OK) return s;
        if ((s = kur_set_graph_csr(c, n, row_ptr, col, labels)) != KUR_OK) return s;
        ++S.builds;
    }
    if (best.l != l0) {
        double ms = 0.0;
        if ((s = ctx_time_steps(c, 3, &ms)) != KUR_OK) return s;
        ++S.timed;
        best.ms = ms;
        if ((s = search_tiles(S, best)) != KUR_OK) return s;
    }
    if ((s = ctx_set_build_options(c, best.l, best.t)) != KUR_OK) return s;
    const bool stored = cache_store(cache_path, key, best);
    fill_report(report, best, ms_default, S, stored ? 0.0 : -1.0, seconds());
    return KUR_OK;
}
