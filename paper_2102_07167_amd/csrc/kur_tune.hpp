// kur_tune.hpp -- hooks into the context for the layout autotuner (autotune.cpp) and the
// shared-graph ensemble path (ensemble.cpp): re-tiling, timing, block densities, the device,
// stream and options of a context; implemented in kur_api.cpp.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/kur.h"

namespace kur {

// Options that only change how rows are grouped into tiles or how the row kernel gathers (no list
// rebuild).
struct TileParams {
    int32_t threads = 512;
    int32_t tile_rows = 256;
    int64_t tile_min_cost = 16384;
    double flat_min_vec = 8.0;
    int32_t xcds = 1;
    int32_t inter_gather = -1;  // inter-block gathers: 1 phases, 0 (sin, cos) pairs, -1 the dtype's default
    bool operator==(const TileParams &o) const
    {
        return threads == o.threads && tile_rows == o.tile_rows && tile_min_cost == o.tile_min_cost &&
               flat_min_vec == o.flat_min_vec && xcds == o.xcds && inter_gather == o.inter_gather;
    }
    bool operator!=(const TileParams &o) const { return !(*this == o); }
};

// Options that change the stored lists (a rebuild from the adjacency).
struct LayoutParams {
    double tau = 0.5;
    int32_t chunk = 4096;
    double mask_min = 2.0;  // bitmask segments from this many list entries per cell (above 1: none)
    bool operator==(const LayoutParams &o) const
    {
        return tau == o.tau && chunk == o.chunk && mask_min == o.mask_min;
    }
    bool operator!=(const LayoutParams &o) const { return !(*this == o); }
};

struct EnsState;                    // ensemble.cpp
void ens_free(EnsState *s);         // ensemble.cpp
EnsState *&ctx_ens_slot(kur_ctx *c);
int ctx_device(const kur_ctx *c);
hipStream_t ctx_stream(const kur_ctx *c);
int ctx_timing(const kur_ctx *c);
int ctx_compensate(const kur_ctx *c);
double ctx_ens_tau(const kur_ctx *c);
void ctx_set_ens_tau(kur_ctx *c, double tau);

bool ctx_is_device(const kur_ctx *c);
bool ctx_has_graph(const kur_ctx *c);
int ctx_esz(const kur_ctx *c);
std::string ctx_arch(const kur_ctx *c);
kur_status ctx_fail(kur_ctx *c, kur_status s, const std::string &msg);
// tile options of the installed layout, and the options the next build will use
TileParams ctx_tile_params(const kur_ctx *c);
LayoutParams ctx_layout_params(const kur_ctx *c);
// sets the options of the next build (validated like kur_set_option)
kur_status ctx_set_build_options(kur_ctx *c, const LayoutParams &l, const TileParams &t);
// whether a layout fits the LDS of a workgroup: the row kernel, and the adjoint kernel when the
// installed graph is symmetric (so that tuning never makes the adjoint unavailable); chunk <= 0:
// the installed chunk width
bool ctx_layout_fits(const kur_ctx *c, int32_t chunk, const TileParams &t);
// re-groups the installed graph's rows into tiles with t (lists untouched)
kur_status ctx_retile(kur_ctx *c, const TileParams &t);
// best of `trials` timings of whole RK4 steps with HIP events, in ms per step; the phases, the
// compensation terms and the winding counts are restored afterwards
kur_status ctx_time_steps(kur_ctx *c, int trials, double *ms_per_step);
// realised density and size of every block of the installed graph, and the densities of its
// nonzero off-diagonal blocks large enough to be made dense
void ctx_block_stats(const kur_ctx *c, std::vector<double> &density, std::vector<int32_t> &size,
                     std::vector<double> &pair_density);
// the chunk width limit of the context's dtype (16-bit LDS byte offsets)
int32_t ctx_max_chunk(const kur_ctx *c);

}  // namespace kur
