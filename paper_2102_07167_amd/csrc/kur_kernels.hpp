// kur_kernels.hpp -- device-side argument blocks and kernel launchers (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kur_internal.hpp"

namespace kur {

// The graph in device memory (block order).
struct DevGraph {
    const BlkInfo *blk;
    const Tile *tiles;
    const int32_t *order;
    const int64_t *seg_ptr;
    const uint16_t *list;
    const int64_t *inter_ptr;
    const int32_t *inter_col;
    int32_t W;
    int32_t tile_rows;
};

// Arguments of one row-kernel launch (one RK stage, or a plain evaluation when stage == 0).
template <typename T>
struct RowArgs {
    int stage;          // 0: write F to kout; 1..4: classical RK4 stage
    int compensate;     // compensated phase update in stage 4
    T dt, half_dt, dt6; // dt, dt/2, dt/6
    T kscale;           // K/N when rowscale == nullptr
    const T *rowscale;  // per-row coupling factor (K/deg_m), or nullptr
    const T *omega;
    T *hi;              // wrapped phase
    T *lo;              // compensation term
    int32_t *wind;      // winding count
    T *ksum;            // k1 + 2 k2 + 2 k3 accumulator
    T *kout;            // stage 0 output
    const void *sc_in;  // (sin, cos) of the stage input
    void *sc_out;       // (sin, cos) of the next stage input
    const void *part_in;
    void *part_out;
};

template <typename T>
hipError_t launch_sc_init(const DevGraph &g, int ntiles, const T *y, void *sc, void *part, int threads, hipStream_t st);
template <typename T>
hipError_t launch_rows(const DevGraph &g, int ntiles, const RowArgs<T> &a, int threads, hipStream_t st);
template <typename T>
hipError_t launch_order(const void *part, int ntiles, int64_t n, double *r, double *psi, int64_t idx, hipStream_t st);
template <typename T>
hipError_t launch_phase_out(int64_t n, const void *hi, const void *lo, const int32_t *wind, int unwrapped, void *out,
                            hipStream_t st);

size_t rows_lds_bytes(int elem_bytes, int W, int tile_rows, int threads);
double two_pi_p1(int elem_bytes);
double two_pi_p2(int elem_bytes);

}  // namespace kur
