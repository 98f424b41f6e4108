// kur_kernels.hpp -- device-side argument blocks and kernel launchers (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kur_internal.hpp"

namespace kur {

// The graph in device memory (block order).
struct DevGraph {
    const BlkInfo *blk;
    const SegD *segd;
    const Grp *grp;
    const Tile *tiles;
    const int32_t *order;
    const int64_t *seg_ptr;
    const uint16_t *list;
    const uint32_t *mask;  // bitmask segments, 4 words per unit (see SegD)
    const int64_t *inter_ptr;
    const int32_t *inter_col;
    int32_t W;
    int32_t tile_rows;
    int32_t nlaunch;  // entries of order (workgroups of a tile launch); -1 entries are empty slots
    void *msum;       // the bitmask items' partial sums (see MaskItem), one (x, y) pair of the dtype
                      // per row, written by k_mask before every tile-kernel launch; null when the
                      // layout has no bitmask segment
    const MaskItem *mitem;  // bitmask items in launch order
    const MaskTile *mtile;  // per tile its items' partial sums
    int32_t nmitem;
    int32_t mask_sub;       // columns of a bitmask sub-chunk
};

// Arguments of one row-kernel launch (one RK stage, or a plain evaluation when stage == 0).
// The coupling factor of row m is K * unit[m] (unit = 1/deg_m) or K * inv_n when unit is null.
template <typename T>
struct RowArgs {
    int stage;          // 0: write F to kout; -1: write the coupling energy (see k_rows); 1..4: RK4 stage
    int compensate;     // compensated phase update in stage 4
    T dt, half_dt, dt6; // dt, dt/2, dt/6
    T K, inv_n;
    const T *unit;
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
    void *ac_out;       // stages 1..4: if not null, ((A sin y)_m, (A cos y)_m) of the stage input
    const T *y_in;      // if not null: the stage input y itself; the inter-block gathers then read
                        // y_l and form (sin y_l, cos y_l) (the same values as sc_in) instead of
                        // reading the pair
    T *y_out;           // stages 1..3: if not null, receives the next stage input y
};

// Arguments of one stage of the embedded Runge-Kutta pair (variable step size). Stage i of s
// stores k_i = F(Y_i) and forms Y_{i+1} = theta + dt sum_{j <= i} coef[j] k_j; the last stage
// forms the candidate theta + dt sum_j coef[j] k_j (coef = the propagated weights) into the
// *_new arrays and the per-tile maximum of |dt sum_j coef2[j] k_j| (coef2 = the difference of
// the two weight rows, the local error estimate).
template <typename T>
struct EmbArgs {
    int stage;          // 1..nstages
    int nstages;
    int compensate;
    T dt;
    T K, inv_n;
    const T *unit;
    const T *omega;
    const T *hi, *lo;         // start of the step (read only)
    const int32_t *wind;
    T *hi_new, *lo_new;       // candidate (last stage)
    int32_t *wind_new;
    T *kbuf;                  // nstages x n stage derivatives
    int64_t n;
    T coef[8];
    T coef2[8];
    T *err_part;              // per tile (last stage)
    const void *sc_in;
    void *sc_out;
    const void *part_in;
    void *part_out;
};

template <typename T>
hipError_t launch_emb(const DevGraph &g, const EmbArgs<T> &a, int threads, hipStream_t st);
// out[0] = max of in[0..n) (n >= 1), one workgroup
template <typename T>
hipError_t launch_max_fold(int64_t n, const T *in, T *out, hipStream_t st);

// Arguments of one reverse RK4 stage (Jacobian-transpose product and adjoint bookkeeping).
template <typename T>
struct VjpArgs {
    int stage;          // 4, 3, 2, 1 (k_vjp); unused by k_vjp_init
    T K, inv_n;
    const T *unit;
    T cl, cm;           // l_{i-1} = cl * lam + cm * mu_i (k_vjp); l_4 = cl * lam (k_vjp_init)
    const void *x_in;   // (w s, w c) at Y_i
    const void *part_in;
    void *x_out;        // the same for the next stage
    void *part_out;
    const void *sc_cur; // (sin, cos) at Y_i
    const void *sc_next;// (sin, cos) of the next stage's state; at stage 1, if not null, the Y_4
                        // of the next reverse step, whose start (k_vjp_init's work) is then done here
    T *lam;             // dL/dtheta at the end of the step; the start of the step after stage 1
    T *lam_acc;         // lam + sum of mu_i
    T *lbuf;            // l_i
    double *g_omega;    // dL/domega, accumulated
    double *gk_part;    // per tile dL/dK, accumulated
    const void *ac_rows;// ((A s)_m, (A c)_m) at Y_i, kept by the forward recompute (the gathers run
                        // over the lists of A^T, which are A's own for symmetric A)
};
template <typename T>
hipError_t launch_sc_init(const DevGraph &g, int ntiles, const T *y, void *sc, void *part, int threads, hipStream_t st);
template <typename T>
hipError_t launch_rows(const DevGraph &g, int ntiles, const RowArgs<T> &a, int threads, hipStream_t st);
template <typename T>
hipError_t launch_order(const void *part, const int64_t *tile_first, const double *inv_n, int n_inst, double *r,
                        double *psi, const int64_t *idx_dev, int64_t idx, hipStream_t st);
hipError_t launch_bump(int64_t *ctr, hipStream_t st);
hipError_t launch_stream_read(const void *p, int64_t words, uint32_t *out, hipStream_t st);
template <typename T>
hipError_t launch_phase_out(int64_t n, const void *hi, const void *lo, const int32_t *wind, int unwrapped, void *out,
                            hipStream_t st);

// nsteps classical RK4 steps of the complete graph (Sec. 2, the classical model through its order
// parameter) in one workgroup that keeps every oscillator's state in registers: per stage a
// fixed-order block sum of (sin y, cos y), then the right-hand side and the stage bookkeeping of
// every row. r and psi are written for steps 0, r_every, 2 r_every, ... below nsteps, and for
// nsteps itself when final_sample (r_every > 0): the kernel stores the mean (sin, cos) of each
// sample there and a one-workgroup pass converts them.
constexpr int kPersistThreads = 512;
constexpr int kPersistMaxRows = 2;  // rows per thread: n <= 1024
template <typename T>
struct PersistArgs {
    int64_t n;
    int64_t nsteps;
    int64_t r_every;
    int final_sample;
    int compensate;
    T dt, half_dt, dt6;
    T K, inv_n;
    const T *unit;
    const T *omega;
    T *hi, *lo;
    int32_t *wind;
    double *r_out, *psi_out;
    T *ck;              // if not null: (hi, lo) before global step s (s a multiple of ck_every) to
    int64_t ck_every;   // ck + 2 n (s / ck_every); step0 is the global index of this launch's
    int64_t step0;      // first step
};
template <typename T>
hipError_t launch_persist_complete(const PersistArgs<T> &a, hipStream_t st);

// The discrete adjoint of the one-workgroup RK4 run of the complete graph (same arithmetic as
// k_vjp on the complete graph's single dense block). One launch sweeps the checkpoint segments
// seg_hi down to seg_lo: each is recomputed from its checkpoint, keeping the (sin, cos) of every
// stage input in ystore, then swept in reverse. lam, g_omega and gk_part carry the state between
// launches.
template <typename T>
struct PersistAdjArgs {
    int64_t n, nsteps, ck_every;
    int64_t seg_hi, seg_lo;
    int compensate;
    T dt, half_dt, dt6, dt3;
    T K, inv_n;
    const T *unit;
    const T *omega;
    const T *ck;        // checkpoint s: (hi, lo) at step s ck_every, at ck + 2 n s
    T *ystore;          // (sin, cos) of the 4 ck_every stage inputs of one segment: 8 ck_every n
    T *lam;             // dL/dtheta at the end of segment seg_hi (in); at the start of seg_lo (out)
    double *g_omega;    // dL/domega, accumulated
    double *gk_part;    // kPersistThreads partial sums of dL/dK, accumulated
};
template <typename T>
hipError_t launch_persist_adjoint(const PersistAdjArgs<T> &a, hipStream_t st);

template <typename T>
hipError_t launch_vjp(const DevGraph &g, int ntiles, const VjpArgs<T> &a, int threads, hipStream_t st);
template <typename T>
hipError_t launch_vjp_init(const DevGraph &g, int ntiles, const VjpArgs<T> &a, int threads, hipStream_t st);

// Dynamic LDS bytes of a tile workgroup gathering nv (sin, cos)-sized pairs per node.
// Diagnostics at the current state: out[0..3) = (sum of unwrapped theta, sum of omega,
// sum_m -omega_m theta_m - K/2 scale_m e_m) with e the rows' coupling energies; part holds
// 3 ceil(n / 256) doubles of scratch.
template <typename T>
hipError_t launch_diag(int64_t n, const void *hi, const void *lo, const int32_t *wind, const void *omega,
                       const void *unit, const void *e, double K, double *part, double *out, hipStream_t st);

size_t rows_lds_bytes(int elem_bytes, int W, int tile_rows, int threads);
double two_pi_p1(int elem_bytes);
double two_pi_p2(int elem_bytes);

}  // namespace kur
