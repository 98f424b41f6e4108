/*
 * kur_oracle.c -- CPU reference for the Kuramoto model on graphs.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously correct definition that the GPU
 * library is checked against. Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it; the library never calls it and shares no code, header or table with it.
 *
 * Everything is IEEE double, plain loops, one term at a time, in the order the definition
 * states. OpenMP only distributes independent rows; every row is summed sequentially in
 * increasing column order, so results do not depend on the thread count.
 *
 * Model (Sec. 3, eq. KuramotoGraph):
 *     theta_m' = omega_m + K / Mscale_m * sum_{l : A_ml = 1} sin(theta_l - theta_m)
 * with uniform scaling Mscale_m = N or non-uniform scaling Mscale_m = sum_l A_ml (a zero row
 * then leaves theta_m' = omega_m). The classical model (Sec. 2, eq. Kuramoto) is the complete
 * graph A_ml = 1 for l != m; the diagonal term sin(0) = 0 is left out (Sec. 2, remark on
 * coinciding indices).
 *
 * Time integration: the classical fourth-order Runge-Kutta method with a fixed step, on the
 * unwrapped phases. Order parameter (Sec. 2, eq. OrderParameter): r e^{i psi} = (1/N) sum e^{i theta}.
 * Gradients: the discrete adjoint of that Runge-Kutta map (the exact derivative of the computed
 * trajectory), built from the Jacobian-transpose product of the right-hand side.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int64_t n;
    int complete;            /* 1: all pairs l != m coupled; row_ptr/col unused */
    const int64_t *row_ptr;  /* CSR, n+1 */
    const int32_t *col;      /* neighbours of row m: col[row_ptr[m] .. row_ptr[m+1]) */
    const int32_t *w;        /* integer value A_ml of every entry (NULL: all 1) */
    int scaling;             /* 0: uniform K/N; 1: K/deg_m with deg_m = sum_l A_ml */
} orc_graph;

static double weight_of(const orc_graph *g, int64_t e) { return g->w ? (double)g->w[e] : 1.0; }

static double row_scale(const orc_graph *g, int64_t m)
{
    if (g->scaling == 0) return 1.0 / (double)g->n;
    double deg = 0.0;
    if (g->complete) {
        deg = (double)(g->n - 1);
    } else {
        for (int64_t e = g->row_ptr[m]; e < g->row_ptr[m + 1]; ++e)
            if (g->col[e] != m) deg += weight_of(g, e);
    }
    return deg > 0 ? 1.0 / deg : 0.0;
}

/* sum_l A_ml sin(theta_l - theta_m), straightforward summation (Sec. 3, eq.
 * KuramotoGraphApproach, first case, applied to the whole row) */
static double coupling_sum(const orc_graph *g, const double *theta, int64_t m)
{
    double acc = 0.0;
    if (g->complete) {
        for (int64_t l = 0; l < g->n; ++l)
            if (l != m) acc += sin(theta[l] - theta[m]);
    } else {
        for (int64_t e = g->row_ptr[m]; e < g->row_ptr[m + 1]; ++e)
            acc += weight_of(g, e) * sin(theta[g->col[e]] - theta[m]);
    }
    return acc;
}

static void rhs(const orc_graph *g, const double *omega, double K, const double *theta, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < g->n; ++m)
        out[m] = omega[m] + K * row_scale(g, m) * coupling_sum(g, theta, m);
}

/* F(theta) for all rows */
void orc_rhs(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
             const double *omega, double K, const double *theta, double *out)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    rhs(&g, omega, K, theta, out);
}

/* F(theta) for a subset of rows: out[i] = F_{rows[i]}(theta) */
void orc_rhs_rows(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
                  const double *omega, double K, const double *theta, int64_t nrows,
                  const int64_t *rows, double *out)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nrows; ++i) {
        int64_t m = rows[i];
        out[i] = omega[m] + K * row_scale(&g, m) * coupling_sum(&g, theta, m);
    }
}

/* threads of the parallel row loops (timing reports only) */
int orc_threads(void) { return omp_get_max_threads(); }

/* r and psi of (1/N) sum_m e^{i theta_m} (Sec. 2, eq. OrderParameter) */
void orc_order_parameter(int64_t n, const double *theta, double *r, double *psi)
{
    double c = 0.0, s = 0.0;
    for (int64_t m = 0; m < n; ++m) {
        c += cos(theta[m]);
        s += sin(theta[m]);
    }
    c /= (double)n;
    s /= (double)n;
    *r = sqrt(c * c + s * s);
    *psi = atan2(s, c);
}

/* One classical RK4 step of size dt; work holds 5n doubles. */
static void rk4_step(const orc_graph *g, const double *omega, double K, double dt, double *theta,
                     double *work)
{
    int64_t n = g->n;
    double *k1 = work, *k2 = work + n, *k3 = work + 2 * n, *k4 = work + 3 * n, *y = work + 4 * n;
    rhs(g, omega, K, theta, k1);
    for (int64_t m = 0; m < n; ++m) y[m] = theta[m] + 0.5 * dt * k1[m];
    rhs(g, omega, K, y, k2);
    for (int64_t m = 0; m < n; ++m) y[m] = theta[m] + 0.5 * dt * k2[m];
    rhs(g, omega, K, y, k3);
    for (int64_t m = 0; m < n; ++m) y[m] = theta[m] + dt * k3[m];
    rhs(g, omega, K, y, k4);
    for (int64_t m = 0; m < n; ++m)
        theta[m] += dt / 6.0 * (k1[m] + 2.0 * k2[m] + 2.0 * k3[m] + k4[m]);
}

/*
 * Integrate nsteps classical RK4 steps in place on the unwrapped phases theta.
 * If r_every > 0, r_out/psi_out (may be NULL) receive r and psi at steps 0, r_every, 2 r_every,
 * ..., i.e. nsteps / r_every + 1 values. Returns 0, or -1 on allocation failure.
 */
int orc_rk4(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
            const double *omega, double K, double dt, int64_t nsteps, int64_t r_every,
            double *theta, double *r_out, double *psi_out)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    double *work = (double *)malloc(sizeof(double) * 5 * (size_t)n);
    if (!work) return -1;
    int64_t k = 0;
    for (int64_t s = 0; s <= nsteps; ++s) {
        if (r_every > 0 && s % r_every == 0) {
            double r, psi;
            orc_order_parameter(n, theta, &r, &psi);
            if (r_out) r_out[k] = r;
            if (psi_out) psi_out[k] = psi;
            ++k;
        }
        if (s < nsteps) rk4_step(&g, omega, K, dt, theta, work);
    }
    free(work);
    return 0;
}

/*
 * The implicit midpoint rule theta_{n+1} = theta_n + dt F((theta_n + theta_{n+1}) / 2), the
 * second-order symmetric integrator, solved by fixed-point iteration on the midpoint Y in the
 * order the iteration is defined: Y = theta_n; repeat iters - 1 times Y = theta_n + dt/2 F(Y);
 * then theta_{n+1} = theta_n + dt F(Y). Samples of (r, psi) as in orc_rk4.
 */
int orc_midpoint(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
                 const double *omega, double K, double dt, int64_t nsteps, int32_t iters, int64_t r_every,
                 double *theta, double *r_out, double *psi_out)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    double *y = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    if (!y) return -1;
    double *f = y + n;
    int64_t k = 0;
    for (int64_t s = 0; s <= nsteps; ++s) {
        if (r_every > 0 && s % r_every == 0) {
            double r, psi;
            orc_order_parameter(n, theta, &r, &psi);
            if (r_out) r_out[k] = r;
            if (psi_out) psi_out[k] = psi;
            ++k;
        }
        if (s == nsteps) break;
        memcpy(y, theta, sizeof(double) * (size_t)n);
        for (int32_t it = 1; it < iters; ++it) {
            rhs(&g, omega, K, y, f);
            for (int64_t m = 0; m < n; ++m) y[m] = theta[m] + 0.5 * dt * f[m];
        }
        rhs(&g, omega, K, y, f);
        for (int64_t m = 0; m < n; ++m) theta[m] += dt * f[m];
    }
    free(y);
    return 0;
}

/*
 * Fehlberg's embedded Runge-Kutta pair of orders 4 and 5 (E. Fehlberg, NASA TR R-315, 1969),
 * written as the tableau c, a (strictly lower triangular), b4 (propagated), b5 (error estimate).
 */
static const double RKF_A[6][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 4, 0, 0, 0, 0, 0},
    {3.0 / 32, 9.0 / 32, 0, 0, 0, 0},
    {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0, 0},
    {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0, 0},
    {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40, 0},
};
static const double RKF_B4[6] = {25.0 / 216, 0, 1408.0 / 2565, 2197.0 / 4104, -1.0 / 5, 0};
static const double RKF_B5[6] = {16.0 / 135, 0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55};

void orc_rkf45_tableau(double *a, double *b4, double *b5)
{
    for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) a[6 * i + j] = RKF_A[i][j];
        b4[i] = RKF_B4[i];
        b5[i] = RKF_B5[i];
    }
}

/*
 * Variable step size integration over [0, t_end] with the pair above, in this order per
 * attempted step of size h = min(dt, t_end - t): k_1 = F(theta), k_i = F(theta + h sum_{j<i}
 * a_ij k_j); local error e = max_m |h sum_j (b5_j - b4_j) k_{j,m}|; accept if e <= atol
 * (theta += h sum_j b4_j k_j, t += h); next dt = h min(4, max(0.2, 0.9 (e/atol)^(-1/5))), 4 when
 * e = 0. stats = (t reached, next dt, accepted, rejected).
 */
int orc_rkf45(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
              const double *omega, double K, double t_end, double dt0, double atol, int64_t max_steps,
              double *theta, double *stats)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    double *k = (double *)malloc(sizeof(double) * 7 * (size_t)n);
    if (!k) return -1;
    double *y = k + 6 * n;
    double t = 0.0, dt = dt0 < t_end ? dt0 : t_end;
    int64_t acc = 0, rej = 0;
    while (t < t_end && acc + rej < max_steps) {
        const double h = dt < t_end - t ? dt : t_end - t;
        rhs(&g, omega, K, theta, k);
        for (int i = 1; i < 6; ++i) {
            for (int64_t m = 0; m < n; ++m) {
                double s = 0.0;
                for (int j = 0; j < i; ++j) s += RKF_A[i][j] * k[j * n + m];
                y[m] = theta[m] + h * s;
            }
            rhs(&g, omega, K, y, k + i * n);
        }
        double err = 0.0;
        for (int64_t m = 0; m < n; ++m) {
            double s = 0.0;
            for (int j = 0; j < 6; ++j) s += (RKF_B5[j] - RKF_B4[j]) * k[j * n + m];
            if (fabs(h * s) > err) err = fabs(h * s);
        }
        const double errn = err / atol;
        if (!(errn == errn) || errn > 1e300) { free(k); return -2; }
        if (errn <= 1.0) {
            for (int64_t m = 0; m < n; ++m) {
                double s = 0.0;
                for (int j = 0; j < 6; ++j) s += RKF_B4[j] * k[j * n + m];
                theta[m] += h * s;
            }
            t = h == t_end - t ? t_end : t + h;  /* a step clamped to the end lands on it */
            ++acc;
        } else {
            ++rej;
        }
        double fac = 4.0;
        if (errn > 0.0) {
            fac = 0.9 * pow(errn, -0.2);
            if (fac < 0.2) fac = 0.2;
            if (fac > 4.0) fac = 4.0;
        }
        dt = h * fac;
    }
    stats[0] = t;
    stats[1] = dt;
    stats[2] = (double)acc;
    stats[3] = (double)rej;
    free(k);
    return 0;
}

/*
 * Jacobian-transpose product out = J(theta)^T lam, with
 *   dF_m/dtheta_l = K s_m A_ml cos(theta_l - theta_m)             (l != m)
 *   dF_m/dtheta_m = -K s_m sum_l A_ml cos(theta_l - theta_m)
 * (s_m the row scale), obtained by differentiating eq. KuramotoGraph term by term. Computed by
 * scattering every row's contributions, so an asymmetric A needs no transpose.
 */
void orc_vjp(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
             double K, const double *theta, const double *lam, double *out)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    memset(out, 0, sizeof(double) * (size_t)n);
    for (int64_t m = 0; m < n; ++m) {
        double w = K * row_scale(&g, m) * lam[m];
        if (w == 0.0) continue;
        if (complete) {
            for (int64_t l = 0; l < n; ++l) {
                if (l == m) continue;
                double c = cos(theta[l] - theta[m]);
                out[l] += w * c;
                out[m] -= w * c;
            }
        } else {
            for (int64_t e = row_ptr[m]; e < row_ptr[m + 1]; ++e) {
                int64_t l = col[e];
                double c = weight_of(&g, e) * cos(theta[l] - theta[m]);
                out[l] += w * c;
                out[m] -= w * c;
            }
        }
    }
}

/* dF/dK = s_m sum_l A_ml sin(theta_l - theta_m) */
static void dfdk(const orc_graph *g, const double *theta, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t m = 0; m < g->n; ++m) out[m] = row_scale(g, m) * coupling_sum(g, theta, m);
}

/*
 * Discrete adjoint of orc_rk4 (no r output). Given dL/dtheta(T) (n values), returns
 * g_theta0 = dL/dtheta(0), g_omega = dL/domega, *g_K = dL/dK.
 *
 * For one step theta+ = theta + dt/6 (k1 + 2k2 + 2k3 + k4), k_i = F(Y_i), Y1 = theta,
 * Y2 = theta + dt/2 k1, Y3 = theta + dt/2 k2, Y4 = theta + dt k3, the chain rule applied in
 * reverse with lam = dL/dtheta+ gives, with l_i = dL/dk_i and mu_i = J(Y_i)^T l_i:
 *   l4 = dt/6 lam,            mu4 = J(Y4)^T l4
 *   l3 = dt/3 lam + dt mu4,   mu3 = J(Y3)^T l3
 *   l2 = dt/3 lam + dt/2 mu3, mu2 = J(Y2)^T l2
 *   l1 = dt/6 lam + dt/2 mu2, mu1 = J(Y1)^T l1
 *   dL/dtheta = lam + mu1 + mu2 + mu3 + mu4,  dL/domega += sum_i l_i,  dL/dK += sum_i <l_i, dF/dK(Y_i)>.
 * The whole forward trajectory is stored ((nsteps+1) n doubles).
 */
int orc_adjoint_rk4(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
                    const double *omega, double K, double dt, int64_t nsteps, const double *theta0,
                    const double *dl_dthetaT, double *g_theta0, double *g_omega, double *g_K)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    size_t N = (size_t)n;
    double *traj = (double *)malloc(sizeof(double) * N * (size_t)(nsteps + 1));
    double *work = (double *)malloc(sizeof(double) * 14 * N);
    if (!traj || !work) { free(traj); free(work); return -1; }
    memcpy(traj, theta0, sizeof(double) * N);
    for (int64_t s = 0; s < nsteps; ++s) {
        memcpy(traj + (size_t)(s + 1) * N, traj + (size_t)s * N, sizeof(double) * N);
        rk4_step(&g, omega, K, dt, traj + (size_t)(s + 1) * N, work);
    }
    double *k1 = work, *k2 = work + N, *k3 = work + 2 * N, *Y2 = work + 3 * N, *Y3 = work + 4 * N,
           *Y4 = work + 5 * N, *lam = work + 6 * N, *l = work + 7 * N, *mu = work + 8 * N,
           *acc = work + 9 * N, *gk = work + 10 * N, *mu_prev = work + 11 * N;
    memcpy(lam, dl_dthetaT, sizeof(double) * N);
    memset(g_omega, 0, sizeof(double) * N);
    double gK = 0.0;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double *th = traj + (size_t)s * N;
        /* recompute the stage states of this step */
        rhs(&g, omega, K, th, k1);
        for (size_t m = 0; m < N; ++m) Y2[m] = th[m] + 0.5 * dt * k1[m];
        rhs(&g, omega, K, Y2, k2);
        for (size_t m = 0; m < N; ++m) Y3[m] = th[m] + 0.5 * dt * k2[m];
        rhs(&g, omega, K, Y3, k3);
        for (size_t m = 0; m < N; ++m) Y4[m] = th[m] + dt * k3[m];
        const double *Ys[4] = {th, Y2, Y3, Y4};
        /* coefficients: l_i = bl_i dt lam + cm_i dt mu_{i+1} */
        const double bl[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
        const double cm[4] = {0.5, 0.5, 1.0, 0.0};
        memcpy(acc, lam, sizeof(double) * N);
        memset(mu_prev, 0, sizeof(double) * N);
        for (int i = 3; i >= 0; --i) {
            for (size_t m = 0; m < N; ++m) l[m] = bl[i] * dt * lam[m] + cm[i] * dt * mu_prev[m];
            orc_vjp(n, complete, row_ptr, col, weight, scaling, K, Ys[i], l, mu);
            dfdk(&g, Ys[i], gk);
            for (size_t m = 0; m < N; ++m) {
                g_omega[m] += l[m];
                gK += l[m] * gk[m];
                acc[m] += mu[m];
            }
            memcpy(mu_prev, mu, sizeof(double) * N);
        }
        memcpy(lam, acc, sizeof(double) * N);
    }
    memcpy(g_theta0, lam, sizeof(double) * N);
    *g_K = gK;
    free(traj);
    free(work);
    return 0;
}

/*
 * Potential (Sec. 3, eq. ExtendedPotentialConservation, uniform scaling and symmetric A):
 *   V = -omega^T theta + K/2 sum_{l,m} Ascaled_ml (1 - cos(theta_l - theta_m))
 * evaluated term by term.
 */
double orc_potential(int64_t n, int complete, const int64_t *row_ptr, const int32_t *col, const int32_t *weight, int scaling,
                     const double *omega, double K, const double *theta)
{
    orc_graph g = {n, complete, row_ptr, col, weight, scaling};
    double lin = 0.0, pair = 0.0;
    for (int64_t m = 0; m < n; ++m) lin += omega[m] * theta[m];
    for (int64_t m = 0; m < n; ++m) {
        double rs = row_scale(&g, m), acc = 0.0;
        if (complete) {
            for (int64_t l = 0; l < n; ++l)
                if (l != m) acc += 1.0 - cos(theta[l] - theta[m]);
        } else {
            for (int64_t e = row_ptr[m]; e < row_ptr[m + 1]; ++e)
                acc += weight_of(&g, e) * (1.0 - cos(theta[col[e]] - theta[m]));
        }
        pair += rs * acc;
    }
    return -lin + 0.5 * K * pair;
}
