/*
 * kurgen.c -- seeded synthetic graph generator for the Kuramoto-on-graphs workloads.
 *
 * Input infrastructure only: this file decides WHICH pairs of oscillators are coupled. It holds
 * no part of the right-hand side, the integrator or the block split; the oracle and the GPU
 * library both consume what it produces.
 *
 * Randomness is counter based: every Bernoulli or uniform draw is the SplitMix64 output function
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014) applied
 * to a key built from (seed, community, pair) or (seed, row, counter). The result therefore does
 * not depend on the number of threads or on the order in which rows are visited.
 *
 * Graph model (stochastic block model in "planted order"):
 *   - community c owns the planted nodes [cptr[c], cptr[c+1]);
 *   - an intra-community pair (i<j, local indices) is an edge iff u(seed, c, i, j) < rho[c];
 *   - a cross-community pair is an edge with probability p_out, drawn row by row with geometric
 *     skips over the upper triangle (exact independent Bernoulli trials, O(edges) work);
 *   - every edge is undirected (symmetric adjacency), no self-loops.
 * A user permutation uperm[p] maps planted node p to its user-facing index.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t sm64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform in [0,1) with 53 random bits */
static inline double u01(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

static inline uint64_t comm_key(uint64_t seed, int64_t c) { return sm64(sm64(seed ^ 0xA5A5A5A5ull) ^ (uint64_t)(c + 1)); }

static inline int intra_edge(uint64_t kc, uint32_t i, uint32_t j, double rho)
{
    uint32_t a = i < j ? i : j, b = i < j ? j : i;
    return u01(sm64(kc ^ (((uint64_t)a << 32) | (uint64_t)b))) < rho;
}

/* Public: is the intra pair (i, j) of community c an edge? (used by tests to cross-check) */
int kg_intra_edge(uint64_t seed, int64_t c, uint32_t i, uint32_t j, double rho)
{
    if (i == j) return 0;
    return intra_edge(comm_key(seed, c), i, j, rho);
}

static inline int64_t comm_of(const int64_t *cptr, int64_t nc, int64_t p)
{
    int64_t lo = 0, hi = nc; /* cptr[lo] <= p < cptr[hi] */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (cptr[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

/* Geometric skipping over q in (p, n): successive successes of Bernoulli(p_out). Returns the
 * number of cross-community successes; writes them to out (if non-NULL). */
static int64_t inter_row(int64_t p, int64_t n, const int64_t *cptr, int64_t nc, double p_out,
                         uint64_t seed, int64_t *out)
{
    if (p_out <= 0.0) return 0;
    int64_t cnt = 0;
    int64_t cp = comm_of(cptr, nc, p);
    uint64_t key = sm64(sm64(seed ^ 0x5A5A5A5Aull) ^ (uint64_t)(p + 1));
    if (p_out >= 1.0) {
        for (int64_t q = p + 1; q < n; ++q)
            if (q < cptr[cp] || q >= cptr[cp + 1]) { if (out) out[cnt] = q; ++cnt; }
        return cnt;
    }
    const double lq = log1p(-p_out);
    uint64_t k = 0;
    int64_t q = p;
    for (;;) {
        double u = u01(sm64(key + 0x9E3779B97F4A7C15ull * (++k)));
        double g = floor(log1p(-u) / lq); /* failures before the next success */
        if (g >= (double)(n - q)) break;
        q += 1 + (int64_t)g;
        if (q >= n) break;
        if (q >= cptr[cp] && q < cptr[cp + 1]) continue; /* intra pairs belong to the intra process */
        if (out) out[cnt] = q;
        ++cnt;
    }
    return cnt;
}

/* Count (pairs_out == NULL) or list the undirected cross-community edges (p<q, planted order).
 * row_off (n+1) receives the per-row offsets into the pair list when pairs_out is NULL.
 * Returns the number of undirected edges. */
int64_t kg_inter_pairs(int64_t n, const int64_t *cptr, int64_t nc, double p_out, uint64_t seed,
                       int64_t *row_off, int64_t *pairs_q)
{
    if (!pairs_q) {
        row_off[0] = 0;
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t p = 0; p < n; ++p) row_off[p + 1] = inter_row(p, n, cptr, nc, p_out, seed, NULL);
        for (int64_t p = 0; p < n; ++p) row_off[p + 1] += row_off[p];
        return row_off[n];
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t p = 0; p < n; ++p) inter_row(p, n, cptr, nc, p_out, seed, pairs_q + row_off[p]);
    return row_off[n];
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Degrees of the symmetric SBM in USER order.
 *   inter_off/inter_q: output of kg_inter_pairs (upper triangle, planted order)
 *   deg_user[n]: receives the degree of every user node
 *   inter_deg[n] (scratch, planted order): receives inter degrees
 */
void kg_sbm_degrees(int64_t n, const int64_t *cptr, int64_t nc, const double *rho, uint64_t seed,
                    const int64_t *inter_off, const int64_t *inter_q, const int32_t *uperm,
                    int64_t *inter_deg, int64_t *deg_user)
{
    memset(inter_deg, 0, sizeof(int64_t) * (size_t)n);
    for (int64_t p = 0; p < n; ++p) {
        inter_deg[p] += inter_off[p + 1] - inter_off[p];
        for (int64_t e = inter_off[p]; e < inter_off[p + 1]; ++e) inter_deg[inter_q[e]] += 1;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < n; ++p) {
        int64_t c = comm_of(cptr, nc, p);
        uint64_t kc = comm_key(seed, c);
        int64_t s = cptr[c + 1] - cptr[c], i = p - cptr[c];
        int64_t d = 0;
        if (rho[c] >= 1.0) d = s - 1;
        else if (rho[c] > 0.0)
            for (int64_t j = 0; j < s; ++j)
                if (j != i && intra_edge(kc, (uint32_t)i, (uint32_t)j, rho[c])) ++d;
        deg_user[uperm[p]] = d + inter_deg[p];
    }
}

/*
 * Fill the USER-order CSR: row_ptr (n+1, prefix of deg_user, computed by the caller) and col
 * (user indices, ascending per row). sym_off (n+1) and sym_nbr (2*E) are caller scratch that
 * receive the inter edges in symmetric planted CSR form. by_user (n) holds, for every
 * community, its local indices ordered by user index, so intra neighbours come out sorted and
 * only the few inter neighbours need sorting and a merge.
 */
void kg_sbm_fill(int64_t n, const int64_t *cptr, int64_t nc, const double *rho, uint64_t seed,
                 const int64_t *inter_off, const int64_t *inter_q, const int32_t *uperm,
                 const int32_t *by_user, const int64_t *row_ptr, int32_t *col, int64_t *sym_off,
                 int64_t *sym_nbr)
{
    /* symmetric planted CSR of the inter edges */
    memset(sym_off, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t p = 0; p < n; ++p)
        for (int64_t e = inter_off[p]; e < inter_off[p + 1]; ++e) {
            sym_off[p + 1] += 1;
            sym_off[inter_q[e] + 1] += 1;
        }
    for (int64_t p = 0; p < n; ++p) sym_off[p + 1] += sym_off[p];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
        memcpy(fill, sym_off, sizeof(int64_t) * (size_t)n);
        for (int64_t p = 0; p < n; ++p)
            for (int64_t e = inter_off[p]; e < inter_off[p + 1]; ++e) {
                int64_t q = inter_q[e];
                sym_nbr[fill[p]++] = q;
                sym_nbr[fill[q]++] = p;
            }
        free(fill);
    }
#pragma omp parallel
    {
        int32_t *ibuf = NULL;
        int64_t icap = 0;
#pragma omp for schedule(dynamic, 64)
        for (int64_t p = 0; p < n; ++p) {
            int64_t c = comm_of(cptr, nc, p);
            uint64_t kc = comm_key(seed, c);
            int64_t s = cptr[c + 1] - cptr[c], i = p - cptr[c];
            int64_t ni = sym_off[p + 1] - sym_off[p];
            if (ni > icap) {
                icap = 2 * ni + 16;
                ibuf = (int32_t *)realloc(ibuf, sizeof(int32_t) * (size_t)icap);
            }
            for (int64_t e = 0; e < ni; ++e) ibuf[e] = uperm[sym_nbr[sym_off[p] + e]];
            qsort(ibuf, (size_t)ni, sizeof(int32_t), cmp_i32);
            int32_t *out = col + row_ptr[uperm[p]];
            const int32_t *ord = by_user + cptr[c];
            int64_t k = 0, e = 0;
            if (rho[c] > 0.0)
                for (int64_t t = 0; t < s; ++t) {
                    int64_t j = ord[t];
                    if (j == i || !(rho[c] >= 1.0 || intra_edge(kc, (uint32_t)i, (uint32_t)j, rho[c]))) continue;
                    int32_t v = uperm[cptr[c] + j];
                    while (e < ni && ibuf[e] < v) out[k++] = ibuf[e++];
                    out[k++] = v;
                }
            while (e < ni) out[k++] = ibuf[e++];
        }
        free(ibuf);
    }
}
