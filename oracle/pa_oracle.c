/*
 * pa_oracle.c -- plain CPU oracle for population-annealing Max-Cut.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do. It shares no code with the device path.
 *
 * What it computes (paper: "New Best-Known Max-Cut Solution for the G63
 * Instance in the G-Set Benchmark", arXiv 2510.21105):
 *
 *   Section 1, eq. (1): the Max-Cut objective
 *       cut(x) = 1/2 * sum_{i<j} w_ij (1 - x_i x_j),  x in {-1,+1}^N.
 *   Section 2: Max-Cut is the ground state of the Ising energy with
 *       antiferromagnetic couplings J_ij = -w_ij, i.e. of
 *       E(x) = sum_{i<j} w_ij x_i x_j,  so  cut = (W_tot - E) / 2,
 *       W_tot = sum_{i<j} w_ij.
 *   Abstract and section 3: the solver is population annealing Monte Carlo
 *   with adaptive control of stochasticity and periodic non-local moves.
 *   The paper names these parts but does not define them; the concrete
 *   integer-exact definitions below are the readings this project adopts
 *   (each listed in the design notes):
 *
 *   RNG   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). A draw for
 *         (tag, sweep s, step k, node i, replica r) is word (r & 3) of
 *         Philox(key = (lo32 seed, hi32 seed),
 *                ctr = (i, s | tag << 16, k, (r >> 2) | inst << 16)).
 *         Tags: 0 Metropolis, 1 initial spins, 2 resampling, 3 non-local
 *         pair seed, 4 single-replica cluster seed, 5 bond activation.
 *   Init  x_i^r = +1 if bit 0 of draw(1, 0, 0, i, r) is set, else -1.
 *   Sweep for each replica, for t = 0..N-1, i = order[t]:
 *         h_i = sum_j w_ij x_j, m = -x_i h_i (the flip changes E by 2m);
 *         accept iff m <= 0, or draw(0, s, k, i, r) < T_k,l(m) where
 *         T(beta, m) = floor(2^32 * exp(-(beta * 2m))) computed in FP64 and
 *         beta = beta_k * gamma^l (gamma^l by l successive FP64 products).
 *         On accept x_i <- -x_i, E += 2m and h_j += 2 w_ij x_i(new).
 *         After every sweep: if min_r E_r < best_E the best becomes
 *         (E, lowest such r, k, s) with a copy of its configuration.
 *   NL    every nl_period steps (after the sweeps of steps k with
 *         (k+1) % nl_period == 0): for p = 0..R/2-1 take replicas a = p,
 *         b = p + R/2; D = {i : x_i^a != x_i^b} in node order; if D is not
 *         empty pick D[floor(draw(3, 0, k, 0, p) * |D| / 2^32)] and flip, in
 *         both replicas, the connected component of that node in the
 *         subgraph induced by D (Houdayer's cluster move). Then the best
 *         check runs again (recorded with sweep index S).
 *   NL, single-replica kind (nl_kind 1, same steps): every replica r on its
 *         own makes one Wolff cluster update at the step's sweep temperature
 *         beta' = beta_k gamma^l. Seed s = floor(draw(4, 0, k, 0, r) * N /
 *         2^32). Each edge {i < j} whose term w_ij x_i x_j is negative (a
 *         satisfied bond of the couplings J = -w) is activated iff
 *         draw(5, j, k, i, r) < Q(beta' |w_ij|), Q(a) = floor(2^32 * (1 -
 *         exp(-2a))) evaluated as -expm1(-2a) in FP64. The connected component
 *         of s in the graph of active bonds is flipped (Wolff's construction
 *         for couplings of either sign: it satisfies detailed balance with
 *         respect to exp(-beta' E) and needs no acceptance test). Then the
 *         best check runs again (recorded with sweep index S).
 *   AS    if the best improved during step k: level l <- 0, stall <- 0;
 *         else stall += 1, and if stall >= P_stall and
 *         frozen_inv * (uphill accepts) < (uphill attempts) during step k
 *         then l <- min(l + 1, l_max) and stall <- 0. The level applies to the
 *         next step's sweeps. Uphill means m > 0.
 *   Adaptive steps (beta_adapt 1): beta[] is an evenly spaced grid of K
 *         inverse temperatures and step k sweeps at the current grid point
 *         g_k (g_0 = 0). Population annealing reweights a step from beta to
 *         beta' by exp(-(beta' - beta) E); a jump of j grid points from g
 *         raises beta by beta_{g+j} - beta_g, which on an evenly spaced grid
 *         is beta_j - beta_0 wherever the jump starts. Grids whose spacings
 *         differ (by more than 1e-9 of the mean spacing plus 8 ulps of the
 *         largest |beta|, the FP64 rounding of a linear grid) are refused.
 *         After step k (if g_k < K-1) the run moves to g_k + j for the
 *         largest j in [1, min(J, K-1-g_k)] whose weights
 *         W_r = floor(2^32 exp(-(dbeta_j (E_r - E_min)))), dbeta_j =
 *         beta_j - beta_0, keep the normalised effective population
 *         (sum W)^2 / (R sum W^2) at or above num/den (exact in 128-bit
 *         integers; j = 1 when none does), and resamples with those weights.
 *         The run ends after the step at the last grid point, so it takes at
 *         most K steps. Without adaptation g_k = k and j = 1.
 *   Resample (steps k < K-1): dbeta = beta_{k+1} - beta_k (FP64);
 *         E_min = min_r E_r; W_r = floor(2^32 * exp(-(dbeta * (E_r - E_min))));
 *         S = sum W (uint64); C_r = W_0 + ... + W_r;
 *         U = word0 | word1 << 32 of Philox(ctr = (0, 2 << 16, k, inst << 16));
 *         u = floor(U * S / 2^64); f(c) = 0 if R*c <= u else
 *         ceil((R*c - u) / S); replica r gets n_r = f(C_r) - f(C_{r-1})
 *         copies in new slots f(C_{r-1}) .. f(C_r)-1 (systematic resampling,
 *         population size fixed at R).
 *
 * Parity status: Philox is pinned by the published known-answer vectors;
 * eq. (1), brute force, closed forms, the Boltzmann distribution, the
 * free-energy estimator and the resampling/cluster invariants pin the rest.
 * The adaptive-stochasticity rule has no definition in the paper; its
 * reading above is pinned by an independent replay of (level, stall) from
 * the per-step statistics (uphill attempts and accepts, best energy).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_STAT_FIELDS 10
/* stats record per step k (int64):
 *   0 E_min   (after sweeps and NL, before resampling)
 *   1 E_sum
 *   2 uphill attempts (m > 0) during the step's sweeps
 *   3 uphill accepts
 *   4 AS level used by the step's sweeps
 *   5 best_E after the step
 *   6 number of replicas with at least one copy (0 on the last step)
 *   7 weight sum S (0 on the last step)
 *   8 grid index of the step's inverse temperature (= k without adaptation)
 *   9 grid points to the next step (1 without adaptation; 0 on the last)  */

/* ------------------------------------------------------------------ RNG */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint32_t oracle_draw(uint64_t seed, uint32_t inst, uint32_t tag, uint32_t sweep,
                     uint32_t step, uint32_t node, uint32_t replica)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { node, sweep | (tag << 16), step, (replica >> 2) | (inst << 16) };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[replica & 3];
}

uint64_t oracle_resample_uniform(uint64_t seed, uint32_t inst, uint32_t step)
{
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t ctr[4] = { 0u, 2u << 16, step, inst << 16 };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return (uint64_t)out[0] | ((uint64_t)out[1] << 32);
}

/* --------------------------------------------------------------- tables */

/* floor(2^32 * exp(-(beta * 2m))) */
uint64_t oracle_threshold(double beta, int32_t m)
{
    double x = exp(-(beta * (double)(2 * m)));
    return (uint64_t)floor(ldexp(x, 32));
}

/* floor(2^32 * exp(-(dbeta * n))) */
uint64_t oracle_weight(double dbeta, int64_t n)
{
    double x = exp(-(dbeta * (double)n));
    return (uint64_t)floor(ldexp(x, 32));
}

double oracle_level_beta(double beta, double gamma, int32_t level)
{
    double g = 1.0;
    for (int32_t l = 0; l < level; ++l) g = g * gamma;
    return beta * g;
}

/* ---------------------------------------------------------------- graph */

int64_t oracle_energy(int32_t n, const int32_t *row_ptr, const int32_t *col,
                      const int8_t *w, const int8_t *x)
{
    int64_t twice = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            twice += (int64_t)w[e] * x[i] * x[col[e]];
    return twice / 2;
}

static void fields(int32_t n, const int32_t *row_ptr, const int32_t *col,
                   const int8_t *w, const int8_t *x, int32_t *h)
{
    for (int32_t i = 0; i < n; ++i) {
        int32_t s = 0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) s += w[e] * x[col[e]];
        h[i] = s;
    }
}

/* ----------------------------------------------------------- resampling */

static uint64_t sys_f(uint64_t c, uint64_t R, uint64_t u, uint64_t S)
{
    uint64_t rc = R * c;
    if (rc <= u) return 0;
    return (rc - u + S - 1) / S;
}

/* Copy counts n[0..R-1] of systematic resampling with weights W and the
 * 64-bit uniform U. Returns the weight sum S (0 if all weights are 0). */
uint64_t oracle_resample_counts(int32_t R, const uint64_t *W, uint64_t U, int32_t *n_out)
{
    uint64_t S = 0;
    for (int32_t r = 0; r < R; ++r) S += W[r];
    if (S == 0) return 0;
    uint64_t u = (uint64_t)(((unsigned __int128)U * S) >> 64);
    uint64_t C = 0, prev = 0;
    for (int32_t r = 0; r < R; ++r) {
        C += W[r];
        uint64_t f = sys_f(C, (uint64_t)R, u, S);
        n_out[r] = (int32_t)(f - prev);
        prev = f;
    }
    return S;
}

/* ------------------------------------------------------ non-local move */

/* Houdayer cluster move on one pair. xa, xb are modified in place.
 * in_cluster (n bytes, may be NULL) receives 1 for flipped nodes.
 * Returns the cluster size (0 when the replicas agree everywhere). */
int32_t oracle_icm_pair(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        int8_t *xa, int8_t *xb, uint32_t draw, uint8_t *in_cluster)
{
    if (n <= 0) return 0;
    int32_t nd = 0;
    for (int32_t i = 0; i < n; ++i) nd += (xa[i] != xb[i]);
    if (in_cluster) memset(in_cluster, 0, (size_t)n);
    if (nd == 0) return 0;
    int64_t pick = (int64_t)(((uint64_t)draw * (uint64_t)nd) >> 32);
    int32_t seed_node = -1;
    for (int32_t i = 0, c = 0; i < n; ++i) {
        if (xa[i] != xb[i]) {
            if (c == pick) { seed_node = i; break; }
            ++c;
        }
    }
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t head = 0, tail = 0;
    queue[tail++] = seed_node;
    seen[seed_node] = 1;
    while (head < tail) {
        int32_t i = queue[head++];
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            if (!seen[j] && xa[j] != xb[j]) { seen[j] = 1; queue[tail++] = j; }
        }
    }
    for (int32_t q = 0; q < tail; ++q) {
        int32_t i = queue[q];
        xa[i] = (int8_t)-xa[i];
        xb[i] = (int8_t)-xb[i];
        if (in_cluster) in_cluster[i] = 1;
    }
    free(seen);
    free(queue);
    return tail;
}

/* floor(2^32 * (1 - exp(-2a))): the probability of activating a satisfied
 * bond of strength a / beta at inverse temperature beta. */
uint64_t oracle_bond_threshold(double a)
{
    double q = -expm1(-2.0 * a);
    return (uint64_t)floor(ldexp(q, 32));
}

/* Wolff cluster update of one replica (Wolff, PRL 62, 361 (1989), with bond
 * activation on satisfied bonds of either sign). x is modified in place;
 * q = oracle_bond_threshold(beta) applies to every edge of weight +-1 and
 * q_of_w (NULL for unit weights) holds thresholds by |w| (index |w|).
 * in_cluster (n bytes, may be NULL) receives 1 for flipped nodes. The bond
 * draws are draw(5, j, step, i, replica) for the edge {i < j}; the seed is
 * floor(draw(4, 0, step, 0, replica) * n / 2^32). Returns the cluster size. */
int32_t oracle_wolff(int32_t n, const int32_t *row_ptr, const int32_t *col, const int8_t *w,
                     int8_t *x, const uint64_t *q_of_w, uint64_t q, uint64_t seed, uint32_t inst,
                     uint32_t step, uint32_t replica, uint8_t *in_cluster)
{
    if (n <= 0) return 0;
    uint32_t d = oracle_draw(seed, inst, 4, 0, step, 0, replica);
    int32_t s = (int32_t)(((uint64_t)d * (uint64_t)n) >> 32);
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t head = 0, tail = 0;
    queue[tail++] = s;
    seen[s] = 1;
    /* Breadth-first growth over active bonds; whether a bond is active
     * depends only on its endpoints' spins before the update and its own
     * draw, so the order of growth does not matter. */
    while (head < tail) {
        int32_t i = queue[head++];
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col[e];
            if (seen[j]) continue;
            if ((int32_t)w[e] * x[i] * x[j] >= 0) continue;           /* not satisfied */
            int32_t lo = i < j ? i : j, hi = i < j ? j : i;
            uint64_t qq = q_of_w ? q_of_w[w[e] < 0 ? -w[e] : w[e]] : q;
            uint32_t u = oracle_draw(seed, inst, 5, (uint32_t)hi, step, (uint32_t)lo, replica);
            if ((uint64_t)u < qq) { seen[j] = 1; queue[tail++] = j; }
        }
    }
    if (in_cluster) memset(in_cluster, 0, (size_t)n);
    for (int32_t t = 0; t < tail; ++t) {
        int32_t i = queue[t];
        x[i] = (int8_t)-x[i];
        if (in_cluster) in_cluster[i] = 1;
    }
    free(seen);
    free(queue);
    return tail;
}

/* Adaptive step: the largest j in [1, jmax] whose weights
 * W_r = floor(2^32 exp(-((beta_j - beta_0)(E_r - emin)))) satisfy
 * den (sum W)^2 >= num R (sum W^2), else 1 (128-bit integers throughout). */
int32_t oracle_adapt_jump(int32_t R, const int32_t *E, int64_t emin, const double *beta, int32_t jmax,
                          int32_t num, int32_t den)
{
    for (int32_t j = jmax; j > 1; --j) {
        double dbeta = beta[j] - beta[0];
        unsigned __int128 S1 = 0, S2 = 0;
        for (int32_t r = 0; r < R; ++r) {
            uint64_t W = oracle_weight(dbeta, (int64_t)E[r] - emin);
            S1 += W;
            S2 += (unsigned __int128)W * W;
        }
        if (S1 * S1 * (unsigned __int128)(uint32_t)den >= (unsigned __int128)(uint32_t)num * (uint32_t)R * S2)
            return j;
    }
    return 1;
}

/* ------------------------------------------------------------ PA driver */

/* 1 if some spacing beta[k+1] - beta[k] differs from the mean spacing
 * (beta[K-1] - beta[0]) / (K-1) by more than 1e-9 of it plus 8 ulps of the
 * largest |beta|. */
static int grid_uneven(const double *beta, int32_t K)
{
    if (K < 3) return 0;
    double h = (beta[K - 1] - beta[0]) / (double)(K - 1);
    double big = fabs(beta[0]) > fabs(beta[K - 1]) ? fabs(beta[0]) : fabs(beta[K - 1]);
    double tol = 1e-9 * fabs(h) + 8.0 * ldexp(big, -52);
    for (int32_t k = 0; k + 1 < K; ++k)
        if (fabs((beta[k + 1] - beta[k]) - h) > tol) return 1;
    return 0;
}

static void best_check(int32_t R, int32_t n, const int32_t *E, const int8_t *x,
                       int64_t *best, int8_t *best_x, int32_t k, int32_t s, int *improved)
{
    int32_t arg = -1;
    int64_t emin = best[0];
    for (int32_t r = 0; r < R; ++r)
        if ((int64_t)E[r] < emin) { emin = E[r]; arg = r; }
    if (arg >= 0) {
        best[0] = emin; best[1] = k; best[2] = s; best[3] = arg;
        memcpy(best_x, x + (size_t)arg * n, (size_t)n);
        *improved = 1;
    }
}

/*
 * Full population-annealing run. Output pointers may be NULL.
 *   x_init  R*n   initial population (replica-major)
 *   x_out   R*n   final population
 *   E_out   R     final energies
 *   best    4     {best_E, step, sweep, replica}; step -1 = initial population
 *   best_x  n     best configuration (+-1)
 *   stats   K*ORACLE_STAT_FIELDS (K*10) per-step records, fields listed at
 *                 ORACLE_STAT_FIELDS
 *   counts  K*R   copy counts n_r of each resampling (row K-1 unused)
 * Returns 0, or a negative value on invalid arguments.
 */
int oracle_run(int32_t n, const int32_t *row_ptr, const int32_t *col, const int8_t *w,
               int32_t K, const double *beta, int32_t S, const int32_t *order,
               int32_t as_enable, int32_t as_stall_steps, int32_t as_max_level,
               int32_t as_frozen_inv, double as_gamma, int32_t nl_period, int32_t nl_kind,
               int32_t beta_adapt, int32_t adapt_jump, int32_t adapt_num, int32_t adapt_den,
               int32_t R, uint64_t seed, uint32_t inst, int32_t nthreads,
               int8_t *x_init, int8_t *x_out, int32_t *E_out, int64_t *best,
               int8_t *best_x, int64_t *stats, int32_t *counts)
{
    if (n <= 0 || K <= 0 || S <= 0 || S > 65535 || R <= 0 || R > 32768 || inst > 65535)
        return -1;
    if (nl_kind != 0 && nl_kind != 1) return -1;
    if (beta_adapt != 0 && beta_adapt != 1) return -1;
    if (beta_adapt && (adapt_jump < 1 || adapt_num < 0 || adapt_den < 1 || adapt_num > adapt_den ||
                       adapt_den > 65536))
        return -1;
    if (nl_period > 0 && nl_kind == 0 && (R & 1)) return -1;
    if (as_enable && (as_stall_steps < 1 || as_max_level < 0 || as_frozen_inv < 1)) return -1;
    for (int32_t k = 0; k < K; ++k) {
        if (!(beta[k] >= 0.0) || !isfinite(beta[k])) return -1;
        if (k > 0 && beta[k] < beta[k - 1]) return -1;
    }
    if (beta_adapt && grid_uneven(beta, K)) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    int32_t dmax = 0;
    for (int32_t i = 0; i < n; ++i)
        if (row_ptr[i + 1] - row_ptr[i] > dmax) dmax = row_ptr[i + 1] - row_ptr[i];
    int32_t lmax = as_enable ? as_max_level : 0;

    int8_t *x = (int8_t *)malloc((size_t)R * n);
    int8_t *x2 = (int8_t *)malloc((size_t)R * n);
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * n);
    int32_t *h2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * n);
    int32_t *E = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int32_t *E2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    uint64_t *Wr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)R);
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    uint64_t *att = (uint64_t *)calloc((size_t)R, sizeof(uint64_t));
    uint64_t *acc = (uint64_t *)calloc((size_t)R, sizeof(uint64_t));
    uint64_t *thr = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(dmax + 1));
    int8_t *bx = best_x ? best_x : (int8_t *)malloc((size_t)n);
    int64_t bbuf[4];
    int64_t *bst = best ? best : bbuf;

    /* initial population */
    for (int32_t r = 0; r < R; ++r) {
        int8_t *xr = x + (size_t)r * n;
        for (int32_t i = 0; i < n; ++i)
            xr[i] = (oracle_draw(seed, inst, 1, 0, 0, (uint32_t)i, (uint32_t)r) & 1u) ? 1 : -1;
        fields(n, row_ptr, col, w, xr, h + (size_t)r * n);
        E[r] = (int32_t)oracle_energy(n, row_ptr, col, w, xr);
    }
    if (x_init) memcpy(x_init, x, (size_t)R * n);
    bst[0] = INT64_MAX; bst[1] = -1; bst[2] = -1; bst[3] = -1;
    int dummy = 0;
    best_check(R, n, E, x, bst, bx, -1, -1, &dummy);

    int32_t level = 0, stall = 0, gk = 0, done = 0;
    for (int32_t k = 0; k < K && !done; ++k) {
        int improved = 0;
        double b = oracle_level_beta(beta[gk], as_gamma, level);
        thr[0] = 0;
        for (int32_t m = 1; m <= dmax; ++m) thr[m] = oracle_threshold(b, m);
        (void)lmax;

        for (int32_t r = 0; r < R; ++r) { att[r] = 0; acc[r] = 0; }
        for (int32_t s = 0; s < S; ++s) {
#pragma omp parallel for schedule(dynamic, 1)
            for (int32_t r = 0; r < R; ++r) {
                int8_t *xr = x + (size_t)r * n;
                int32_t *hr = h + (size_t)r * n;
                int32_t e = E[r];
                uint64_t a_up = 0, c_up = 0;
                for (int32_t t = 0; t < n; ++t) {
                    int32_t i = order ? order[t] : t;
                    int32_t m = -xr[i] * hr[i];
                    int accept;
                    if (m <= 0) {
                        accept = 1;
                    } else {
                        ++a_up;
                        accept = thr[m] != 0 &&
                                 (uint64_t)oracle_draw(seed, inst, 0, (uint32_t)s, (uint32_t)k,
                                                       (uint32_t)i, (uint32_t)r) < thr[m];
                        c_up += (uint64_t)accept;
                    }
                    if (accept) {
                        xr[i] = (int8_t)-xr[i];
                        e += 2 * m;
                        for (int32_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q)
                            hr[col[q]] += 2 * w[q] * xr[i];
                    }
                }
                E[r] = e;
                att[r] += a_up;
                acc[r] += c_up;
            }
            best_check(R, n, E, x, bst, bx, k, s, &improved);
        }
        uint64_t att_up = 0, acc_up = 0;
        for (int32_t r = 0; r < R; ++r) { att_up += att[r]; acc_up += acc[r]; }

        if (nl_period > 0 && (k + 1) % nl_period == 0 && nl_kind == 1) {
            uint64_t q = oracle_bond_threshold(b);
#pragma omp parallel for schedule(dynamic, 1)
            for (int32_t r = 0; r < R; ++r) {
                int8_t *xr = x + (size_t)r * n;
                if (oracle_wolff(n, row_ptr, col, w, xr, NULL, q, seed, inst, (uint32_t)k,
                                 (uint32_t)r, NULL) > 0) {
                    E[r] = (int32_t)oracle_energy(n, row_ptr, col, w, xr);
                    fields(n, row_ptr, col, w, xr, h + (size_t)r * n);
                }
            }
            best_check(R, n, E, x, bst, bx, k, S, &improved);
        } else if (nl_period > 0 && (k + 1) % nl_period == 0) {
            int32_t half = R / 2;
#pragma omp parallel for schedule(dynamic, 1)
            for (int32_t p = 0; p < half; ++p) {
                int8_t *xa = x + (size_t)p * n;
                int8_t *xb = x + (size_t)(p + half) * n;
                uint32_t d = oracle_draw(seed, inst, 3, 0, (uint32_t)k, 0, (uint32_t)p);
                if (oracle_icm_pair(n, row_ptr, col, xa, xb, d, NULL) > 0) {
                    E[p] = (int32_t)oracle_energy(n, row_ptr, col, w, xa);
                    E[p + half] = (int32_t)oracle_energy(n, row_ptr, col, w, xb);
                    fields(n, row_ptr, col, w, xa, h + (size_t)p * n);
                    fields(n, row_ptr, col, w, xb, h + (size_t)(p + half) * n);
                }
            }
            best_check(R, n, E, x, bst, bx, k, S, &improved);
        }

        int64_t emin = INT64_MAX, esum = 0;
        for (int32_t r = 0; r < R; ++r) {
            if (E[r] < emin) emin = E[r];
            esum += E[r];
        }
        int32_t level_used = level;
        if (as_enable) {
            if (improved) {
                level = 0;
                stall = 0;
            } else {
                stall += 1;
                if (stall >= as_stall_steps &&
                    (unsigned __int128)(uint64_t)as_frozen_inv * acc_up < (unsigned __int128)att_up) {
                    level = level + 1 < as_max_level ? level + 1 : as_max_level;
                    stall = 0;
                }
            }
        }

        int64_t parents = 0;
        uint64_t wsum = 0;
        int32_t jump = 0;
        const int32_t g_used = gk;
        if (gk < K - 1) {
            double dbeta;
            if (!beta_adapt) {
                jump = 1;
                dbeta = beta[gk + 1] - beta[gk];
                for (int32_t r = 0; r < R; ++r) Wr[r] = oracle_weight(dbeta, (int64_t)E[r] - emin);
            } else {
                int32_t jmax = K - 1 - gk < adapt_jump ? K - 1 - gk : adapt_jump;
                jump = oracle_adapt_jump(R, E, emin, beta, jmax, adapt_num, adapt_den);
                dbeta = beta[jump] - beta[0];
                for (int32_t r = 0; r < R; ++r) Wr[r] = oracle_weight(dbeta, (int64_t)E[r] - emin);
            }
            gk += jump;
            uint64_t U = oracle_resample_uniform(seed, inst, (uint32_t)k);
            wsum = oracle_resample_counts(R, Wr, U, cnt);
            int32_t slot = 0;
            for (int32_t r = 0; r < R; ++r) {
                if (cnt[r] > 0) ++parents;
                for (int32_t c = 0; c < cnt[r]; ++c, ++slot) {
                    memcpy(x2 + (size_t)slot * n, x + (size_t)r * n, (size_t)n);
                    memcpy(h2 + (size_t)slot * n, h + (size_t)r * n, sizeof(int32_t) * (size_t)n);
                    E2[slot] = E[r];
                }
            }
            if (counts) memcpy(counts + (size_t)k * R, cnt, sizeof(int32_t) * (size_t)R);
            int8_t *tx = x; x = x2; x2 = tx;
            int32_t *th = h; h = h2; h2 = th;
            int32_t *te = E; E = E2; E2 = te;
        }
        else {
            done = 1;
        }
        if (stats) {
            int64_t *st = stats + (size_t)k * ORACLE_STAT_FIELDS;
            st[0] = emin; st[1] = esum; st[2] = (int64_t)att_up; st[3] = (int64_t)acc_up;
            st[4] = level_used; st[5] = bst[0]; st[6] = parents; st[7] = (int64_t)wsum;
            st[8] = g_used; st[9] = jump;
        }
    }
    if (x_out) memcpy(x_out, x, (size_t)R * n);
    if (E_out) memcpy(E_out, E, sizeof(int32_t) * (size_t)R);

    free(x); free(x2); free(h); free(h2); free(E); free(E2); free(Wr); free(cnt);
    free(att); free(acc); free(thr);
    if (!best_x) free(bx);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
