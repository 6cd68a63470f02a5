/*
 * CPU oracle for exact edge posteriors in Bayesian networks.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it. It shares no code, header, table or layout
 * with the GPU library.
 *
 * Plain and slow on purpose: FP64 log-space throughout, full n-bit subset
 * masks (variable i <-> bit i), untruncated zeta transforms, layers of the
 * subset lattice enumerated by scanning every mask. It follows the steps of
 * Algorithm 1 (Koivisto's forward-backward programme, Sec. 2.2) in order:
 *
 *   1. local scores B_i(G) = rho_i(G) p(x_i | x_G) for |G| <= d      (Eq. 6)
 *   2. A_i(S) = q_i(S) sum_{G subset S, |G|<=d} B_i(G)                (Eq. 7)
 *   3. F(S) = sum_{i in S} A_i(S - i) F(S - i), F(empty) = 1          (Eq. 9)
 *   4. backward function, stored prefix-indexed:
 *        Rp(S) := R(V - S) = sum_{i not in S} A_i(S) Rp(S + i),
 *        Rp(V) = 1                                                    (Eq. 10)
 *   5. Gamma_v(G) = sum_{G subset S subset V-v} q_v(S) F(S) Rp(S + v) (Eq. 12)
 *   6. P(u->v, D) = sum_{G containing u, |G|<=d} B_v(G) Gamma_v(G)    (Eq. 11)
 *   7. P(u->v | D) = P(u->v, D) / F(V)
 *
 * The local marginal likelihood is BDeu (Dirichlet hyperparameters
 * ess / (q r_i)) or K2 (all hyperparameters 1); the paper leaves it open
 * (Sec. 2.1). The order-modular prior functions q_i and rho_i (Eq. 4) are
 * taken to depend on subset size only: log q(k), k = 0..n-1, and
 * log rho(k), k = 0..d.
 *
 * A last section writes out the generic subset transforms of Def. 1 and
 * Def. 2 (and their inverses) as plain sums over subsets or supersets.
 *
 * Parity pins for this file live in the test suite: brute force over all
 * orders and over all DAGs, exact rational BDeu values, the m = 0 closed
 * form, the Gamma-free identity and the lattice invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_NEG_INF (-INFINITY)

/* log(exp(a) + exp(b)) */
static double lae(double a, double b)
{
    if (a == OR_NEG_INF) return b;
    if (b == OR_NEG_INF) return a;
    double m = a > b ? a : b;
    return m + log1p(exp(-fabs(a - b)));
}

static int popc(uint64_t x) { return __builtin_popcountll(x); }

/* Threads an OpenMP region of the oracle will use. */
int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ------------------------------------------------------------------ */
/* Step 1: local marginal likelihood log p(x_i | x_G) (Eq. 6).          */
/* ------------------------------------------------------------------ */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Counts N_jk (parent configuration j, child value k) by sorting the
 * per-sample keys key = j * r_i + k, then the Dirichlet-multinomial
 * marginal likelihood. Parent configurations never observed contribute 0.
 * kind 0 = BDeu(ess), kind 1 = K2.
 */
static double local_score(int n, int m, const uint8_t *data, const uint8_t *arity,
                          int i, uint64_t G, int kind, double ess, uint64_t *keys)
{
    (void)n;
    if (m == 0) return 0.0;
    double ri = (double)arity[i];
    double q = 1.0;
    for (int p = 0; p < n; ++p)
        if ((G >> p) & 1) q *= (double)arity[p];
    for (int s = 0; s < m; ++s) {
        uint64_t j = 0;
        for (int p = 0; p < n; ++p)
            if ((G >> p) & 1) j = j * arity[p] + data[(size_t)p * m + s];
        keys[s] = j * (uint64_t)arity[i] + data[(size_t)i * m + s];
    }
    qsort(keys, (size_t)m, sizeof(uint64_t), cmp_u64);
    double a_j, a_jk;
    if (kind == 0) { a_j = ess / q; a_jk = ess / (q * ri); }
    else { a_j = ri; a_jk = 1.0; }
    double lg_aj = lgamma(a_j), lg_ajk = lgamma(a_jk);
    double total = 0.0;
    int s = 0;
    while (s < m) {
        uint64_t j = keys[s] / arity[i];
        int nj = 0;
        while (s < m && keys[s] / arity[i] == j) {
            uint64_t key = keys[s];
            int njk = 0;
            while (s < m && keys[s] == key) { ++njk; ++s; }
            total += lgamma(a_jk + njk) - lg_ajk;
            nj += njk;
        }
        total += lg_aj - lgamma(a_j + nj);
    }
    return total;
}

/*
 * out[i * 2^n + G] = log p(x_i | x_G) for every G not containing i with
 * |G| <= d; every other entry is -inf. The prior rho is NOT included.
 */
int or_local_scores(int n, int m, const uint8_t *data, const uint8_t *arity, int d,
                    int kind, double ess, double *out, int nthreads)
{
    if (n < 1 || n > 30 || m < 0 || d < 0) return -1;
    set_threads(nthreads);
    const uint64_t N = 1ull << n;
    for (uint64_t x = 0; x < (uint64_t)n * N; ++x) out[x] = OR_NEG_INF;
    int err = 0;
#pragma omp parallel
    {
        uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
        if (!keys) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t x = 0; x < (int64_t)((uint64_t)n * N); ++x) {
            if (!keys) continue;
            int i = (int)(x / N);
            uint64_t G = (uint64_t)x % N;
            if ((G >> i) & 1) continue;
            if (popc(G) > d) continue;
            out[x] = local_score(n, m, data, arity, i, G, kind, ess, keys);
        }
        free(keys);
    }
    return err ? -2 : 0;
}

/* ------------------------------------------------------------------ */
/* Steps 2-7 from given log B_i(G).                                   */
/* ------------------------------------------------------------------ */

/*
 * Inputs:
 *   logB[i * 2^n + G] = log B_i(G) (prior rho included) for G not
 *     containing i and |G| <= d; all other entries must be -inf.
 *   log_q[k] = log q(k), k = 0..n-1 (NULL: q == 1).
 * Outputs:
 *   post[u * n + v] = P(u -> v | D); diagonal 0.
 *   diag[0] = log F(V)
 *   diag[1] = log Rp(empty) - log F(V)                      (should be 0)
 *   diag[2] = max_k |log sum_{|S|=k} F(S) Rp(S) - log F(V)| (should be 0)
 *   diag[3] = max_v |log sum_G B_v(G) Gamma_v(G) - log F(V)| (should be 0)
 *   diag[4] = max |P - P_gamma_free| if gamma_free_check, else -1
 *   Optional dumps (NULL to skip), all log-space:
 *     alpha_out[i * 2^n + S]  log A_i(S)   (-inf for S containing i)
 *     F_out[S], Rp_out[S]
 *     gamma_out[v * 2^n + G]  log Gamma_v(G) for |G| <= d, v not in G; else -inf
 * Returns 0 on success, negative on bad arguments or allocation failure.
 */
int or_posteriors_from_scores(int n, int d, const double *logB, const double *log_q,
                              double *post, double *diag, double *alpha_out,
                              double *F_out, double *Rp_out, double *gamma_out,
                              int gamma_free_check, int nthreads)
{
    if (n < 1 || n > 30 || d < 0) return -1;
    set_threads(nthreads);
    const uint64_t N = 1ull << n;
    const uint64_t FULL = N - 1;
    double lq[64];
    for (int k = 0; k <= n; ++k) lq[k] = (log_q && k < n) ? log_q[k] : 0.0;

    /* Keep the scores of every family with |G| <= d before the transform
     * (the alpha buffer may be the score buffer itself). */
    uint64_t K = 0;
    for (uint64_t G = 0; G < N; ++G)
        if (popc(G) <= d) ++K;
    uint64_t *fam = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)K);
    double *famB = (double *)malloc(sizeof(double) * (size_t)n * K);
    double *A = alpha_out ? alpha_out : (double *)malloc(sizeof(double) * (size_t)n * N);
    double *F = F_out ? F_out : (double *)malloc(sizeof(double) * (size_t)N);
    double *Rp = Rp_out ? Rp_out : (double *)malloc(sizeof(double) * (size_t)N);
    if (!fam || !famB || !A || !F || !Rp) {
        free(fam);
        free(famB);
        if (!alpha_out) free(A);
        if (!F_out) free(F);
        if (!Rp_out) free(Rp);
        return -2;
    }
    {
        uint64_t c = 0;
        for (uint64_t G = 0; G < N; ++G)
            if (popc(G) <= d) fam[c++] = G;
        for (int i = 0; i < n; ++i)
            for (uint64_t c2 = 0; c2 < K; ++c2)
                famB[(size_t)i * K + c2] = logB[(size_t)i * N + fam[c2]];
    }

    /* Step 2: A_i by an untruncated upward zeta over every bit j != i.
     * The input is zero (log -inf) for |G| > d and for G containing i, so
     * summing over all subsets equals the truncated sum of Eq. 7. */
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
        double *a = A + (size_t)i * N;
        if (a != logB + (size_t)i * N)
            memcpy(a, logB + (size_t)i * N, sizeof(double) * (size_t)N);
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const uint64_t bj = 1ull << j;
            for (uint64_t S = 0; S < N; ++S)
                if (S & bj) a[S] = lae(a[S], a[S ^ bj]);
        }
        for (uint64_t S = 0; S < N; ++S) {
            if ((S >> i) & 1) a[S] = OR_NEG_INF;
            else if (a[S] != OR_NEG_INF) a[S] += lq[popc(S)];
        }
    }

    /* Step 3: forward F, one popcount layer at a time (Eq. 9). */
    F[0] = 0.0;
    for (int k = 1; k <= n; ++k) {
#pragma omp parallel for schedule(static)
        for (int64_t Si = 0; Si < (int64_t)N; ++Si) {
            uint64_t S = (uint64_t)Si;
            if (popc(S) != k) continue;
            double acc = OR_NEG_INF;
            for (int i = 0; i < n; ++i)
                if ((S >> i) & 1) {
                    uint64_t T = S ^ (1ull << i);
                    acc = lae(acc, A[(size_t)i * N + T] + F[T]);
                }
            F[S] = acc;
        }
    }

    /* Step 4: backward, prefix-indexed: Rp(S) = R(V - S) (Eq. 10). */
    Rp[FULL] = 0.0;
    for (int k = n - 1; k >= 0; --k) {
#pragma omp parallel for schedule(static)
        for (int64_t Si = 0; Si < (int64_t)N; ++Si) {
            uint64_t S = (uint64_t)Si;
            if (popc(S) != k) continue;
            double acc = OR_NEG_INF;
            for (int i = 0; i < n; ++i)
                if (!((S >> i) & 1))
                    acc = lae(acc, A[(size_t)i * N + S] + Rp[S | (1ull << i)]);
            Rp[S] = acc;
        }
    }

    const double logFV = F[FULL];
    double maxlayer = 0.0;
    for (int k = 0; k <= n; ++k) {
        double acc = OR_NEG_INF;
        for (uint64_t S = 0; S < N; ++S)
            if (popc(S) == k) acc = lae(acc, F[S] + Rp[S]);
        double r = fabs(acc - logFV);
        if (r > maxlayer) maxlayer = r;
    }

    /* Steps 5-7 per endpoint v: product, downward zeta over every bit
     * j != v (the untruncated transform restricted to |G| <= d equals the
     * truncated one of Eq. 12), then the edge sums of Eq. 11. */
    double maxtot = 0.0;
    int err = 0;
    for (uint64_t x = 0; x < (uint64_t)n * n; ++x) post[x] = 0.0;
#pragma omp parallel
    {
        double *g = (double *)malloc(sizeof(double) * (size_t)N);
        double *acc = (double *)malloc(sizeof(double) * (size_t)n);
        if (!g || !acc) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int v = 0; v < n; ++v) {
            if (!g || !acc) continue;
            const uint64_t bv = 1ull << v;
            for (uint64_t S = 0; S < N; ++S)
                g[S] = (S & bv) ? OR_NEG_INF : lq[popc(S)] + F[S] + Rp[S | bv];
            for (int j = 0; j < n; ++j) {
                if (j == v) continue;
                const uint64_t bj = 1ull << j;
                for (uint64_t S = 0; S < N; ++S)
                    if (!(S & bj)) g[S] = lae(g[S], g[S | bj]);
            }
            for (int u = 0; u < n; ++u) acc[u] = OR_NEG_INF;
            double tot = OR_NEG_INF;
            const double *B = famB + (size_t)v * K;
            for (uint64_t c = 0; c < K; ++c) {
                const uint64_t G = fam[c];
                if (G & bv) continue;
                if (gamma_out) gamma_out[(size_t)v * N + G] = g[G];
                double w = B[c] + g[G];
                tot = lae(tot, w);
                for (int u = 0; u < n; ++u)
                    if ((G >> u) & 1) acc[u] = lae(acc[u], w);
            }
            if (gamma_out)
                for (uint64_t G = 0; G < N; ++G)
                    if ((G & bv) || popc(G) > d) gamma_out[(size_t)v * N + G] = OR_NEG_INF;
            for (int u = 0; u < n; ++u)
                post[(size_t)u * n + v] = (u == v) ? 0.0 : exp(acc[u] - logFV);
            double r = fabs(tot - logFV);
#pragma omp critical
            {
                if (r > maxtot) maxtot = r;
            }
        }
        free(g);
        free(acc);
    }

    /* Independent cross-check that never forms Gamma: grouping the orders
     * by the predecessor set S of v, P(u->v, D) equals
     *   sum_{S not containing v, u in S} F(S) Rp(S + v)
     *       * (A_v(S) - q(|S|) / q(|S| - 1) * A_v(S - u)),
     * where the bracket is q(|S|) sum_{G subset S, u in G} B_v(G). */
    double maxgf = -1.0;
    if (gamma_free_check && !err) {
        maxgf = 0.0;
#pragma omp parallel for schedule(dynamic, 1)
        for (int v = 0; v < n; ++v) {
            const uint64_t bv = 1ull << v;
            const double *a = A + (size_t)v * N;
            for (int u = 0; u < n; ++u) {
                if (u == v) continue;
                const uint64_t bu = 1ull << u;
                double acc = OR_NEG_INF;
                for (uint64_t S = 0; S < N; ++S) {
                    if ((S & bv) || !(S & bu)) continue;
                    int k = popc(S);
                    double hi = a[S];
                    double lo = a[S ^ bu] + lq[k] - lq[k - 1];
                    if (hi == OR_NEG_INF) continue;
                    double diff;
                    if (lo == OR_NEG_INF) diff = hi;
                    else if (lo >= hi) continue;
                    else diff = hi + log1p(-exp(lo - hi));
                    acc = lae(acc, F[S] + Rp[S | bv] + diff);
                }
                double p2 = exp(acc - logFV);
                double r = fabs(p2 - post[(size_t)u * n + v]);
#pragma omp critical
                {
                    if (r > maxgf) maxgf = r;
                }
            }
        }
    }

    if (diag) {
        diag[0] = logFV;
        diag[1] = Rp[0] - logFV;
        diag[2] = maxlayer;
        diag[3] = maxtot;
        diag[4] = maxgf;
    }
    free(fam);
    free(famB);
    if (!alpha_out) free(A);
    if (!F_out) free(F);
    if (!Rp_out) free(Rp);
    return err ? -2 : 0;
}

/*
 * Whole method from data: log B_i(G) = log rho(|G|) + log p(x_i | x_G)
 * (log_rho NULL: rho(k) = 1 / C(n-1, k)), then steps 2-7.
 * The score array lives in the alpha buffer's place, so the peak memory is
 * about 2 n 2^n doubles.
 */
int or_edge_posteriors(int n, int m, const uint8_t *data, const uint8_t *arity, int d,
                       int kind, double ess, const double *log_rho, const double *log_q,
                       double *post, double *diag, int nthreads)
{
    if (n < 1 || n > 30 || d < 0) return -1;
    if (d > n - 1) d = n - 1;
    const uint64_t N = 1ull << n;
    double *B = (double *)malloc(sizeof(double) * (size_t)n * N);
    if (!B) return -2;
    int rc = or_local_scores(n, m, data, arity, d, kind, ess, B, nthreads);
    if (rc) { free(B); return rc; }
    double lr[64];
    for (int k = 0; k <= d; ++k) {
        if (log_rho) lr[k] = log_rho[k];
        else lr[k] = -(lgamma((double)n) - lgamma((double)k + 1) - lgamma((double)(n - k)));
    }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < (int64_t)((uint64_t)n * N); ++x)
        if (B[x] != OR_NEG_INF) B[x] += lr[popc((uint64_t)x % N)];
    /* B doubles as the alpha buffer: the scores needed later are copied
     * into compact per-node lists before the transform overwrites them. */
    rc = or_posteriors_from_scores(n, d, B, log_q, post, diag, B, NULL, NULL, NULL, 0,
                                   nthreads);
    free(B);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Generic subset sums (Def. 1 and Def. 2 written out as sums).         */
/* ------------------------------------------------------------------ */

/* Compensated (Neumaier) running sum, so the reference value is exact to a
 * few units in the last place whatever the number of terms. */
typedef struct { double s, c; } or_acc;
static void acc_add(or_acc *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/*
 * One output of a subset transform of x (2^nbits values, x[S] for the subset
 * S given by the index bits), straight from its definition:
 *   kind 0 (upward zeta, Def. 1):   sum over S subset T with |S| <= d
 *                                   (d < 0: no bound) of x[S]
 *   kind 1 (downward zeta, Def. 2): sum over S superset T of x[S]
 *   kind 2 (inverse of kind 0 without bound):
 *                                   sum over S subset T of (-1)^|T-S| x[S]
 *   kind 3 (inverse of kind 1):     sum over S superset T of (-1)^|S-T| x[S]
 * absval != 0 sums |x[S]| instead, without signs (the scale of the
 * rounding error).
 * Subsets of T are enumerated as sub = (sub - 1) & T; supersets as the
 * union of T with the subsets of its complement.
 */
static double subset_sum_one(int nbits, int kind, int d, const double *x, uint64_t T, int absval)
{
    const uint64_t full = (nbits == 64) ? ~0ull : ((1ull << nbits) - 1);
    const int down = kind == 1 || kind == 3;
    const int alt = kind == 2 || kind == 3;
    const uint64_t free_bits = down ? (full & ~T) : T;
    or_acc a = {0.0, 0.0};
    uint64_t sub = free_bits;
    for (;;) {
        const uint64_t S = down ? (T | sub) : sub;
        if (!(kind == 0 && d >= 0 && popc(S) > d)) {
            double v = absval ? fabs(x[S]) : x[S];
            if (alt && !absval && (popc(down ? (S & ~T) : (T & ~S)) & 1)) v = -v;
            acc_add(&a, v);
        }
        if (sub == 0) break;
        sub = (sub - 1) & free_bits;
    }
    return a.s + a.c;
}

/* Every output: out[T] for all 2^nbits subsets T (x and out distinct). */
int or_subset_sums(int nbits, int kind, int d, const double *x, double *out, int absval,
                   int nthreads)
{
    if (nbits < 0 || nbits > 30 || kind < 0 || kind > 3) return -1;
    set_threads(nthreads);
    const int64_t N = (int64_t)1 << nbits;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t T = 0; T < N; ++T) out[T] = subset_sum_one(nbits, kind, d, x, (uint64_t)T, absval);
    return 0;
}

/* Selected outputs: out[k] for the subsets Ts[k], k < nT. The caller keeps
 * the enumeration small (few members of T for kinds 0 and 2, few
 * non-members for kinds 1 and 3). */
int or_subset_sums_at(int nbits, int kind, int d, const double *x, const uint64_t *Ts,
                      int64_t nT, double *out, int absval, int nthreads)
{
    if (nbits < 0 || nbits > 40 || kind < 0 || kind > 3) return -1;
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nT; ++k) out[k] = subset_sum_one(nbits, kind, d, x, Ts[k], absval);
    return 0;
}
