/*
 * bn.h -- C ABI of the MI355X edge-posterior library (libbnpost.so).
 *
 * Computes exact posterior probabilities P(u -> v | D) of all n(n-1)
 * directed edges of a Bayesian network from discrete data, by the
 * forward-backward dynamic programme over the subset lattice (Algorithm 1,
 * Sec. 2.2 of Chen, Tian, Nikolova and Aluru, "A Parallel Algorithm for
 * Exact Bayesian Structure Discovery in Bayesian Networks"):
 *
 *   local scores  B_i(G) = rho(|G|) p(x_i | x_G),  |G| <= d        (Eq. 6)
 *   upward zeta   A_i(S) = q(|S|) sum_{G subset S, |G|<=d} B_i(G)  (Eq. 7)
 *   forward       F(S)   = sum_{i in S} A_i(S-i) F(S-i)            (Eq. 9)
 *   backward      R(S), stored prefix-indexed as Rp(S) = R(V-S)    (Eq. 10)
 *   downward zeta Gamma_v(G) = sum_{G subset S subset V-v}
 *                               q(|S|) F(S) Rp(S+v),  |G| <= d     (Eq. 12)
 *   edges         P(u->v|D) = sum_{G containing u} B_v(G) Gamma_v(G) / F(V)
 *                                                            (Eq. 11)
 *
 * Conventions for every call:
 *   - variable i <-> bit i of a subset mask; data column i = variable i;
 *   - the caller owns every buffer; the library keeps no caller pointer
 *     after a call returns (the server copies what it needs at submit);
 *   - all arguments are validated before any device work; on an error
 *     nothing is written and no device state changes;
 *   - on BN_OK every output is complete;
 *   - the order-modular prior (Eq. 4) is taken to depend on subset size:
 *     q_i(S) = q(|S|) and rho_i(G) = rho(|G|).
 */
#ifndef BN_H
#define BN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
/* In C++ the enumerations get a fixed 32-bit underlying type, so that every
 * int32 a C caller passes is a value of the type (the library rejects the
 * unknown ones with BN_EINVAL); in C an enumeration is an int already. */
#define BN_ENUM_BASE : int32_t
#else
#define BN_ENUM_BASE
#endif

typedef enum BN_ENUM_BASE {
    BN_OK = 0,
    BN_EINVAL = -1,     /* invalid argument (see each call)                        */
    BN_ENOMEM = -2,     /* the problem's footprint exceeds device memory or budget */
    BN_EDEVICE = -3,    /* a HIP runtime call failed                               */
    BN_EAGAIN = -4,     /* serving: result not ready yet                           */
    BN_ECANCELED = -5,  /* serving: request dropped by bn_server_destroy           */
    BN_EINTERNAL = -6   /* internal error                                          */
} bn_status;

typedef enum BN_ENUM_BASE {
    BN_FP64_LOG = 0,    /* every lattice value as an FP64 natural logarithm         */
    BN_FP32_SCALED = 1  /* values stored as an FP32 significand + 8-bit exponent
                           (units of 2^64) per entry, on top of exact per-node (B_i)
                           and per-layer (q) power-of-two scales; products and the
                           sweep sums in FP32 significands with integer exponents.
                           FP64 in the log-gamma score sums, the scale exponents,
                           the final 1/F(V) step and the zeta adds inside a tile
                           (plain doubles under one power-of-two scale per tile,
                           or the FP32 form itself where the tile's range does
                           not fit one FP64 scale)                                */
} bn_precision;

typedef enum BN_ENUM_BASE {
    BN_SCORE_BDEU = 0,  /* Dirichlet hyperparameters ess / (q r_i)               */
    BN_SCORE_K2 = 1     /* all Dirichlet hyperparameters 1                       */
} bn_score;

/*
 * The problem statement of Sec. 2.1: discrete data D over n variables with
 * arities, an in-degree bound d, an order-modular prior and a local score.
 */
typedef struct {
    int32_t n;             /* number of variables, 2..31                             */
    int32_t m;             /* number of samples, >= 0 (m = 0: every score is 0)      */
    const uint8_t *data;   /* column-major n*m: data[i*m + s] < arity[i]. Host memory
                              for bn_local_scores, bn_edge_posteriors and
                              bn_serve_submit; DEVICE memory for
                              bn_edge_posteriors_dev                                 */
    const uint8_t *arity;  /* host, n entries, each 2..255                           */
    int32_t d;             /* in-degree bound, >= 0; values above n-1 act as n-1     */
    int32_t score;         /* bn_score                                               */
    double ess;            /* BDeu equivalent sample size, > 0 (ignored for K2)      */
    const double *log_rho; /* host or NULL; d+1 values log rho(k), k = 0..min(d,n-1);
                              NULL: rho(k) = 1 / C(n-1, k)                           */
    const double *log_q;   /* host or NULL; n values log q(k), k = 0..n-1;
                              NULL: q == 1                                           */
} bn_problem;

/* Filled by the solve calls when a non-NULL pointer is passed. */
typedef struct {
    double log_LV;                 /* natural log of F(V) = P(D)                     */
    double max_invariant_residual; /* max over: |log Rp(empty) - log F(V)|,
                                      |log sum_{|S|=k} F(S)Rp(S) - log F(V)| (all k),
                                      |log sum_G B_v(G)Gamma_v(G) - log F(V)| (all v) */
    uint64_t saturated;            /* FP32-scaled: entries clamped at the top of
                                      the exponent range                             */
    uint64_t flushed;              /* FP32-scaled: nonzero entries rounded to 0 below
                                      the bottom of the exponent range               */
    double ms_scores, ms_alpha, ms_fwd, ms_bwd, ms_gamma, ms_edges, ms_total;
    double ms_queue;               /* serving: submit -> admission (host clock)      */
    double ms_latency;             /* serving: submit -> completion observed          */
    uint64_t fallback_tiles;       /* zeta tiles (alpha, Gamma) whose range did not fit
                                      one FP64 scale and were recomputed in the solve's
                                      own number system                              */
} bn_report;

/* Number of parent sets of one node: K(n-1, d) = sum_{k<=min(d,n-1)} C(n-1, k).
 * Returns 0 for n < 1 or d < 0. */
size_t bn_num_parent_sets(int32_t n, int32_t d);

/*
 * Local scores (Eq. 6 without the prior factor): log p(x_i | x_G) for every
 * node i and every G subset V-{i} with |G| <= d.
 *   log_score: host, n * K(n-1,d) doubles, written as log_score[i*K + r].
 *   Ranking r of a parent set: G is written as a mask over the n-1 other
 *   variables in increasing order (bit p <-> variable p if p < i, else p+1);
 *   r = sum_{k' < |G|} C(n-1, k') + sum_t C(c_t, t), where c_1 < ... < c_|G|
 *   are the set bit positions (sets by size, then in colex order).
 * Runs on the current HIP device and blocks until done.
 * BN_EINVAL: NULL pointers, n out of range, arity out of range, a data value
 * >= its arity, ess <= 0 (BDeu), d < 0, a family with more than 16384
 * (parent configuration, child value) bins, or more than 2^31 - 1 families.
 */
bn_status bn_local_scores(const bn_problem *p, double *log_score);

/* Device workspace needed by bn_edge_posteriors_dev for a given problem
 * shape. The sample count m enters because the workspace also holds the
 * score step's per-sample tables (bit planes of binary data and log-gamma
 * values up to m). BN_EINVAL for n outside 2..31, d < 0, m < 0, an unknown
 * precision or a NULL bytes. */
bn_status bn_workspace_bytes(int32_t n, int32_t d, int32_t m, bn_precision prec,
                             size_t *bytes);

/*
 * All n(n-1) edge posteriors from host data: the whole of Algorithm 1 (local
 * scores by Eq. 6, alpha by Eq. 7, the forward and backward sums of Eqs. 9
 * and 10, Gamma by Eq. 12, and P(u -> v | D) by Eq. 11, divided by F(V) =
 * P(D)). Allocates its own device workspace, copies the data, runs every
 * step on the current HIP device and blocks until done.
 *   post: host, n*n doubles, post[u*n + v] = P(u -> v | D); diagonal 0.
 *   rep:  nullable; per-phase times are measured with HIP events.
 * BN_EINVAL as for bn_local_scores (and a bad precision); BN_ENOMEM when
 * the workspace does not fit in device memory.
 */
bn_status bn_edge_posteriors(const bn_problem *p, bn_precision prec, double *post,
                             bn_report *rep);

/*
 * Posterior of every parent set of every node, P(G_v = G | D) for |G| <= d
 * (the parent-set feature of Sec. 2.1, Eq. 5: the same Gamma_v as the edge
 * sums, P(G_v = G | D) = B_v(G) Gamma_v(G) / F(V)). Any feature of one
 * node's parent set is a sum of these; the edge posterior P(u -> v | D) is
 * the sum over the sets G containing u.
 *   ps:   host, n * K(n-1,d) doubles, ps[v*K + r] for the parent set of rank
 *         r (the ranking of bn_local_scores); each row sums to 1.
 *   post: host n*n doubles as for bn_edge_posteriors, or NULL.
 *   rep:  nullable, as for bn_edge_posteriors.
 * Errors as for bn_edge_posteriors (BN_EINVAL when ps is NULL).
 */
bn_status bn_parent_set_posteriors(const bn_problem *p, bn_precision prec, double *ps,
                                   double *post, bn_report *rep);

struct bn_timer;

/*
 * The computation of bn_edge_posteriors (Algorithm 1; Eqs. 6, 7, 9-12) with
 * caller-supplied device memory and stream, in stream order: nothing is
 * allocated and nothing waits. p->data must point to DEVICE memory (n*m
 * bytes); arity, log_rho and log_q are host arrays (consumed before the
 * call returns). Results go to device buffers, and per-phase times to an
 * optional bn_timer rather than a bn_report, which would need a wait;
 * the caller synchronises the stream before reading any of them.
 *   dev_ws/ws_bytes: device workspace of at least bn_workspace_bytes().
 *   hip_stream:      a hipStream_t (NULL: the default stream).
 *   dev_post:        DEVICE, n*n doubles, written as for bn_edge_posteriors.
 *   dev_diag:        DEVICE or NULL; 8 doubles: [0] log F(V), [1] max invariant
 *                    residual, [2] saturated count, [3] flushed count,
 *                    [4] |log Rp(empty) - log F(V)|, [5] max layer-sum residual,
 *                    [6] max edge-sum residual, [7] fallback tiles (bn_report).
 *   timer:           NULL, or a bn_timer to receive per-phase HIP events.
 * Enqueues the work and returns without waiting; the results are valid after
 * the stream is synchronised. Data values are not range-checked on the host
 * (they live on the device); out-of-range values give undefined scores but
 * never out-of-bounds accesses.
 */
bn_status bn_edge_posteriors_dev(const bn_problem *p, bn_precision prec, void *dev_ws,
                                 size_t ws_bytes, void *hip_stream, double *dev_post,
                                 double *dev_diag, struct bn_timer *timer);

/*
 * Allocation-free variant of bn_edge_posteriors_dev, for callers that cannot
 * allocate device memory during a solve: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc. The workspace is a static
 * device array of BN_NOALLOC_MAX_BYTES inside the library (one per GPU,
 * held from the library's loading until the process ends); the call itself
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *   p, prec:    as for bn_edge_posteriors_dev (p->data in DEVICE memory).
 *   hip_stream: a hipStream_t (NULL: the default stream).
 *   dev_post:   DEVICE, n*n doubles, as for bn_edge_posteriors_dev.
 *   dev_diag:   DEVICE or NULL, 8 doubles, as for bn_edge_posteriors_dev.
 * Enqueues the work and returns without waiting; the results are valid after
 * the stream is synchronised, and bit-identical to bn_edge_posteriors_dev on
 * the same inputs. Every call on one GPU shares that GPU's array: calls whose
 * work overlaps on the device (other streams, or other threads, before the
 * previous call's stream has finished) race and give undefined results.
 * Each solve initialises everything it reads, so the previous call's
 * contents need no clearing.
 * BN_EINVAL as for bn_edge_posteriors_dev; BN_ENOMEM when the problem's
 * workspace (bn_workspace_bytes) exceeds BN_NOALLOC_MAX_BYTES (256 MiB;
 * with d = 3 and m <= 2000 that admits n <= 21 in either form);
 * BN_EDEVICE when the array's device address cannot be obtained.
 */
#define BN_NOALLOC_MAX_BYTES ((size_t)256 << 20)
bn_status bn_edge_posteriors_noalloc(const bn_problem *p, bn_precision prec, void *hip_stream,
                                     double *dev_post, double *dev_diag);

/*
 * Phase timer: HIP events that bn_edge_posteriors_dev records on the solve's
 * own stream between its phases when a non-NULL timer is passed (recording
 * does not synchronise). Create it on the device that runs the solves.
 * bn_timer_read, valid once that stream has been synchronised, returns the
 * milliseconds of the last solve that used the timer:
 *   ms[0] parameters, tables, local scores and prior/gauges (Eq. 6)
 *   ms[1] alpha, truncated upward zeta (Eq. 7, Alg. 2): one kernel launch
 *   ms[2] forward sweep, all layers (Eq. 9)
 *   ms[3] backward sweep, all layers (Eq. 10)
 *   ms[4] Gamma: product and truncated downward zeta (Eq. 12, Alg. 3)
 *   ms[5] edge sums, invariants and diagnostics (Eq. 11)
 *   ms[6] total
 *   ms[7] the Gamma in-tile kernel alone (one launch; part of ms[4]): the
 *         products and the zeta over the low tile bits (the recomputation of
 *         fallback tiles, if any, is not included)
 *   ms[8] the alpha tile kernel alone (one launch; part of ms[1]): the zeta
 *         over the low tile bits and the store of alpha (its seed gather and
 *         any fallback tiles are not included)
 */
typedef struct bn_timer bn_timer;
bn_status bn_timer_create(bn_timer **timer);
bn_status bn_timer_destroy(bn_timer *timer);
bn_status bn_timer_read(const bn_timer *timer, double ms[9]);

/*
 * Serving: a server thread batches solves of mixed n, m and arity as they
 * arrive (continuous batching). Requests are admitted when their device
 * footprint fits in mem_budget_bytes (0: 90% of free device memory) and
 * fewer than max_active are in flight; admitted requests advance phase by
 * phase, interleaved on several streams.
 */
bn_status bn_server_create(size_t mem_budget_bytes, int32_t max_active, void **server);
/* Copies the problem's inputs; non-blocking. BN_ENOMEM if the request could
 * never fit in the budget; BN_EINVAL as for bn_edge_posteriors. */
bn_status bn_serve_submit(void *server, const bn_problem *p, bn_precision prec,
                          uint64_t *ticket);
/* Waits up to timeout_us (0: no wait, < 0: forever). BN_OK: post (host n*n)
 * and rep (nullable) are written and the ticket is released. BN_EAGAIN: not
 * done yet. BN_ECANCELED: dropped by destroy. BN_EINVAL: unknown ticket. */
bn_status bn_serve_poll(void *server, uint64_t ticket, double *post, bn_report *rep,
                        int32_t timeout_us);
/* Stops the server; pending requests resolve to BN_ECANCELED. */
bn_status bn_server_destroy(void *server);

/*
 * Posterior expectation of a modular feature f(G) = prod_i f_i(G_i), a
 * product of one factor per node that depends only on that node's parent
 * set (Sec. 2.1; for a 0/1 feature it is the posterior probability P(f | D),
 * Eqs. 1-2). With the order-modular prior (Eq. 4) f enters Eq. 5 next to
 * B_i, so P(f, D) is the forward sum L(V) of Eq. 9 run on f_i(G) B_i(G);
 * the result is P(f, D) / P(D). Two forward-only runs (alpha and the
 * forward sweep; no backward sweep or Gamma). Examples: f_v(G) = [u in G]
 * gives P(u -> v | D); f_v(G) = [u not in G] for several pairs gives the
 * probability that none of those edges is present.
 *   log_f: host, n * K(n-1,d) doubles, log f_i(G) for the parent set of rank
 *          r (the ranking of bn_local_scores) at log_f[i*K + r]; -inf where
 *          f_i(G) = 0, 0 where it is 1. Read only.
 *   expectation: host, one double, E[f | D] (0 when P(f, D) = 0).
 *   log_pair: nullable host double[2], {log P(D), log P(f, D)} up to the
 *          same constant.
 * Allocates and frees its own workspace; blocks until done. BN_EINVAL as for
 * bn_edge_posteriors, and for a NULL log_f or expectation or an entry of
 * log_f that is NaN or +inf (checked before any device work).
 */
bn_status bn_modular_feature_posterior(const bn_problem *p, bn_precision prec,
                                       const double *log_f, double *expectation,
                                       double *log_pair);

/*
 * Subset transforms of a device array x of 2^nbits doubles, x[S] for the
 * subset S given by the bits of the index, in place on the given stream
 * (NULL: the default stream); returns without waiting.
 *   BN_ZETA_UP      t(T) = sum_{S subset T, |S| <= d} x(S) for every T: the
 *                   truncated upward zeta transform (Def. 1, Alg. 2); d < 0
 *                   or d >= nbits: untruncated.
 *   BN_ZETA_DOWN    t(T) = sum_{S superset T} x(S): the downward zeta
 *                   transform (Def. 2, Alg. 3). Def. 2 requires the outputs
 *                   with |T| <= d only; every output is computed.
 *   BN_MOBIUS_UP    the inverse of the untruncated upward transform,
 *                   t(T) = sum_{S subset T} (-1)^{|T - S|} x(S).
 *   BN_MOBIUS_DOWN  the inverse of the downward transform.
 * nbits in 1..32. BN_EINVAL: NULL array, nbits out of range, an unknown
 * kind, or a truncated (0 <= d < nbits) Moebius transform. Summation is in
 * FP64 in a fixed order (deterministic).
 */
typedef enum BN_ENUM_BASE {
    BN_ZETA_UP = 0,
    BN_ZETA_DOWN = 1,
    BN_MOBIUS_UP = 2,
    BN_MOBIUS_DOWN = 3
} bn_subset_kind;
bn_status bn_subset_transform(double *dev_x, int32_t nbits, bn_subset_kind kind, int32_t d,
                              void *hip_stream);

/*
 * Measurement, not a step of the solve: the blocked 0/1 contraction against
 * the register pass for one in-tile zeta step. For every 16-entry group g of
 * the device array x (16 * groups doubles), y(g, T) = sum_{S subset T}
 * x(g, S) over the four low index bits (Def. 1, untruncated), by
 *   method 0  four add steps over the 16 values one lane holds (the form of
 *             the library's in-tile passes), groups staged through LDS so
 *             that loads and stores are coalesced;
 *   method 1  the 16-column group matrix times the 16 x 16 subset-inclusion
 *             matrix on the FP64 matrix cores (four 16x16x4 products per 16
 *             groups).
 * reps > 1 repeats the arithmetic on values held in registers (method 0
 * applies the transform reps times in a row, method 1 accumulates reps equal
 * products), so that large reps times the arithmetic alone; reps = 1 is one
 * HBM pass and its y is the transform. groups: a multiple of 16 in
 * 16..2^32; reps in 1..4096. The caller owns x and y (disjoint, device
 * memory). Blocks until the kernel has finished; *ms receives its time
 * (HIP events on the stream; NULL: the default stream). BN_EINVAL for NULL
 * pointers or out-of-range arguments.
 */
bn_status bn_zeta4_probe(const double *dev_x, double *dev_y, uint64_t groups, int32_t method,
                         int32_t reps, void *hip_stream, float *ms);

/*
 * The zeta transforms of bn_subset_transform (BN_ZETA_UP, truncated when
 * 0 <= d < nbits, Def. 1 and Alg. 2; BN_ZETA_DOWN, Def. 2 and Alg. 3) on
 * non-negative values in the library's FP32-scaled storage, in place: entry
 * S is dev_f[S] * 2^(64 * (dev_b[S] - 200)), dev_b[S] = 0 meaning 0; both
 * planes hold 2^nbits entries (5 bytes per entry instead of 8). Negative
 * significands are taken as 0 (the number system has no sign), so the
 * Moebius kinds are not offered (BN_EINVAL). Each add aligns the smaller
 * operand to the larger exponent by an exact power of two and rounds to
 * FP32, so an output's relative error is at most about nbits * 2^-24 plus
 * terms below 2^-64 of the output. Outputs beyond the byte's range are
 * clamped and counted: dev_counts (NULL: not counted; else two device
 * uint64) receives += saturations in [0] and flushes of nonzero values to 0
 * in [1]. Enqueued on the stream (NULL: the default stream); returns without
 * waiting. nbits in 1..32; BN_EINVAL for NULL planes or nbits out of range.
 */
bn_status bn_subset_transform_x32(float *dev_f, uint8_t *dev_b, int32_t nbits,
                                  bn_subset_kind kind, int32_t d,
                                  unsigned long long *dev_counts, void *hip_stream);

const char *bn_status_string(bn_status s);

#ifdef __cplusplus
}
#endif

#endif /* BN_H */
