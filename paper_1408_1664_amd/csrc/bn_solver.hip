// Host side of the library: problem validation, the plan (tile sizes and
// workspace layout), the launch sequence and the C ABI of bn.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/bn.h"
#include "bn_device.h"
#include "bn_kernels.h"
#include "bn_solver.h"

namespace bnk {

static uint64_t binom_u64(int a, int b) {
    if (b < 0 || b > a) return 0;
    uint64_t r = 1;
    for (int k = 1; k <= b; ++k) r = r * (uint64_t)(a - b + k) / (uint64_t)k;
    return r;
}
static uint64_t kcount_u64(int w, int t) {
    uint64_t s = 0;
    for (int k = 0; k <= t && k <= w; ++k) s += binom_u64(w, k);
    return s;
}
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// BN_LOG_LEVEL (read once): 0 or unset, silent; 1, each solve's plan on
// stderr; 2, also the report of each blocking solve.
static int log_level() {
    static const int lv = [] {
        const char *e = getenv("BN_LOG_LEVEL");
        return e ? atoi(e) : 0;
    }();
    return lv;
}

// Host-side ranges for a marker trace (rocprofv3 --marker-trace): the
// enqueue phases of a solve and the wait of the blocking calls.
struct Range {
    explicit Range(const char *m) { roctxRangePushA(m); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

// Parameters passed by value to the parameter kernel (host arrays are
// consumed at launch, so no caller pointer is kept).
struct ParamBlock {
    uint8_t arity[32];
    double log_rho[33];
    double log_q[32];
    int has_rho, has_q;
};

__global__ void k_params(ParamBlock pb, int n, int d, uint8_t *arity, double *log_rho,
                         double *log_q, unsigned long long *cnt) {
    const int t = threadIdx.x;
    if (t < n) {
        arity[t] = pb.arity[t];
        log_q[t] = pb.has_q ? pb.log_q[t] : 0.0;
    }
    if (t <= d) {
        // default rho(k) = 1 / C(n-1, k)
        log_rho[t] = pb.has_rho ? pb.log_rho[t]
                                : -(lgamma((double)n) - lgamma((double)t + 1.0) -
                                    lgamma((double)(n - t)));
    }
    if (t < 2) cnt[t] = 0ull;
}

bn_status validate(const bn_problem *p, bool host_data, bool check_values) {
    if (!p) return BN_EINVAL;
    if (p->n < 2 || p->n > 31) return BN_EINVAL;
    if (p->m < 0) return BN_EINVAL;
    if (p->d < 0) return BN_EINVAL;
    if (p->score != BN_SCORE_BDEU && p->score != BN_SCORE_K2) return BN_EINVAL;
    if (p->score == BN_SCORE_BDEU && !(p->ess > 0.0 && std::isfinite(p->ess))) return BN_EINVAL;
    if (!p->arity) return BN_EINVAL;
    if (p->m > 0 && !p->data) return BN_EINVAL;
    const int n = p->n;
    const int d = std::min(p->d, n - 1);
    for (int i = 0; i < n; ++i)
        if (p->arity[i] < 2) return BN_EINVAL;
    if (p->log_rho)
        for (int k = 0; k <= d; ++k)
            if (std::isnan(p->log_rho[k]) || p->log_rho[k] == HUGE_VAL) return BN_EINVAL;
    if (p->log_q)
        for (int k = 0; k < n; ++k)
            if (std::isnan(p->log_q[k]) || p->log_q[k] == HUGE_VAL) return BN_EINVAL;
    // one workgroup per family must fit one grid dimension
    if ((double)n * (double)kcount_u64(n - 1, d) > 2147483647.0) return BN_EINVAL;
    // histogram bins of the largest family of each node
    for (int i = 0; i < n; ++i) {
        std::vector<int> ar;
        for (int j = 0; j < n; ++j)
            if (j != i) ar.push_back(p->arity[j]);
        std::sort(ar.rbegin(), ar.rend());
        double bins = p->arity[i];
        for (int k = 0; k < d; ++k) bins *= ar[k];
        if (bins > kMaxBins) return BN_EINVAL;
    }
    if (host_data && check_values && p->m > 0) {
        for (int i = 0; i < n; ++i) {
            const uint8_t *col = p->data + (size_t)i * p->m;
            const uint8_t r = p->arity[i];
            for (int s = 0; s < p->m; ++s)
                if (col[s] >= r) return BN_EINVAL;
        }
    }
    return BN_OK;
}

// fuse: 1 for the fused sweeps (alpha never materialised), 0 for alpha in
// HBM, -1 to decide (see make_plan)
static Plan plan_of(int n, int d_in, int m, bn_precision prec, bool with_data, bool with_post,
                    int fuse) {
    Plan P{};
    P.n = n;
    P.m = m;
    P.d = std::min(d_in, n - 1);
    P.N = n - 1;
    P.x32 = (prec == BN_FP32_SCALED);
    const int N = P.N, d = P.d;
    P.K = (uint32_t)kcount_u64(N, d);
    P.bA = N >= 13 ? 13 : N;      // alpha tile: 13 bits, or the whole lattice when smaller
    // sweep tile: 9 bits for the large FP32-scaled lattices (more workgroups
    // per CU for an HBM-bound sweep); 10 below n = 23 (one launch fewer per
    // sweep where launches dominate) and for the log form, whose log-add
    // cross terms want all 256 threads busy (4 entries each)
    P.bL = std::min(n, (P.x32 && n >= 23) ? 9 : 10);
    P.bG = n >= 12 ? 12 : n;      // Gamma tile: 12 bits, or the whole lattice when smaller
    P.aG = 12;
    // Tuning / test override "bA,bL,bG,aG" (each clamped to its valid range);
    // lets small problems exercise every tiling path.
    if (const char *tb = getenv("BN_TILE_BITS")) {
        int v[4] = {P.bA, P.bL, P.bG, P.aG};
        if (sscanf(tb, "%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3]) == 4) {
            (void)v[0];
            // at most 11 sweep bits: the in-tile alpha slices (bL 2^(bL-1)
            // entries) and the tile must fit the 160 KB of LDS
            P.bL = std::max(2, std::min(std::min(v[1], n), 11));
            (void)v[2];
            P.aG = std::max(1, std::min(v[3], 12));
        }
    }
    // Linear tiles for the alpha and Gamma in-tile zetas (with fallback).
    // BN_LINEAR_TILES=0 turns them off, =force sends every tile to the
    // fallback path (tests of that path).
    P.lin_mode = 1;
    if (const char *lt = getenv("BN_LINEAR_TILES")) {
        if (!strcmp(lt, "0")) P.lin_mode = 0;
        else if (!strcmp(lt, "force")) P.lin_mode = 2;
    }
    // Alpha never materialised (FP32-scaled form with linear tiles on): the
    // sweeps rebuild alpha from the seeds of 9-bit blocks.
    P.fused = fuse == 1 && P.x32 && P.lin_mode != 0 && n >= 10;
    if (P.fused) P.bL = 9;
    P.KS9 = (P.fused && d > 0) ? (uint32_t)kcount_u64(9, d - 1) : 0;
    P.KG = (uint32_t)kcount_u64(P.bG, d);
    P.KA = (uint32_t)kcount_u64(P.aG, d);
    P.W = std::max(std::max(P.bA, P.bG), P.aG);
    P.W = std::max(P.W, 1);
    {
        GammaGeom &g = P.gg;
        memset(&g, 0, sizeof(g));
        uint64_t y1 = 0, y2 = 0;
        int hmax1 = 0;
        for (int v = 0; v < n; ++v) {
            g.bv[v] = v < P.bG ? P.bG - 1 : P.bG;
            g.hv[v] = N - g.bv[v];
            const uint64_t kg = kcount_u64(g.bv[v], d);
            g.y1off[v] = y1;
            g.kg4[v] = (uint32_t)kg & ~3u;
            y1 += kg << g.hv[v];
            const bool two = g.hv[v] > P.aG;
            g.y2off[v] = y2;
            if (two) y2 += (kg * P.KA) << (g.hv[v] - P.aG);
            else hmax1 = std::max(hmax1, g.hv[v]);
            g.blk1[v + 1] = g.blk1[v] + (two ? 0 : (uint32_t)kg);
            g.blkA[v + 1] = g.blkA[v] + (two ? (uint32_t)(kg << (g.hv[v] - P.aG)) : 0);
            const uint32_t items4 = g.kg4[v] / 4 + ((uint32_t)kg - g.kg4[v]);
            g.blk1x4[v + 1] = g.blk1x4[v] + (two ? 0 : items4);
            g.blkAx4[v + 1] = g.blkAx4[v] + (two ? items4 << (g.hv[v] - P.aG) : 0);
            g.blkB[v + 1] = g.blkB[v] + (two ? (uint32_t)kg : 0);
        }
        g.KT = P.KG;
        g.npat = (uint32_t)kcount_u64(std::max(P.bG - 1, 0), d);
        g.hmax1 = hmax1;
        P.y1_elems = y1;
        P.y2_elems = y2;
        P.two_level = y2 > 0;
    }
    const int nh = n - P.bL;
    P.tiles.resize(nh + 1);
    for (int h = 0; h <= nh; ++h) P.tiles[h] = (uint32_t)binom_u64(nh, h);

    const uint64_t NN = 1ull << N, NS = 1ull << n;
    const size_t V = 8;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align256(bytes);
        return r;
    };
    P.o_binom = take(33 * 33 * 4);
    P.o_lorder = take(((size_t)1 << P.bL) * 2);
    P.o_loff = take((P.bL + 2) * 4);
    P.o_pat = take(((size_t)1 << P.W) * 2);
    P.o_seed = take(P.KG * 4);
    P.o_famask = take((size_t)P.K * 4);
    P.o_seedA = take(kcount_u64(P.bA, d) * 4);
    P.o_items = take(kcount_u64(N - P.bA, d) * 4);
    P.o_ordC = take(256);
    P.o_hord = take(((size_t)4) << (n - P.bL));
    P.o_glo = take(512 * 4);
    P.o_arity = take(64);
    P.o_rho = take(34 * 8);
    P.o_q = take(32 * 8);
    P.o_cnt = take(4 * 8);
    P.o_diag = take(16 * 8);
    P.o_resid = take(32 * 8);
    P.o_layer = take(33 * 32 * V);     // layer sums of L(S) Rp(S), 32 tile ranges each
    P.o_qt = take(32 * V);
    P.o_gexp = take(64 * 8);
    P.o_logp = take((size_t)n * P.K * 8);
    // binary bit planes, then log-gamma tables (10 x (m + 1) doubles)
    P.o_bits = take((size_t)2 * n * ((std::max(m, 1) + 31) / 32) * 4 + (size_t)10 * (m + 1) * 8);
    // everything the local-score step touches lies below this offset
    P.o_scores_end = o;
    P.o_beta = take((size_t)n * P.K * V);
    if (P.x32) {
        P.o_alpha_f = P.fused ? 0 : take((size_t)n * NN * 4);
        P.o_alpha_b = P.fused ? 0 : take((size_t)n * NN);
        P.o_L_f = take(NS * 4);
        P.o_L_b = take(NS);
        P.o_R_f = take(NS * 4);
        P.o_R_b = take(NS);
    } else {
        P.o_alpha_f = take((size_t)n * NN * 8);
        P.o_L_f = take(NS * 8);
        P.o_R_f = take(NS * 8);
    }
    P.o_Y1 = take((size_t)P.y1_elems * V);
    if (P.two_level) P.o_Y2 = take((size_t)P.y2_elems * V);
    P.o_gam = take((size_t)n * P.K * V);
    P.o_part = take(std::max(((size_t)1 << nh) * (P.bL + 1),
                             n >= 12 ? ((size_t)1 << (n - 12)) * 13 : (size_t)0) * V);
    P.o_fbA = P.fused ? take(8) : (P.bA == 13 ? take(4 * (1 + ((size_t)n << (N - 13)))) : 0);
    P.o_betal = (P.bA == 13 || P.fused) ? take((size_t)n * P.K * 8) : 0;
    // Linear alpha tiles keep their seeds (K(13, d) doubles per tile) in the
    // workspace when those take at most 16 GiB; otherwise alpha runs in the
    // number system proper.
    P.KS = (P.bA == 13 && d > 0) ? (uint32_t)kcount_u64(13, d - 1) : 0;   // seeds of size < d
    const uint64_t zs_bytes = P.bA == 13 ? ((uint64_t)n << (N - 13)) * P.KS * 8 : 0;
    P.alpha_lin = !P.fused && P.lin_mode != 0 && P.bA == 13 && zs_bytes <= (16ull << 30);
    // the fused path builds its 9-bit block seeds from the same 13-bit seeds
    const bool zs13 = P.fused && P.bA == 13 && d > 0 && zs_bytes <= (16ull << 30);
    P.o_Zs = (P.alpha_lin || zs13) ? take(zs_bytes) : 0;
    // seeds of the 9-bit blocks: K(9, d - 1) of 8 bytes per block, 2^(n - 10)
    // blocks per node
    const uint64_t nz9 = P.fused ? ((uint64_t)n << (N - 9)) * P.KS9 : 0;
    P.o_zw9 = P.fused ? take(nz9 * 8) : 0;
    P.o_emax = take(32 * 4);
    P.o_flin = take(64 * 4);
    P.o_anc = take(32 * 8);
    P.o_linok = take(32 * 4);
    // Gamma lists: endpoints for a second scale (at most one entry per tile and
    // endpoint), tiles for the fallback (one per failed second chance, and one
    // per tile when every tile is forced there)
    P.o_fbG = P.bG == 12 ? take(4 * (1 + ((size_t)(n + 1) << (n - 12)))) : 0;
    P.o_rtG = P.bG == 12 ? take(4 * (1 + ((size_t)n << (n - 12)))) : 0;
    if (with_post) P.o_post = take((size_t)n * n * 8);
    if (with_post) P.o_ps = take((size_t)n * P.K * 8);
    if (with_data) P.o_data = take((size_t)n * (size_t)std::max(m, 1));
    P.total = o;
    P.max_bins = 1;
    return P;
}

// Materialised alpha costs 2.9x the fused path's HBM footprint but measures
// faster (n = 30: 103.7 against 120.4 ms; n = 25: 5.6 against 6.9 ms), so
// the fused sweeps are taken only where alpha would not fit: from n = 23
// when the materialised workspace exceeds kFuseAboveBytes (a device of
// 288 GB, less room for the caller's own buffers) and the fused one is
// smaller. BN_FUSED_ALPHA=1 takes the fused path from n = 10, =0 never
// (tests, measurements).
static constexpr size_t kFuseAboveBytes = 240ull << 30;

Plan make_plan(int n, int d_in, int m, bn_precision prec, bool with_data, bool with_post) {
    if (const char *fa = getenv("BN_FUSED_ALPHA")) {
        if (!strcmp(fa, "0")) return plan_of(n, d_in, m, prec, with_data, with_post, 0);
        if (!strcmp(fa, "1")) return plan_of(n, d_in, m, prec, with_data, with_post, 1);
    }
    Plan P = plan_of(n, d_in, m, prec, with_data, with_post, 0);
    if (n >= 23 && P.x32 && P.lin_mode != 0 && P.total > kFuseAboveBytes) {
        // the block seeds, K(9, d - 1) of 8 bytes per 512 entries, outgrow
        // alpha's 5 bytes per entry from d = 6: keep the smaller plan
        Plan F = plan_of(n, d_in, m, prec, with_data, with_post, 1);
        if (F.total < P.total) P = F;
    }
    return P;
}

static int max_bins_of(const bn_problem *p, int d) {
    int best = 1;
    for (int i = 0; i < p->n; ++i) {
        std::vector<int> ar;
        for (int j = 0; j < p->n; ++j)
            if (j != i) ar.push_back(p->arity[j]);
        std::sort(ar.rbegin(), ar.rend());
        long bins = p->arity[i];
        for (int k = 0; k < d; ++k) bins *= ar[k];
        best = (int)std::max<long>(best, bins);
    }
    return best;
}

static Tables tables_of(const Plan &P, char *ws) {
    Tables tb;
    tb.binom = reinterpret_cast<uint32_t *>(ws + P.o_binom);
    tb.lorder = reinterpret_cast<uint16_t *>(ws + P.o_lorder);
    tb.loff = reinterpret_cast<uint32_t *>(ws + P.o_loff);
    tb.pat = reinterpret_cast<uint16_t *>(ws + P.o_pat);
    tb.seedmask = reinterpret_cast<uint32_t *>(ws + P.o_seed);
    tb.famask = reinterpret_cast<uint32_t *>(ws + P.o_famask);
    tb.seedA = reinterpret_cast<uint32_t *>(ws + P.o_seedA);
    tb.items = reinterpret_cast<uint32_t *>(ws + P.o_items);
    tb.ordC = reinterpret_cast<uint8_t *>(ws + P.o_ordC);
    tb.hord = reinterpret_cast<uint32_t *>(ws + P.o_hord);
    return tb;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e__ = (x);                       \
        if (e__ != hipSuccess) return BN_EDEVICE;   \
    } while (0)

// Enqueue parameters, tables and local scores on stream st.
static bn_status enqueue_scores(const Plan &P, const bn_problem *p, const uint8_t *dev_data,
                                char *ws, hipStream_t st) {
    ParamBlock pb{};
    for (int i = 0; i < P.n; ++i) pb.arity[i] = p->arity[i];
    pb.has_rho = p->log_rho != nullptr;
    pb.has_q = p->log_q != nullptr;
    if (p->log_rho)
        for (int k = 0; k <= P.d; ++k) pb.log_rho[k] = p->log_rho[k];
    if (p->log_q)
        for (int k = 0; k < P.n; ++k) pb.log_q[k] = p->log_q[k];
    auto *cnt = reinterpret_cast<unsigned long long *>(ws + P.o_cnt);
    hipLaunchKernelGGL(k_params, dim3(1), dim3(64), 0, st, pb, P.n, P.d,
                       reinterpret_cast<uint8_t *>(ws + P.o_arity),
                       reinterpret_cast<double *>(ws + P.o_rho),
                       reinterpret_cast<double *>(ws + P.o_q), cnt);
    HIPCHK(hipGetLastError());
    Tables tb = tables_of(P, ws);
    HIPCHK(launch_setup(tb, P.bL, P.W, P.bG, P.bA, P.d, P.N, P.K, st));
    const int kind = p->score == BN_SCORE_K2 ? 1 : 0;
    // all-binary data with d <= 4: the bit-plane counting path; one arity r
    // for every variable and d <= 4: log-gamma tables (q = r^k)
    bool uniform = P.d <= 4;
    for (int i = 1; i < P.n && uniform; ++i) uniform = p->arity[i] == p->arity[0];
    bool binary = P.m > 0 && uniform && p->arity[0] == 2;
    if (const char *e = getenv("BN_SCORE_BITS"))
        if (e[0] == '0') binary = false;
    if (const char *e = getenv("BN_SCORE_TABLES"))
        if (e[0] == '0') uniform = false;
    uint32_t *bits = reinterpret_cast<uint32_t *>(ws + P.o_bits);
    double *lgt = reinterpret_cast<double *>(bits + (size_t)2 * P.n * ((std::max(P.m, 1) + 31) / 32));
    HIPCHK(launch_scores(P.n, P.m, dev_data, reinterpret_cast<const uint8_t *>(ws + P.o_arity), P.K,
                         kind, p->ess, tb.famask, max_bins_of(p, P.d),
                         reinterpret_cast<double *>(ws + P.o_logp), st, binary ? bits : nullptr,
                         uniform ? p->arity[0] : 0, lgt));
    return BN_OK;
}

static LatticeArgs lattice_args(const Plan &P, char *ws, double *dev_post, double *dev_diag,
                                double *dev_ps) {
    LatticeArgs a{};
    a.n = P.n;
    a.d = P.d;
    a.K = P.K;
    a.bA = P.bA;
    a.bL = P.bL;
    a.bG = P.bG;
    a.aG = P.aG;
    a.KG = P.KG;
    a.KA = P.KA;
    a.npatA = (uint32_t)kcount_u64(std::max(P.bA - 1, 0), P.d);
    a.nitA = (uint32_t)kcount_u64(P.N - P.bA, P.d);
    a.gauge = P.x32 ? 1 : 0;
    a.tb = tables_of(P, ws);
    a.logp = reinterpret_cast<const double *>(ws + P.o_logp);
    a.log_rho = reinterpret_cast<const double *>(ws + P.o_rho);
    a.log_q = reinterpret_cast<const double *>(ws + P.o_q);
    a.beta = ws + P.o_beta;
    a.qt = ws + P.o_qt;
    a.Y1 = ws + P.o_Y1;
    a.Y2 = P.two_level ? ws + P.o_Y2 : nullptr;
    a.gam = ws + P.o_gam;
    a.part = ws + P.o_part;
    a.layer = ws + P.o_layer;
    a.gauge_exp = reinterpret_cast<double *>(ws + P.o_gexp);
    a.post = dev_post;
    a.ps = dev_ps;
    a.resid = reinterpret_cast<double *>(ws + P.o_resid);
    a.diag = dev_diag ? dev_diag : reinterpret_cast<double *>(ws + P.o_diag);
    a.cnt = reinterpret_cast<unsigned long long *>(ws + P.o_cnt);
    a.tiles_per_layer = P.tiles.data();
    a.gg = P.gg;
    a.lin_mode = P.lin_mode;
    a.fbA = (P.bA == 13 || P.fused) ? reinterpret_cast<uint32_t *>(ws + P.o_fbA) : nullptr;
    a.fbG = P.bG == 12 ? reinterpret_cast<uint32_t *>(ws + P.o_fbG) : nullptr;
    a.rtG = P.bG == 12 ? reinterpret_cast<uint32_t *>(ws + P.o_rtG) : nullptr;
    a.betal = (P.bA == 13 || P.fused) ? reinterpret_cast<double *>(ws + P.o_betal) : nullptr;
    a.anc = ws + P.o_anc;
    a.linok = reinterpret_cast<int *>(ws + P.o_linok);
    a.Zs = P.o_Zs ? reinterpret_cast<double *>(ws + P.o_Zs) : nullptr;
    a.KS = P.KS;
    a.fused = P.fused ? 1 : 0;
    a.KS9 = P.KS9;
    a.zw9 = P.fused ? reinterpret_cast<void *>(ws + P.o_zw9) : nullptr;
    a.emax = reinterpret_cast<int *>(ws + P.o_emax);
    a.flin = reinterpret_cast<int *>(ws + P.o_flin);
    a.glo = reinterpret_cast<uint32_t *>(ws + P.o_glo);
    return a;
}

// The backward sweep of a large lattice runs on a second stream of the
// device (one per device, created on first use, default priority), forked
// after alpha and joined before Gamma, so that the small layers of the two
// sweeps overlap. From n = 24 (smaller lattices are dispatch-bound and are
// served many at a time on streams of their own); BN_SWEEP_FORK=0 keeps
// both sweeps on the caller's stream. Solves that run at the same time on
// one device share that second stream (their backward sweeps then queue
// behind each other).
constexpr int kSweepForkFromN = 24;
static std::mutex g_side_mu;
static hipStream_t g_side[64] = {};
static hipStream_t side_stream(const Plan &P) {
    if (P.n < kSweepForkFromN || P.fused) return nullptr;
    static const bool on = [] {
        const char *e = getenv("BN_SWEEP_FORK");
        return !(e && e[0] == '0');
    }();
    if (!on) return nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (!g_side[dev] && hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking) != hipSuccess)
        g_side[dev] = nullptr;
    return g_side[dev];
}

static bn_status run_lattice(const Plan &P, char *ws, LatticeArgs a, hipStream_t st,
                             PhaseEvents *ev) {
    a.side = side_stream(P);
    hipError_t e;
    if (P.x32) {
        PolX32::Store al{reinterpret_cast<float *>(ws + P.o_alpha_f),
                         reinterpret_cast<uint8_t *>(ws + P.o_alpha_b)};
        PolX32::Store L{reinterpret_cast<float *>(ws + P.o_L_f),
                        reinterpret_cast<uint8_t *>(ws + P.o_L_b)};
        PolX32::Store R{reinterpret_cast<float *>(ws + P.o_R_f),
                        reinterpret_cast<uint8_t *>(ws + P.o_R_b)};
        e = launch_lattice<PolX32>(a, al, L, R, st, ev);
    } else {
        PolLog::Store al{reinterpret_cast<double *>(ws + P.o_alpha_f)};
        PolLog::Store L{reinterpret_cast<double *>(ws + P.o_L_f)};
        PolLog::Store R{reinterpret_cast<double *>(ws + P.o_R_f)};
        e = launch_lattice<PolLog>(a, al, L, R, st, ev);
    }
    return e == hipSuccess ? BN_OK : BN_EDEVICE;
}

bn_status enqueue_solve(const Plan &P, const bn_problem *p, const uint8_t *dev_data, char *ws,
                        hipStream_t st, double *dev_post, double *dev_diag, PhaseEvents *ev,
                        double *dev_ps) {
    if (log_level() >= 1)
        fprintf(stderr,
                "[bn] solve n=%d m=%d d=%d %s alpha=%s tiles alpha/sweep/gamma=%d/%d/%d "
                "linear_tiles=%d workspace=%.3f GiB\n",
                P.n, P.m, P.d, P.x32 ? "fp32_scaled" : "fp64_log",
                P.fused ? "fused" : "materialised", P.bA, P.bL, P.bG, P.lin_mode,
                (double)P.total / (double)(1ull << 30));
    Range r("bn.enqueue_solve");
    if (ev && ev->ev[0]) HIPCHK(hipEventRecord(ev->ev[0], st));
    bn_status s;
    {
        Range rs("bn.enqueue_scores");
        s = enqueue_scores(P, p, dev_data, ws, st);
    }
    if (s != BN_OK) return s;
    const LatticeArgs a = lattice_args(P, ws, dev_post, dev_diag, dev_ps);
    Range rl("bn.enqueue_lattice");
    return run_lattice(P, ws, a, st, ev);
}

bn_status local_scores_host(const bn_problem *p, double *log_score) {
    bn_status s = validate(p, true, true);
    if (s != BN_OK) return s;
    if (!log_score) return BN_EINVAL;
    Plan P = make_plan(p->n, p->d, p->m, BN_FP64_LOG, true, false);
    // the parameters, tables, counters and scores all lie below o_scores_end
    char *ws = nullptr;
    const size_t small = P.o_scores_end;
    size_t data_bytes = (size_t)P.n * std::max(P.m, 1);
    if (hipMalloc(&ws, small + align256(data_bytes)) != hipSuccess) return BN_ENOMEM;
    uint8_t *dev_data = reinterpret_cast<uint8_t *>(ws + small);
    hipStream_t st = nullptr;
    bn_status rs = BN_OK;
    if (P.m > 0 &&
        hipMemcpyAsync(dev_data, p->data, (size_t)P.n * P.m, hipMemcpyHostToDevice, st) !=
            hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK) rs = enqueue_scores(P, p, dev_data, ws, st);
    if (rs == BN_OK &&
        hipMemcpyAsync(log_score, ws + P.o_logp, (size_t)P.n * P.K * 8, hipMemcpyDeviceToHost,
                       st) != hipSuccess)
        rs = BN_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) rs = BN_EDEVICE;
    (void)hipFree(ws);
    return rs;
}

bn_status edge_posteriors_host(const bn_problem *p, bn_precision prec, double *post,
                               bn_report *rep, double *ps) {
    bn_status s = validate(p, true, true);
    if (s != BN_OK) return s;
    if (!post && !ps) return BN_EINVAL;
    if (prec != BN_FP64_LOG && prec != BN_FP32_SCALED) return BN_EINVAL;
    Plan P = make_plan(p->n, p->d, p->m, prec, true, true);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return BN_EDEVICE;
    if (P.total > free_b) return BN_ENOMEM;
    char *ws = nullptr;
    if (hipMalloc(&ws, P.total) != hipSuccess) return BN_ENOMEM;
    hipStream_t st = nullptr;
    PhaseEvents ev{};
    bool timing = rep != nullptr;
    if (timing)
        for (int k = 0; k < 7; ++k) (void)hipEventCreate(&ev.ev[k]);
    uint8_t *dev_data = reinterpret_cast<uint8_t *>(ws + P.o_data);
    double *dev_post = reinterpret_cast<double *>(ws + P.o_post);
    double *dev_diag = reinterpret_cast<double *>(ws + P.o_diag);
    double *dev_ps = ps ? reinterpret_cast<double *>(ws + P.o_ps) : nullptr;
    bn_status rs = BN_OK;
    if (P.m > 0 &&
        hipMemcpyAsync(dev_data, p->data, (size_t)P.n * P.m, hipMemcpyHostToDevice, st) !=
            hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK)
        rs = enqueue_solve(P, p, dev_data, ws, st, dev_post, dev_diag, timing ? &ev : nullptr,
                           dev_ps);
    double diag[16] = {0};
    if (rs == BN_OK && post &&
        hipMemcpyAsync(post, dev_post, (size_t)P.n * P.n * 8, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK && ps &&
        hipMemcpyAsync(ps, dev_ps, (size_t)P.n * P.K * 8, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK &&
        hipMemcpyAsync(diag, dev_diag, 8 * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
        rs = BN_EDEVICE;
    {
        Range rw("bn.wait");
        if (hipStreamSynchronize(st) != hipSuccess) rs = BN_EDEVICE;
    }
    if (rs == BN_OK && rep) {
        memset(rep, 0, sizeof(*rep));
        rep->log_LV = diag[0];
        rep->max_invariant_residual = diag[1];
        rep->saturated = (uint64_t)diag[2];
        rep->flushed = (uint64_t)diag[3];
        rep->fallback_tiles = (uint64_t)diag[7];
        float ms[7] = {0};
        for (int k = 1; k < 7; ++k) (void)hipEventElapsedTime(&ms[k], ev.ev[k - 1], ev.ev[k]);
        float tot = 0;
        (void)hipEventElapsedTime(&tot, ev.ev[0], ev.ev[6]);
        rep->ms_scores = ms[1];
        rep->ms_alpha = ms[2];
        rep->ms_fwd = ms[3];
        rep->ms_bwd = ms[4];
        rep->ms_gamma = ms[5];
        rep->ms_edges = ms[6];
        rep->ms_total = tot;
        if (log_level() >= 2)
            fprintf(stderr,
                    "[bn] report log_L(V)=%.9f residual=%.3e saturated=%llu flushed=%llu "
                    "fallback=%llu ms scores/alpha/fwd/bwd/gamma/edges/total="
                    "%.3f/%.3f/%.3f/%.3f/%.3f/%.3f/%.3f\n",
                    rep->log_LV, rep->max_invariant_residual,
                    (unsigned long long)rep->saturated, (unsigned long long)rep->flushed,
                    (unsigned long long)rep->fallback_tiles, rep->ms_scores, rep->ms_alpha,
                    rep->ms_fwd, rep->ms_bwd, rep->ms_gamma, rep->ms_edges, rep->ms_total);
        if (log_level() >= 2 && P.bG == 12) {
            // list heads: Gamma endpoints given a second scale, Gamma items and
            // alpha tiles (or, fused, blocks) recomputed in the number system
            uint32_t cnt[3] = {0, 0, 0};
            (void)hipMemcpy(&cnt[0], ws + P.o_rtG, 4, hipMemcpyDeviceToHost);
            (void)hipMemcpy(&cnt[1], ws + P.o_fbG, 4, hipMemcpyDeviceToHost);
            if (P.o_fbA) (void)hipMemcpy(&cnt[2], ws + P.o_fbA, 4, hipMemcpyDeviceToHost);
            fprintf(stderr, "[bn] lists gamma_second_scale=%u gamma_fallback=%u alpha_fallback=%u\n",
                    cnt[0], cnt[1], cnt[2]);
        }
    }
    if (timing)
        for (int k = 0; k < 7; ++k) (void)hipEventDestroy(ev.ev[k]);
    (void)hipFree(ws);
    return rs;
}

// E[f | D] of a modular feature: two forward-only runs on one workspace, the
// second with log f added to the log scores (f_i(G) B_i(G) in place of
// B_i(G)); out = exp(log P(f, D) - log P(D)).
bn_status feature_posterior_host(const bn_problem *p, bn_precision prec, const double *log_f,
                                 double *out, double *log_pair) {
    bn_status s = validate(p, true, true);
    if (s != BN_OK) return s;
    if (!log_f || !out) return BN_EINVAL;
    if (prec != BN_FP64_LOG && prec != BN_FP32_SCALED) return BN_EINVAL;
    Plan P = make_plan(p->n, p->d, p->m, prec, true, true);
    const size_t cnt = (size_t)P.n * P.K;
    for (size_t x = 0; x < cnt; ++x)
        if (std::isnan(log_f[x]) || log_f[x] == HUGE_VAL) return BN_EINVAL;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return BN_EDEVICE;
    if (P.total > free_b) return BN_ENOMEM;
    char *ws = nullptr;
    if (hipMalloc(&ws, P.total) != hipSuccess) return BN_ENOMEM;
    hipStream_t st = nullptr;
    uint8_t *dev_data = reinterpret_cast<uint8_t *>(ws + P.o_data);
    double *dev_diag = reinterpret_cast<double *>(ws + P.o_diag);
    double *dev_f = reinterpret_cast<double *>(ws + P.o_ps);   // n*K doubles, unused here
    LatticeArgs a = lattice_args(P, ws, nullptr, dev_diag, nullptr);
    a.fwd_only = 1;
    double d0[8] = {0}, d1[8] = {0};
    bn_status rs = BN_OK;
    if (P.m > 0 &&
        hipMemcpyAsync(dev_data, p->data, (size_t)P.n * P.m, hipMemcpyHostToDevice, st) !=
            hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK) rs = enqueue_scores(P, p, dev_data, ws, st);
    if (rs == BN_OK) rs = run_lattice(P, ws, a, st, nullptr);
    if (rs == BN_OK && hipMemcpyAsync(d0, dev_diag, 64, hipMemcpyDeviceToHost, st) != hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK &&
        hipMemcpyAsync(dev_f, log_f, cnt * 8, hipMemcpyHostToDevice, st) != hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK &&
        launch_add_log(reinterpret_cast<double *>(ws + P.o_logp), dev_f, cnt, st) != hipSuccess)
        rs = BN_EDEVICE;
    if (rs == BN_OK) rs = run_lattice(P, ws, a, st, nullptr);
    if (rs == BN_OK && hipMemcpyAsync(d1, dev_diag, 64, hipMemcpyDeviceToHost, st) != hipSuccess)
        rs = BN_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) rs = BN_EDEVICE;
    (void)hipFree(ws);
    if (rs != BN_OK) return rs;
    *out = d1[0] > -HUGE_VAL ? std::exp(d1[0] - d0[0]) : 0.0;
    if (log_pair) {
        log_pair[0] = d0[0];
        log_pair[1] = d1[0];
    }
    return BN_OK;
}

// ------------------------------------------------ allocation-free variant
// The workspace of bn_edge_posteriors_noalloc: a static device array. Each
// GPU the library runs on holds its own copy, at its own address, from the
// loading of the library until the process ends. In host code the array's
// name is only a stand-in for the symbol; the device address comes from
// hipGetSymbolAddress, once per device, and is the only form that reaches a
// kernel.
static __device__ __align__(256) unsigned char scratch[BN_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (resolved on the
// first call on that device, with that device current).
static bn_status scratch_of_current_device(char **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BN_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return BN_EDEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = reinterpret_cast<char *>(g_scratch_ptr[dev]);
    return BN_OK;
}

bn_status edge_posteriors_noalloc(const bn_problem *p, bn_precision prec, void *hip_stream,
                                  double *dev_post, double *dev_diag) {
    bn_status s = validate(p, false, false);
    if (s != BN_OK) return s;
    if (!dev_post) return BN_EINVAL;
    if (prec != BN_FP64_LOG && prec != BN_FP32_SCALED) return BN_EINVAL;
    Plan P = make_plan(p->n, p->d, p->m, prec, false, false);
    if (P.total > (size_t)BN_NOALLOC_MAX_BYTES) return BN_ENOMEM;
    char *ws = nullptr;
    s = scratch_of_current_device(&ws);
    if (s != BN_OK) return s;
    // Every kernel of the solve initialises what it later reads (counters,
    // lists and partial sums included), so the previous call's contents need
    // no clearing.
    return enqueue_solve(P, p, p->data, ws, reinterpret_cast<hipStream_t>(hip_stream), dev_post,
                         dev_diag, nullptr);
}

bn_status edge_posteriors_dev(const bn_problem *p, bn_precision prec, void *dev_ws,
                              size_t ws_bytes, void *hip_stream, double *dev_post,
                              double *dev_diag, PhaseEvents *ev) {
    bn_status s = validate(p, false, false);
    if (s != BN_OK) return s;
    if (!dev_ws || !dev_post) return BN_EINVAL;
    if (prec != BN_FP64_LOG && prec != BN_FP32_SCALED) return BN_EINVAL;
    Plan P = make_plan(p->n, p->d, p->m, prec, false, false);
    if (ws_bytes < P.total) return BN_EINVAL;
    return enqueue_solve(P, p, p->data, reinterpret_cast<char *>(dev_ws),
                         reinterpret_cast<hipStream_t>(hip_stream), dev_post, dev_diag, ev);
}

}  // namespace bnk

// ------------------------------------------------------------------ C ABI
extern "C" {

size_t bn_num_parent_sets(int32_t n, int32_t d) {
    if (n < 1 || d < 0) return 0;
    return (size_t)bnk::kcount_u64(n - 1, std::min(d, n - 1));
}

bn_status bn_local_scores(const bn_problem *p, double *log_score) {
    return bnk::local_scores_host(p, log_score);
}

bn_status bn_workspace_bytes(int32_t n, int32_t d, int32_t m, bn_precision prec, size_t *bytes) {
    if (!bytes || n < 2 || n > 31 || d < 0 || m < 0) return BN_EINVAL;
    if (prec != BN_FP64_LOG && prec != BN_FP32_SCALED) return BN_EINVAL;
    *bytes = bnk::make_plan(n, d, m, prec, false, false).total;
    return BN_OK;
}

bn_status bn_edge_posteriors(const bn_problem *p, bn_precision prec, double *post,
                             bn_report *rep) {
    if (!post) return BN_EINVAL;
    return bnk::edge_posteriors_host(p, prec, post, rep, nullptr);
}

bn_status bn_parent_set_posteriors(const bn_problem *p, bn_precision prec, double *ps,
                                   double *post, bn_report *rep) {
    if (!ps) return BN_EINVAL;
    return bnk::edge_posteriors_host(p, prec, post, rep, ps);
}

bn_status bn_modular_feature_posterior(const bn_problem *p, bn_precision prec,
                                       const double *log_f, double *expectation,
                                       double *log_pair) {
    return bnk::feature_posterior_host(p, prec, log_f, expectation, log_pair);
}

bn_status bn_edge_posteriors_noalloc(const bn_problem *p, bn_precision prec, void *hip_stream,
                                     double *dev_post, double *dev_diag) {
    return bnk::edge_posteriors_noalloc(p, prec, hip_stream, dev_post, dev_diag);
}

struct bn_timer {
    bnk::PhaseEvents ev;
};

bn_status bn_edge_posteriors_dev(const bn_problem *p, bn_precision prec, void *dev_ws,
                                 size_t ws_bytes, void *hip_stream, double *dev_post,
                                 double *dev_diag, bn_timer *timer) {
    return bnk::edge_posteriors_dev(p, prec, dev_ws, ws_bytes, hip_stream, dev_post, dev_diag,
                                    timer ? &timer->ev : nullptr);
}

bn_status bn_timer_create(bn_timer **timer) {
    if (!timer) return BN_EINVAL;
    bn_timer *t = new bn_timer();
    for (int k = 0; k < 10; ++k) {
        if (hipEventCreate(&t->ev.ev[k]) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(t->ev.ev[j]);
            delete t;
            return BN_EDEVICE;
        }
    }
    *timer = t;
    return BN_OK;
}

bn_status bn_timer_destroy(bn_timer *timer) {
    if (!timer) return BN_EINVAL;
    for (int k = 0; k < 10; ++k) (void)hipEventDestroy(timer->ev.ev[k]);
    delete timer;
    return BN_OK;
}

bn_status bn_timer_read(const bn_timer *timer, double ms[9]) {
    if (!timer || !ms) return BN_EINVAL;
    for (int k = 1; k < 7; ++k) {
        float x = 0;
        if (hipEventElapsedTime(&x, timer->ev.ev[k - 1], timer->ev.ev[k]) != hipSuccess)
            return BN_EDEVICE;
        ms[k - 1] = x;
    }
    float tot = 0;
    if (hipEventElapsedTime(&tot, timer->ev.ev[0], timer->ev.ev[6]) != hipSuccess)
        return BN_EDEVICE;
    ms[6] = tot;
    float gt = 0;
    if (hipEventElapsedTime(&gt, timer->ev.ev[4], timer->ev.ev[7]) != hipSuccess)
        return BN_EDEVICE;
    ms[7] = gt;
    float at = 0;
    if (hipEventElapsedTime(&at, timer->ev.ev[8], timer->ev.ev[9]) != hipSuccess)
        return BN_EDEVICE;
    ms[8] = at;
    return BN_OK;
}

const char *bn_status_string(bn_status s) {
    switch (s) {
        case BN_OK: return "ok";
        case BN_EINVAL: return "invalid argument";
        case BN_ENOMEM: return "out of device memory or budget";
        case BN_EDEVICE: return "HIP runtime error";
        case BN_EAGAIN: return "not ready";
        case BN_ECANCELED: return "canceled";
        case BN_EINTERNAL: return "internal error";
    }
    return "unknown status";
}

}  // extern "C"
