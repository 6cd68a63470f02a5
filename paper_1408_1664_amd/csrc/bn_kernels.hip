// HIP kernels (gfx950) for the exact edge-posterior programme.
//
// Lattice layout in HBM (variable i <-> bit i):
//   alpha_i : node-major, 2^(n-1) entries per node, indexed by the subset S
//             of the other n-1 variables with bit i removed (compress_bit).
//   L, Rp   : 2^n entries indexed by the subset mask.
//   scores, beta, Gamma : per node, K(n-1,d) parent sets ranked by size then
//             colex order of the compressed mask.
//
// Tiling: a tile is 2^b consecutive masks (the low b bits vary inside a
// workgroup, the high bits select the tile). Every kernel runs 256 threads.
#include <algorithm>
#include <type_traits>

#include "bn_device.h"
#include "bn_kernels.h"

namespace bnk {

constexpr int kThreads = 256;

// ----------------------------------------------------------- block reduce
// Deterministic tree reduction over the 256 threads of a block (fixed order).
template <class T, class Op>
__device__ inline T block_reduce(T v, T *scratch, Op op) {
    const int t = threadIdx.x;
    scratch[t] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (t < s) scratch[t] = op(scratch[t], scratch[t + s]);
        __syncthreads();
    }
    T r = scratch[0];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ setup
// Lane order of the Gamma tile's layout C, where lane t holds the 8-bit
// pattern p = ordC[t] of tile bits 0..7 and reads its 16 doubles at padded
// slots r * 272 + p + p / 16. The patterns with at most d ones fill the first
// 2 * ceil(nlive / 64) groups of 32 lanes (so the same number of waves holds
// them as in popcount order), each going to the group with room where the
// fewest patterns already share its bank pair (p + p / 16) mod 32; the other
// patterns fill the remaining lanes. Computed once per d on the host.
struct LaneOrder {
    uint8_t p[256];
};

static LaneOrder lane_order_c(int d) {
    LaneOrder o{};
    int cntb[8][32] = {}, fill[8] = {};
    int nl = 0;
    for (int p = 0; p < 256; ++p) nl += __builtin_popcount(p) <= d ? 1 : 0;
    const int ng = std::min(8, 2 * ((nl + 63) / 64));
    for (int k = 0; k <= 8; ++k) {
        for (int p = 0; p < 256; ++p) {
            if (__builtin_popcount(p) != k) continue;
            int best = -1;
            if (k <= d) {
                const int f = (p + (p >> 4)) & 31;
                for (int g = 0; g < ng; ++g)
                    if (fill[g] < 32 && (best < 0 || cntb[g][f] < cntb[best][f])) best = g;
                ++cntb[best][f];
            } else {
                best = 0;
                while (fill[best] == 32) ++best;
            }
            o.p[best * 32 + fill[best]++] = (uint8_t)p;
        }
    }
    return o;
}

// C(a, b) for a, b <= 32, built at compile time (row by row, Pascal's rule)
// and read from constant memory by the table kernel.
struct BinomTable {
    uint32_t v[33 * 33];
};
static constexpr BinomTable make_binom() {
    BinomTable t{};
    for (int a = 0; a <= 32; ++a) {
        t.v[a * 33] = 1;
        for (int b = 1; b <= a; ++b)
            t.v[a * 33 + b] = t.v[(a - 1) * 33 + b - 1] + (b < a ? t.v[(a - 1) * 33 + b] : 0u);
    }
    return t;
}
static_assert(make_binom().v[5 * 33 + 2] == 10u && make_binom().v[32 * 33 + 16] == 601080390u &&
                  make_binom().v[32 * 33 + 32] == 1u && make_binom().v[3 * 33 + 5] == 0u,
              "binomial table");
__constant__ BinomTable kBinomTab = make_binom();

// Masks over w bits with at most d ones (every mask when d >= w), ranked by
// size then colex order (numeric order within a size): out[rank] = mask, for
// the masks x in [x0, x0 + 256).
__device__ inline void ranked_chunk(const uint32_t *bn, int w, int d, uint32_t x,
                                    uint32_t *out) {
    if (x >= (1u << w)) return;
    const int k = __popc(x);
    if (k > d) return;
    uint32_t r = Kcount(bn, w, k - 1);
    int j = 0;
    for (int p = 0; p < w; ++p)
        if ((x >> p) & 1) r += C(bn, p, ++j);
    out[r] = x;
}

// Every per-problem table in one launch; the grid is split into ranges of
// workgroups, one range per table (TableGrid), all reading the binomials
// from constant memory:
//   binomials, layer offsets and popcount-ordered masks of the sweep tile,
//   patterns of at most d ones over W bits (numeric order: the w-bit
//   patterns are exactly the first K(w, d) entries), the lane order of the
//   Gamma tile's layout C and its ranked seed masks (range S);
//   the alpha tile's ranked seed masks over bA bits (range A);
//   the ranked high-bit items of an alpha tile over n - 1 - bA bits (I);
//   the compressed parent-set masks in rank order, K(n - 1, d) (F);
//   the sweep tiles' high parts over n - bL bits by popcount, then colex (H).
struct TableGrid {
    uint32_t s, a, i, f, h;   // cumulative ends of the ranges
};
__global__ void k_tables(Tables tb, LaneOrder oc, TableGrid g, int bL, int W, int bG, int bA,
                         int d, int N, uint32_t K) {
    const uint32_t *bn = kBinomTab.v;
    const uint32_t blk = blockIdx.x;
    const int t = threadIdx.x;
    if (blk < g.s) {
        __shared__ uint32_t loff[34];
        if (blk == 0)
            for (int x = t; x < 33 * 33; x += kThreads) tb.binom[x] = bn[x];
        if (t == 0) {
            uint32_t acc = 0;
            for (int l = 0; l <= bL; ++l) {
                loff[l] = acc;
                acc += C(bn, bL, l);
            }
            loff[bL + 1] = acc;
        }
        __syncthreads();
        if (blk == 0 && t <= bL + 1) tb.loff[t] = loff[t];
        const uint32_t x0 = blk * kThreads + t, step = g.s * kThreads;
        // popcount-ordered tile masks: position = offset of the layer + colex rank
        for (uint32_t x = x0; x < (1u << bL); x += step) {
            int k = __popc(x);
            uint32_t r = 0;
            int j = 0;
            for (int p = 0; p < bL; ++p)
                if ((x >> p) & 1) r += C(bn, p, ++j);
            tb.lorder[loff[k] + r] = (uint16_t)x;
        }
        // patterns with at most d ones over W bits, numeric order
        for (uint32_t x = x0; x < (1u << W); x += step) {
            int ones = __popc(x);
            if (ones > d) continue;
            uint32_t pos = 0;
            int above = 0;
            for (int p = W - 1; p >= 0; --p) {
                if ((x >> p) & 1) {
                    if (d - above >= 0) pos += Kcount(bn, p, d - above);
                    ++above;
                }
            }
            tb.pat[pos] = (uint16_t)x;
        }
        // lane order of the Gamma tile's layout C (lane_order_c)
        if (blk == 0) tb.ordC[t] = oc.p[t];
        // ranked seed masks of the Gamma tile (bG bits): size, then colex
        for (uint32_t x = x0; x < (1u << bG); x += step) ranked_chunk(bn, bG, d, x, tb.seedmask);
    } else if (blk < g.a) {
        ranked_chunk(bn, bA, d, (blk - g.s) * kThreads + t, tb.seedA);
    } else if (blk < g.i) {
        ranked_chunk(bn, N - bA, d, (blk - g.a) * kThreads + t, tb.items);
    } else if (blk < g.f) {
        // compressed parent-set masks in rank order
        const uint32_t r = (blk - g.i) * kThreads + t;
        if (r >= K) return;
        int k = 0;
        uint32_t off = 0;
        while (k < d && r >= off + C(bn, N, k)) off += C(bn, N, k++);
        int pos[32];
        colex_unrank(bn, r - off, k, pos);
        uint32_t msk = 0;
        for (int q = 0; q < k; ++q) msk |= 1u << pos[q];
        tb.famask[r] = msk;
    } else {
        ranked_chunk(bn, N + 1 - bL, 64, (blk - g.f) * kThreads + t, tb.hord);
    }
}

// ------------------------------------------------------ a1: local scores
// One workgroup per family (i, G): integer counts N_jk in an LDS histogram,
// then the Dirichlet-multinomial log marginal likelihood in FP64.
__global__ void k_scores(int n, int m, const uint8_t *__restrict__ data,
                         const uint8_t *__restrict__ arity, uint32_t K, int kind, double ess,
                         const uint32_t *__restrict__ famask, double *__restrict__ out) {
    extern __shared__ int hist[];
    __shared__ double red[kThreads];
    __shared__ int par[32];
    __shared__ int npar_s;
    __shared__ int q_s;
    const uint32_t fam = blockIdx.x;
    const int i = fam / K;
    const uint32_t r = fam % K;
    const int t = threadIdx.x;
    if (t == 0) {
        uint32_t msk = famask[r];
        int np = 0, q = 1;
        // mixed radix: the highest variable index is the most significant digit
        for (int p = 30; p >= 0; --p)
            if ((msk >> p) & 1) {
                int var = p < i ? p : p + 1;
                par[np++] = var;
                q *= arity[var];
            }
        npar_s = np;
        q_s = q;
    }
    __syncthreads();
    const int np = npar_s, q = q_s, ri = arity[i];
    const int bins = q * ri;
    for (int b = t; b < bins; b += kThreads) hist[b] = 0;
    __syncthreads();
    const uint8_t *xi = data + (size_t)i * m;
    for (int s = t; s < m; s += kThreads) {
        int key = 0;
        for (int p = 0; p < np; ++p) {
            int var = par[p];
            key = key * arity[var] + data[(size_t)var * m + s];
        }
        const int bin = key * ri + xi[s];
        if (bin < bins) atomicAdd(&hist[bin], 1);  // values >= arity are ignored
    }
    __syncthreads();
    double a_j, a_jk;
    if (kind == 0) {
        a_j = ess / q;
        a_jk = ess / ((double)q * ri);
    } else {
        a_j = ri;
        a_jk = 1.0;
    }
    const double lg_aj = lgamma(a_j), lg_ajk = lgamma(a_jk);
    double acc = 0.0;
    for (int j = t; j < q; j += kThreads) {
        int nj = 0;
        double s = 0.0;
        for (int k = 0; k < ri; ++k) {
            int c = hist[j * ri + k];
            if (c) {
                s += lgamma(a_jk + c) - lg_ajk;
                nj += c;
            }
        }
        if (nj) acc += s + lg_aj - lgamma(a_j + nj);
    }
    double tot = block_reduce(acc, red, [](double a, double b) { return a + b; });
    if (t == 0) out[fam] = tot;
}

// The same scores, four families per workgroup, one wave each, for
// histograms of at most kScoreWaveBins bins (every family of the problem):
// a quarter of the workgroups and no workgroup barriers. Parents, counts and
// the wave's sum stay within the wave (LDS accesses of one wave run in
// order; the wave barriers keep the compiler from moving them). Each lane
// takes four samples per step, with every load of the step issued before
// the counts. When every variable has the same arity (lgt non-null, d <= 4),
// the log-gamma values come from the tables of k_lgamma_table: a family with
// k parents has q = r^k configurations, so its hyperparameters depend on k
// alone; the table entries are the same lgamma values, so the sums are too.
constexpr int kScoreWaveBins = 2048;
__global__ void __launch_bounds__(kThreads)
k_scores_w(int n, int m, const uint8_t *__restrict__ data, const uint8_t *__restrict__ arity,
           uint32_t K, int kind, double ess, const uint32_t *__restrict__ famask, int max_bins,
           const double *__restrict__ lgt, double *__restrict__ out) {
    extern __shared__ int hist_all[];
    __shared__ int par_all[4][32];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const uint32_t fam = blockIdx.x * 4u + (uint32_t)w;
    if (fam >= (uint32_t)n * K) return;          // whole waves
    int *hist = hist_all + w * max_bins;
    int *par = par_all[w];
    const int i = fam / K;
    const uint32_t msk = famask[fam % K];
    // parents in mixed-radix order: the highest variable index is the most
    // significant digit; lane p < 31 tests bit 30 - p
    const bool has = l < 31 && ((msk >> (30 - l)) & 1);
    const uint64_t ball = __ballot(has);
    const int np = __popcll(ball);
    if (has) {
        const int p = 30 - l;
        par[__popcll(ball & ((1ull << l) - 1))] = p < i ? p : p + 1;
    }
    __builtin_amdgcn_wave_barrier();
    int q = 1;
    for (int p = 0; p < np; ++p) q *= arity[par[p]];
    const int ri = arity[i];
    const int bins = q * ri;
    for (int b = l; b < bins; b += 64) hist[b] = 0;
    __builtin_amdgcn_wave_barrier();
    const uint8_t *xi = data + (size_t)i * m;
    constexpr int U = 4;
    for (int s0 = l; s0 < m; s0 += 64 * U) {
        int key[U];
#pragma unroll
        for (int u = 0; u < U; ++u) key[u] = 0;
        for (int p = 0; p < np; ++p) {
            const int var = par[p];
            const int ar = arity[var];
            const uint8_t *row = data + (size_t)var * m;
            int x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int s = s0 + 64 * u;
                x[u] = s < m ? row[s] : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) key[u] = key[u] * ar + x[u];
        }
        int xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int s = s0 + 64 * u;
            xv[u] = s < m ? (int)xi[s] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int bin = key[u] * ri + xv[u];
            // samples past the end count nowhere; values >= arity are ignored
            if (s0 + 64 * u < m && bin < bins) atomicAdd(&hist[bin], 1);
        }
    }
    __builtin_amdgcn_wave_barrier();
    double acc = 0.0;
    if (lgt) {
        const int m1 = m + 1;
        const double *lj = lgt + (size_t)(2 * np) * m1, *ljk = lj + m1;
        const double lg_aj = lj[0], lg_ajk = ljk[0];
        for (int j = l; j < q; j += 64) {
            int nj = 0;
            double sj = 0.0;
            for (int k = 0; k < ri; ++k) {
                const int c = hist[j * ri + k];
                if (c) {
                    sj += ljk[c] - lg_ajk;
                    nj += c;
                }
            }
            if (nj) acc += sj + lg_aj - lj[nj];
        }
    } else {
        double a_j, a_jk;
        if (kind == 0) {
            a_j = ess / q;
            a_jk = ess / ((double)q * ri);
        } else {
            a_j = ri;
            a_jk = 1.0;
        }
        const double lg_aj = lgamma(a_j), lg_ajk = lgamma(a_jk);
        for (int j = l; j < q; j += 64) {
            int nj = 0;
            double sj = 0.0;
            for (int k = 0; k < ri; ++k) {
                const int c = hist[j * ri + k];
                if (c) {
                    sj += lgamma(a_jk + c) - lg_ajk;
                    nj += c;
                }
            }
            if (nj) acc += sj + lg_aj - lgamma(a_j + nj);
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (l == 0) out[fam] = acc;
}

// ----------------------------------------------- prep: prior and gauges
// log B_i(G) = log rho(|G|) + log p(x_i|x_G); beta_i = B_i / 2^E_i with
// E_i = round(max_G log2 B_i(G)) in the scaled form (0 in log form); the same
// for q(k) with a per-layer exponent F_k.
// Scores of one row per workgroup row (blockIdx.x = node), kPrepChunk
// entries per workgroup (blockIdx.y).
constexpr uint32_t kPrepChunk = 2048;
template <class P>
__global__ void k_prep(int n, int d, uint32_t K, const uint32_t *binom,
                       const double *__restrict__ logp, const double *__restrict__ log_rho,
                       const double *__restrict__ log_q, int gauge,
                       typename P::V *__restrict__ beta, typename P::V *__restrict__ qt,
                       double *__restrict__ gauge_exp, uint32_t *fbA, uint32_t *fbG,
                       uint32_t *rtG) {
    __shared__ double red[kThreads];
    const int i = blockIdx.x;
    const uint32_t chunk = blockIdx.y;      // entries [chunk * kPrepChunk, ...) of row i
    const int t = threadIdx.x;
    if (i == 0 && chunk == 0 && t == 0) {
        if (fbA) fbA[0] = 0;
        if (fbG) fbG[0] = 0;
        if (rtG) rtG[0] = 0;
    }
    const int N = n - 1;
    // cum[k] = K(N, k): the parent sets of rank below it have at most k members
    __shared__ uint32_t cum[33];
    if (t <= d && t < 33) cum[t] = Kcount(binom, N, t);
    __syncthreads();
    auto size_of = [&](uint32_t r) {
        int k = 0;
        while (k < d && r >= cum[k]) ++k;
        return k;
    };
    // the row's maximum (every chunk of the row reads the whole row)
    double mx = -__builtin_huge_val();
    for (uint32_t r = t; r < K; r += kThreads)
        mx = fmax(mx, log_rho[size_of(r)] + logp[(size_t)i * K + r]);
    mx = block_reduce(mx, red, [](double a, double b) { return fmax(a, b); });
    const double E = (gauge && mx > -1e300) ? rint(mx * 1.4426950408889634074) : 0.0;
    const uint32_t r1 = min(K, (chunk + 1) * kPrepChunk);
    for (uint32_t r = chunk * kPrepChunk + t; r < r1; r += kThreads) {
        const double lb = log_rho[size_of(r)] + logp[(size_t)i * K + r];
        beta[(size_t)i * K + r] = P::from_log(lb - E * 0.69314718055994530942);
    }
    if (chunk == 0 && t == 0) gauge_exp[i] = E;
    if (i == 0 && chunk == 0) {
        for (int k = t; k < n; k += kThreads) {
            double lq = log_q[k];
            double F = (gauge && lq > -1e300) ? rint(lq * 1.4426950408889634074) : 0.0;
            qt[k] = P::from_log(lq - F * 0.69314718055994530942);
            gauge_exp[n + k] = F;
        }
    }
}

// ------------------------------------------------ a2: alpha (upward zeta)
__device__ inline double shfl_xor_v(double v, int m) { return __shfl_xor(v, m); }
__device__ inline X32 shfl_xor_v(X32 v, int m) {
    return X32{__shfl_xor(v.f, m), __shfl_xor(v.e, m)};
}

// Padded LDS index for 2^13-entry tiles: one spare slot every 32 entries
// keeps the transposed accesses of the alpha tile nearly free of bank
// conflicts.
__device__ inline uint32_t pad32(uint32_t x) { return x + (x >> 5); }

template <class P, int NR>
__device__ inline void reg_zeta_up(typename P::V *v, int q) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if ((r >> q) & 1) v[r] = P::add(v[r], v[r ^ (1 << q)]);
}

// Workgroup (i, H): the tile of node i's lattice (n-1 bits) whose high
// N-13 bits are H; tile entry x = the low 13 bits, 256 threads x 32 entries.
//  1. Seeds Z(G_L) = sum_{G_H subset H, |G_H| <= d-|G_L|} beta_i(G_H + G_L)
//     for every |G_L| <= d. The G_H are the small masks over H's bits (a
//     ranked table); their contribution to the rank of G_L + G_H is
//     tabulated once per workgroup, so a (seed, G_H) pair costs one LDS
//     read and one beta gather. Each seed is summed by a group of lanes and
//     reduced by cross-lane shuffles.
//  2. Upward zeta over the 13 tile bits in registers, in three layouts:
//     bits 0..4 (thread t holds x = ord8[t]*32 + r; ord8 lists the 8-bit
//     patterns by popcount, so the waves whose entries are all structural
//     zeros -- more than d ones above bit 4, Def. 1 -- skip it), bits 5..9
//     and bits 10..12 (x = r*256 + t), with two LDS transposes.
//  3. alpha = q(|S|) * t(S), stored coalesced from the last layout.
template <class P>
__device__ __forceinline__ void alpha_tile(int n, int d, uint32_t K, int use_prk, const Tables &tb,
                                           const typename P::V *__restrict__ beta,
                                           const typename P::V *__restrict__ qt,
                                           const typename P::Store &alpha,
                                           unsigned long long *cnt, uint32_t blk) {
    using V = typename P::V;
    constexpr int bA = 13, NR = 32;
    extern __shared__ unsigned char smem[];
    V *tile = reinterpret_cast<V *>(smem);                         // pad32(2^13)
    uint32_t *sbin = reinterpret_cast<uint32_t *>(tile + 8192 + 256);
    uint16_t *prk = reinterpret_cast<uint16_t *>(sbin + 33 * 33);  // (d+1) x items
    __shared__ int hb[32];
    __shared__ uint32_t offN[34];
    __shared__ V sq[32];
    __shared__ uint8_t ord8[256];
    const int N = n - 1;
    const int hA = N - bA;
    const int i = blk >> hA;
    const uint32_t H = blk & ((1u << hA) - 1);
    const int t = threadIdx.x;
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    if (t < hA && ((H >> t) & 1)) hb[__popc(H & ((1u << t) - 1))] = bA + t;
    if (t < n) sq[t] = qt[t];
    for (uint32_t x = t; x < 8192 + 256; x += kThreads) tile[x] = P::zero();
    __syncthreads();
    const uint32_t *bn = sbin;
    const int h = __popc(H);
    if (t <= d + 1) offN[t] = Kcount(bn, N, t - 1);
    {   // ord8: 8-bit patterns by popcount (then value)
        const int k = __popc(t);
        uint32_t r = Kcount(bn, 8, k - 1);
        int j = 0;
        for (int p = 0; p < 8; ++p)
            if ((t >> p) & 1) r += C(bn, p, ++j);
        ord8[r] = (uint8_t)t;
    }
    // partial ranks of the high-bit items: prk[s * nit + it] = sum_q C(hb[e_q], s + q)
    const uint32_t nit = Kcount(bn, h, d);
    for (uint32_t it = t; use_prk && it < nit; it += kThreads) {
        int k = 0;
        uint32_t off = 0, toff = 0;
        while (it >= off + C(bn, h, k)) {
            off += C(bn, h, k);
            toff += C(bn, hA, k);
            ++k;
        }
        const uint32_t m = tb.items[toff + (it - off)];
        for (int s = 0; s + k <= d; ++s) {
            uint32_t r = 0, mm = m;
            int q = 0;
            while (mm) {
                const int e = __ffs(mm) - 1;
                mm &= mm - 1;
                r += C(bn, hb[e], s + (++q));
            }
            prk[s * nit + it] = (uint16_t)r;
        }
    }
    __syncthreads();
    const V *bi = beta + (size_t)i * K;

    // 1. seeds, one size class s = |G_L| at a time
    for (int s = 0; s <= d && s <= bA; ++s) {
        const uint32_t nseed = C(bn, bA, s);
        const uint32_t items = Kcount(bn, h, d - s);    // G_H with |G_H| <= d - s
        int grp = 1;                                    // lanes per seed, power of 2 <= 64
        while (grp < 64 && (uint32_t)grp < items && (uint32_t)(grp * 2) * nseed <= kThreads)
            grp *= 2;
        const uint32_t per_round = kThreads / grp;
        const uint32_t seedoff = Kcount(bn, bA, s - 1);
        for (uint32_t base = 0; base < nseed; base += per_round) {
            const uint32_t seed = base + t / grp;
            const int lane = t % grp;
            V acc = P::zero();
            if (seed < nseed) {
                constexpr int B = 4;
                for (uint32_t it0 = lane; it0 < items; it0 += B * grp) {
                    V bv[B];
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        const uint32_t it = it0 + u * grp;
                        if (it < items) {
                            // size of item it: items are ordered by size
                            int k = 0;
                            uint32_t off = 1, toff = 0;
                            while (it >= off) {
                                toff += C(bn, hA, k);
                                off += C(bn, h, ++k);
                            }
                            uint32_t pr;
                            if (use_prk) {
                                pr = prk[s * nit + it];
                            } else {
                                uint32_t m = tb.items[toff + it - (off - C(bn, h, k))];
                                pr = 0;
                                int q = 0;
                                while (m) {
                                    const int e = __ffs(m) - 1;
                                    m &= m - 1;
                                    pr += C(bn, hb[e], s + (++q));
                                }
                            }
                            bv[u] = bi[offN[s + k] + seed + pr];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < B; ++u)
                        if (it0 + u * grp < items) acc = P::add(acc, bv[u]);
                }
            }
            for (int w = grp / 2; w > 0; w >>= 1) acc = P::add(acc, shfl_xor_v(acc, w));
            if (lane == 0 && seed < nseed) tile[pad32(tb.seedA[seedoff + seed])] = acc;
        }
    }
    __syncthreads();

    // 2. upward zeta in registers
    V v[NR];
    const uint32_t pt = ord8[t];
    const bool live = __popc(pt) <= d;    // bits 5..12 of every entry this thread holds
    if (__any(live)) {
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = tile[pad32((pt << 5) | r)];
#pragma unroll
        for (int q = 0; q < 5; ++q) reg_zeta_up<P, NR>(v, q);
#pragma unroll
        for (int r = 0; r < NR; ++r) tile[pad32((pt << 5) | r)] = v[r];
    }
    __syncthreads();
    const uint32_t tlo = t & 31, thi = t >> 5;   // layout B: x = thi*1024 + r*32 + tlo
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = tile[pad32((thi << 10) | (r << 5) | tlo)];
#pragma unroll
    for (int q = 0; q < 5; ++q) reg_zeta_up<P, NR>(v, q);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) tile[pad32((thi << 10) | (r << 5) | tlo)] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = tile[pad32(r * kThreads + t)];
#pragma unroll
    for (int q = 2; q < 5; ++q) reg_zeta_up<P, NR>(v, q);     // tile bits 10..12

    // 3. alpha = q(|S|) t(S)
    const uint64_t base = ((uint64_t)i << N) | ((uint64_t)H << bA);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const uint32_t x = r * kThreads + t;
        P::store(alpha, base + x, P::mul(sq[h + __popc(x)], v[r]), cnt);
    }
}

template <class P>
__global__ void __launch_bounds__(kThreads)
k_alpha(int n, int d, uint32_t K, int use_prk, Tables tb, const typename P::V *__restrict__ beta,
        const typename P::V *__restrict__ qt, typename P::Store alpha,
        unsigned long long *cnt) {
    alpha_tile<P>(n, d, K, use_prk, tb, beta, qt, alpha, cnt, blockIdx.x);
}

// Recomputation of the tiles listed by k_alpha_lin (list[0] entries,
// list[1 + j] = i * 2^(N-13) + H): the grid walks the list.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_alpha_fb(int n, int d, uint32_t K, int use_prk, Tables tb,
           const typename P::V *__restrict__ beta, const typename P::V *__restrict__ qt,
           typename P::Store alpha, unsigned long long *cnt, const uint32_t *list) {
    const uint32_t ntile = list[0];
    for (uint32_t it = blockIdx.x; it < ntile; it += gridDim.x) {
        __syncthreads();
        alpha_tile<P>(n, d, K, use_prk, tb, beta, qt, alpha, cnt, list[1 + it]);
    }
}

// A double held in LDS as two 32-bit words (4-byte alignment): it moves with
// 32-bit LDS instructions. The alpha tile's transposes run at about twice
// the speed this way than with 64-bit LDS instructions.
struct W2 {
    uint32_t lo, hi;
};
__device__ inline W2 w2_of(double x) {
    W2 w;
    __builtin_memcpy(&w, &x, 8);
    return w;
}
__device__ inline double dbl_of(W2 w) {
    double x;
    __builtin_memcpy(&x, &w, 8);
    return x;
}
// The same, as two separate planes of 32-bit words: every access is then a
// 32-bit LDS instruction on consecutive or 33-strided words, free of bank
// conflicts under the pad32 layout.
__device__ inline void put_w2(uint32_t *lo, uint32_t *hi, uint32_t ix, double x) {
    const W2 w = w2_of(x);
    lo[ix] = w.lo;
    hi[ix] = w.hi;
}
__device__ inline double get_w2(const uint32_t *lo, const uint32_t *hi, uint32_t ix) {
    return dbl_of(W2{lo[ix], hi[ix]});
}

__device__ inline void fb_push(uint32_t *fb, uint32_t id) {
    const uint32_t k = atomicAdd(fb, 1u);
    fb[1 + k] = id;
}

template <int NR>
__device__ inline void lin_zeta_up(double *v, int q) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if ((r >> q) & 1) v[r] += v[r ^ (1 << q)];
}

// Per-node scale for the linear alpha tiles. Every alpha_i(S) / q(|S|) is a
// sum of B_i(G) over G subset S that includes B_i(empty), and none exceeds
// K(n-1, d) max_G B_i(G). Node i therefore gets one power of two (a log
// offset for the log-space system) that puts B_i(empty) near 2^-1000, and
// the node is held in plain doubles when max_G B_i(G) / B_i(empty) is below
// 2^1900: no partial sum can then leave the double range (K(n-1, d) <
// 2^31). betal_i(r) = B_i(r) under that scale. Nodes that do not qualify
// (linok = 0) are computed in the number system proper.
// emax (nullable) receives floor(log2 max_G B_i(G)) + 1 per node (the bound
// the fused sweeps test their blocks against).
template <class P>
__global__ void k_prep_lin(int n, uint32_t K, const typename P::V *__restrict__ beta,
                           double *__restrict__ betal, typename P::Anchor *__restrict__ anc,
                           int *__restrict__ linok, int *__restrict__ emax) {
    using A = typename P::Anchor;
    __shared__ double red[kThreads];
    __shared__ int sok;
    __shared__ A sT;
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    const typename P::V *bi = beta + (size_t)i * K;
    double mx = -1e300;
    for (uint32_t r = t; r < K; r += kThreads) mx = fmax(mx, P::log2_of(bi[r]));
    mx = block_reduce(mx, red, [](double a, double b) { return fmax(a, b); });
    if (t == 0) {
        A T{};
        const bool ok = P::anchor_of(bi[0], &T) && mx - P::log2_of(bi[0]) <= 1900.0;
        sok = ok ? 1 : 0;
        sT = T;
        anc[i] = T;
        linok[i] = sok;
        if (emax) emax[i] = mx > -1e300 ? (int)mx + 1 : -(1 << 26);
    }
    __syncthreads();
    if (!sok) return;
    const A T = sT;
    for (uint32_t r = t; r < K; r += kThreads) betal[(size_t)i * K + r] = P::to_lin(bi[r], T);
}

// Binomial coefficient for small arguments; folds to a constant when its
// arguments are compile-time constants.
__host__ __device__ constexpr uint32_t cbin(int a, int b) {
    if (b < 0 || b > a) return 0;
    uint32_t r = 1;
    for (int k = 1; k <= b; ++k) r = r * (uint32_t)(a - b + k) / (uint32_t)k;
    return r;
}

// Colex rank of the set bits of a 5-bit mask (bit p is element p).
__host__ __device__ constexpr uint32_t colex5(uint32_t r) {
    uint32_t c = 0;
    int j = 0;
    for (int p = 0; p < 5; ++p)
        if ((r >> p) & 1) c += cbin(p, ++j);
    return c;
}

// Seeds of the linear alpha tiles, in a kernel of their own (the gather of
// k_alpha's first step, at high occupancy). For tile (i, H) and every G_L
// over the 13 tile bits with |G_L| < d,
//   Zs[(i, H)][rank(G_L)] = sum_{G_H subset H, |G_H| <= d - |G_L|} betal_i(G_H + G_L),
// rank = size, then colex order. A seed with |G_L| = d is betal_i(G_L)
// itself, the same for every H: k_alpha_lin reads those from betal. For one G_H the G_L of one size s give a
// contiguous run of ranks of G_H + G_L, so consecutive lanes take
// consecutive G_L (coalesced loads) and groups of lanes split the G_H;
// their partial sums meet in LDS in a fixed order.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_alpha_seeds(int n, int d, uint32_t K, uint32_t KS, int use_prk, Tables tb,
              const double *__restrict__ betal, const int *__restrict__ linok,
              double *__restrict__ Zs) {
    constexpr int bA = 13;
    extern __shared__ unsigned char smem[];
    uint32_t *sbin = reinterpret_cast<uint32_t *>(smem);
    uint16_t *prk = reinterpret_cast<uint16_t *>(sbin + 33 * 33);  // (d+1) x items
    __shared__ int hb[32];
    __shared__ uint32_t offN[34];
    __shared__ double part[kThreads];
    const int N = n - 1;
    const int hA = N - bA;
    const int i = blockIdx.x >> hA;
    const uint32_t H = blockIdx.x & ((1u << hA) - 1);
    const int t = threadIdx.x;
    if (!linok[i]) return;
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    if (t < hA && ((H >> t) & 1)) hb[__popc(H & ((1u << t) - 1))] = bA + t;
    __syncthreads();
    const uint32_t *bn = sbin;
    const int h = __popc(H);
    if (t <= d + 1) offN[t] = Kcount(bn, N, t - 1);
    const uint32_t nit = Kcount(bn, h, d);
    uint8_t *itk = reinterpret_cast<uint8_t *>(prk + (use_prk ? (size_t)(d + 1) * nit : 0));
    for (uint32_t it = t; use_prk && it < nit; it += kThreads) {
        int k = 0;
        uint32_t off = 0, toff = 0;
        while (it >= off + C(bn, h, k)) {
            off += C(bn, h, k);
            toff += C(bn, hA, k);
            ++k;
        }
        itk[it] = (uint8_t)k;
        const uint32_t m = tb.items[toff + (it - off)];
        for (int s = 0; s + k <= d; ++s) {
            uint32_t r = 0, mm = m;
            int q = 0;
            while (mm) {
                const int e = __ffs(mm) - 1;
                mm &= mm - 1;
                r += C(bn, hb[e], s + (++q));
            }
            prk[s * nit + it] = (uint16_t)r;
        }
    }
    __syncthreads();
    const double *bi = betal + (size_t)i * K;
    double *out = Zs + (size_t)blockIdx.x * KS;
    for (int s = 0; s < d && s <= bA; ++s) {
        const uint32_t nseed = C(bn, bA, s);
        const uint32_t items = Kcount(bn, h, d - s);
        const uint32_t seedoff = Kcount(bn, bA, s - 1);
        for (uint32_t base = 0; base < nseed; base += kThreads) {
            const uint32_t cnt = min(nseed - base, (uint32_t)kThreads);
            const uint32_t ni = kThreads / cnt;        // lanes per seed
            const uint32_t seed = base + t % cnt, il = t / cnt;
            double acc = 0.0;
            if (il < ni) {
                constexpr int B = 8;
                for (uint32_t it0 = il; it0 < items; it0 += B * ni) {
                    double bv[B];
#pragma unroll
                    for (int u = 0; u < B; ++u) {
                        const uint32_t it = it0 + u * ni;
                        bv[u] = 0.0;
                        if (it < items) {
                            int k;
                            uint32_t pr;
                            if (use_prk) {
                                k = itk[it];
                                pr = prk[s * nit + it];
                            } else {
                                k = 0;
                                uint32_t off = 1, toff = 0;
                                while (it >= off) {
                                    toff += C(bn, hA, k);
                                    off += C(bn, h, ++k);
                                }
                                uint32_t m = tb.items[toff + it - (off - C(bn, h, k))];
                                pr = 0;
                                int q = 0;
                                while (m) {
                                    const int e = __ffs(m) - 1;
                                    m &= m - 1;
                                    pr += C(bn, hb[e], s + (++q));
                                }
                            }
                            bv[u] = bi[offN[s + k] + seed + pr];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < B; ++u) acc += bv[u];
                }
            }
            if (ni == 1) {
                if (il == 0) out[seedoff + seed] = acc;
            } else {
                part[t] = acc;
                __syncthreads();
                if ((uint32_t)t < cnt) {
                    double z = 0.0;
                    for (uint32_t j = 0; j < ni; ++j) z += part[j * cnt + t];
                    out[seedoff + base + t] = z;
                }
                __syncthreads();
            }
        }
    }
}

// Store NR doubles of a thread (entry r at index base + r * stride, scaled
// by q(|r| + const), qr indexed by the popcount of r) in the solve's number
// system. The X32 form checks the exponent range once per thread and takes
// the per-entry saturation / flush path only when some entry needs it.
template <class P, int NR>
__device__ inline void store_tile_lin(const typename P::Store &st, uint64_t ubase,
                                      uint32_t toff, uint32_t stride, const double *v,
                                      const typename P::V *qr, typename P::Anchor T,
                                      unsigned long long *cnt) {
    uint32_t nsat = 0, nfl = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r)
        P::store_lin_q(st, ubase + (toff + (uint32_t)r * stride), v[r],
                       qr[__builtin_popcount(r)], T, nsat, nfl);
    if (cnt && (nsat | nfl)) {
        if (nsat) atomicAdd(cnt, (unsigned long long)nsat);
        if (nfl) atomicAdd(cnt + 1, (unsigned long long)nfl);
    }
}

template <int NR>
__device__ inline void store_tile_lin_x32(const PolX32::Store &st, uint64_t ubase,
                                          uint32_t toff, uint32_t stride, const double *v,
                                          const X32 *qr, int T, unsigned long long *cnt) {
    float *fp = st.f + ubase;           // uniform bases, 32-bit per-thread offsets
    uint8_t *bp = st.b + ubase;
    int b[NR];
    bool ok = true;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const X32 q = qr[__builtin_popcount(r)];
        const double z = v[r] * (double)q.f;
        int k;
        const float f = PolX32::lin_encode(z, &k);
        b[r] = ((T + q.e) >> 6) + k + kX32Bias;
        ok = ok && z > 0.0 && b[r] >= 1 && b[r] <= 255;
        fp[toff + (uint32_t)r * stride] = f;      // rewritten below if out of range
    }
    if (ok) {
#pragma unroll
        for (int r = 0; r < NR; ++r) bp[toff + (uint32_t)r * stride] = (uint8_t)b[r];
    } else {
        uint32_t nsat = 0, nfl = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
            PolX32::store_lin_q(st, ubase + (toff + (uint32_t)r * stride), v[r],
                                qr[__builtin_popcount(r)], T, nsat, nfl);
        if (cnt && (nsat | nfl)) {
            if (nsat) atomicAdd(cnt, (unsigned long long)nsat);
            if (nfl) atomicAdd(cnt + 1, (unsigned long long)nfl);
        }
    }
}

template <>
__device__ inline void store_tile_lin<PolX32, 16>(const PolX32::Store &st, uint64_t ubase,
                                                  uint32_t toff, uint32_t stride,
                                                  const double *v, const X32 *qr, int T,
                                                  unsigned long long *cnt) {
    store_tile_lin_x32<16>(st, ubase, toff, stride, v, qr, T, cnt);
}

// Padded LDS index for 2^12-entry halves: one spare word every 16.
__device__ inline uint32_t pad16(uint32_t x) { return x + (x >> 4); }

// Colex rank of the set bits of a 4-bit mask (bit p is element p).
__host__ __device__ constexpr uint32_t colex4(uint32_t r) {
    uint32_t c = 0;
    int j = 0;
    for (int p = 0; p < 4; ++p)
        if ((r >> p) & 1) c += cbin(p, ++j);
    return c;
}

__host__ __device__ constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Padded LDS index: one spare slot every 16 entries.
__device__ inline uint32_t padx(uint32_t x) { return x + (x >> 4); }

// Seeds of the linear alpha tiles by blocks of tiles (same outputs as
// k_alpha_seeds). Workgroup (i, Hh) covers the 2^b tiles H = Hh * 2^b + Hl
// (4 <= b <= 8 low bits of H). With G_H = G_lo + G_hi, G_lo over the
// b low bits of H and G_hi over the rest,
//   Z(H, G_L) = sum_{G_lo subset Hl} F(G_lo),
//   F(G_lo) = sum_{G_hi subset Hh, |G_hi| <= d - |G_L| - |G_lo|} betal_i(G_L + G_lo + G_hi),
// i.e. an upward zeta over the b low bits of a vector that is nonzero only
// where |G_L| + |G_lo| <= d. The seeds go in chunks of 16: thread (g, u) holds
// F for seed g and G_lo = u * 16 + r in 16 registers (bits 0..3), then, after
// an LDS transpose, bits 4..b-1. Score ranks are size, then colex: the part
// of G_hi (with the size offset) comes from a table built per workgroup,
// hiP[m][j] for the j-th subset of Hh and m smaller elements. Workgroup
// (i, Hh, y) takes every gridDim.y-th chunk from chunk y.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_alpha_seeds_blk(int n, int d, uint32_t K, uint32_t KS, int b, uint32_t nhiMax, Tables tb,
                  const double *__restrict__ betal, const int *__restrict__ linok,
                  double *__restrict__ Zs) {
    constexpr int bA = 13;
    extern __shared__ unsigned char smem[];
    double *buf = reinterpret_cast<double *>(smem);                   // 16 x 256, padx
    uint32_t *sbin = reinterpret_cast<uint32_t *>(buf + 4096 + 256);  // 33 x 33
    uint32_t *hiP = sbin + 33 * 33;                                   // (d + 1) x nhiMax
    __shared__ uint32_t hcnt[34];
    __shared__ int hpos[32];
    __shared__ int snh;
    const int N = n - 1, hA = N - bA, hh = hA - b;
    const int i = blockIdx.x >> hh;
    const uint32_t Hh = blockIdx.x & ((1u << hh) - 1);
    const int t = threadIdx.x;
    if (!linok[i]) return;
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    if (t == 0) {
        int c = 0;
        for (int p = 0; p < hh; ++p)
            if ((Hh >> p) & 1) hpos[c++] = bA + b + p;   // mask positions of Hh's elements
        snh = c;
    }
    __syncthreads();
    const uint32_t *bn = sbin;
    const int nh = snh;
    const uint32_t nhi = Kcount(bn, nh, d);
    if (t <= d) hcnt[t] = Kcount(bn, nh, t);         // subsets of Hh with at most t elements
    for (uint32_t j = t; j < nhi; j += kThreads) {
        int k = 0;
        uint32_t off = 0;
        while (j >= off + C(bn, nh, k)) off += C(bn, nh, k++);
        int el[8];
        colex_unrank(bn, j - off, k, el);
        for (int m = 0; m <= d; ++m) {
            uint32_t r = (m + k >= 1) ? Kcount(bn, N, m + k - 1) : 0u;
            for (int q = 0; q < k; ++q) r += C(bn, hpos[el[q]], m + q + 1);
            hiP[m * nhiMax + j] = r;
        }
    }
    __syncthreads();
    const double *bi = betal + (size_t)i * K;
    const uint32_t g = t >> 4, u = t & 15;
    const uint32_t nu = 1u << (b - 4);                 // thread values of G_lo bits 4..b-1
    const uint64_t tile0 = (uint64_t)blockIdx.x << b;  // tile index (i, Hh, Hl = 0)
    const uint32_t nent = 16u << b;
    // chunks of 16 seed ranks, split over gridDim.y workgroups of the same tiles
    for (uint32_t c0 = 16 * blockIdx.y; c0 < KS; c0 += 16 * gridDim.y) {
        const uint32_t rk = c0 + g;
        double v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = 0.0;
        if (rk < KS && u < nu) {
            const uint32_t GL = tb.seedA[rk];
            const int s = __popc(GL);
            const uint32_t cl = rk - Kcount(bn, bA, s - 1);   // colex rank of G_L
            for (int r = 0; r < 16; ++r) {
                const uint32_t Glo = (u << 4) | (uint32_t)r;
                const int m = s + __popc(Glo);
                if (m > d) continue;
                uint32_t lp = cl;
                int q = s;
                uint32_t rest = Glo;
                while (rest) {
                    const int p = __ffs(rest) - 1;
                    rest &= rest - 1;
                    lp += C(bn, bA + p, ++q);
                }
                const uint32_t *hp = hiP + m * nhiMax;
                const uint32_t nsub = hcnt[d - m];
                double acc = 0.0;
                for (uint32_t jj = 0; jj < nsub; ++jj) acc += bi[lp + hp[jj]];
                v[r] = acc;
            }
        }
        // upward zeta over G_lo bits 0..3
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if ((r >> q) & 1) v[r] += v[r ^ (1 << q)];
        if (u < nu) {
#pragma unroll
            for (int r = 0; r < 16; ++r) buf[padx((g << 8) | (u << 4) | (uint32_t)r)] = v[r];
        }
        __syncthreads();
        // thread (g, u = G_lo bits 0..3), registers r = G_lo bits 4..b-1
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = ((uint32_t)r < nu) ? buf[padx((g << 8) | ((uint32_t)r << 4) | u)] : 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < b - 4) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    if ((r >> q) & 1) v[r] += v[r ^ (1 << q)];
            }
        }
        __syncthreads();
        // tile-major for the stores: entry (Hl, g) at Hl * 16 + g
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if ((uint32_t)r < nu) buf[padx((((uint32_t)r << 4) | u) * 16 + g)] = v[r];
        __syncthreads();
        for (uint32_t e = t; e < nent; e += kThreads) {
            const uint32_t Hl = e >> 4, gg = e & 15;
            if (c0 + gg < KS) Zs[(tile0 | Hl) * KS + c0 + gg] = buf[padx(e)];
        }
        __syncthreads();
    }
}

// One 12-bit half of a linear alpha tile (see k_alpha_lin).
template <class P, int hb>
__device__ __forceinline__ void alpha_lin_half(int d, const double *__restrict__ zs,
                                               const double *__restrict__ zd,
                                               const typename P::V *sq, const uint16_t *ctab,
                                               const uint16_t *cb,
                                               const uint32_t *k13, uint32_t *tlo_,
                                               uint32_t *thi_, uint32_t pt, int h,
                                               uint64_t base, typename P::Anchor T,
                                               typename P::Store alpha,
                                               unsigned long long *cnt) {
    using V = typename P::V;
    constexpr int NR = 16;
    const int t = threadIdx.x;
    const int kp = __popc(pt);
    const uint32_t tlo = t & 15, thi = t >> 4;
    const int kh = __popc(thi);
    // pad16 indices written as a lane base plus a constant per register, so
    // that the constants fold into the LDS offsets:
    //   A: pad16(pt * 16 + r) = 17 pt + r,
    //   B: pad16(thi * 256 + r * 16 + tlo) = 272 thi + tlo + 17 r,
    //   C: pad16(r * 256 + t) = t + t / 16 + 272 r
    const uint32_t ib = thi * 272 + tlo, ic = t + (t >> 4);
    double v[NR];
    // ---- layout A: y = pt * 16 + r, tile bits 0..3. The upper half starts
    //      from its own seeds plus the lower half's (the zeta step over
    //      tile bit 12 commutes with the others).
    if (__any(kp <= d)) {
        // colex terms of pt's bits (tile bits 4..11) with m ones below them,
        // and of bit 12 on top for the upper half's second seed
        uint32_t off[5], offu[5], cpt[5], cup[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            off[m] = k13[min(kp + m, 14)];
            offu[m] = k13[min(kp + m + 1, 14)];
            cpt[m] = ctab[m * 256 + pt];
            cup[m] = cpt[m] + cb[12 * 14 + min(kp + m + 1, 13)];
        }
        // every load is issued (clamped to a valid index of zd) before any is
        // used; seeds of size d come from zd, smaller ones from zs
        double u[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int m = __builtin_popcount(r);
            const uint32_t il = (kp + m <= d) ? off[m] + colex4(r) + cpt[m] : 0u;
            const uint32_t iu = (hb && kp + m + 1 <= d) ? offu[m] + colex4(r) + cup[m] : 0u;
            v[r] = (kp + m < d ? zs : zd)[il];
            u[r] = (kp + m + 1 < d ? zs : zd)[iu];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int m = __builtin_popcount(r);
            const double lo = (kp + m <= d) ? v[r] : 0.0;
            const double up = (hb && kp + m + 1 <= d) ? u[r] : 0.0;
            v[r] = lo + up;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) lin_zeta_up<NR>(v, q);
        if (kp <= d) {
#pragma unroll
            for (int r = 0; r < NR; ++r) put_w2(tlo_, thi_, pt * 17 + r, v[r]);
        }
    }
    __syncthreads();
    // ---- layout B: y = thi * 256 + r * 16 + tlo, tile bits 4..7
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = get_w2(tlo_, thi_, ib + r * 17);
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (kh + __builtin_popcount(r) > d) v[r] = 0.0;      // slot never written
#pragma unroll
    for (int q = 0; q < 4; ++q) lin_zeta_up<NR>(v, q);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) put_w2(tlo_, thi_, ib + r * 17, v[r]);
    __syncthreads();
    // ---- layout C: y = r * 256 + t, tile bits 8..11
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = get_w2(tlo_, thi_, ic + r * 272);
#pragma unroll
    for (int q = 0; q < 4; ++q) lin_zeta_up<NR>(v, q);
    // ---- alpha = q(|S|) t(S), |S| = h + hb + |t| + |r|
    V qr[5];
    const int ht = h + hb + __popc(t);
#pragma unroll
    for (int m = 0; m < 5; ++m) qr[m] = sq[min(ht + m, 31)];
    if constexpr (std::is_same<P, PolX32>::value) {
        // Significands go out from layout C (256 B per wave store); the
        // exponent bytes are transposed through LDS so that each thread
        // stores 16 consecutive bytes (1 KB per wave store): byte stores of
        // 64 B per wave would cost partial-line reads and writes in L2.
        const uint64_t ub = base + hb * 4096;
        float *fp = alpha.f + ub;
        uint8_t *bytes = reinterpret_cast<uint8_t *>(tlo_);
        uint32_t nsat = 0, nfl = 0, bq[NR];
        double qf[5];
        int qb[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            qf[m] = (double)qr[m].f;
            qb[m] = ((T + qr[m].e) >> 6) + kX32Bias;
        }
        // fast path: every entry positive with its byte in 1..255
        float fq[NR];
        bool ok = true;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int m = __builtin_popcount(r);
            const double z = v[r] * qf[m];
            int k;
            fq[r] = PolX32::lin_encode(z, &k);
            bq[r] = (uint32_t)(qb[m] + k);
            ok = ok && z > 0.0 && bq[r] - 1u < 255u;
        }
        if (!ok) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double z = v[r] * qf[__builtin_popcount(r)];
                const int b = (int)bq[r];
                const bool zero = !(z > 0.0);
                const bool fl = !zero && b < 1;
                const bool sat = !zero && b > 255;
                nfl += fl ? 1u : 0u;
                nsat += sat ? 1u : 0u;
                fq[r] = (zero || fl) ? 0.0f : (sat ? 4.0e9f : fq[r]);
                bq[r] = (zero || fl) ? 0u : (sat ? 255u : (uint32_t)b);
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) fp[(uint32_t)(r * kThreads + t)] = fq[r];
        __syncthreads();                      // every layout-C read of the planes is done
#pragma unroll
        for (int r = 0; r < NR; ++r) bytes[r * kThreads + t] = (uint8_t)bq[r];
        __syncthreads();
        reinterpret_cast<uint4 *>(alpha.b + ub)[t] = reinterpret_cast<const uint4 *>(bytes)[t];
        if (cnt && (nsat | nfl)) {
            if (nsat) atomicAdd(cnt, (unsigned long long)nsat);
            if (nfl) atomicAdd(cnt + 1, (unsigned long long)nfl);
        }
    } else {
        store_tile_lin<P, NR>(alpha, base + hb * 4096, t, kThreads, v, qr, T, cnt);
    }
    __syncthreads();
}

// Linear-tile form of k_alpha. A workgroup takes 2^tl consecutive tiles (i, H)
// of one node in turn, each the same 13-bit tile as k_alpha's, run
// as two 12-bit halves x = hb * 4096 + y through one half-size LDS buffer,
// which lets four workgroups share a CU. The zeta step over tile bit 12 is
// taken first: the upper half starts from its seeds plus the lower half's.
// The seeds come from k_alpha_seeds, already as
// doubles under the node's scale (k_prep_lin), and the upward zeta runs on
// doubles, one FP64 add per step, in three layouts of a half (256 threads x
// 16 entries): A, y = pattern * 16 + r (bits 0..3 in registers; patterns of
// bits 4..11 by popcount, so waves holding only structural zeros skip it),
// seeds read straight from Zs; B, y = thi * 256 + r * 16 + tlo (bits 4..7),
// which skips slots that still hold structural zeros, so the LDS buffer never
// needs clearing; C, y = r * 256 + t (bits 8..11), stored from there. Tiles
// of nodes without a linear scale go to the fallback list for k_alpha_fb;
// force_fb sends every tile there (tests).
// Four workgroups per CU (LDS allows it): registers are capped to match.
template <class P>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_alpha_lin(int n, int d, uint32_t KS, int force_fb, int tl, const double *__restrict__ Zs,
            const double *__restrict__ betal, uint32_t K, uint32_t offd,
            const typename P::Anchor *__restrict__ anc, const int *__restrict__ linok,
            const typename P::V *__restrict__ qt, typename P::Store alpha,
            unsigned long long *cnt, uint32_t *fb) {
    using V = typename P::V;
    using A = typename P::Anchor;
    constexpr int bA = 13, NR = 16;
    extern __shared__ unsigned char smem[];
    // a half's doubles as two planes of 32-bit words (pad16 indices)
    uint32_t *tlo_ = reinterpret_cast<uint32_t *>(smem);
    uint32_t *thi_ = tlo_ + 4096 + 256;
    __shared__ V sq[32];
    __shared__ uint8_t ord8[256];
    __shared__ uint16_t cb[14 * 14];      // C(a, b), a, b <= 13
    __shared__ uint32_t k13[15];          // K(13, k - 1) = sum_{j < k} C(13, j)
    // ctab[m * 256 + p]: colex terms of the 8-bit pattern p at tile bits
    // 4..11 with m ones below it (kept in LDS rather than in registers
    // across the tile loop)
    __shared__ uint16_t ctab[5 * 256];
    const int N = n - 1;
    const int hA = N - bA;
    const uint32_t tile0 = blockIdx.x << tl;   // 2^tl consecutive tiles of one node
    const int i = tile0 >> hA;
    const int t = threadIdx.x;
    if (force_fb || !linok[i]) {
        if (t < (1 << tl)) fb_push(fb, tile0 + t);
        return;
    }
    const A T = anc[i];
    if (t < n) sq[t] = qt[t];
    if (t < 14 * 14) cb[t] = (uint16_t)cbin(t / 14, t % 14);
    if (t < 15) {
        uint32_t o = 0;
        for (int j = 0; j < t; ++j) o += cbin(13, j);
        k13[t] = o;
    }
    __syncthreads();
    {   // ord8: 8-bit patterns by popcount (then value)
        const int k = __popc(t);
        uint32_t r = 0;
        for (int j = 0; j < k; ++j) r += cb[8 * 14 + j];
        int j = 0;
        for (int p = 0; p < 8; ++p)
            if ((t >> p) & 1) r += cb[p * 14 + (++j)];
        ord8[r] = (uint8_t)t;
    }
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        uint32_t c = 0;
        int j = m;
        for (int p = 0; p < 8; ++p)
            if ((t >> p) & 1) c += cb[(4 + p) * 14 + (++j)];
        ctab[m * 256 + t] = (uint16_t)c;
    }
    __syncthreads();
    // size-d seeds: betal_i(G_L) at rank offd + colex(G_L), offd = K(N, d - 1);
    // indexed like zs (k13[d] + colex), so the base is shifted by k13[d]
    const double *zd = betal + (size_t)i * K + offd - k13[min(d, 14)];
    const uint32_t pt = ord8[t];
    for (int j = 0; j < (1 << tl); ++j) {
        const uint32_t tile = tile0 + j;
        const uint32_t H = tile & ((1u << hA) - 1);
        const int h = __popc(H);
        const double *zs = Zs + (size_t)tile * KS;
        const uint64_t base = ((uint64_t)i << N) | ((uint64_t)H << bA);
        alpha_lin_half<P, 0>(d, zs, zd, sq, ctab, cb, k13, tlo_, thi_, pt, h, base, T, alpha, cnt);
        alpha_lin_half<P, 1>(d, zs, zd, sq, ctab, cb, k13, tlo_, thi_, pt, h, base, T, alpha, cnt);
    }
}

// Generic form for lattices smaller than the 13-bit tile (n - 1 < 13): one
// tile of bA = n - 1 bits, seeds as above, truncated zeta in LDS.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_alpha_small(int n, int d, uint32_t K, Tables tb, const typename P::V *__restrict__ beta,
              const typename P::V *__restrict__ qt, typename P::Store alpha,
              unsigned long long *cnt) {
    using V = typename P::V;
    extern __shared__ unsigned char smem[];
    V *tile = reinterpret_cast<V *>(smem);
    __shared__ V sq[32];
    const int N = n - 1;
    const int bA = N;
    const int i = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t *bn = tb.binom;
    if (t < n) sq[t] = qt[t];
    const V *bi = beta + (size_t)i * K;
    // with no high bits every seed is a single family: Z(G) = beta_i(G)
    for (uint32_t x = t; x < (1u << bA); x += kThreads) tile[x] = P::zero();
    __syncthreads();
    for (uint32_t r = t; r < K; r += kThreads) tile[tb.famask[r]] = bi[r];
    __syncthreads();
    for (int j = 0; j < bA; ++j) {
        const uint32_t cntj = Kcount(bn, bA - 1 - j, d) << j;
        for (uint32_t idx = t; idx < cntj; idx += kThreads) {
            const uint32_t lo = idx & ((1u << j) - 1);
            const uint32_t S = ((uint32_t)tb.pat[idx >> j] << (j + 1)) | (1u << j) | lo;
            tile[S] = P::add(tile[S], tile[S ^ (1u << j)]);
        }
        __syncthreads();
    }
    const uint64_t base = (uint64_t)i << N;
    for (uint32_t x = t; x < (1u << bA); x += kThreads)
        P::store(alpha, base + x, P::mul(sq[__popc(x)], tile[x]), cnt);
}

// ------------------------------------------- a3/a4: sweep helpers
// In-tile alpha slices in LDS. The FP32-scaled form keeps the stored form,
// a plane of significands and a plane of exponent bytes (5 bytes per entry,
// so more workgroups share a CU); the log form keeps the values.
template <class P>
struct SliceLds {
    typename P::V *v;
    __device__ SliceLds(void *base, uint32_t) : v(reinterpret_cast<typename P::V *>(base)) {}
    __device__ typename P::V at(uint32_t k) const { return v[k]; }
    __device__ void put4(uint32_t e, const typename P::Raw4 &r) { P::decode4_nz(r, v + e); }
    __device__ void put(uint32_t e, const typename P::Store &s, uint64_t i) { v[e] = P::load(s, i); }
    static constexpr size_t bytes_per_entry = sizeof(typename P::V);
};
template <>
struct SliceLds<PolX32> {
    float *f;
    uint8_t *b;
    __device__ SliceLds(void *base, uint32_t total)
        : f(reinterpret_cast<float *>(base)), b(reinterpret_cast<uint8_t *>(f + total)) {}
    // factor of a product only: a stored zero has significand 0
    __device__ X32 at(uint32_t k) const { return X32{f[k], ((int)b[k] - kX32Bias) << 6}; }
    __device__ void put4(uint32_t e, const PolX32::Raw4 &r) {
        *reinterpret_cast<float4 *>(f + e) = r.f;
        *reinterpret_cast<uint32_t *>(b + e) = r.b;
    }
    __device__ void put(uint32_t e, const PolX32::Store &s, uint64_t i) {
        f[e] = s.f[i];
        b[e] = s.b[i];
    }
    static constexpr size_t bytes_per_entry = 5;
};

// Stage alpha_i(Hf + Lo') (Lo' without bit i) for the bL tile bits into LDS:
// slice i is the contiguous block alpha_i[(Hf >> 1) + k], k < 2^(bL-1).
// All loads of a thread are issued before any is stored.
template <class P>
__device__ inline void stage_alpha(const typename P::Store &alpha, uint64_t NN, uint64_t Hf,
                                   int bL, SliceLds<P> &la) {
    const uint32_t half = 1u << (bL - 1);
    const uint32_t total = (uint32_t)bL * half;
    const int t = threadIdx.x;
    if (half >= 4) {
        constexpr int U = 5;                  // batches of 4 entries in flight per thread
        for (uint32_t e0 = 4 * t; e0 < total; e0 += 4 * kThreads * U) {
            typename P::Raw4 raw[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t e = e0 + 4 * kThreads * u;
                if (e < total)
                    raw[u] = P::load4_raw(alpha, (uint64_t)(e >> (bL - 1)) * NN + (Hf >> 1) +
                                                     (e & (half - 1)));
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t e = e0 + 4 * kThreads * u;
                if (e < total) la.put4(e, raw[u]);   // product factors only
            }
        }
    } else {
        for (uint32_t e = t; e < total; e += kThreads)
            la.put(e, alpha, (uint64_t)(e >> (bL - 1)) * NN + (Hf >> 1) + (e & (half - 1)));
    }
}

// acc[k] += sum over the listed nodes i of alpha_i[ai(i) + k] * X[xi(i) + k], k < 4,
// four nodes per batch of loads.
template <class P, class AI, class XI>
__device__ inline void cross_terms(const typename P::Store &alpha, const typename P::Store &X,
                                   const int *nodes, int cnt, AI ai, XI xi,
                                   typename P::Acc *acc) {
    using V = typename P::V;
    constexpr int B = 4;
    for (int q0 = 0; q0 < cnt; q0 += B) {
        typename P::Raw4 ra[B], rx[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (q0 + u < cnt) {
                const int i = nodes[q0 + u];
                ra[u] = P::load4_raw(alpha, ai(i));
                rx[u] = P::load4_raw(X, xi(i));
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            if (q0 + u < cnt) {
                V a[4], x[4];
                P::decode4_nz(ra[u], a);
                P::decode4_nz(rx[u], x);
#pragma unroll
                for (int k = 0; k < 4; ++k) P::acc_add(acc[k], P::mul_raw(a[k], x[k]));
            }
        }
    }
}

// ------------------------------------------- a3: forward sweep, one layer
// Workgroup = tile H with |H| = h (H over the n-bL high bits), in colex
// order: consecutive workgroups, which run at the same time on the eight
// XCDs, take tiles that share most of their L blocks (a mapping that gave
// each XCD a contiguous eighth of the layer cut the L2 misses by 10% but
// measured 5% slower). Cross-tile terms (i in H) stream contiguous 2^bL blocks of alpha_i and L, four
// consecutive entries per thread; in-tile terms (i among the low bits) use
// the tile's alpha slices staged in LDS and run popcount layer by popcount
// layer. Requires bL >= 2.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_fwd(int n, int bL, int h, uint32_t hoff, Tables tb, typename P::Store alpha,
      typename P::Store L, unsigned long long *cnt) {
    using V = typename P::V;
    extern __shared__ unsigned char smem[];
    const uint32_t half = 1u << (bL - 1);
    const uint32_t T = 1u << bL;
    SliceLds<P> la(smem, (uint32_t)bL * half);   // bL * half entries
    V *lt = reinterpret_cast<V *>(smem + align16(SliceLds<P>::bytes_per_entry * bL * half));
    uint16_t *lord = reinterpret_cast<uint16_t *>(lt + T);
    __shared__ uint32_t loff[34];
    __shared__ int pos[32];
    const int t = threadIdx.x;
    const uint64_t NN = 1ull << (n - 1);
    if (t == 0) {
        uint32_t Hm = tb.hord[hoff + blockIdx.x];   // H over the high bits
        for (int q = 0; q < h; ++q) {
            pos[q] = bL + __ffs(Hm) - 1;            // node indices of H
            Hm &= Hm - 1;
        }
    }
    if (t < bL + 2) loff[t] = tb.loff[t];
    for (uint32_t x = t; x < T; x += kThreads) lord[x] = tb.lorder[x];
    __syncthreads();
    uint64_t Hf = 0;
    for (int q = 0; q < h; ++q) Hf |= 1ull << pos[q];
    stage_alpha<P>(alpha, NN, Hf, bL, la);
    // cross-tile terms: alpha_i(S - i) L(S - i) for i in H
    for (uint32_t lo = 4 * t; lo < T; lo += 4 * kThreads) {
        typename P::Acc acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = P::acc_of((Hf == 0 && lo + k == 0) ? P::one() : P::zero());
        cross_terms<P>(alpha, L, pos, h,
                       [&](int i) { return (uint64_t)i * NN + compress_bit((Hf ^ (1ull << i)) | lo, i); },
                       [&](int i) { return (Hf ^ (1ull << i)) | lo; }, acc);
#pragma unroll
        for (int k = 0; k < 4; ++k) lt[lo + k] = P::norm_v(P::acc_value(acc[k]));
    }
    __syncthreads();
    for (int l = 1; l <= bL; ++l) {
        for (uint32_t idx = loff[l] + t; idx < loff[l + 1]; idx += kThreads) {
            const uint32_t lo = lord[idx];
            typename P::Acc acc = P::acc_of(lt[lo]);
            uint32_t rest = lo;
            while (rest) {
                const int i = __ffs(rest) - 1;
                rest &= rest - 1;
                const uint32_t Tm = lo ^ (1u << i);
                P::acc_add(acc, P::mul_raw(la.at(i * half + (uint32_t)compress_bit(Tm, i)), lt[Tm]));
            }
            lt[lo] = P::norm_v(P::acc_value(acc));
        }
        __syncthreads();
    }
    for (uint32_t lo = 4 * t; lo < T; lo += 4 * kThreads) P::store4(L, Hf | lo, lt + lo, cnt);
}

// ----------------------------------------- a4: backward sweep, one layer
// Rp(S) = sum_{i not in S} alpha_i(S) Rp(S + i), Rp(V) = 1; layers run from
// the top. Same tiling as the forward sweep, mirrored. Requires bL >= 2.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_bwd(int n, int bL, int h, uint32_t hoff, Tables tb, typename P::Store alpha,
      typename P::Store R, unsigned long long *cnt) {
    using V = typename P::V;
    extern __shared__ unsigned char smem[];
    const uint32_t half = 1u << (bL - 1);
    const uint32_t T = 1u << bL;
    SliceLds<P> la(smem, (uint32_t)bL * half);
    V *lt = reinterpret_cast<V *>(smem + align16(SliceLds<P>::bytes_per_entry * bL * half));
    uint16_t *lord = reinterpret_cast<uint16_t *>(lt + T);
    __shared__ uint32_t loff[34];
    __shared__ int pos[32];
    __shared__ int outs[32];
    __shared__ int nout_s;
    const int t = threadIdx.x;
    const int nh = n - bL;
    const uint64_t NN = 1ull << (n - 1);
    if (t == 0) {
        const uint32_t Hm = tb.hord[hoff + blockIdx.x];   // H over the high bits
        uint32_t rest = Hm;
        for (int q = 0; q < h; ++q) {
            pos[q] = __ffs(rest) - 1;
            rest &= rest - 1;
        }
        int no = 0;
        for (int p = 0; p < nh; ++p)
            if (!((Hm >> p) & 1)) outs[no++] = bL + p;   // nodes above the tile, not in H
        nout_s = no;
    }
    if (t < bL + 2) loff[t] = tb.loff[t];
    for (uint32_t x = t; x < T; x += kThreads) lord[x] = tb.lorder[x];
    __syncthreads();
    uint64_t Hf = 0;
    for (int q = 0; q < h; ++q) Hf |= 1ull << (bL + pos[q]);
    const int nout = nout_s;
    const uint64_t highall = ((1ull << nh) - 1) << bL;
    stage_alpha<P>(alpha, NN, Hf, bL, la);
    for (uint32_t lo = 4 * t; lo < T; lo += 4 * kThreads) {
        typename P::Acc acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[k] = P::acc_of((Hf == highall && lo + k == T - 1) ? P::one() : P::zero());
        const uint64_t Sm = Hf | lo;
        cross_terms<P>(alpha, R, outs, nout,
                       [&](int i) { return (uint64_t)i * NN + compress_bit(Sm, i); },
                       [&](int i) { return Sm | (1ull << i); }, acc);
#pragma unroll
        for (int k = 0; k < 4; ++k) lt[lo + k] = P::norm_v(P::acc_value(acc[k]));
    }
    __syncthreads();
    for (int l = bL - 1; l >= 0; --l) {
        for (uint32_t idx = loff[l] + t; idx < loff[l + 1]; idx += kThreads) {
            const uint32_t lo = lord[idx];
            typename P::Acc acc = P::acc_of(lt[lo]);
            uint32_t rest = (T - 1) & ~lo;
            while (rest) {
                const int i = __ffs(rest) - 1;
                rest &= rest - 1;
                P::acc_add(acc, P::mul_raw(la.at(i * half + (uint32_t)compress_bit(lo, i)),
                                           lt[lo | (1u << i)]));
            }
            lt[lo] = P::norm_v(P::acc_value(acc));
        }
        __syncthreads();
    }
    for (uint32_t lo = 4 * t; lo < T; lo += 4 * kThreads) P::store4(R, Hf | lo, lt + lo, cnt);
}

// ---------------------------------------- a5 + a6: Gamma, in-tile part
// Layout of Y1_v (K(bv, d) ranks x 2^hv values of Hc). The ranks below
// kg4 (K(bv, d) rounded down to a multiple of 4) sit in groups of four: group
// j holds, for every Hc, the values of ranks 4j .. 4j + 3 side by side. A
// Gamma tile workgroup writes one Hc of every rank, so its stores leave as
// 32-byte runs instead of single 8-byte values. The ranks from kg4 on follow
// as plain rows of 2^hv values.
__device__ __forceinline__ size_t y1_at(uint32_t rank, uint64_t Hc, int hv, uint32_t kg4) {
    return rank < kg4 ? ((((size_t)rank >> 2) << (hv + 2)) | ((size_t)Hc << 2) | (rank & 3u))
                      : (((size_t)rank << hv) + Hc);
}
// distance between the entries of consecutive Hc of one rank
__device__ __forceinline__ uint32_t y1_stride(uint32_t rank, uint32_t kg4) {
    return rank < kg4 ? 4u : 1u;
}
// Workgroup order of the kernels that read Y1 rows: a workgroup's index
// within endpoint v, local (rank-major: s * 2^hB + Ht), becomes the
// (rank, Ht) item it takes, such that the four ranks of a group (same Ht)
// run 8 workgroups apart, on one XCD, where its L2 serves the group's
// 32-byte runs to all four. A bijection on [0, K(bv, d) 2^hB): whole octets
// of (group, Ht) pairs first, then the rest of the grouped ranks with the
// four ranks side by side, then the plain rows unchanged.
__device__ __forceinline__ uint32_t y1_reader_item(uint32_t local, int hB, uint32_t kg4) {
    const uint32_t G = (kg4 >> 2) << hB;        // (group, Ht) pairs
    const uint32_t full = (G >> 3) << 5;        // locals of whole octets
    if (local >= 4 * G) return local;
    uint32_t gH, q;
    if (local < full) {
        q = (local >> 3) & 3u;
        gH = ((local >> 5) << 3) | (local & 7u);
    } else {
        const uint32_t x = local - full;
        q = x & 3u;
        gH = ((G >> 3) << 3) + (x >> 2);
    }
    return ((((gH >> hB) << 2) | q) << hB) | (gH & ((1u << hB) - 1u));
}

// In-register downward zeta step over register bit q of NR = 2^RB entries,
// skipped when that register bit carries the endpoint itself.
template <class P, int NR>
__device__ inline void reg_zeta_down(typename P::V *g, int q) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!((r >> q) & 1)) g[r] = P::add(g[r], g[r | (1 << q)]);
}

// Padded LDS index: one spare slot every 16 entries keeps the transposed
// reads of the Gamma tile free of heavy bank conflicts.

// Workgroup = full-mask tile H of 2^12 masks (the low 12 bits vary), 256
// threads x 16 entries. L(H + x) and Rp(H + x) stay in registers for the
// whole workgroup; every endpoint v not in H is served in turn:
//   g_v(S) = q(|S|) L(S) Rp(S + v) for S = H + x. For v a tile bit, x runs
//   over the entries without bit v and Rp(S + v) is the partner entry (same
//   thread for a register bit, else read through LDS). For v above the tile
//   Rp(S + v) is the tile H + v, prefetched while the previous endpoint is
//   reduced. Products are left unnormalised (add() aligns exactly).
//   Downward zeta over the tile bits other than v, entirely in registers:
//   layout A holds tile bits 8..11 in the register index (x = r*256 + t),
//   layout B bits 4..7 (x = t_hi*256 + r*16 + t_lo), layout C bits 0..3
//   (x = t*16 + r); two LDS transposes move between them.
//   The entries with at most d ones (Def. 2: Gamma_v(G) is needed for
//   |G| <= d only) go from registers to Y1_v[seed][Hc_v].
template <class P>
__device__ __forceinline__ void gamma_tile(int n, int d, const GammaGeom &gg, const Tables &tb,
                                           const typename P::Store &L,
                                           const typename P::Store &R,
                                           const typename P::V *__restrict__ qt,
                                           typename P::V *__restrict__ Y1,
                                           typename P::V *__restrict__ part, uint32_t H,
                                           int only_v = -1) {
    using V = typename P::V;
    using Raw = typename P::Raw;
    constexpr int bT = 12, NR = 16;
    extern __shared__ unsigned char smem[];
    V *gb = reinterpret_cast<V *>(smem);                       // padded 2^12 entries
    uint32_t *sbin = reinterpret_cast<uint32_t *>(gb + 4096 + 256);
    uint32_t *seedT = sbin + 33 * 33;                          // K(12, d) ranked masks
    __shared__ V sq[32];
    __shared__ uint32_t offT[34], offT1[34];
    const int t = threadIdx.x;
    const uint64_t Hf = (uint64_t)H << bT;
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    for (uint32_t x = t; x < gg.KT; x += kThreads) seedT[x] = tb.seedmask[x];
    if (t < n) sq[t] = qt[t];
    V Lr[NR], Rr[NR], g[NR];
    Raw Rv[NR];                               // next endpoint's Rp tile, undecoded
    const int hpc = __popcll(Hf);
    {
        Raw l0[NR], r0[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t x = r * kThreads + t;
            l0[r] = P::load_raw(L, Hf | x);
            r0[r] = P::load_raw(R, Hf | x);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            Lr[r] = P::decode_raw(l0[r]);
            Rr[r] = P::decode_raw(r0[r]);
        }
    }
    // next endpoint above the tile, not in H (only_v itself when it is one)
    int vn = only_v >= bT ? only_v : bT;
    while (vn < n && ((Hf >> vn) & 1)) ++vn;
    if (vn < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r) Rv[r] = P::load_raw(R, Hf | (r * kThreads + t) | (1ull << vn));
    }
    {   // invariant partials: sum of L(S) Rp(S) over the tile, per |x| (x = r*256 + t)
        V lr[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) lr[k] = P::zero();
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const V prod = P::mul(Lr[r], Rr[r]);
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (__popc(r) == k) lr[k] = P::add(lr[k], prod);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) gb[t * 5 + k] = lr[k];
        __syncthreads();
        {   // layer l = t / 16 of the tile: 16 lanes x 16 slots, then a lane tree
            const int l = t >> 4, j = t & 15;
            V acc = P::zero();
            if (l <= bT) {
                for (int u = j; u < kThreads; u += 16) {
                    const int k = l - __popc(u);
                    if (k >= 0 && k <= 4) acc = P::add(acc, gb[u * 5 + k]);
                }
            }
            for (int w = 8; w > 0; w >>= 1) acc = P::add(acc, shfl_xor_v(acc, w));
            if (l <= bT && j == 0) part[(size_t)H * (bT + 1) + l] = acc;
        }
    }
    __syncthreads();
    if (t <= d + 1) {
        offT[t] = Kcount(sbin, bT, t - 1);
        offT1[t] = Kcount(sbin, bT - 1, t - 1);
    }
    const uint32_t tlo = t & 15, thi = t >> 4;
    for (int v = only_v >= 0 ? only_v : 0; v < (only_v >= 0 ? only_v + 1 : n); ++v) {
        const bool low = v < bT;
        if (!low && ((Hf >> v) & 1)) continue;
        // ---- g in layout A
        if (low && v < 8) {
            // partner Rp(S + v) lives in another thread: exchange through LDS
#pragma unroll
            for (int r = 0; r < NR; ++r) gb[padx(r * kThreads + t)] = Rr[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const uint32_t x = r * kThreads + t;
                g[r] = ((x >> v) & 1) ? P::zero()
                                      : P::mul_raw(sq[hpc + __popc(x)],
                                                   P::mul_raw(Lr[r], gb[padx(x | (1u << v))]));
            }
            __syncthreads();
        } else if (low) {
            // v is register bit q: the partner is register r + 2^q of this thread
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (v - 8 != q) continue;
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    g[r] = ((r >> q) & 1) ? P::zero()
                                          : P::mul_raw(sq[hpc + __popc(r * kThreads + t)],
                                                       P::mul_raw(Lr[r], Rr[r | (1 << q)]));
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r)
                g[r] = P::mul_raw(sq[hpc + __popc(r * kThreads + t)],
                                  P::mul_raw(Lr[r], P::decode_raw(Rv[r])));
            vn = v + 1;                       // prefetch the next endpoint's Rp tile
            while (vn < n && ((Hf >> vn) & 1)) ++vn;
            if (vn < n) {
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    Rv[r] = P::load_raw(R, Hf | (r * kThreads + t) | (1ull << vn));
            }
        }
        // ---- tile bits 8..11 (layout A)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v != 8 + q) reg_zeta_down<P, NR>(g, q);
        // ---- A -> B, tile bits 4..7
#pragma unroll
        for (int r = 0; r < NR; ++r) gb[padx(r * kThreads + t)] = g[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) g[r] = gb[padx((thi << 8) | (r << 4) | tlo)];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v != 4 + q) reg_zeta_down<P, NR>(g, q);
        __syncthreads();
        // ---- B -> C, tile bits 0..3
#pragma unroll
        for (int r = 0; r < NR; ++r) gb[padx((thi << 8) | (r << 4) | tlo)] = g[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) g[r] = gb[padx((t << 4) | r)];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v != q) reg_zeta_down<P, NR>(g, q);
        // ---- outputs: entries with at most d ones, read back through LDS
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) gb[padx((t << 4) | r)] = g[r];
        __syncthreads();
        const int hv = gg.hv[v];
        const uint32_t Hc = low ? H : (uint32_t)compress_bit(H, v - bT);
        V *dst = Y1 + gg.y1off[v];
        for (uint32_t si = t; si < gg.KT; si += kThreads) {
            const uint32_t msk = seedT[si];
            uint32_t rank = si;
            if (low) {
                if ((msk >> v) & 1) continue;
                const uint32_t cm = (uint32_t)compress_bit(msk, v);
                rank = offT1[__popc(cm)];
                int k = 0;
                uint32_t rest = cm;
                while (rest) {
                    const int p = __ffs(rest) - 1;
                    rest &= rest - 1;
                    rank += C(sbin, p, ++k);
                }
            }
            dst[y1_at(rank, Hc, hv, gg.kg4[v])] = P::norm_v(gb[padx(msk)]);
        }
        __syncthreads();
    }
}

// Consecutive tiles run on the same XCD so that its L2 merges the 8-byte Y1
// writes of neighbouring tiles.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_gamma_tile(int n, int d, GammaGeom gg, Tables tb, typename P::Store L, typename P::Store R,
             const typename P::V *__restrict__ qt, typename P::V *__restrict__ Y1,
             typename P::V *__restrict__ part) {
    const uint32_t nblk = 1u << (n - 12);
    uint32_t H = blockIdx.x;
    if (nblk >= 64) H = (blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
    gamma_tile<P>(n, d, gg, tb, L, R, qt, Y1, part, H);
}

// Recomputation in the number system proper of the listed work (list[0]
// entries, list[1 + j] = H * 64 + e: tile H, every endpoint for e = 0, else
// endpoint e - 1 alone): the grid walks the list.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_gamma_tile_fb(int n, int d, GammaGeom gg, Tables tb, typename P::Store L,
                typename P::Store R, const typename P::V *__restrict__ qt,
                typename P::V *__restrict__ Y1, typename P::V *__restrict__ part,
                const uint32_t *list) {
    const uint32_t ntile = list[0];
    for (uint32_t it = blockIdx.x; it < ntile; it += gridDim.x) {
        __syncthreads();
        const uint32_t item = list[1 + it];
        gamma_tile<P>(n, d, gg, tb, L, R, qt, Y1, part, item >> 6, (int)(item & 63) - 1);
    }
}

template <int NR>
__device__ inline void lin_zeta_down(double *g, int q) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
        if (!((r >> q) & 1)) g[r] += g[r | (1 << q)];
}

// Linear-tile form of k_gamma_tile (same tiles and outputs). For endpoint v
// every needed output Gamma_v(G_L) of the tile is a sum over supersets of
// G_L that includes g_v(H + top), top = every tile bit but v. So the
// products are scaled by one power of two (a log offset for the log-space
// system) that puts g_v(H + top) near 2^-1000 (within 2^-1032 .. 2^-968 in the
// FP32-scaled form, whose scales are multiples of 64), and the downward zeta
// runs on plain doubles: one FP64 add per step. Products far below
// g_v(H + top) may lose bits to the subnormal range, each at most 2^-1075;
// over the at most 2^11 terms of an output (which is at least g_v(H + top))
// that is at most 2^-32 of the output in the FP32-scaled form, below the
// 2^-24 rounding of its stored significand, and 2^-64 in the log form. If
// Gamma_v(H + empty), the largest entry, overflows after
// the scaling, or g_v(H + top) is zero, the endpoint's outputs are not stored
// and (H, v) goes to the list of k_gamma_tile_retry. force_fb sends every
// tile to the fallback list of k_gamma_tile_fb, which recomputes all of its
// endpoints (tests).
// Layouts (x the 12 tile bits, 256 threads x 16 entries):
//   A  x = t * 16 + r      bits 0..3 in registers; products formed here. Each
//      thread owns 16 consecutive masks, so L, Rp and the partners Rp(x + v)
//      move as 16-entry vector loads: the thread's own Rp block for a
//      register bit, the block of thread t + 2^(v-4) for tile bits 4..11,
//      the tile H + v above the tile; one endpoint ahead of their use.
//   B  x = thi * 256 + r * 16 + tlo, bits 4..7 in registers;
//   C  x = r * 256 + p, p the thread's pattern of bits 0..7 (lane order
//      ordC), bits 8..11 in registers. Only outputs with at most d ones are
//      needed and bits 0..7 are final by then, so threads whose pattern has
//      more than d ones skip C (whole waves for small d).
// The kernel below wraps this body with its register cap.
template <class P, bool kSplit>
__device__ __forceinline__ void
gamma_tile_lin_body(int n, int d, int force_fb, int vsplit, GammaGeom gg, Tables tb,
                    typename P::Store L, typename P::Store R, const typename P::V *__restrict__ qt,
                    typename P::V *__restrict__ Y1, typename P::V *__restrict__ part,
                    uint32_t *fb, uint32_t *rt) {
    using V = typename P::V;
    using R16 = typename P::Raw16;
    using A = typename P::Anchor;
    constexpr int bT = 12, NR = 16;
    extern __shared__ unsigned char smem[];
    double *gb = reinterpret_cast<double *>(smem);             // padded 2^12 entries
    V *gv = reinterpret_cast<V *>(smem);                       // same slots, as values
    uint32_t *sbin = reinterpret_cast<uint32_t *>(gb + 4096 + 256);
    uint32_t *seedT = sbin + 33 * 33;                          // K(12, d) ranked masks
    __shared__ V sq[32];
    __shared__ uint32_t offT[34], offT1[34];
    __shared__ A sT[32];
    __shared__ int sok[32];
    __shared__ int sfail;
    const int t = threadIdx.x;
    const int hbits = n - bT;
    const uint32_t nblk = 1u << hbits;
    // vsplit workgroups share a tile, workgroup v0 taking the endpoints
    // v = v0 (mod vsplit); the first of them also writes the tile's partials
    const int vs = kSplit ? vsplit : 1;
    const uint32_t blk = kSplit ? blockIdx.x / (uint32_t)vs : blockIdx.x;
    const int v0 = kSplit ? (int)(blockIdx.x % (uint32_t)vs) : 0;
    uint32_t H = blk;
    if (nblk >= 64) H = (blk & 7) * (nblk >> 3) + (blk >> 3);
    const uint64_t Hf = (uint64_t)H << bT;
    const uint64_t x0 = Hf | ((uint32_t)t << 4);   // the thread's first mask in layout A
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    for (uint32_t x = t; x < gg.KT; x += kThreads) seedT[x] = tb.seedmask[x];
    if (t < n) sq[t] = qt[t];
    if (t == 0) sfail = force_fb && v0 == 0 ? 1 : 0;
    R16 Lw, Rown, Rv;                         // own L and Rp blocks; partners of the next endpoint
    const int hpc = __popcll(Hf);
    // the workgroup's first endpoint, and the partner block it needs
    int vfirst = v0;
    while (vfirst < n && vfirst >= bT && ((Hf >> vfirst) & 1)) vfirst += vs;
    {
        Lw = P::load16_raw(L, x0);
        Rown = P::load16_raw(R, x0);
        Rv = Rown;                            // a register bit needs no partner block
        if (vfirst >= 4 && vfirst < bT)
            Rv = P::load16_raw(R, Hf | ((uint32_t)(t | (1 << (vfirst - 4))) << 4));
        else if (vfirst >= bT && vfirst < n)
            Rv = P::load16_raw(R, x0 | (1ull << vfirst));
        __syncthreads();                      // sbin
        // invariant partials: sum of L(S) Rp(S) over the tile, per |x|; the
        // thread's entries have |x| = |t| + |r|
        V lr[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) lr[k] = P::zero();
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const V prod = P::mul(P::at16(Lw, r), P::at16(Rown, r));
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (__builtin_popcount(r) == k) lr[k] = P::add(lr[k], prod);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) gv[t * 5 + k] = lr[k];
        __syncthreads();
        {   // layer l = t / 16 of the tile: 16 lanes x 16 slots, then a lane tree
            const int l = t >> 4, j = t & 15;
            V acc = P::zero();
            if (l <= bT) {
                for (int u = j; u < kThreads; u += 16) {
                    const int k = l - __popc(u);
                    if (k >= 0 && k <= 4) acc = P::add(acc, gv[u * 5 + k]);
                }
            }
            for (int w = 8; w > 0; w >>= 1) acc = P::add(acc, shfl_xor_v(acc, w));
            if (l <= bT && j == 0 && v0 == 0) part[(size_t)H * (bT + 1) + l] = acc;
        }
    }
    // scale of endpoint v: g_v at the top of the tile
    if (t < n) {
        const int v = t;
        const uint32_t all = (1u << bT) - 1;
        int ok = 0;
        A T{};
        if (v < bT) {
            const V a = P::mul(P::mul(sq[hpc + bT - 1], P::load(L, Hf | (all & ~(1u << v)))),
                               P::load(R, Hf | all));
            ok = P::anchor_of(a, &T) ? 1 : 0;
        } else if (!((Hf >> v) & 1)) {
            const V a = P::mul(P::mul(sq[hpc + bT], P::load(L, Hf | all)),
                               P::load(R, Hf | all | (1ull << v)));
            ok = P::anchor_of(a, &T) ? 1 : 0;
        }
        sT[v] = T;
        sok[v] = ok;
    }
    if (t <= d + 1) {
        offT[t] = Kcount(sbin, bT, t - 1);
        offT1[t] = Kcount(sbin, bT - 1, t - 1);
    }
    __syncthreads();
    // q(|S|) for the thread's entries in layout A: |S| = |H| + |t| + |r|
    // q(|S|) L(S) for the thread's entries, the factor every endpoint shares
    V qL[NR];
    {
        const int ht = hpc + __popc(t);
        V qa[5];
#pragma unroll
        for (int m = 0; m < 5; ++m) qa[m] = sq[min(ht + m, 31)];
#pragma unroll
        for (int r = 0; r < NR; ++r) qL[r] = P::mul_raw(qa[__builtin_popcount(r)], P::at16_nz(Lw, r));
    }
    const uint32_t tlo = t & 15, thi = t >> 4;
    const uint32_t pc = tb.ordC[t];
    const bool liveC = __popc(pc) <= d;
    // padx indices as a lane base plus a constant per register (folded into
    // the LDS offsets): A, padx(t * 16 + r) = 17 t + r; B, padx(thi * 256 +
    // r * 16 + tlo) = 272 thi + tlo + 17 r; C, padx(r * 256 + pc) =
    // pc + pc / 16 + 272 r
    const uint32_t iA = 17 * t, iB = 272 * thi + tlo, iC = pc + (pc >> 4);
    auto endpoint = [&](const int v) {
        const bool low = v < bT;
        if (!low && ((Hf >> v) & 1)) return;
        const A T = sT[v];
        const int okv = sok[v];
        // ---- products in layout A (entries with bit v are not in the lattice)
        double g[NR];
        if (v < 4) {
            // the partner of register r is register r + 2^v of the own block
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (v != q) continue;
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    g[r] = ((r >> q) & 1) ? 0.0
                                          : P::prod2_lin(qL[r], P::at16_nz(Rown, r | (1 << q)), T);
            }
        } else {
            const bool excl = low && ((t >> (v - 4)) & 1);
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double pr =
                    P::prod2_lin(qL[r], P::at16_nz(Rv, r), T);
                g[r] = excl ? 0.0 : pr;
            }
        }
        {   // partners of the next endpoint (none needed for register bits)
            int vn = v + vs;
            while (vn < n && vn >= bT && ((Hf >> vn) & 1)) vn += vs;
            if (vn >= 4 && vn < bT) {
                // tile bit vn: the block of thread t + 2^(vn-4) (own block if set)
                Rv = P::load16_raw(R, Hf | ((uint32_t)(t | (1 << (vn - 4))) << 4));
            } else if (vn >= bT && vn < n) {
                Rv = P::load16_raw(R, x0 | (1ull << vn));
            }
        }
        // ---- tile bits 0..3 (layout A)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v != q) lin_zeta_down<NR>(g, q);
        // ---- A -> B, tile bits 4..7
#pragma unroll
        for (int r = 0; r < NR; ++r) gb[iA + r] = g[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) g[r] = gb[iB + r * 17];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (v != 4 + q) lin_zeta_down<NR>(g, q);
        // B-layout slots belong to one thread each: written back in place
#pragma unroll
        for (int r = 0; r < NR; ++r) gb[iB + r * 17] = g[r];
        __syncthreads();
        // ---- B -> C, tile bits 8..11, live patterns only; results stay in place
        if (liveC) {
#pragma unroll
            for (int r = 0; r < NR; ++r) g[r] = gb[iC + r * 272];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v != 8 + q) lin_zeta_down<NR>(g, q);
#pragma unroll
            for (int r = 0; r < NR; ++r) gb[iC + r * 272] = g[r];
        }
        __syncthreads();
        // ---- outputs: entries with at most d ones, read back through LDS.
        // Gamma_v(H + empty) bounds every entry of the tile.
        const bool fine = okv && gb[padx(0)] <= 1.0e300;
        if (!fine) {
            if (t == 0) fb_push(rt, (H << 5) | (uint32_t)v);   // k_gamma_tile_retry
        } else {
            const int hv = gg.hv[v];
            const uint32_t Hc = low ? H : (uint32_t)compress_bit(H, v - bT);
            V *dst = Y1 + gg.y1off[v];
            for (uint32_t si = t; si < gg.KT; si += kThreads) {
                const uint32_t msk = seedT[si];
                uint32_t rank = si;
                if (low) {
                    if ((msk >> v) & 1) continue;
                    const uint32_t cm = (uint32_t)compress_bit(msk, v);
                    rank = offT1[__popc(cm)];
                    int k = 0;
                    uint32_t rest = cm;
                    while (rest) {
                        const int p = __ffs(rest) - 1;
                        rest &= rest - 1;
                        rank += C(sbin, p, ++k);
                    }
                }
                dst[y1_at(rank, Hc, hv, gg.kg4[v])] = P::from_lin(gb[padx(msk)], T);
            }
        }
        __syncthreads();
    };
    // the own Rp block is a partner only for the register bits 0..3: with a
    // loop of their own, it is dead in the loops over the other endpoints;
    // the tile bits and the bits above the tile get a loop each as well
    if constexpr (kSplit) {
        int v = v0;
        for (; v < 4 && v < n; v += vs) endpoint(v);
        for (; v < bT && v < n; v += vs) endpoint(v);
        for (; v < n; v += vs) endpoint(v);
    } else {
        for (int v = 0; v < 4 && v < n; ++v) endpoint(v);
        for (int v = 4; v < bT && v < n; ++v) endpoint(v);
        for (int v = bT; v < n; ++v) endpoint(v);
    }
    if (t == 0 && sfail) fb_push(fb, H << 6);             // every endpoint
}

// Three waves per SIMD (168 registers, some spill), which measured faster
// than two without spills: more waves hide the barrier and load latency of
// the endpoint loops.
template <class P, bool kSplit>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_gamma_tile_lin(int n, int d, int force_fb, int vsplit, GammaGeom gg, Tables tb,
                 typename P::Store L,
                 typename P::Store R, const typename P::V *__restrict__ qt,
                 typename P::V *__restrict__ Y1, typename P::V *__restrict__ part,
                 uint32_t *fb, uint32_t *rt) {
    gamma_tile_lin_body<P, kSplit>(n, d, force_fb, vsplit, gg, tb, L, R, qt, Y1, part, fb, rt);
}

// Second chance for the endpoints that k_gamma_tile_lin could not scale from
// g_v(H + top) (list[0] items, list[1 + j] = H * 32 + v; the grid walks the
// list). The scale now comes from the largest product of the tile, which
// keeps Gamma_v(H + empty) finite; the outputs are stored only if every
// needed one is at least 2^-1000, since the products that fell below 2^-1074
// (at most 4096) then change none by more than 2^-62 of itself. Outputs below
// that get a third chance under the first scale (below); an endpoint with an
// output valid under neither goes to the fallback list of k_gamma_tile_fb.
// Same layouts as k_gamma_tile_lin, layout C for every thread.
template <class P>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gamma_tile_retry(int n, int d, GammaGeom gg, Tables tb, typename P::Store L,
                   typename P::Store R, const typename P::V *__restrict__ qt,
                   typename P::V *__restrict__ Y1, const uint32_t *list, uint32_t *fb) {
    using V = typename P::V;
    using R16 = typename P::Raw16;
    using A = typename P::Anchor;
    constexpr int bT = 12, NR = 16;
    extern __shared__ unsigned char smem[];
    double *gb = reinterpret_cast<double *>(smem);             // padded 2^12 entries
    uint32_t *sbin = reinterpret_cast<uint32_t *>(gb + 4096 + 256);
    uint32_t *seedT = sbin + 33 * 33;                          // K(12, d) ranked masks
    __shared__ V sq[32];
    __shared__ uint32_t offT1[34];
    __shared__ int smax;
    __shared__ A sT2;
    const uint32_t t = threadIdx.x;
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    for (uint32_t x = t; x < gg.KT; x += kThreads) seedT[x] = tb.seedmask[x];
    if (t < (uint32_t)n) sq[t] = qt[t];
    __syncthreads();
    if (t <= (uint32_t)d + 1) offT1[t] = Kcount(sbin, bT - 1, (int)t - 1);
    const uint32_t tlo = t & 15, thi = t >> 4;
    const uint32_t nitem = list[0];
    for (uint32_t it = blockIdx.x; it < nitem; it += gridDim.x) {
        __syncthreads();
        const uint32_t item = list[1 + it];
        const uint32_t H = item >> 5;
        const int v = (int)(item & 31);
        const bool low = v < bT;
        const uint64_t Hf = (uint64_t)H << bT;
        const uint64_t x0 = Hf | (t << 4);
        const int ht = __popcll(Hf) + __popc(t);
        const R16 Lw = P::load16_raw(L, x0);
        const R16 Rown = P::load16_raw(R, x0);
        R16 Rv = Rown;
        if (v >= 4)
            Rv = P::load16_raw(R, low ? Hf | ((uint64_t)(t | (1u << (v - 4))) << 4) : x0 | (1ull << v));
        const bool excl = v >= 4 && low && ((t >> (v - 4)) & 1);
        // products q(|S|) L(S) Rp(S + v) as undecoded values, and their largest
        V pv[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r)
            pv[r] = P::mul_raw(sq[min(ht + __builtin_popcount(r), 31)], P::at16_nz(Lw, r));
        if (v < 4) {
            // the partner of register r is register r + 2^v of the own block
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (v != q) continue;
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    pv[r] = ((r >> q) & 1) ? P::zero()
                                           : P::mul_raw(pv[r], P::at16_nz(Rown, r | (1 << q)));
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r)
                pv[r] = excl ? P::zero() : P::mul_raw(pv[r], P::at16_nz(Rv, r));
        }
        double mx = -1e300;
#pragma unroll
        for (int r = 0; r < NR; ++r) mx = fmax(mx, P::log2_of(pv[r]));
        if (t == 0) smax = -(1 << 30);
        __syncthreads();
        atomicMax(&smax, (int)fmax(mx, -1073741824.0));
        __syncthreads();
        const bool any = smax > -(1 << 29);
        const A T = P::anchor_high(smax);
        // downward zeta of the products under scale Ts over the tile bits
        // but v, into gb (layout C for every thread)
        auto zeta3 = [&](const A Ts) {
            double g[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r) g[r] = P::prod2_lin(pv[r], P::one(), Ts);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v != q) lin_zeta_down<NR>(g, q);
#pragma unroll
            for (int r = 0; r < NR; ++r) gb[padx((t << 4) | r)] = g[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NR; ++r) g[r] = gb[padx((thi << 8) | (r << 4) | tlo)];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v != 4 + q) lin_zeta_down<NR>(g, q);
#pragma unroll
            for (int r = 0; r < NR; ++r) gb[padx((thi << 8) | (r << 4) | tlo)] = g[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NR; ++r) g[r] = gb[padx((r << 8) | t)];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (v != 8 + q) lin_zeta_down<NR>(g, q);
#pragma unroll
            for (int r = 0; r < NR; ++r) gb[padx((r << 8) | t)] = g[r];
            __syncthreads();
        };
        zeta3(T);
        bool small = !(any && gb[padx(0)] <= 1.0e300);
        for (uint32_t si = t; si < gg.KT && !small; si += kThreads) {
            const uint32_t msk = seedT[si];
            if (low && ((msk >> v) & 1)) continue;
            small = !(gb[padx(msk)] >= 0x1p-1000);
        }
        // Third chance for outputs below 2^-1000 under the largest product's
        // scale: a pass under the scale of g_v(H + top) (every needed output
        // holds that term, so it is at least about 2^-1000 there; an output
        // that overflows there is at least 2^-1000 under the first scale when
        // the two scales lie less than 2024 binary orders apart). Each needed
        // output is taken from the pass where it is at least 2^-1000 and
        // finite; an endpoint with an output valid in neither goes to
        // k_gamma_tile_fb. Outputs of the first pass wait in registers
        // (at most 4 per thread, K(12, d) <= 1024).
        constexpr int kMaxOut = 4;
        double keep1[kMaxOut];
        A T2 = T;
        bool two = false;
        if (__syncthreads_or(small ? 1 : 0)) {
            bool ok = any && gg.KT <= kMaxOut * kThreads;
            if (ok) {
                // g_v(H + top): top = every tile bit but v, entry x_top of layout A
                const uint32_t xtop = low ? (0xfffu & ~(1u << v)) : 0xfffu;
                if (t == (xtop >> 4)) {
                    A Tt{};
                    V top = P::zero();
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        if ((uint32_t)r == (xtop & 15u)) top = pv[r];
                    smax = P::anchor_of(top, &Tt) ? 1 : 0;
                    sT2 = Tt;
                }
                __syncthreads();
                ok = smax != 0;
                T2 = sT2;
            }
            if (ok) {
#pragma unroll
                for (int k = 0; k < kMaxOut; ++k) {
                    const uint32_t si = t + k * kThreads;
                    keep1[k] = si < gg.KT ? gb[padx(seedT[si])] : 0.0;
                }
                __syncthreads();                  // gb is rewritten by the second pass
                zeta3(T2);
                bool fail = false;
#pragma unroll
                for (int k = 0; k < kMaxOut; ++k) {
                    const uint32_t si = t + k * kThreads;
                    if (si >= gg.KT) continue;
                    const uint32_t msk = seedT[si];
                    if (low && ((msk >> v) & 1)) continue;
                    const double y2 = gb[padx(msk)];
                    fail = fail || !(keep1[k] >= 0x1p-1000 || (y2 >= 0x1p-1000 && y2 <= 1.0e300));
                }
                ok = __syncthreads_or(fail ? 1 : 0) == 0;
            }
            if (!ok) {
                if (t == 0) fb_push(fb, (H << 6) | (uint32_t)(v + 1));   // this endpoint only
                continue;
            }
            two = true;
        }
        const int hv = gg.hv[v];
        const uint32_t Hc = low ? H : (uint32_t)compress_bit(H, v - bT);
        V *dst = Y1 + gg.y1off[v];
        auto rank_of = [&](uint32_t si, uint32_t msk) {
            uint32_t rank = si;
            if (low) {
                const uint32_t cm = (uint32_t)compress_bit(msk, v);
                rank = offT1[__popc(cm)];
                int k = 0;
                uint32_t rest = cm;
                while (rest) {
                    const int p = __ffs(rest) - 1;
                    rest &= rest - 1;
                    rank += C(sbin, p, ++k);
                }
            }
            return rank;
        };
        if (two) {
#pragma unroll
            for (int k = 0; k < kMaxOut; ++k) {
                const uint32_t si = t + k * kThreads;
                if (si >= gg.KT) break;
                const uint32_t msk = seedT[si];
                if (low && ((msk >> v) & 1)) continue;
                const bool first = keep1[k] >= 0x1p-1000;
                dst[y1_at(rank_of(si, msk), Hc, hv, gg.kg4[v])] =
                    P::from_lin(first ? keep1[k] : gb[padx(msk)], first ? T : T2);
            }
        } else {
            for (uint32_t si = t; si < gg.KT; si += kThreads) {
                const uint32_t msk = seedT[si];
                if (low && ((msk >> v) & 1)) continue;
                dst[y1_at(rank_of(si, msk), Hc, hv, gg.kg4[v])] = P::from_lin(gb[padx(msk)], T);
            }
        }
    }
}

// ------------------------- a5 + a6: Gamma, in-tile part, tiles of any size
// Generic form used when the lattice is smaller than the 12-bit tile of
// k_gamma_tile (n < 12): the whole lattice is one tile of bT = n bits.
// Workgroup = full-mask tile H (the low bT bits vary; entry x = reg * 256 + t)
// and, when the lattice is that one tile, one endpoint (vsplit = n workgroups;
// otherwise vsplit = 1). L(H + x) and Rp(H + x) stay in registers for the
// whole workgroup; each of its endpoints v not in H is served in turn:
//   g_v(S) = q(|S|) L(S) Rp(S + v) for S = H + x. For v a tile bit, x runs
//   over the entries without bit v and Rp(S + v) is the partner entry: the
//   same thread's register when v is a register bit, else read through LDS.
//   For v above the tile Rp(S + v) is the tile H + v, prefetched while the
//   previous endpoint is reduced. Products are left unnormalised: the
//   alignment in add() is exact for any FP32 significand.
//   Truncated downward zeta over the tile bits other than v: the register
//   bits densely, then the low 8 bits in LDS, where bit j only updates masks
//   with at most d ones among the bits already processed (Def. 2; the
//   predicate of Alg. 3).
//   The entries with at most d ones go to Y1_v[seed][Hc_v].
// Consecutive tiles run on the same XCD so that its L2 merges the 8-byte Y1
// writes of neighbouring tiles.
template <class P, int RB>
__global__ void __launch_bounds__(kThreads)
k_gamma_tile_gen(int n, int d, int bT, int vsplit, GammaGeom gg, Tables tb, typename P::Store L,
             typename P::Store R, const typename P::V *__restrict__ qt,
             typename P::V *__restrict__ Y1) {
    using V = typename P::V;
    constexpr int NR = 1 << RB;
    extern __shared__ unsigned char smem[];
    const uint32_t T = 1u << bT;
    V *gb = reinterpret_cast<V *>(smem);
    uint32_t *sbin = reinterpret_cast<uint32_t *>(gb + T);
    uint32_t *seedT = sbin + 33 * 33;
    uint16_t *spat = reinterpret_cast<uint16_t *>(seedT + gg.KT);
    __shared__ V sq[32];
    const int t = threadIdx.x;
    const int lb = bT < 8 ? bT : 8;          // thread bits of the tile
    const int hbits = n - bT;
    const uint32_t nblk = 1u << hbits;
    // vsplit workgroups share a tile, workgroup v0 taking the endpoints
    // v = v0 (mod vsplit)
    const uint32_t blk = blockIdx.x / (uint32_t)vsplit;
    const int v0 = (int)(blockIdx.x % (uint32_t)vsplit);
    uint32_t H = blk;
    if (nblk >= 64) H = (blk & 7) * (nblk >> 3) + (blk >> 3);
    const uint64_t Hf = (uint64_t)H << bT;
    for (int x = t; x < 33 * 33; x += kThreads) sbin[x] = tb.binom[x];
    for (uint32_t x = t; x < gg.KT; x += kThreads) seedT[x] = tb.seedmask[x];
    for (uint32_t x = t; x < gg.npat; x += kThreads) spat[x] = tb.pat[x];
    if (t < n) sq[t] = qt[t];
    using Raw = typename P::Raw;
    V Lr[NR], Rr[NR], g[NR];
    Raw Rv[NR];                               // next endpoint's Rp tile, undecoded
    uint32_t pc[NR];
    const bool full = RB > 0 || T >= kThreads;   // every (r, t) maps to an entry
    {
        Raw l0[NR], r0[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t x = r * kThreads + t;
            pc[r] = __popcll(Hf | x);
            if (full || x < T) {
                l0[r] = P::load_raw(L, Hf | x);
                r0[r] = P::load_raw(R, Hf | x);
            }
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            Lr[r] = P::decode_raw(l0[r]);
            Rr[r] = P::decode_raw(r0[r]);
        }
    }
    int vn = v0;                              // next endpoint above the tile, not in H
    while (vn < bT) vn += vsplit;
    while (vn < n && ((Hf >> vn) & 1)) vn += vsplit;
    if (vn < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t x = r * kThreads + t;
            if (full || x < T) Rv[r] = P::load_raw(R, Hf | x | (1ull << vn));
        }
    }
    __syncthreads();
    const uint32_t *bn = sbin;
    for (int v = v0; v < n; v += vsplit) {
        const bool low = v < bT;
        if (!low && ((Hf >> v) & 1)) continue;
        if (low && v < lb) {
            // partner Rp(S + v) lives in another thread: exchange through LDS
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const uint32_t x = r * kThreads + t;
                if (full || x < T) gb[x] = Rr[r];
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const uint32_t x = r * kThreads + t;
                if (!full && x >= T) continue;
                if ((x >> v) & 1) {
                    g[r] = P::zero();
                } else {
                    g[r] = P::mul_raw(sq[pc[r]], P::mul_raw(Lr[r], gb[x | (1u << v)]));
                }
            }
            __syncthreads();
        } else if (low) {
            // v is register bit q: the partner is register r + 2^q of this thread
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                if (v - lb != q) continue;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    if ((r >> q) & 1) {
                        g[r] = P::zero();
                    } else {
                        const uint32_t x = r * kThreads + t;
                        if (full || x < T)
                            g[r] = P::mul_raw(sq[pc[r]], P::mul_raw(Lr[r], Rr[r | (1 << q)]));
                    }
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const uint32_t x = r * kThreads + t;
                if (full || x < T)
                    g[r] = P::mul_raw(sq[pc[r]], P::mul_raw(Lr[r], P::decode_raw(Rv[r])));
            }
            vn = v + vsplit;                  // prefetch the next endpoint's Rp tile
            while (vn < n && ((Hf >> vn) & 1)) vn += vsplit;
            if (vn < n) {
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const uint32_t x = r * kThreads + t;
                    if (full || x < T) Rv[r] = P::load_raw(R, Hf | x | (1ull << vn));
                }
            }
        }
        // register bits (downward, dense), skipping bit v
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (low && v == lb + q) continue;
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (!((r >> q) & 1)) g[r] = P::add(g[r], g[r | (1 << q)]);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t x = r * kThreads + t;
            if (full || x < T) gb[x] = g[r];
        }
        __syncthreads();
        // thread bits in LDS, truncated on the bits already processed
        for (int j = 0; j < lb; ++j) {
            if (j == v) continue;
            const int fb = lb - 1 - j;           // free bits above j
            const uint32_t cnt = Kcount(bn, j + RB, d) << fb;
            const uint32_t jm = (1u << j) - 1, fm = (1u << fb) - 1;
            for (uint32_t idx = t; idx < cnt; idx += kThreads) {
                const uint32_t p = spat[idx >> fb];
                const uint32_t Tm = (p & jm) | ((p >> j) << lb) | ((idx & fm) << (j + 1));
                gb[Tm] = P::add(gb[Tm], gb[Tm | (1u << j)]);
            }
            __syncthreads();
        }
        // outputs: masks with at most d ones (and without bit v)
        const int hv = gg.hv[v];
        const uint32_t Hc = low ? H : (uint32_t)compress_bit(H, v - bT);
        V *dst = Y1 + gg.y1off[v];
        for (uint32_t si = t; si < gg.KT; si += kThreads) {
            const uint32_t msk = seedT[si];
            uint32_t rank = si;
            if (low) {
                if ((msk >> v) & 1) continue;
                const uint32_t cm = (uint32_t)compress_bit(msk, v);
                const int sg = __popc(cm);
                rank = Kcount(bn, bT - 1, sg - 1);
                int k = 0;
                uint32_t rest = cm;
                while (rest) {
                    const int p = __ffs(rest) - 1;
                    rest &= rest - 1;
                    rank += C(bn, p, ++k);
                }
            }
            dst[y1_at(rank, Hc, hv, gg.kg4[v])] = P::norm_v(gb[msk]);
        }
        __syncthreads();
    }
}

// Output rank (within node v's ranked parent sets) of G_L + (high pattern
// x shifted by shift), |G_L| = sigma with colex rank cl.
__device__ inline uint32_t out_rank(const uint32_t *bn, int N, int sigma, uint32_t cl,
                                    uint32_t x, int shift) {
    int k = 0;
    uint32_t r = cl;
    while (x) {
        const int p = __ffs(x) - 1;
        x &= x - 1;
        r += C(bn, shift + p, sigma + (++k));
    }
    return Kcount(bn, N, sigma + k - 1) + r;
}

// Seed of endpoint v's compressed tile: size class and colex rank of the
// s-th ranked mask over bv bits.
__device__ inline void seed_of(const uint32_t *bn, int bv, uint32_t s, int *sigma, uint32_t *cl) {
    int k = 0;
    uint32_t off = 0;
    while (s >= off + C(bn, bv, k)) off += C(bn, bv, k++);
    *sigma = k;
    *cl = s - off;
}

// Locate (v, local index) of a flat block index over per-v block counts.
__device__ inline int find_v(const uint32_t *pref, int n, uint32_t b) {
    int v = 0;
    while (v + 1 < n + 1 && pref[v + 1] <= b) ++v;
    return v;
}

// ---------------------------------- a6: Gamma, high bits, one level
// Workgroup (v, seed): the vector Y1_v[seed][.] over v's hv high bits;
// truncated downward zeta keeping |G_H| <= d - |G_L|; writes Gamma_v.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_gamma_high1(int n, int d, uint32_t K, GammaGeom gg, Tables tb,
              const typename P::V *__restrict__ Y1, typename P::V *__restrict__ gam) {
    using V = typename P::V;
    extern __shared__ unsigned char smem[];
    V *vec = reinterpret_cast<V *>(smem);
    const int N = n - 1;
    const int v = find_v(gg.blk1, n, blockIdx.x);
    const uint32_t s = y1_reader_item(blockIdx.x - gg.blk1[v], 0, gg.kg4[v]);
    const int t = threadIdx.x;
    const uint32_t *bn = tb.binom;
    const int bv = gg.bv[v], hv = gg.hv[v];
    int sigma;
    uint32_t cl;
    seed_of(bn, bv, s, &sigma, &cl);
    const int tr = d - sigma;
    const V *src = Y1 + gg.y1off[v] + y1_at(s, 0, hv, gg.kg4[v]);
    const uint32_t st = y1_stride(s, gg.kg4[v]);
    for (uint32_t x = t; x < (1u << hv); x += kThreads) vec[x] = src[(size_t)x * st];
    __syncthreads();
    for (int j = 0; j < hv; ++j) {
        const uint32_t cntj = Kcount(bn, j, d);  // walk the d-table, skip > tr
        const uint32_t tot = cntj << (hv - 1 - j);
        for (uint32_t idx = t; idx < tot; idx += kThreads) {
            const uint32_t hi = idx / cntj;
            const uint32_t p = tb.pat[idx - hi * cntj];
            if (__popc(p) > tr) continue;
            const uint32_t Tm = (hi << (j + 1)) | p;
            vec[Tm] = P::add(vec[Tm], vec[Tm | (1u << j)]);
        }
        __syncthreads();
    }
    const uint32_t npat = Kcount(bn, hv, d);
    for (uint32_t idx = t; idx < npat; idx += kThreads) {
        const uint32_t x = tb.pat[idx];
        if (__popc(x) > tr) continue;
        gam[(size_t)v * K + out_rank(bn, N, sigma, cl, x, bv)] = vec[x];
    }
}

// ------------------------------- a6: Gamma, high bits, two levels (A, B)
// Level A, workgroup (v, seed, Ht): the low a bits of Hc; output for every
// a-bit pattern p with at most d ones: Y2_v[seed][p][Ht].
template <class P>
__global__ void __launch_bounds__(kThreads)
k_gamma_highA(int n, int d, int a, uint32_t KA, GammaGeom gg, Tables tb,
              const typename P::V *__restrict__ Y1, typename P::V *__restrict__ Y2) {
    using V = typename P::V;
    extern __shared__ unsigned char smem[];
    V *vec = reinterpret_cast<V *>(smem);
    const int v = find_v(gg.blkA, n, blockIdx.x);
    const int bv = gg.bv[v], hv = gg.hv[v];
    const int hB = hv - a;
    const uint32_t local = y1_reader_item(blockIdx.x - gg.blkA[v], hB, gg.kg4[v]);
    const uint32_t Ht = local & ((1u << hB) - 1);
    const uint32_t s = local >> hB;
    const int t = threadIdx.x;
    const uint32_t *bn = tb.binom;
    int sigma;
    uint32_t cl;
    seed_of(bn, bv, s, &sigma, &cl);
    const int tr = d - sigma;
    const V *src = Y1 + gg.y1off[v] + y1_at(s, (uint64_t)Ht << a, hv, gg.kg4[v]);
    const uint32_t st = y1_stride(s, gg.kg4[v]);
    for (uint32_t x = t; x < (1u << a); x += kThreads) vec[x] = src[(size_t)x * st];
    __syncthreads();
    for (int j = 0; j < a; ++j) {
        const uint32_t cntj = Kcount(bn, j, d);
        const uint32_t tot = cntj << (a - 1 - j);
        for (uint32_t idx = t; idx < tot; idx += kThreads) {
            const uint32_t hi = idx / cntj;
            const uint32_t p = tb.pat[idx - hi * cntj];
            if (__popc(p) > tr) continue;
            const uint32_t Tm = (hi << (j + 1)) | p;
            vec[Tm] = P::add(vec[Tm], vec[Tm | (1u << j)]);
        }
        __syncthreads();
    }
    V *dst = Y2 + gg.y2off[v];
    for (uint32_t pi = t; pi < KA; pi += kThreads)
        dst[(((size_t)s * KA + pi) << hB) + Ht] = vec[tb.pat[pi]];
}

// Dense downward zeta over 12 bits: src[x], x < 2^12, into vec[padx(x)]
// (256 threads x 16 entries; bits 0..3, 4..7, 8..11 in three layouts joined
// through LDS). An entry with at most d - sigma ones receives the same
// additions in the same order as in the truncated pass of k_gamma_high1 /
// k_gamma_highA, so the results agree exactly; the other entries are
// computed too and never read. No pattern table, division or skip test per
// update. Ends with a barrier.
template <class P>
__device__ __forceinline__ void dense_zeta_down12_regs(typename P::V (&g)[16],
                                                       typename P::V *vec, uint32_t t) {
    constexpr int NR = 16;
    auto zeta4 = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (!((r >> q) & 1)) g[r] = P::add(g[r], g[r | (1 << q)]);
    };
    zeta4();                                            // bits 0..3
#pragma unroll
    for (int r = 0; r < NR; ++r) vec[padx((t << 4) | r)] = g[r];
    __syncthreads();
    const uint32_t tlo = t & 15, thi = t >> 4;
#pragma unroll
    for (int r = 0; r < NR; ++r) g[r] = vec[padx((thi << 8) | (r << 4) | tlo)];
    zeta4();                                            // bits 4..7
#pragma unroll
    for (int r = 0; r < NR; ++r) vec[padx((thi << 8) | (r << 4) | tlo)] = g[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) g[r] = vec[padx((r << 8) | t)];
    zeta4();                                            // bits 8..11
#pragma unroll
    for (int r = 0; r < NR; ++r) vec[padx((r << 8) | t)] = g[r];
    __syncthreads();
}

// The same zeta from layout C (g[r] = entry r * 256 + t, so that the loads
// of consecutive lanes touch consecutive entries), its bits in the order
// 8..11, 4..7, 0..3; the results end in vec[padx(x)] as above.
template <class P>
__device__ __forceinline__ void dense_zeta_down12_regsC(typename P::V (&g)[16],
                                                        typename P::V *vec, uint32_t t) {
    constexpr int NR = 16;
    auto zeta4 = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (!((r >> q) & 1)) g[r] = P::add(g[r], g[r | (1 << q)]);
    };
    zeta4();                                            // bits 8..11
#pragma unroll
    for (int r = 0; r < NR; ++r) vec[padx((r << 8) | t)] = g[r];
    __syncthreads();
    const uint32_t tlo = t & 15, thi = t >> 4;
#pragma unroll
    for (int r = 0; r < NR; ++r) g[r] = vec[padx((thi << 8) | (r << 4) | tlo)];
    zeta4();                                            // bits 4..7
#pragma unroll
    for (int r = 0; r < NR; ++r) vec[padx((thi << 8) | (r << 4) | tlo)] = g[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NR; ++r) g[r] = vec[padx((t << 4) | r)];
    zeta4();                                            // bits 0..3
#pragma unroll
    for (int r = 0; r < NR; ++r) vec[padx((t << 4) | r)] = g[r];
    __syncthreads();
}

template <class P>
__device__ __forceinline__ void dense_zeta_down12(const typename P::V *__restrict__ src,
                                                  uint32_t stride, typename P::V *vec,
                                                  uint32_t t) {
    typename P::V g[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) g[r] = src[(size_t)((t << 4) | r) * stride];
    dense_zeta_down12_regs<P>(g, vec, t);
}

// The FP32-scaled form of the dense 12-bit passes over the grouped ranks of
// Y1: a workgroup loads the four ranks of a group at once (32 bytes per
// entry, each byte read once, consecutive lanes on consecutive entries) and
// runs the zeta for each in turn; the ranks
// past the groups take one workgroup each. item: the workgroup's index within
// endpoint v; the grouped items come first, (group, Ht) with Ht fastest.
// Calls out(s, Ht) after the zeta of rank s has left vec (ends with a barrier).
template <class Out>
__device__ __forceinline__ void dense_zeta_down12_x4(const X32 *__restrict__ Y1v, int hv, int hB,
                                                     uint32_t kg4, uint32_t item, X32 *vec,
                                                     uint32_t t, Out out) {
    const uint32_t G = (kg4 >> 2) << hB;
    const uint32_t hmask = (1u << hB) - 1u;
    if (item < G) {
        const uint32_t s0 = (item >> hB) << 2, Ht = item & hmask;
        const uint4 *src = reinterpret_cast<const uint4 *>(Y1v + y1_at(s0, (uint64_t)Ht << 12, hv, kg4));
        uint4 raw[16][2];                     // entry r * 256 + t: ranks s0, s0 + 1 | s0 + 2, s0 + 3
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            raw[r][0] = src[2 * ((r << 8) | t)];
            raw[r][1] = src[2 * ((r << 8) | t) + 1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            X32 g[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint4 w = raw[r][q >> 1];
                g[r] = (q & 1) ? X32{__uint_as_float(w.z), (int)w.w}
                               : X32{__uint_as_float(w.x), (int)w.y};
            }
            dense_zeta_down12_regsC<PolX32>(g, vec, t);
            out(s0 + q, Ht);
            __syncthreads();                  // vec is read by out()
        }
    } else {
        const uint32_t x = item - G;
        const uint32_t s = kg4 + (x >> hB), Ht = x & hmask;
        const X32 *src = Y1v + y1_at(s, (uint64_t)Ht << 12, hv, kg4);
        X32 g[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) g[r] = src[(r << 8) | t];
        dense_zeta_down12_regsC<PolX32>(g, vec, t);
        out(s, Ht);
    }
}

// Plain doubles for dense_zeta_down12_regs.
struct Lin64 {
    using V = double;
    __device__ static inline V add(V a, V b) { return a + b; }
};

// Level A for a = 12 in the log form. The row's logarithms become plain
// doubles under one scale, exp(x - M) 2^960 with M the row's largest (so the
// sum of 4096 of them stays below 2^972), the dense 12-bit zeta runs in FP64
// adds, and the outputs go back as logarithms. They are kept only if every
// needed output (at most d - sigma ones) is at least 2^-1000: the values that
// fell below 2^-1074 (at most 4096) then change none by more than 2^-62 of
// itself. Otherwise, or always with force_trunc (tests), the workgroup runs
// the truncated log-add pass of k_gamma_highA on the row.
__global__ void __launch_bounds__(kThreads)
k_gamma_highA12_log(int n, int d, uint32_t KA, int force_trunc, GammaGeom gg, Tables tb,
                    const double *__restrict__ Y1, double *__restrict__ Y2) {
    constexpr int a = 12;
    extern __shared__ unsigned char smem[];
    double *vec = reinterpret_cast<double *>(smem);   // 2^12 entries, padx or plain
    __shared__ double red[kThreads];
    const int v = find_v(gg.blkA, n, blockIdx.x);
    const int bv = gg.bv[v], hv = gg.hv[v];
    const int hB = hv - a;
    const uint32_t local = y1_reader_item(blockIdx.x - gg.blkA[v], hB, gg.kg4[v]);
    const uint32_t Ht = local & ((1u << hB) - 1);
    const uint32_t s = local >> hB;
    const uint32_t t = threadIdx.x;
    const uint32_t *bn = tb.binom;
    int sigma;
    uint32_t cl;
    seed_of(bn, bv, s, &sigma, &cl);
    const int tr = d - sigma;
    const double *src = Y1 + gg.y1off[v] + y1_at(s, (uint64_t)Ht << a, hv, gg.kg4[v]);
    const uint32_t st = y1_stride(s, gg.kg4[v]);
    double *dst = Y2 + gg.y2off[v];
    auto out_at = [&](uint32_t pi) -> double & { return dst[(((size_t)s * KA + pi) << hB) + Ht]; };
    double g[16];
    double mx = -__builtin_huge_val();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        g[r] = src[(size_t)((t << 4) | r) * st];
        mx = fmax(mx, g[r]);
    }
    mx = block_reduce(mx, red, [](double x, double y) { return fmax(x, y); });
    if (!(mx > -1e300)) {                            // an empty row: every output is zero
        for (uint32_t pi = t; pi < KA; pi += kThreads) out_at(pi) = -__builtin_huge_val();
        return;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) g[r] = g[r] > -1e300 ? ldexp(exp(g[r] - mx), 960) : 0.0;
    dense_zeta_down12_regs<Lin64>(g, vec, t);
    bool small = false;
    for (uint32_t pi = t; pi < KA; pi += kThreads) {
        const uint32_t x = tb.pat[pi];
        if (__popc(x) <= tr) small = small || !(vec[padx(x)] >= 0x1p-1000);
    }
    if (!__syncthreads_or(small || force_trunc ? 1 : 0)) {
        const double off = mx - 960.0 * 0.69314718055994530942;
        for (uint32_t pi = t; pi < KA; pi += kThreads) {
            const double y = vec[padx(tb.pat[pi])];
            out_at(pi) = y > 0.0 ? log(y) + off : -__builtin_huge_val();
        }
        return;
    }
    // the truncated log-add pass of k_gamma_highA
    for (uint32_t x = t; x < (1u << a); x += kThreads) vec[x] = src[(size_t)x * st];
    __syncthreads();
    for (int j = 0; j < a; ++j) {
        const uint32_t cntj = Kcount(bn, j, d);
        const uint32_t tot = cntj << (a - 1 - j);
        for (uint32_t idx = t; idx < tot; idx += kThreads) {
            const uint32_t hi = idx / cntj;
            const uint32_t p = tb.pat[idx - hi * cntj];
            if (__popc(p) > tr) continue;
            const uint32_t Tm = (hi << (j + 1)) | p;
            vec[Tm] = PolLog::add(vec[Tm], vec[Tm | (1u << j)]);
        }
        __syncthreads();
    }
    for (uint32_t pi = t; pi < KA; pi += kThreads) out_at(pi) = vec[tb.pat[pi]];
}

// Level A for a = 12, FP32-scaled form: the outputs of k_gamma_highA from
// the dense zeta, over groups of ranks.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_gamma_highA12(int n, uint32_t KA, GammaGeom gg, Tables tb, const X32 *__restrict__ Y1,
                   X32 *__restrict__ Y2) {
    extern __shared__ unsigned char smem[];
    X32 *vec = reinterpret_cast<X32 *>(smem);   // 2^12 entries at padx indices
    const int v = find_v(gg.blkAx4, n, blockIdx.x);
    const int hB = gg.hv[v] - 12;
    const uint32_t t = threadIdx.x;
    X32 *dst = Y2 + gg.y2off[v];
    dense_zeta_down12_x4(Y1 + gg.y1off[v], gg.hv[v], hB, gg.kg4[v], blockIdx.x - gg.blkAx4[v],
                         vec, t, [&](uint32_t s, uint32_t Ht) {
                             for (uint32_t pi = t; pi < KA; pi += kThreads)
                                 dst[(((size_t)s * KA + pi) << hB) + Ht] = vec[padx(tb.pat[pi])];
                         });
}

// One level with hv = 12 (every one-level endpoint when n = 25), FP32-scaled
// form: the outputs of k_gamma_high1 from the dense zeta, over groups of ranks.
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_gamma_high1_12(int n, int d, uint32_t K, GammaGeom gg, Tables tb,
                    const X32 *__restrict__ Y1, X32 *__restrict__ gam) {
    extern __shared__ unsigned char smem[];
    X32 *vec = reinterpret_cast<X32 *>(smem);   // 2^12 entries at padx indices
    const int N = n - 1;
    const int v = find_v(gg.blk1x4, n, blockIdx.x);
    const uint32_t t = threadIdx.x;
    const uint32_t *bn = tb.binom;
    const int bv = gg.bv[v];
    const uint32_t npat = Kcount(bn, 12, d);
    dense_zeta_down12_x4(Y1 + gg.y1off[v], 12, 0, gg.kg4[v], blockIdx.x - gg.blk1x4[v], vec, t,
                         [&](uint32_t s, uint32_t) {
                             int sigma;
                             uint32_t cl;
                             seed_of(bn, bv, s, &sigma, &cl);
                             const int tr = d - sigma;
                             for (uint32_t idx = t; idx < npat; idx += kThreads) {
                                 const uint32_t x = tb.pat[idx];
                                 if (__popc(x) > tr) continue;
                                 gam[(size_t)v * K + out_rank(bn, N, sigma, cl, x, bv)] =
                                     vec[padx(x)];
                             }
                         });
}

// Level B, workgroup (v, seed): for each a-bit pattern p and each output
// pattern y over the remaining hB bits, the superset sum over y' of y. With
// hB <= 6 a wave takes 64 / 2^hB patterns p at a time, 2^hB lanes each: lane
// y of a pattern loads entry y of its row (coalesced loads) and the downward
// zeta over the hB bits runs across those lanes by shuffles. Larger hB
// (n = 31) sums each output's supersets in turn.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_gamma_highB(int n, int d, int a, uint32_t KA, uint32_t K, GammaGeom gg, Tables tb,
              const typename P::V *__restrict__ Y2, typename P::V *__restrict__ gam) {
    using V = typename P::V;
    const int N = n - 1;
    const int v = find_v(gg.blkB, n, blockIdx.x);
    const uint32_t s = blockIdx.x - gg.blkB[v];
    const int bv = gg.bv[v], hv = gg.hv[v];
    const int hB = hv - a;
    const int t = threadIdx.x;
    const uint32_t *bn = tb.binom;
    int sigma;
    uint32_t cl;
    seed_of(bn, bv, s, &sigma, &cl);
    const int tr = d - sigma;
    const uint32_t ny = 1u << hB;
    const V *base = Y2 + gg.y2off[v];
    if (hB <= 6) {
        // lane = (pattern slot, y): 64 / 2^hB patterns per wave step
        const uint32_t lane = t & 63, y = lane & (ny - 1), sub = lane >> hB;
        const uint32_t ppw = 64u >> hB;
        for (uint32_t p0 = (t >> 6) * ppw; p0 < KA; p0 += (kThreads / 64) * ppw) {
            const uint32_t pi = p0 + sub;
            const uint32_t p = pi < KA ? tb.pat[pi] : 0u;
            const int pp = __popc(p);
            const bool need = pi < KA && pp <= tr;
            V x = need ? base[(((size_t)s * KA + pi) << hB) + y] : P::zero();
            for (int b = 0; b < hB; ++b) {
                const V o = shfl_xor_v(x, 1 << b);
                if (!((y >> b) & 1)) x = P::add(x, o);
            }
            if (need && pp + __popc(y) <= tr)
                gam[(size_t)v * K + out_rank(bn, N, sigma, cl, p | (y << a), bv)] = x;
        }
        return;
    }
    for (uint32_t idx = t; idx < KA * ny; idx += kThreads) {
        const uint32_t pi = idx / ny;
        const uint32_t y = idx - pi * ny;
        const uint32_t p = tb.pat[pi];
        if (__popc(p) + __popc(y) > tr) continue;
        const V *src = base + (((size_t)s * KA + pi) << hB);
        typename P::Acc acc = P::acc_of(P::zero());
        const uint32_t free_bits = (ny - 1) & ~y;
        uint32_t sub = 0;   // all supersets y | sub, sub a submask of free_bits, ascending
        while (true) {
            P::acc_add(acc, src[y | sub]);
            if (sub == free_bits) break;
            sub = (sub - free_bits) & free_bits;
        }
        gam[(size_t)v * K + out_rank(bn, N, sigma, cl, p | (y << a), bv)] = P::acc_value(acc);
    }
}

// ------------------------------------------------------------ a7: edges
// Workgroup (v, j): w_v(G) = beta_v(G) Gamma_v(G). j = 0: sum_G w_v(G)
// against L(V) (the residual) and, when asked for, the parent-set
// posteriors w_v(G) / L(V); j = u + 1: P(u->v) = sum_{G containing u}
// w_v(G) / L(V), the last division in FP64.
template <class P>
__global__ void __launch_bounds__(kThreads)
k_edges(int n, uint32_t K, const uint32_t *__restrict__ famask,
        const typename P::V *__restrict__ beta, const typename P::V *__restrict__ gam,
        typename P::Store L, double *__restrict__ post, double *__restrict__ resid,
        double *__restrict__ ps) {
    using V = typename P::V;
    __shared__ V red[kThreads];
    const int v = blockIdx.x;
    const int u = (int)blockIdx.y - 1;
    const int t = threadIdx.x;
    if (u == v) {
        if (t == 0) post[(size_t)u * n + v] = 0.0;
        return;
    }
    const V LV = P::load(L, (1ull << n) - 1);
    auto add = [](V a, V b) { return P::add(a, b); };
    // parent-set posteriors P(G_v = G | D) = w_v(G) / L(V), when asked for
    if (ps && u < 0) {
        for (uint32_t r = t; r < K; r += kThreads) {
            const double lr =
                P::log_ratio(P::mul(beta[(size_t)v * K + r], gam[(size_t)v * K + r]), LV);
            ps[(size_t)v * K + r] = (lr > -1e300) ? exp(lr) : 0.0;
        }
    }
    const int pu = u < v ? u : u - 1;
    typename P::Acc acc = P::acc_of(P::zero());
    for (uint32_t r = t; r < K; r += kThreads) {
        if (u >= 0 && !((famask[r] >> pu) & 1)) continue;
        P::acc_add(acc, P::mul(beta[(size_t)v * K + r], gam[(size_t)v * K + r]));
    }
    const V tot = block_reduce(P::acc_value(acc), red, add);
    if (t == 0) {
        const double lr = P::log_ratio(tot, LV);
        if (u < 0) resid[v] = fabs(lr);
        else post[(size_t)u * n + v] = (lr > -1e300) ? exp(lr) : 0.0;
    }
}

// -------------------------------------------------------- invariants
// Per tile H (blockIdx.x) and in-tile layer l (blockIdx.y): sum of
// L(S) Rp(S); then per layer k of the whole lattice. Every layer sum must
// equal L(V).
template <class P>
__global__ void __launch_bounds__(kThreads)
k_inv1(int n, int bL, Tables tb, typename P::Store L, typename P::Store R,
       typename P::V *__restrict__ part) {
    using V = typename P::V;
    __shared__ V red[kThreads];
    const uint64_t Hf = (uint64_t)blockIdx.x << bL;
    const int l = blockIdx.y;
    const int t = threadIdx.x;
    auto add = [](V a, V b) { return P::add(a, b); };
    V acc = P::zero();
    for (uint32_t idx = tb.loff[l] + t; idx < tb.loff[l + 1]; idx += kThreads) {
        const uint64_t S = Hf | tb.lorder[idx];
        acc = P::add(acc, P::mul(P::load(L, S), P::load(R, S)));
    }
    V s = block_reduce(acc, red, add);
    if (t == 0) part[(size_t)blockIdx.x * (bL + 1) + l] = s;
}

// Workgroup (k, c): the layer-k sum over the c-th of kInvChunks ranges of
// tiles, to layer[k * kInvChunks + c]; k_finalize adds the ranges in order.
constexpr int kInvChunks = 32;
template <class P>
__global__ void __launch_bounds__(kThreads)
k_inv2(int n, int bL, const typename P::V *__restrict__ part, typename P::V *__restrict__ layer) {
    using V = typename P::V;
    __shared__ V red[kThreads];
    const int k = blockIdx.x;
    const int c = blockIdx.y;
    const int t = threadIdx.x;
    const uint32_t ntile = 1u << (n - bL);
    const uint32_t per = (ntile + kInvChunks - 1) / kInvChunks;
    const uint32_t h0 = c * per, h1 = min(ntile, h0 + per);
    auto add = [](V a, V b) { return P::add(a, b); };
    V acc = P::zero();
    for (uint32_t H = h0 + t; H < h1; H += kThreads) {
        const int l = k - __popc(H);
        if (l < 0 || l > bL) continue;
        acc = P::add(acc, part[(size_t)H * (bL + 1) + l]);
    }
    V s = block_reduce(acc, red, add);
    if (t == 0) layer[k * kInvChunks + c] = s;
}

// diag: [0] log L(V), [1] max residual, [2] saturated, [3] flushed,
//       [4] |log Rp(0) - log L(V)|, [5] max layer residual, [6] max edge-sum residual
template <class P>
__global__ void k_finalize(int n, typename P::Store L, typename P::Store R,
                           const typename P::V *__restrict__ layer,
                           const double *__restrict__ resid, const double *__restrict__ gauge_exp,
                           const unsigned long long *__restrict__ cnt,
                           const uint32_t *__restrict__ fbA, const uint32_t *__restrict__ fbG,
                           double *__restrict__ diag) {
    using V = typename P::V;
    const int t = threadIdx.x;
    const V LV = P::load(L, (1ull << n) - 1);
    // lane k sums layer k's chunks in order; the largest deviation over the
    // wave (one wave of 64 lanes, n + 1 <= 32 layers)
    double rl = 0.0;
    if (t <= n) {
        V lk = layer[t * kInvChunks];
        for (int c = 1; c < kInvChunks; ++c) lk = P::add(lk, layer[t * kInvChunks + c]);
        rl = fabs(P::log_ratio(lk, LV));
    }
    for (int o = 32; o > 0; o >>= 1) rl = fmax(rl, __shfl_xor(rl, o));
    if (t != 0) return;
    double g = 0.0;
    for (int k = 0; k < 2 * n; ++k) g += gauge_exp[k];
    const double rLR = fabs(P::log_ratio(P::load(R, 0), LV));
    double re = 0.0;
    for (int v = 0; v < n; ++v) re = fmax(re, resid[v]);
    diag[0] = P::to_log(LV) + g * 0.69314718055994530942;
    diag[1] = fmax(rLR, fmax(rl, re));
    diag[2] = (double)cnt[0];
    diag[3] = (double)cnt[1];
    diag[4] = rLR;
    diag[5] = rl;
    diag[6] = re;
    diag[7] = (double)((fbA ? fbA[0] : 0u) + (fbG ? fbG[0] : 0u));
}

// Forward-only runs (modular features): diag[0] = log L(V) with the gauges,
// [2] / [3] the saturation and flush counts, [7] the fallback tiles; the
// invariant entries are 0 (no backward sweep to check against).
template <class P>
__global__ void k_log_LV(int n, typename P::Store L, const double *__restrict__ gauge_exp,
                         const unsigned long long *__restrict__ cnt,
                         const uint32_t *__restrict__ fbA, double *__restrict__ diag) {
    if (threadIdx.x != 0) return;
    double g = 0.0;
    for (int k = 0; k < 2 * n; ++k) g += gauge_exp[k];
    diag[0] = P::to_log(P::load(L, (1ull << n) - 1)) + g * 0.69314718055994530942;
    diag[1] = diag[4] = diag[5] = diag[6] = 0.0;
    diag[2] = (double)cnt[0];
    diag[3] = (double)cnt[1];
    diag[7] = (double)(fbA ? fbA[0] : 0u);
}

__global__ void k_add_log(double *__restrict__ logp, const double *__restrict__ log_f,
                          size_t count) {
    for (size_t x = (size_t)blockIdx.x * kThreads + threadIdx.x; x < count;
         x += (size_t)gridDim.x * kThreads)
        logp[x] += log_f[x];
}

hipError_t launch_add_log(double *logp, const double *log_f, size_t count, hipStream_t st) {
    const unsigned g = (unsigned)std::min<size_t>((count + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_add_log, dim3(std::max(g, 1u)), dim3(kThreads), 0, st, logp, log_f,
                       count);
    return hipGetLastError();
}

// ------------------------------------------- a1: local scores, binary data
// All-binary data as two bit planes per variable: plane 1 marks the samples
// with value 1, plane 0 those with value 0 (a value out of range is in
// neither, and so ignored, as in k_scores). W 32-bit words per plane.
__global__ void k_pack2(int n, int m, int W, const uint8_t *__restrict__ data,
                        uint32_t *__restrict__ bits) {
    const uint32_t id = blockIdx.x * kThreads + threadIdx.x;
    if (id >= (uint32_t)(n * W)) return;
    const int j = id / W, w = id % W;
    uint32_t one = 0, zero = 0;
    for (int b = 0; b < 32; ++b) {
        const int s = w * 32 + b;
        if (s >= m) break;
        const uint8_t x = data[(size_t)j * m + s];
        one |= (uint32_t)(x == 1) << b;
        zero |= (uint32_t)(x == 0) << b;
    }
    bits[((size_t)j * 2 + 1) * W + w] = one;
    bits[((size_t)j * 2 + 0) * W + w] = zero;
}

// One step of count_cells2's butterfly, at lane bit B.
template <int KP, int B>
__device__ inline void count_scatter(uint32_t *cnt, int lane) {
    constexpr int sft = 1 << B;
    if constexpr (B >= KP) {
#pragma unroll
        for (int c = 0; c < (2 << KP); ++c) cnt[c] += __shfl_xor(cnt[c], sft, 16);
    } else {
        // held: the 2^(B+1) configurations agreeing with the lane above bit
        // B, counts at 2 * (configuration mod 2^(B+1)) + v
        constexpr int half = 2 << B;
        const bool up = (lane >> B) & 1;
#pragma unroll
        for (int c = 0; c < half; ++c) {
            const uint32_t keep = up ? cnt[c + half] : cnt[c];
            const uint32_t send = up ? cnt[c] : cnt[c + half];
            cnt[c] = keep + __shfl_xor(send, sft, 16);
        }
    }
}

// Counts of one family of k parents over words w = lane, lane + 16, ...:
// cell (c << 1) | v, c the parents' values as bits, v the child's value, is
// the popcount of the AND of the matching planes. The 16 lanes' partial
// counts are then summed and scattered by a butterfly that, at lane bit b,
// halves the configurations a lane keeps by configuration bit b (b < k), or
// sums all it holds (b >= k): lane L < 2^k ends with the two counts of
// configuration L in cnt[0] and cnt[1].
template <int KP>
__device__ inline void count_cells2(const uint32_t *__restrict__ bits, int W, int lane,
                                    int child, const int *par, uint32_t *cnt) {
    constexpr int NC = 2 << KP;
#pragma unroll
    for (int c = 0; c < NC; ++c) cnt[c] = 0;
    for (int w = lane; w < W; w += 16) {
        uint32_t a[NC];
        a[0] = bits[((size_t)child * 2 + 0) * W + w];
        a[1] = bits[((size_t)child * 2 + 1) * W + w];
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const uint32_t p0 = bits[((size_t)par[j] * 2 + 0) * W + w];
            const uint32_t p1 = bits[((size_t)par[j] * 2 + 1) * W + w];
            const int half = 2 << j;
#pragma unroll
            for (int c = 0; c < NC / 2; ++c) {
                if (c < half) {
                    a[c + half] = a[c] & p1;
                    a[c] = a[c] & p0;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) cnt[c] += __popc(a[c]);
    }
    count_scatter<KP, 3>(cnt, lane);
    count_scatter<KP, 2>(cnt, lane);
    count_scatter<KP, 1>(cnt, lane);
    count_scatter<KP, 0>(cnt, lane);
}

// Log-gamma tables of the score paths for data whose variables all have
// arity r: for k = 0..4 parents (q = r^k configurations),
// lgt[(2k) * (m+1) + c] = lgamma(a_j + c) and lgt[(2k+1) * (m+1) + c] =
// lgamma(a_jk + c), c = 0..m, with the BDeu (a_j = ess / q, a_jk =
// ess / (q r)) or K2 (a_j = r, a_jk = 1) hyperparameters.
__global__ void k_lgamma_table(int m, int r, int kind, double ess, double *__restrict__ lgt) {
    const int m1 = m + 1;
    for (int x = blockIdx.x * kThreads + threadIdx.x; x < 10 * m1; x += gridDim.x * kThreads) {
        const int row = x / m1, c = x - row * m1, k = row >> 1;
        int qi = 1;
        for (int j = 0; j < k; ++j) qi *= r;
        const double a = (row & 1) ? (kind == 0 ? ess / ((double)qi * r) : 1.0)
                                   : (kind == 0 ? ess / qi : (double)r);
        lgt[x] = lgamma(a + c);
    }
}

// BDeu / K2 log marginal likelihood of one family from its cell counts
// (all variables binary: q = 2^k configurations, r = 2 values); lane L < q
// takes configuration L (the counts count_cells2 left it), partial sums met
// by a fixed butterfly. The log-gamma values come from the tables of
// k_lgamma_table.
template <int KP>
__device__ inline double family_score2(const uint32_t *cnt, int lane, const double *lgt,
                                       int m1) {
    constexpr int Q = 1 << KP;
    const double *lj = lgt + (2 * KP) * m1, *ljk = lgt + (2 * KP + 1) * m1;
    const double lg_aj = lj[0], lg_ajk = ljk[0];
    double acc = 0.0;
    if (lane < Q) {
        const uint32_t c0 = cnt[0], c1 = cnt[1];
        const uint32_t nj = c0 + c1;
        if (nj) {
            double s = lg_aj - lj[nj];
            if (c0) s += ljk[c0] - lg_ajk;
            if (c1) s += ljk[c1] - lg_ajk;
            acc += s;
        }
    }
    for (int sft = 8; sft > 0; sft >>= 1) acc += __shfl_xor(acc, sft, 16);
    return acc;
}

// Local scores of all-binary data with d <= 4: 16 lanes per family, 16
// families per workgroup, counts from the bit planes of k_pack2.
__global__ void __launch_bounds__(kThreads)
k_scores2(int n, int W, int m, uint32_t K, const uint32_t *__restrict__ famask,
          const uint32_t *__restrict__ bits, const double *__restrict__ lgt,
          double *__restrict__ out) {
    const int g = threadIdx.x >> 4, lane = threadIdx.x & 15;
    const uint32_t fam = blockIdx.x * 16 + g;
    if (fam >= (uint32_t)n * K) return;      // whole 16-lane groups leave together
    const int i = fam / K;
    const uint32_t r = fam % K;
    const uint32_t msk = famask[r];
    int par[4];
    int k = 0;
    for (int p = 0; p < 31 && k < 4; ++p)
        if ((msk >> p) & 1) par[k++] = p < i ? p : p + 1;
    uint32_t cnt[32];
    double sc = 0.0;
    switch (k) {
        case 0: count_cells2<0>(bits, W, lane, i, par, cnt); sc = family_score2<0>(cnt, lane, lgt, m + 1); break;
        case 1: count_cells2<1>(bits, W, lane, i, par, cnt); sc = family_score2<1>(cnt, lane, lgt, m + 1); break;
        case 2: count_cells2<2>(bits, W, lane, i, par, cnt); sc = family_score2<2>(cnt, lane, lgt, m + 1); break;
        case 3: count_cells2<3>(bits, W, lane, i, par, cnt); sc = family_score2<3>(cnt, lane, lgt, m + 1); break;
        default: count_cells2<4>(bits, W, lane, i, par, cnt); sc = family_score2<4>(cnt, lane, lgt, m + 1); break;
    }
    if (lane == 0) out[fam] = sc;
}

// -------------------------------------------------------------- launchers
// Raise a kernel's dynamic LDS limit to what a workgroup may hold (the
// device's per-block maximum less the kernel's static LDS), once per kernel
// and process: the limit is an upper bound only, the launch size decides the
// allocation, and no launch pays for the call.
template <auto Kernel>
static void allow_big_lds() {
    static const bool once = [] {
        int dev = 0, mx = 0;
        hipFuncAttributes fa{};
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&mx, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) ==
                hipSuccess &&
            hipFuncGetAttributes(&fa, (const void *)Kernel) == hipSuccess)
            (void)hipFuncSetAttribute((const void *)Kernel,
                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                      mx - (int)fa.sharedSizeBytes);
        (void)hipGetLastError();
        return true;
    }();
    (void)once;
}

#define BN_CHECK_LAUNCH() \
    do {                                                   \
        hipError_t e_ = hipGetLastError();                 \
        if (e_ != hipSuccess) return e_;                   \
    } while (0)

hipError_t launch_setup(const Tables &tb, int bL, int W, int bG, int bA, int d, uint32_t N,
                        uint32_t K, hipStream_t st) {
    static const struct OrdTable {
        LaneOrder o[9];
        OrdTable() {
            for (int d = 0; d <= 8; ++d) o[d] = lane_order_c(d);
        }
    } ord_tables;
    auto blocks = [](uint64_t count) { return (uint32_t)((count + kThreads - 1) / kThreads); };
    // range S: one workgroup per 256 masks of its largest table
    const int wmax = std::max(std::max(bL, W), bG);
    TableGrid g;
    g.s = std::max(1, (1 << wmax) / kThreads);
    g.a = g.s + blocks(1ull << bA);
    g.i = g.a + blocks(1ull << (N - bA));
    g.f = g.i + blocks(K);
    g.h = g.f + blocks(1ull << (N + 1 - bL));
    hipLaunchKernelGGL(k_tables, dim3(g.h), dim3(kThreads), 0, st, tb,
                       ord_tables.o[std::min(std::max(d, 0), 8)], g, bL, W, bG, bA, d, (int)N, K);
    BN_CHECK_LAUNCH();
    return hipSuccess;
}

uint32_t hord_offset(int nh, int h) {
    uint64_t s = 0, c = 1;
    for (int k = 0; k < h; ++k) {
        s += c;
        c = c * (uint64_t)(nh - k) / (uint64_t)(k + 1);
    }
    return (uint32_t)s;
}

hipError_t launch_scores(int n, int m, const uint8_t *data, const uint8_t *arity, uint32_t K,
                         int kind, double ess, const uint32_t *famask, int max_bins,
                         double *out, hipStream_t st, uint32_t *bits, int uniform_r,
                         double *lgt) {
    const dim3 tgrid((unsigned)std::min((10 * (m + 1) + kThreads - 1) / kThreads, 1024));
    if (bits) {
        // all-binary data, d <= 4: counts from bit planes
        const int W = (m + 31) / 32;
        hipLaunchKernelGGL(k_pack2, dim3((unsigned)((n * W + kThreads - 1) / kThreads)),
                           dim3(kThreads), 0, st, n, m, W, data, bits);
        BN_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_lgamma_table, tgrid, dim3(kThreads), 0, st, m, 2, kind, ess, lgt);
        BN_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_scores2, dim3((unsigned)((n * K + 15) / 16)), dim3(kThreads), 0, st,
                           n, W, m, K, famask, (const uint32_t *)bits, (const double *)lgt, out);
        BN_CHECK_LAUNCH();
        return hipSuccess;
    }
    if (max_bins <= kScoreWaveBins) {
        const double *tab = nullptr;
        if (uniform_r > 0) {
            hipLaunchKernelGGL(k_lgamma_table, tgrid, dim3(kThreads), 0, st, m, uniform_r, kind,
                               ess, lgt);
            BN_CHECK_LAUNCH();
            tab = lgt;
        }
        hipLaunchKernelGGL(k_scores_w, dim3((unsigned)((n * (uint64_t)K + 3) / 4)), dim3(kThreads),
                           (size_t)4 * max_bins * sizeof(int), st, n, m, data, arity, K, kind, ess,
                           famask, max_bins, tab, out);
    } else
        hipLaunchKernelGGL(k_scores, dim3((unsigned)(n * K)), dim3(kThreads),
                           (size_t)max_bins * sizeof(int), st, n, m, data, arity, K, kind, ess,
                           famask, out);
    BN_CHECK_LAUNCH();
    return hipSuccess;
}

// sum_{k <= t} C(w, k) on the host (0 for t < 0)
static uint32_t host_kcount(int w, int t) {
    uint64_t sum = 0, c = 1;
    for (int k = 0; k <= t && k <= w; ++k) {
        sum += c;
        c = c * (uint64_t)(w - k) / (uint64_t)(k + 1);
    }
    return (uint32_t)sum;
}

template <class P>
static hipError_t launch_gamma_edges(const LatticeArgs &a, const typename P::Store &L,
                                     const typename P::Store &R, hipStream_t st,
                                     PhaseEvents *ev);
static hipError_t launch_lattice_fused(const LatticeArgs &a, const PolX32::Store &L,
                                       const PolX32::Store &R, hipStream_t st,
                                       PhaseEvents *ev);

// Fork of a second stream off the solve's stream and its join: two events
// (no timing), destroyed when the helper goes out of scope (HIP releases an
// event recorded and waited on only after the waits are satisfied).
struct SweepFork {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t open(hipStream_t st, hipStream_t side) {
        hipError_t e = hipEventCreateWithFlags(&e0, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&e1, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(side, e0, 0);
        return e;
    }
    hipError_t join(hipStream_t st, hipStream_t side) {
        hipError_t e = hipEventRecord(e1, side);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, e1, 0);
        return e;
    }
    ~SweepFork() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

template <class P>
hipError_t launch_lattice(const LatticeArgs &a, const typename P::Store &alpha,
                          const typename P::Store &L, const typename P::Store &R,
                          hipStream_t st, PhaseEvents *ev) {
    using V = typename P::V;
    const int n = a.n, N = n - 1, d = a.d;
    const Tables &tb = a.tb;
    V *beta = reinterpret_cast<V *>(a.beta);
    V *qt = reinterpret_cast<V *>(a.qt);
    V *Y1 = reinterpret_cast<V *>(a.Y1);
    V *Y2 = reinterpret_cast<V *>(a.Y2);
    V *gam = reinterpret_cast<V *>(a.gam);
    V *part = reinterpret_cast<V *>(a.part);
    V *layer = reinterpret_cast<V *>(a.layer);
    auto rec = [&](int idx) {
        if (ev && ev->ev[idx]) (void)hipEventRecord(ev->ev[idx], st);
    };
    hipLaunchKernelGGL(k_prep<P>, dim3(n, (a.K + kPrepChunk - 1) / kPrepChunk), dim3(kThreads),
                       0, st, n, d, a.K,
                       (const uint32_t *)tb.binom, (const double *)a.logp,
                       (const double *)a.log_rho, (const double *)a.log_q, a.gauge, beta, qt,
                       a.gauge_exp, a.fbA, a.fbG, a.rtG);
    BN_CHECK_LAUNCH();
    rec(1);
    if constexpr (std::is_same<P, PolX32>::value) {
        if (a.fused) return launch_lattice_fused(a, L, R, st, ev);
    }
    if (a.bA == 13) {
        const uint32_t nit = (uint32_t)a.nitA;
        // the partial-rank table is used when ranks fit 16 bits and it fits 12 KB
        const int use_prk = (a.K < 65536u && (size_t)(d + 1) * nit * 2 <= 12288) ? 1 : 0;
        const size_t sm = sizeof(V) * (8192 + 256) + 33 * 33 * 4 +
                          (use_prk ? (size_t)(d + 1) * nit * 2 : 0);
        const unsigned nblkA = (unsigned)(n << (N - 13));
        if (a.lin_mode && a.Zs) {
            using A = typename P::Anchor;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_prep_lin<P>), dim3(n), dim3(kThreads), 0, st, n,
                               a.K, (const V *)beta, a.betal, (A *)a.anc, a.linok, nullptr);
            BN_CHECK_LAUNCH();
            // block-wise seeds: 2^bS tiles per workgroup, 4 <= bS <= 8, with at
            // least 4 high bits left so that the grid holds n * 16 workgroups
            const int hA = N - 13, bS = hA - 4 < 8 ? hA - 4 : 8;
            const uint32_t nhiMax = bS >= 4 ? host_kcount(hA - bS, d) : 0u;
            if (a.KS > 0 && bS >= 4 && d <= 7 && (size_t)(d + 1) * nhiMax <= 4096) {
                const size_t smB = 8 * (4096 + 256) + 33 * 33 * 4 + (size_t)(d + 1) * nhiMax * 4;
                // few blocks of tiles (n < 26): their chunks of seed ranks
                // spread over more workgroups
                const unsigned nbS = (unsigned)(n << (hA - bS));
                const unsigned ySplit = std::min((a.KS + 15) / 16, std::max(1u, 2048u / nbS));
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha_seeds_blk<P>),
                                   dim3(nbS, ySplit), dim3(kThreads), smB, st, n,
                                   d, a.K, a.KS, bS, nhiMax, tb, (const double *)a.betal,
                                   (const int *)a.linok, a.Zs);
            } else if (a.KS > 0) {
                const size_t smS = 33 * 33 * 4 + (use_prk ? (size_t)(d + 1) * nit * 2 + nit : 0);
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha_seeds<P>), dim3(nblkA), dim3(kThreads),
                                   smS, st, n, d, a.K, a.KS, use_prk, tb, (const double *)a.betal,
                                   (const int *)a.linok, a.Zs);
            }
            BN_CHECK_LAUNCH();
            const size_t smL = 8 * (4096 + 256);
            allow_big_lds<k_alpha_lin<P>>();
            rec(8);
            // 2^tl tiles per workgroup share its set-up (tables in LDS, the
            // colex terms of the thread's pattern)
            // (tl < hA keeps the shift count nonnegative: at n = 14 there
            // is a single tile per node and tl stays 0)
            int tl = 0;
            while (tl < 6 && tl < hA && ((uint64_t)n << (hA - tl - 1)) >= 4096) ++tl;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha_lin<P>), dim3(nblkA >> tl), dim3(kThreads), smL,
                               st, n, d, a.KS, a.lin_mode == 2 ? 1 : 0, tl, (const double *)a.Zs,
                               (const double *)a.betal, a.K,
                               host_kcount(N, d - 1), (const A *)a.anc, (const int *)a.linok, (const V *)qt, alpha,
                               a.cnt, a.fbA);
            BN_CHECK_LAUNCH();
            rec(9);
            // tiles the linear form could not hold: a grid that walks the list
            allow_big_lds<k_alpha_fb<P>>();
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha_fb<P>), dim3(std::min(nblkA, 1024u)),
                               dim3(kThreads), sm, st, n, d, a.K, use_prk, tb, (const V *)beta,
                               (const V *)qt, alpha, a.cnt, (const uint32_t *)a.fbA);
        } else {
            allow_big_lds<k_alpha<P>>();
            rec(8);
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha<P>), dim3(nblkA), dim3(kThreads), sm, st,
                               n, d, a.K, use_prk, tb, (const V *)beta, (const V *)qt, alpha,
                               a.cnt);
            BN_CHECK_LAUNCH();
            rec(9);
        }
    } else {
        rec(8);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha_small<P>), dim3((unsigned)n), dim3(kThreads),
                           sizeof(V) << N, st, n, d, a.K, tb, (const V *)beta, (const V *)qt,
                           alpha, a.cnt);
        BN_CHECK_LAUNCH();
        rec(9);
    }
    BN_CHECK_LAUNCH();
    rec(2);
    const int nh = n - a.bL;
    const size_t smL = align16(SliceLds<P>::bytes_per_entry * ((size_t)a.bL << (a.bL - 1))) +
                       sizeof(V) * ((size_t)1 << a.bL) + 2 * ((size_t)1 << a.bL);
    // The backward sweep needs alpha but not L: with a.side set it runs on that
    // stream, forked after alpha and joined before Gamma, so that its small
    // layers overlap the forward sweep's.
    SweepFork fork;
    hipStream_t sb = st;
    if (a.side && !a.fwd_only) {
        const hipError_t e = fork.open(st, a.side);
        if (e != hipSuccess) return e;
        sb = a.side;
    }
    for (int h = 0; h <= nh; ++h) {
        const unsigned nb = a.tiles_per_layer[h];
        hipLaunchKernelGGL(k_fwd<P>, dim3(nb), dim3(kThreads), smL, st, n, a.bL, h,
                           hord_offset(nh, h), tb, alpha, L, a.cnt);
        BN_CHECK_LAUNCH();
    }
    rec(3);
    if (a.fwd_only) {
        hipLaunchKernelGGL(k_log_LV<P>, dim3(1), dim3(64), 0, st, n, L,
                           (const double *)a.gauge_exp, (const unsigned long long *)a.cnt,
                           (const uint32_t *)a.fbA, a.diag);
        BN_CHECK_LAUNCH();
        rec(6);
        return hipSuccess;
    }
    for (int h = nh; h >= 0; --h) {
        const unsigned nb = a.tiles_per_layer[h];
        hipLaunchKernelGGL(k_bwd<P>, dim3(nb), dim3(kThreads), smL, sb, n, a.bL, h,
                           hord_offset(nh, h), tb, alpha, R, a.cnt);
        BN_CHECK_LAUNCH();
    }
    if (sb != st) {
        const hipError_t e = fork.join(st, sb);
        if (e != hipSuccess) return e;
    }
    rec(4);
    return launch_gamma_edges<P>(a, L, R, st, ev);
}

// Gamma (Eq. 12), edges (Eq. 11) and the invariants, after both sweeps.
template <class P>
static hipError_t launch_gamma_edges(const LatticeArgs &a, const typename P::Store &L,
                                     const typename P::Store &R, hipStream_t st,
                                     PhaseEvents *ev) {
    using V = typename P::V;
    const int n = a.n, d = a.d;
    const int nh = n - a.bL;
    const Tables &tb = a.tb;
    V *beta = reinterpret_cast<V *>(a.beta);
    V *qt = reinterpret_cast<V *>(a.qt);
    V *Y1 = reinterpret_cast<V *>(a.Y1);
    V *Y2 = reinterpret_cast<V *>(a.Y2);
    V *gam = reinterpret_cast<V *>(a.gam);
    V *part = reinterpret_cast<V *>(a.part);
    V *layer = reinterpret_cast<V *>(a.layer);
    auto rec = [&](int idx) {
        if (ev && ev->ev[idx]) (void)hipEventRecord(ev->ev[idx], st);
    };
    {
        const GammaGeom &gg = a.gg;
        if (a.bG == 12) {
            const size_t sm = sizeof(V) * (4096 + 256) + 33 * 33 * 4 + (size_t)gg.KT * 4;
            const unsigned nblkG = 1u << (n - 12);
            allow_big_lds<k_gamma_tile<P>>();
            if (a.lin_mode) {
                // few tiles: their endpoints are split over several
                // workgroups, so that about 512 run (a larger target, 1536,
                // made n = 22 slower: the split form spills more registers
                // and repeats the tile's set-up)
                const unsigned vsplit =
                    std::min((unsigned)n, std::max(1u, (512u + nblkG - 1) / nblkG));
                if (vsplit > 1) {
                    allow_big_lds<k_gamma_tile_lin<P, true>>();
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gamma_tile_lin<P, true>),
                                       dim3(nblkG * vsplit), dim3(kThreads), sm, st, n, d,
                                       a.lin_mode == 2 ? 1 : 0, (int)vsplit, gg, tb, L, R,
                                       (const V *)qt, Y1, part, a.fbG, a.rtG);
                } else {
                    allow_big_lds<k_gamma_tile_lin<P, false>>();
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gamma_tile_lin<P, false>), dim3(nblkG),
                                       dim3(kThreads), sm, st, n, d, a.lin_mode == 2 ? 1 : 0, 1,
                                       gg, tb, L, R, (const V *)qt, Y1, part, a.fbG, a.rtG);
                }
                BN_CHECK_LAUNCH();
                rec(7);
                allow_big_lds<k_gamma_tile_retry<P>>();
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gamma_tile_retry<P>),
                                   dim3(std::min(nblkG, 1024u)), dim3(kThreads), sm, st, n, d, gg,
                                   tb, L, R, (const V *)qt, Y1, (const uint32_t *)a.rtG, a.fbG);
                BN_CHECK_LAUNCH();
                allow_big_lds<k_gamma_tile_fb<P>>();
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gamma_tile_fb<P>),
                                   dim3(std::min(nblkG, 1024u)), dim3(kThreads), sm, st, n, d, gg,
                                   tb, L, R, (const V *)qt, Y1, part, (const uint32_t *)a.fbG);
            } else {
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gamma_tile<P>), dim3(nblkG), dim3(kThreads),
                                   sm, st, n, d, gg, tb, L, R, (const V *)qt, Y1, part);
            }
        } else {
            const int bT = a.bG;
            const size_t sm = sizeof(V) * ((size_t)1 << bT) + 33 * 33 * 4 + (size_t)gg.KT * 4 +
                              (size_t)gg.npat * 2;
            // a lattice of one tile: one workgroup per endpoint
            const int vsplit = n == bT ? n : 1;
            const dim3 g((1u << (n - bT)) * (unsigned)vsplit);
            const int RB = bT > 8 ? bT - 8 : 0;
#define BN_GTILE(rb)                                                                           \
    allow_big_lds<k_gamma_tile_gen<P, rb>>();                                                  \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gamma_tile_gen<P, rb>), g, dim3(kThreads), sm, st, n, \
                       d, bT, vsplit, gg, tb, L, R, (const V *)qt, Y1)
            switch (RB) {
                case 0: BN_GTILE(0); break;
                case 1: BN_GTILE(1); break;
                case 2: BN_GTILE(2); break;
                default: BN_GTILE(3); break;
            }
#undef BN_GTILE
        }
        BN_CHECK_LAUNCH();
        if (!(a.bG == 12 && a.lin_mode)) rec(7);
        if (gg.blk1[n] > 0) {
            // every one-level endpoint with 12 high bits (n = 25): the dense
            // form, as for level A
            bool all12 = std::is_same<P, PolX32>::value;
            for (int v = 0; v < n && all12; ++v)
                if (gg.blk1[v + 1] > gg.blk1[v]) all12 = gg.hv[v] == 12;
            if constexpr (std::is_same<P, PolX32>::value) {
                if (all12)
                    hipLaunchKernelGGL(k_gamma_high1_12, dim3(gg.blk1x4[n]), dim3(kThreads),
                                       sizeof(V) * (4096 + 256), st, n, d, a.K, gg, tb,
                                       (const V *)Y1, gam);
            }
            if (!all12)
                hipLaunchKernelGGL(k_gamma_high1<P>, dim3(gg.blk1[n]), dim3(kThreads),
                                   sizeof(V) << gg.hmax1, st, n, d, a.K, gg, tb, (const V *)Y1,
                                   gam);
            BN_CHECK_LAUNCH();
        }
        if (gg.blkA[n] > 0) {
            // dense 12-bit form for the FP32-scaled system; the log form keeps the
            // truncated pass (its log-adds are costly enough that the skipped
            // entries matter more than the indexing)
            bool dense = false;
            if constexpr (std::is_same<P, PolX32>::value) {
                if (a.aG == 12) {
                    dense = true;
                    hipLaunchKernelGGL(k_gamma_highA12, dim3(gg.blkAx4[n]), dim3(kThreads),
                                       sizeof(V) * (4096 + 256), st, n, a.KA, gg, tb,
                                       (const V *)Y1, Y2);
                }
            }
            if constexpr (std::is_same<P, PolLog>::value) {
                // plain doubles under a scale, as the linear tiles (off with them)
                if (a.aG == 12 && a.lin_mode != 0) {
                    dense = true;
                    hipLaunchKernelGGL(k_gamma_highA12_log, dim3(gg.blkA[n]), dim3(kThreads),
                                       sizeof(double) * (4096 + 256), st, n, d, a.KA,
                                       a.lin_mode == 2 ? 1 : 0, gg, tb, (const double *)Y1,
                                       (double *)Y2);
                }
            }
            if (!dense)
                hipLaunchKernelGGL(k_gamma_highA<P>, dim3(gg.blkA[n]), dim3(kThreads),
                                   sizeof(V) << a.aG, st, n, d, a.aG, a.KA, gg, tb,
                                   (const V *)Y1, Y2);
            BN_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_gamma_highB<P>, dim3(gg.blkB[n]), dim3(kThreads), 0, st, n, d,
                               a.aG, a.KA, a.K, gg, tb, (const V *)Y2, gam);
            BN_CHECK_LAUNCH();
        }
    }
    rec(5);
    hipLaunchKernelGGL(k_edges<P>, dim3(n, n + 1), dim3(kThreads), 0, st, n, a.K,
                       (const uint32_t *)tb.famask, (const V *)beta, (const V *)gam, L, a.post,
                       a.resid, a.ps);
    BN_CHECK_LAUNCH();
    // layer sums of L(S) Rp(S): partials per tile come from the Gamma tile
    // kernel (12-bit tiles) or from k_inv1 (sweep tiles, small lattices)
    int bI = 12;
    if (a.bG != 12) {
        bI = a.bL;
        hipLaunchKernelGGL(k_inv1<P>, dim3(1u << nh, a.bL + 1), dim3(kThreads), 0, st, n, a.bL,
                           tb, L, R, part);
        BN_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_inv2<P>, dim3(n + 1, kInvChunks), dim3(kThreads), 0, st, n, bI,
                       (const V *)part, layer);
    BN_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_finalize<P>, dim3(1), dim3(64), 0, st, n, L, R, (const V *)layer,
                       (const double *)a.resid, (const double *)a.gauge_exp,
                       (const unsigned long long *)a.cnt, (const uint32_t *)a.fbA,
                       (const uint32_t *)a.fbG, a.diag);
    BN_CHECK_LAUNCH();
    rec(6);
    return hipSuccess;
}

// The FP32-scaled lattice with alpha never materialised: per-node linear
// scales and bounds, the 9-bit block seeds (timer entries 8 and 9 bracket
// them), then the fused sweeps, one launch per layer.
static hipError_t launch_lattice_fused(const LatticeArgs &a, const PolX32::Store &L,
                                       const PolX32::Store &R, hipStream_t st,
                                       PhaseEvents *ev) {
    const int n = a.n;
    auto rec = [&](int idx) {
        if (ev && ev->ev[idx]) (void)hipEventRecord(ev->ev[idx], st);
    };
    FusedArgs f{};
    f.n = n;
    f.d = a.d;
    f.K = a.K;
    f.KS = a.KS9;
    f.offd = host_kcount(n - 1, a.d - 1);
    f.force_slow = a.lin_mode == 2 ? 1 : 0;
    f.zw = a.zw9;
    f.flin = a.flin;
    f.beta = reinterpret_cast<const X32 *>(a.beta);
    f.qt = reinterpret_cast<const X32 *>(a.qt);
    f.betal = a.betal;
    f.anc = reinterpret_cast<const int *>(a.anc);
    f.linok = a.linok;
    f.emax = a.emax;
    f.nslow = a.fbA;
    f.glo = a.glo;
    f.binom = a.tb.binom;
    f.lorder = a.tb.lorder;
    f.loff = a.tb.loff;
    f.hord = a.tb.hord;
    f.cnt = a.cnt;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_prep_lin<PolX32>), dim3(n), dim3(kThreads), 0, st, n,
                       a.K, (const X32 *)a.beta, a.betal, (int *)a.anc, a.linok, a.emax);
    BN_CHECK_LAUNCH();
    rec(8);
    // the alpha tiles' seeds by blocks of 13-bit tiles (doubles, linear-scale
    // nodes), when the grouped kernel applies; the 9-bit seeds come from them
    const double *zs13 = nullptr;
    if (a.Zs && a.KS > 0 && a.lin_mode != 2) {
        const int N = n - 1, d = a.d, hA = N - 13, bS = hA - 4 < 8 ? hA - 4 : 8;
        const uint32_t nhiMax = bS >= 4 ? host_kcount(hA - bS, d) : 0u;
        if (bS >= 4 && d <= 7 && (size_t)(d + 1) * nhiMax <= 4096) {
            const size_t smB = 8 * (4096 + 256) + 33 * 33 * 4 + (size_t)(d + 1) * nhiMax * 4;
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_alpha_seeds_blk<PolX32>),
                               dim3((unsigned)(n << (hA - bS))), dim3(kThreads), smB, st, n, d,
                               a.K, a.KS, bS, nhiMax, a.tb, (const double *)a.betal,
                               (const int *)a.linok, a.Zs);
            BN_CHECK_LAUNCH();
            zs13 = a.Zs;
        }
    }
    {
        const hipError_t e = launch_fused_seeds(f, zs13, a.KS, st);
        if (e != hipSuccess) return e;
    }
    rec(9);
    rec(2);
    const int nh = n - 9;
    for (int h = 0; h <= nh; ++h) {
        const hipError_t e = launch_fused_sweep(f, true, h, a.tiles_per_layer[h], L, st);
        if (e != hipSuccess) return e;
    }
    rec(3);
    if (a.fwd_only) {
        hipLaunchKernelGGL(k_log_LV<PolX32>, dim3(1), dim3(64), 0, st, n, L,
                           (const double *)a.gauge_exp, (const unsigned long long *)a.cnt,
                           (const uint32_t *)a.fbA, a.diag);
        BN_CHECK_LAUNCH();
        rec(6);
        return hipSuccess;
    }
    for (int h = nh; h >= 0; --h) {
        const hipError_t e = launch_fused_sweep(f, false, h, a.tiles_per_layer[h], R, st);
        if (e != hipSuccess) return e;
    }
    rec(4);
    return launch_gamma_edges<PolX32>(a, L, R, st, ev);
}

template hipError_t launch_lattice<PolLog>(const LatticeArgs &, const PolLog::Store &,
                                           const PolLog::Store &, const PolLog::Store &,
                                           hipStream_t, PhaseEvents *);
template hipError_t launch_lattice<PolX32>(const LatticeArgs &, const PolX32::Store &,
                                           const PolX32::Store &, const PolX32::Store &,
                                           hipStream_t, PhaseEvents *);

}  // namespace bnk
