// Forward and backward sweeps (Eqs. 9 and 10) of the FP32-scaled form with
// alpha never materialised: every sweep tile rebuilds the alpha blocks it
// multiplies from compressed seeds, so the n 2^(n-1) entries of alpha are
// neither written to nor read from HBM.
//
// Seeds. Node i's lattice (the n-1 other variables, bit i removed) is cut
// into blocks of its 9 low compressed bits; block B holds the sets S = H' + lo
// whose high part H' is given by the bits of B. Splitting G = G_L + G_H (G_L
// over the 9 low bits, G_H over H'), the upward zeta of Eq. 7 restricted to
// one block is
//   alpha_i(H' + lo) = q(|H'| + |lo|) sum_{G_L subset lo, |G_L| <= d} Z_i(B, G_L),
//   Z_i(B, G_L)      = sum_{G_H subset H', |G_H| <= d - |G_L|} B_i(G_L + G_H),
// a zeta over 9 bits of K(9, d) seeds (Def. 1 with the bits split at 9, as
// Alg. 2 splits them between processors). A seed with |G_L| = d is B_i(G_L)
// itself, the same for every block, and is read from the scores; the K(9,
// d-1) others of each block are built once per solve and stored, 8 bytes
// each. From n = 22 they come from the seeds of 13-bit tiles (k_fseeds_13:
// a truncated zeta over compressed bits 9..12 of those), otherwise, and for
// the nodes outside the linear form, one at a time (k_fseeds_gen).
//
// Arithmetic. A node whose scores span at most 2^1800 (flin) runs in plain
// doubles under one power of two per node that puts B_i(empty) within
// [2^-968, 2^-904]: every alpha of the node is a sum that includes
// B_i(empty) and none exceeds 2^31 max_G B_i(G), so the zeta adds stay
// normal doubles, and so do the products with the L (Rp) significands
// (|f| within 2^+-32). Its seeds and size-d scores are doubles under that
// scale. Any other node runs in the number system itself (X32 seeds, X32
// adds). The cross terms of a tile are summed as a double and a power-of-two
// exponent per entry (aligned adds); the in-tile alpha slices and the tile's
// values go back to the 5-byte form, and the in-tile dynamic programme is
// the one of the materialised sweeps.
//
// Sweep tiles are the 9 low bits of the full mask under a high part H of
// popcount h (one launch per layer, as k_fwd / k_bwd). For a cross node i
// (a bit of H in the forward sweep, a high bit outside H in the backward
// one) the tile needs alpha_i over one whole block; for an in-tile node i < 9
// it needs half a block: the block's compressed bit 8 is the full mask's
// bit 9, the lowest bit of H. A wave rebuilds one block at a time. The
// block's seeds and size-d scores arrive as coalesced loads issued one block
// ahead, go to a wave-private LDS area, and each lane picks its entries
// from there (the pattern is the same for every block); the zeta then runs
// over three register layouts joined by two transposes through a second
// wave-private LDS buffer:
//   X: lane l, register r -> lo = (l & 3) | (r << 2) | ((l >> 2) << 5)   bits 2..4
//   Y: lo = (l & 31) | (r << 5) | ((l >> 5) << 8)                       bits 5..7
//   Z: lo = (r & 3) | (l << 2) | ((r >> 2) << 8)                        bits 0, 1, 8
// Layout Z gives each lane two runs of four consecutive entries, which meet
// the L (Rp) blocks as 16-byte loads, issued before the block's zeta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "bn_device.h"
#include "bn_kernels.h"

namespace bnk {

namespace {

constexpr int kT = 256;        // threads per workgroup (4 waves)
constexpr int kFB = 9;         // block bits = sweep tile bits
constexpr int kFT = 1 << kFB;  // entries per block
constexpr int kPad = 557;      // padded 8-byte slots of a wave's transpose buffer
// staging loads per lane and block: K(9, d) <= 64 NP (3 for d <= 3, 4 for
// d = 4, 8 up to d = 9); a template parameter of the sweep kernel
constexpr int npre_of(int d) { return d <= 3 ? 3 : (d == 4 ? 4 : 8); }
constexpr double kTwo64 = 18446744073709551616.0;   // 2^64: the fused scale per node
constexpr int kSeedTiles = 8;  // 13-bit tiles per workgroup of k_fseeds_13

// Slot of entry x in a wave's transpose buffer: within each row of 32
// eight-byte slots, x's low bits are XORed with its row (t = x >> 5) as
// t & 3 into bits 0..1 and t & 7 into bits 2..4. For each of the layouts X,
// Y and Z, the 32 lanes of a half wave then reach 32 distinct slots modulo
// 32, i.e. all 64 four-byte banks, so a 64-bit access takes two passes.
__device__ inline uint32_t fslot(uint32_t x) {
    const uint32_t t = x >> 5;
    return x ^ ((t & 3u) | ((t & 7u) << 2));
}

__host__ __device__ constexpr uint32_t fbin(int a, int b) {
    if (b < 0 || b > a) return 0;
    uint32_t r = 1;
    for (int k = 1; k <= b; ++k) r = r * (uint32_t)(a - b + k) / (uint32_t)k;
    return r;
}
// K(w, k) = sum_{j <= k} C(w, j) (0 for k < 0)
__host__ __device__ constexpr uint32_t fkw(int w, int k) {
    uint32_t s = 0;
    for (int j = 0; j <= k && j <= w; ++j) s += fbin(w, j);
    return s;
}
// colex rank of the set bits of a mask below bit 13 (bit p is element p)
__device__ inline uint32_t fcolex(uint32_t m) {
    uint32_t c = 0;
    int j = 0;
    while (m) {
        const int p = __ffs(m) - 1;
        m &= m - 1;
        c += fbin(p, ++j);
    }
    return c;
}

// A double or an X32 value as two 32-bit words, for the transposes (32-bit
// LDS instructions) and the 8-byte seed slots.
struct U2 {
    uint32_t a, b;
};
__device__ inline U2 u2_of(double x) {
    U2 w;
    __builtin_memcpy(&w, &x, 8);
    return w;
}
__device__ inline double dbl_of(U2 w) {
    double x;
    __builtin_memcpy(&x, &w, 8);
    return x;
}
__device__ inline U2 u2_of(X32 x) { return U2{__float_as_uint(x.f), (uint32_t)x.e}; }
__device__ inline X32 x32_of(U2 w) { return X32{__uint_as_float(w.a), (int)w.b}; }

// c ? y : x by bit masks (c is 0 or 1): a plain select that the compiler
// cannot turn into an indexed scratch array
__device__ inline U2 pick(uint32_t c, U2 x, U2 y) {
    const uint32_t m = 0u - c;
    return U2{(x.a & ~m) | (y.a & m), (x.b & ~m) | (y.b & m)};
}

// The two arithmetics of a block: plain doubles (one add per zeta step) and
// the number system itself.
struct LinA {
    using V = double;
    __device__ static V add(V a, V b) { return a + b; }
    __device__ static U2 pack(V v) { return u2_of(v); }
    __device__ static V unpack(U2 w) { return dbl_of(w); }
};
struct X32A {
    using V = X32;
    __device__ static V add(V a, V b) { return PolX32::add(a, b); }
    __device__ static U2 pack(V v) { return u2_of(v); }
    __device__ static V unpack(U2 w) { return x32_of(w); }
};

template <class A>
__device__ inline void zeta_reg(typename A::V *v, int q) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if ((r >> q) & 1) v[r] = A::add(v[r], v[r ^ (1 << q)]);
}

__device__ inline uint32_t lay_x(uint32_t l, uint32_t r) { return (l & 3) | (r << 2) | ((l >> 2) << 5); }
__device__ inline uint32_t lay_y(uint32_t l, uint32_t r) { return (l & 31) | (r << 5) | ((l >> 5) << 8); }
__device__ inline uint32_t lay_z(uint32_t l, uint32_t r) { return (r & 3) | (l << 2) | ((r >> 2) << 8); }

// Zeta over the 9 block bits of v (layout X in, layout Z out) through the
// wave's buffer (kPad 8-byte slots, one 64-bit LDS access per entry). The
// wave barriers keep the compiler from moving LDS accesses across the
// transposes; the hardware runs a wave's LDS instructions in order.
template <class A>
__device__ inline void block_zeta(typename A::V *v, uint32_t *pa, uint32_t *, uint32_t l) {
    uint64_t *pz = reinterpret_cast<uint64_t *>(pa);
#pragma unroll
    for (int q = 0; q < 3; ++q) zeta_reg<A>(v, q);          // bits 2, 3, 4
#pragma unroll
    for (int r = 0; r < 8; ++r) pz[fslot(lay_x(l, r))] = __builtin_bit_cast(uint64_t, v[r]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r)
        v[r] = __builtin_bit_cast(typename A::V, pz[fslot(lay_y(l, r))]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 3; ++q) zeta_reg<A>(v, q);          // bits 5, 6, 7
#pragma unroll
    for (int r = 0; r < 8; ++r) pz[fslot(lay_y(l, r))] = __builtin_bit_cast(uint64_t, v[r]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r)
        v[r] = __builtin_bit_cast(typename A::V, pz[fslot(lay_z(l, r))]);
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < 3; ++q) zeta_reg<A>(v, q);          // bits 0, 1, 8
}

struct FSweep {
    int n, d;
    uint32_t K;          // parent sets per node
    uint32_t KS;         // stored seeds per block, K(9, d - 1)
    uint32_t C9;         // size-d seeds of a block, C(9, d)
    uint32_t offd;       // rank of the first size-d parent set, K(n - 1, d - 1)
    const U2 *zw;        // seeds [node][block][rank], double (flin) or X32
    const double *betal; // scores under the node's linear scale (flin nodes)
    const X32 *beta;     // gauged scores
    const X32 *qt;       // q(k), gauged
    const int *anc;      // per-node linear scales (the fused scale is anc - 64)
    const int *flin;     // per-node flags: the node runs in plain doubles
    const uint32_t *glo; // slot of block entry lo among its block's staged seeds
    const uint16_t *lorder;
    const uint32_t *loff;
    const uint32_t *hord;
    uint32_t *nslow;     // blocks run in the number system
    unsigned long long *cnt;
};

// One block's staging values, loaded one block ahead: lane l holds entries
// l + 64 j of the list [the KS stored seeds, the C9 size-d scores] (entries
// past the list load seed 0 and are staged into slots nobody reads). The
// loads are issued unconditionally and nothing reads them before the next
// block, so they stay in flight while the current block computes.
template <int NP>
struct Pre {
    uint64_t v[NP];
};

// The per-wave state of a tile's sweep.
struct Ctx {
    const int *items;     // LDS: the tile's items (in-tile nodes, then cross nodes)
    int nitems;
    uint64_t Hf;          // the tile's high part (full mask)
    uint32_t hbit;        // Hf's bit 9
    uint32_t l;           // lane
    uint32_t gsl[8];      // staging slot of each layout-X entry of the lane
    uint32_t *pa, *pb;    // the wave's transpose buffer (two planes)
    U2 *stg;              // the wave's staging area (inside the transpose buffer)
    const int *sanc;      // LDS: per-node linear scales
    float *laf;           // LDS: in-tile alpha slices, significands ...
    uint8_t *lab;         // ... and exponent bytes
    uint32_t nsat, nfl;
};

// node and block of item it (the same for every lane: read into scalar
// registers)
template <bool FWD>
__device__ inline void item_of(const Ctx &c, int it, int *i_, uint64_t *B_) {
    const int i = __builtin_amdgcn_readfirstlane(c.items[it]);
    // in-tile node: block Hf >> 10; cross node: (S - i) or S in i's lattice
    const uint64_t Bc = compress_bit(FWD ? (c.Hf ^ (1ull << i)) : c.Hf, i) >> kFB;
    *i_ = i;
    *B_ = i < kFB ? (c.Hf >> (kFB + 1)) : Bc;
}

template <int NP, bool LIN>
__device__ inline void prefetch(const FSweep &a, int i, uint64_t B, uint32_t l, Pre<NP> &p) {
    const uint64_t nblk = 1ull << (a.n - 1 - kFB);
    const uint64_t *sq = reinterpret_cast<const uint64_t *>(a.zw + ((uint64_t)i * nblk + B) * a.KS);
    const size_t bo = (size_t)i * a.K + a.offd;
    const uint64_t *bp = LIN ? reinterpret_cast<const uint64_t *>(a.betal + bo)
                             : reinterpret_cast<const uint64_t *>(a.beta + bo);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const uint32_t e = l + 64 * j;
        const uint64_t *src = e < a.KS ? sq + e : (e < a.KS + a.C9 ? bp + (e - a.KS) : sq);
        p.v[j] = *src;
    }
}

// Stage the prefetched values of a block (a linear node's size-d scores
// scaled by 2^64 to the fused scale) and the zero slot, then gather the
// lane's layout-X entries.
template <int NP, bool LIN>
__device__ inline void stage_gather(const FSweep &a, const Ctx &c, const Pre<NP> &p,
                                    typename std::conditional<LIN, double, X32>::type *v) {
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const uint32_t e = c.l + 64 * j;
        const uint64_t x = p.v[j];
        if (LIN) {
            const double y = __builtin_bit_cast(double, x) * kTwo64;
            c.stg[e] = __builtin_bit_cast(U2, e >= a.KS ? __builtin_bit_cast(uint64_t, y) : x);
        } else {
            c.stg[e] = __builtin_bit_cast(U2, x);
        }
    }
    c.stg[64 * NP] = LIN ? U2{0u, 0u} : u2_of(PolX32::zero());
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        if constexpr (LIN) v[r] = dbl_of(c.stg[c.gsl[r]]);
        else v[r] = x32_of(c.stg[c.gsl[r]]);
    }
    __builtin_amdgcn_wave_barrier();
}

// a block entry (alpha without its factor q) in the number system: LIN
// from a double under the scale 2^T, else from an X32
__device__ inline X32 alpha_x32(double y, int T) { return PolX32::from_lin(y, T); }
__device__ inline X32 alpha_x32(X32 y, int) { return PolX32::norm(y); }

// The items of a wave: the in-tile items (a half block each, into the LDS
// slices), then the cross items (a whole block each, times the L (Rp) block,
// into the wave's sums). LIN: every node in plain doubles; otherwise every
// node in the number system itself.
template <bool FWD, int NP, bool LIN>
__device__ inline void sweep_items(const FSweep &a, Ctx &c, PolX32::Store X, uint32_t *nslow,
                                   double *accs, int *acce) {
    using A = typename std::conditional<LIN, LinA, X32A>::type;
    using V = typename A::V;
    const uint32_t l = c.l;
    Pre<NP> pre;
    int it = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // the wave
    int i;
    uint64_t B;
    item_of<FWD>(c, it, &i, &B);   // it < 9 <= nitems
    prefetch<NP, LIN>(a, i, B, l, pre);
    // in-tile items (the first 9)
    for (; it < kFB; it += 4) {
        item_of<FWD>(c, it, &i, &B);
        V v[8];
        stage_gather<NP, LIN>(a, c, pre, v);
        {   // the next item's loads, always issued (the last item reloads
            // itself) so that no branch makes the compiler wait for them
            int i2;
            uint64_t B2;
            item_of<FWD>(c, min(it + 4, c.nitems - 1), &i2, &B2);
            prefetch<NP, LIN>(a, i2, B2, l, pre);
        }
        if (!LIN && l == 0) atomicAdd(nslow, 1u);
        block_zeta<A>(v, c.pa, c.pb, l);
        const int T = c.sanc[i] - 64;   // B_i(empty) within [2^-968, 2^-904]
        // keep the half whose bit 8 is Hf's bit 9, in the 5-byte form
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const V y = __builtin_bit_cast(V, pick(c.hbit, __builtin_bit_cast(U2, v[j]),
                                                   __builtin_bit_cast(U2, v[4 + j])));
            const X32 x = alpha_x32(y, T);
            const uint32_t k = i * 256 + 4 * l + j;
            const int bb = (x.e >> 6) + kX32Bias;
            const bool zero = !(x.f > 0.0f);
            const bool fl = !zero && bb < 1, sat = !zero && bb > 255;
            c.nfl += fl ? 1u : 0u;
            c.nsat += sat ? 1u : 0u;
            c.laf[k] = (zero || fl) ? 0.0f : (sat ? 4.0e9f : x.f);
            c.lab[k] = (uint8_t)((zero || fl) ? 0 : (sat ? 255 : bb));
        }
        __builtin_amdgcn_wave_barrier();
    }
    // cross items
    for (; it < c.nitems; it += 4) {
        item_of<FWD>(c, it, &i, &B);
        // the L (Rp) block, issued before the zeta
        const uint64_t xb = FWD ? (c.Hf ^ (1ull << i)) : (c.Hf | (1ull << i));
        typename PolX32::Raw4 rx[2];
#pragma unroll
        for (int half = 0; half < 2; ++half) rx[half] = PolX32::load4_raw(X, xb + 256 * half + 4 * l);
        V v[8];
        stage_gather<NP, LIN>(a, c, pre, v);
        {   // the next item's loads, always issued (the last item reloads
            // itself) so that no branch makes the compiler wait for them
            int i2;
            uint64_t B2;
            item_of<FWD>(c, min(it + 4, c.nitems - 1), &i2, &B2);
            prefetch<NP, LIN>(a, i2, B2, l, pre);
        }
        if (!LIN && l == 0) atomicAdd(nslow, 1u);
        block_zeta<A>(v, c.pa, c.pb, l);
        const int T = c.sanc[i] - 64;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const float4 f = rx[half].f;
            const uint32_t e4 = rx[half].b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = 4 * half + j;
                const float lf = j == 0 ? f.x : j == 1 ? f.y : j == 2 ? f.z : f.w;
                const int le = (int)((e4 >> (8 * j)) & 0xffu) << 6;
                double tv;
                int te;
                if constexpr (LIN) {
                    tv = v[r] * (double)lf;
                    te = T + le - (kX32Bias << 6);
                } else {
                    tv = (double)v[r].f * (double)lf;
                    te = v[r].e + le - (kX32Bias << 6);
                }
                const int em = max(acce[r], te);
                accs[r] = ldexp(accs[r], acce[r] - em) + ldexp(tv, te - em);
                acce[r] = em;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

// One sweep layer of the fused form: FWD = Eq. 9 (L), else Eq. 10 (Rp).
// Workgroup = tile H (entry hoff + blockIdx.x of the high-part order: the
// layer-h masks over the n - 9 high bits). Items: the 9 in-tile nodes, then
// the cross nodes; wave w takes items w, w + 4, ... Each cross item adds
// alpha_i * X over the whole tile to the wave's sums; the four waves' sums
// then meet in LDS in a fixed order (bitwise deterministic) and the in-tile
// layers run as in k_fwd / k_bwd. Every node runs in plain doubles when
// all_lin (flin[32]) is set, else in the number system.
template <bool FWD, int NP>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_fsweep(FSweep a, int h, uint32_t hoff, PolX32::Store X) {
    extern __shared__ unsigned char smem[];
    uint32_t *zbuf = reinterpret_cast<uint32_t *>(smem);             // 4 waves x 2 planes x kPad
    float *laf = reinterpret_cast<float *>(zbuf + 8 * kPad);          // 9 x 256 slice significands
    uint8_t *lab = reinterpret_cast<uint8_t *>(laf + 9 * 256);        // 9 x 256 slice bytes
    X32 *lt = reinterpret_cast<X32 *>(lab + 9 * 256);                 // 512 tile values
    uint16_t *lord = reinterpret_cast<uint16_t *>(lt + kFT);          // 512 masks, by layer
    __shared__ uint32_t loff[kFB + 2];
    __shared__ int items[32];
    __shared__ int nitems_s;
    __shared__ X32 sq[32];       // q(k), gauged
    __shared__ int sanc[32];
    const int n = a.n, nh = n - kFB;
    const int t = threadIdx.x, w = t >> 6;
    const uint32_t Hm = a.hord[hoff + blockIdx.x];  // H over the high bits
    const bool all_lin = a.flin[32] != 0;
    if (t < kFB + 2) loff[t] = a.loff[t];
    if (t < n) {
        sq[t] = a.qt[t];
        sanc[t] = a.anc[t];
    }
    for (uint32_t x = t; x < kFT; x += kT) lord[x] = a.lorder[x];
    if (t == 0) {
        int c = 0;
        for (int i = 0; i < kFB; ++i) items[c++] = i;                  // in-tile nodes
        for (int p = 0; p < nh; ++p)                                   // cross nodes
            if ((((Hm >> p) & 1) != 0) == FWD) items[c++] = kFB + p;
        nitems_s = c;
    }
    Ctx c;
    c.l = t & 63;
    // the staging slot of each of the lane's layout-X entries (the zero
    // slot for entries with more than d elements)
#pragma unroll
    for (int r = 0; r < 8; ++r) c.gsl[r] = a.glo[lay_x(c.l, (uint32_t)r)];
    __syncthreads();
    c.items = items;
    c.nitems = nitems_s;
    c.Hf = (uint64_t)Hm << kFB;
    c.hbit = Hm & 1u;
    c.pa = zbuf + w * 2 * kPad;
    c.pb = c.pa + kPad;
    // a wave's staged seeds share its transpose buffer: the staged entries
    // are read (in program order) before the first transpose writes
    c.stg = reinterpret_cast<U2 *>(c.pa);
    c.sanc = sanc;
    c.laf = laf;
    c.lab = lab;
    c.nsat = c.nfl = 0;
    // cross sums of this wave, layout Z: value = s * 2^E
    double accs[8];
    int acce[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        accs[r] = 0.0;
        acce[r] = -(1 << 26);
    }
    if (all_lin) sweep_items<FWD, NP, true>(a, c, X, a.nslow, accs, acce);
    else sweep_items<FWD, NP, false>(a, c, X, a.nslow, accs, acce);
    const uint64_t Hf = c.Hf;
    const uint32_t l = c.l;
    uint32_t *pa = c.pa, *pb = c.pb;
    __syncthreads();
    // the four waves' cross sums as X32 (s 2^E normalised; E is a multiple
    // of 64), met in wave order
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const uint32_t s = lay_z(l, (uint32_t)r);
        const U2 u = u2_of(PolX32::from_lin(accs[r], acce[r]));
        pa[s] = u.a;
        pb[s] = u.b;
    }
    __syncthreads();
    // Every term of one tile entry's sum carries the same q: q(|S| - 1) in
    // the forward sweep (alpha_i(S - i)), q(|S|) in the backward one
    // (alpha_i(S)). The blocks and slices leave q out; it is applied once per
    // entry, after the cross sums (four waves, in wave order) and the in-tile
    // terms. The base entry (L of the empty set, Rp of V) is 1.
    auto finish = [&](uint32_t lo, X32 s) {
        const bool base = FWD ? (Hf == 0 && lo == 0)
                              : (Hf == (((1ull << nh) - 1) << kFB) && lo == kFT - 1);
        const int m = h + __popc(lo) - (FWD ? 1 : 0);
        return base ? PolX32::one() : PolX32::norm(PolX32::mul_raw(sq[max(m, 0)], s));
    };
    for (uint32_t lo = t; lo < kFT; lo += kT) {
        X32 s = PolX32::zero();
        for (int ww = 0; ww < 4; ++ww)
            s = PolX32::add(s, x32_of(U2{zbuf[ww * 2 * kPad + lo], zbuf[ww * 2 * kPad + kPad + lo]}));
        // entries without in-tile terms are final here
        lt[lo] = (FWD ? lo == 0 : lo == kFT - 1) ? finish(lo, s) : s;
    }
    __syncthreads();
    // in-tile layers (the slice of node i holds alpha_i(H + lo') / q, lo'
    // without bit i, at its compressed 8-bit index)
    if (FWD) {
        for (int ly = 1; ly <= kFB; ++ly) {
            for (uint32_t idx = loff[ly] + t; idx < loff[ly + 1]; idx += kT) {
                const uint32_t lo = lord[idx];
                X32 s = lt[lo];
                uint32_t rest = lo;
                while (rest) {
                    const int i = __ffs(rest) - 1;
                    rest &= rest - 1;
                    const uint32_t Tm = lo ^ (1u << i);
                    const uint32_t k = i * 256 + (uint32_t)compress_bit(Tm, i);
                    const X32 al{laf[k], ((int)lab[k] - kX32Bias) << 6};
                    s = PolX32::add(s, PolX32::mul_raw(al, lt[Tm]));
                }
                lt[lo] = finish(lo, s);
            }
            __syncthreads();
        }
    } else {
        for (int ly = kFB - 1; ly >= 0; --ly) {
            for (uint32_t idx = loff[ly] + t; idx < loff[ly + 1]; idx += kT) {
                const uint32_t lo = lord[idx];
                X32 s = lt[lo];
                uint32_t rest = (kFT - 1) & ~lo;
                while (rest) {
                    const int i = __ffs(rest) - 1;
                    rest &= rest - 1;
                    const uint32_t k = i * 256 + (uint32_t)compress_bit(lo, i);
                    const X32 al{laf[k], ((int)lab[k] - kX32Bias) << 6};
                    s = PolX32::add(s, PolX32::mul_raw(al, lt[lo | (1u << i)]));
                }
                lt[lo] = finish(lo, s);
            }
            __syncthreads();
        }
    }
    for (uint32_t lo = 4 * t; lo < kFT; lo += 4 * kT) PolX32::store4(X, Hf | lo, lt + lo, a.cnt);
    if (c.nsat | c.nfl) {
        if (c.nsat) atomicAdd(a.cnt, (unsigned long long)c.nsat);
        if (c.nfl) atomicAdd(a.cnt + 1, (unsigned long long)c.nfl);
    }
}

// ------------------------------------------------------------------ seeds
namespace {

// size and colex rank of the seed of rank rk among the sets over w bits
// with fewer than d elements (size, then colex order)
__device__ inline void seed_rank(int w, uint32_t rk, int *s, uint32_t *cl) {
    int k = 0;
    while (rk >= fkw(w, k)) ++k;
    *s = k;
    *cl = rk - fkw(w, k - 1);
}

}  // namespace

// Seeds of the 9-bit blocks of the linear-form nodes from the seeds of their
// 13-bit tiles (the alpha tiles' seeds: doubles under the node's linear
// scale, sizes below d). With G_B over the tile's compressed bits 9..12,
//   Z9(16 T + Bl, G_L) = sum_{G_B subset Bl, |G_B| <= d - |G_L|} Z13(T, G_L + G_B),
// Z13 of size d being the score itself: an upward zeta over 4 bits of a
// 16-entry vector. Lane g of a wave takes seed rank g of tile T (one wave
// per tile); the 16 x K(9, d - 1) outputs of a tile are contiguous and leave
// through LDS as coalesced stores, scaled by 2^64 to the fused scale.
__global__ void __launch_bounds__(64)
k_fseeds_13(int n, int d, uint32_t K, uint32_t KS9, uint32_t KS13, uint32_t offd,
            const double *__restrict__ zs13, const double *__restrict__ betal,
            const int *__restrict__ flin, U2 *__restrict__ zw) {
    extern __shared__ unsigned char smem[];
    const int N = n - 1, hA = N - 13;
    const int l = threadIdx.x;
    double *buf = reinterpret_cast<double *>(smem);   // 16 x KS9
    const uint64_t ntiles = (uint64_t)n << hA;
    // kSeedTiles consecutive tiles (node, 13-bit tile) per workgroup
    for (uint64_t tile = (uint64_t)blockIdx.x * kSeedTiles;
         tile < ntiles && tile < (uint64_t)(blockIdx.x + 1) * kSeedTiles; ++tile) {
        const int i = (int)(tile >> hA);
        if (!flin[i]) continue;
        const double *z = zs13 + tile * KS13;
        const double *bd = betal + (size_t)i * K + offd;
        for (uint32_t g0 = 0; g0 < KS9; g0 += 64) {
            const uint32_t g = g0 + l;
            if (g < KS9) {
                int s;
                uint32_t cl;
                seed_rank(kFB, g, &s, &cl);
                double v[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = s + __builtin_popcount(r);
                    double x = 0.0;
                    if (m <= d) {
                        uint32_t c = cl;
                        int j = s;
#pragma unroll
                        for (int p = 0; p < 4; ++p)
                            if ((r >> p) & 1) c += fbin(kFB + p, ++j);
                        x = m < d ? z[fkw(13, m - 1) + c] : bd[c];
                    }
                    v[r] = x;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < 16; ++r)
                        if ((r >> q) & 1) v[r] += v[r ^ (1 << q)];
#pragma unroll
                for (int r = 0; r < 16; ++r) buf[r * KS9 + g] = v[r] * kTwo64;
            }
        }
        __builtin_amdgcn_wave_barrier();
        U2 *out = zw + tile * 16 * KS9;   // blocks 16 T .. 16 T + 15 of node i
        for (uint32_t e = l; e < 16 * KS9; e += 64) out[e] = u2_of(buf[e]);
        __builtin_amdgcn_wave_barrier();
    }
}

// Seeds one at a time: for every node when the 13-bit seeds are not built,
// and otherwise for the nodes outside the linear form. A linear-form node's
// seeds are summed as doubles from its linear scores (scaled by 2^64 to the
// fused scale), any other node's in the number system itself. Each seed
// enumerates the subsets G_H of its block's high part by size, as masks over
// the block's set bits stepped in colex order (Gosper's rule).
__global__ void __launch_bounds__(kT)
k_fseeds_gen(int n, int d, uint32_t K, uint32_t KS, int skip_lin, const uint32_t *__restrict__ binom,
             const X32 *__restrict__ beta, const double *__restrict__ betal,
             const int *__restrict__ flin, U2 *__restrict__ zw) {
    const int N = n - 1, hA = N - kFB;
    const uint64_t items = ((uint64_t)KS) << hA;
    for (int i = 0; i < n; ++i) {
        const bool lin = flin[i] != 0;
        if (skip_lin && lin) continue;
        const X32 *bi = beta + (size_t)i * K;
        const double *bl = betal + (size_t)i * K;
        for (uint64_t it = (uint64_t)blockIdx.x * kT + threadIdx.x; it < items;
             it += (uint64_t)gridDim.x * kT) {
            const uint64_t B = it / KS;
            const uint32_t rk = (uint32_t)(it - B * KS);
            int s;
            uint32_t cl;
            seed_rank(kFB, rk, &s, &cl);
            int hp[32];
            int nb = 0;
            for (int p = 0; p < hA; ++p)
                if ((B >> p) & 1) hp[nb++] = kFB + p;
            X32 acc = PolX32::zero();
            double accd = 0.0;
            for (int k = 0; k <= d - s && k <= nb; ++k) {
                const uint32_t base = Kcount(binom, N, s + k - 1) + cl;
                uint32_t c = (1u << k) - 1;   // k-subset of the nb elements
                while (true) {
                    uint32_t r = base;
                    int j = s;
                    uint32_t rest = c;
                    while (rest) {
                        const int e = __ffs(rest) - 1;
                        rest &= rest - 1;
                        r += C(binom, hp[e], ++j);
                    }
                    if (lin) accd += bl[r];
                    else acc = PolX32::add(acc, bi[r]);
                    if (k == 0) break;
                    const uint32_t lowb = c & (0u - c), rip = c + lowb;   // next k-subset
                    c = (((rip ^ c) >> 2) / lowb) | rip;
                    if (c >> nb) break;
                }
            }
            zw[((uint64_t)i << hA) * KS + it] = lin ? u2_of(accd * kTwo64)
                                                    : u2_of(PolX32::norm(acc));
        }
    }
}

// Per-node flags of the fused form: node i runs in plain doubles when it has
// a linear scale and max_G B_i(G) / B_i(empty) <= 2^1800 (emax - 1 is
// floor(log2 max_G B_i(G)); the linear scale puts B_i(empty) within
// [2^-1032, 2^-968], the fused one 2^64 higher).
// force_slow clears every flag (tests of the number-system path); flin[32]
// is set when every node qualifies (the fused sweeps then run every block in
// plain doubles, else every block in the number system). Also the
// slot table of the staged seeds: block entry lo (a set over the 9 block
// bits) has stored seed K(9, |lo| - 1) + colex(lo) when |lo| < d, size-d
// score KS + colex(lo) when |lo| = d, and the zero slot zslot else.
__global__ void k_fused_flags(int n, int d, uint32_t K, uint32_t KS, uint32_t zslot,
                              int force_slow, const X32 *__restrict__ beta,
                              const int *__restrict__ linok, const int *__restrict__ emax,
                              int *__restrict__ flin, uint32_t *__restrict__ glo) {
    const int t = threadIdx.x;
    for (uint32_t lo = t; lo < kFT; lo += kT) {
        const int m = __popc(lo);
        const uint32_t cl = fcolex(lo);
        glo[lo] = m < d ? fkw(kFB, m - 1) + cl : (m == d ? KS + cl : zslot);
    }
    __shared__ int all;
    if (t == 0) all = 1;
    __syncthreads();
    int ok = 0;
    if (t < n) {
        const X32 b0 = beta[(size_t)t * K];
        const double l0 = PolX32::log2_of(b0);
        ok = (!force_slow && linok[t] && b0.f > 0.0f && (double)(emax[t] - 1) - l0 <= 1800.0)
                 ? 1 : 0;
        if (!ok) atomicAnd(&all, 0);
    }
    __syncthreads();
    // the sweeps run every node in one arithmetic: a node's flag stays set
    // only when every node qualifies, so that seeds and blocks agree
    if (t < n) flin[t] = all ? ok : 0;
    if (t == 0) flin[32] = all;
}

// -------------------------------------------------------------- launchers
hipError_t launch_fused_seeds(const FusedArgs &f, const double *zs13, uint32_t KS13,
                              hipStream_t st) {
    const int n = f.n, N = n - 1, d = f.d;
    hipLaunchKernelGGL(k_fused_flags, dim3(1), dim3(kT), 0, st, n, d, f.K, f.KS,
                       (uint32_t)(64 * npre_of(d)), f.force_slow, f.beta, f.linok, f.emax, f.flin,
                       f.glo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (f.KS == 0) return hipSuccess;   // d = 0: the only seed is B_i(empty)
    U2 *zw = reinterpret_cast<U2 *>(f.zw);
    const bool from13 = zs13 != nullptr && !f.force_slow;
    if (from13) {
        const uint64_t tiles = (uint64_t)n << (N - 13);
        const size_t sm = (size_t)16 * f.KS * 8;     // d <= 7: at most 59.6 KB
        hipLaunchKernelGGL(k_fseeds_13, dim3((unsigned)((tiles + kSeedTiles - 1) / kSeedTiles)),
                           dim3(64), sm, st, n, d, f.K, f.KS, KS13, f.offd, zs13, f.betal, f.flin,
                           zw);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int hA = N - kFB;
    const uint64_t items = (uint64_t)f.KS << hA;
    const unsigned grid = (unsigned)std::min<uint64_t>((items + kT - 1) / kT, 8192);
    hipLaunchKernelGGL(k_fseeds_gen, dim3(grid), dim3(kT), 0, st, n, d, f.K, f.KS,
                       from13 ? 1 : 0, f.binom, f.beta, f.betal, f.flin, zw);
    return hipGetLastError();
}

size_t fused_sweep_lds(int) {
    static_assert((64 * 8 + 1) * 8 <= 2 * kPad * 4, "staging fits a wave's transpose buffer");
    return (size_t)8 * kPad * 4 + 9 * 256 * 4 + 9 * 256 + (size_t)kFT * sizeof(X32) + kFT * 2;
}

hipError_t launch_fused_sweep(const FusedArgs &f, bool forward, int h, unsigned tiles,
                              PolX32::Store X, hipStream_t st) {
    FSweep a{};
    a.n = f.n;
    a.d = f.d;
    a.K = f.K;
    a.KS = f.KS;
    a.C9 = fbin(kFB, f.d);
    a.offd = f.offd;
    a.zw = reinterpret_cast<const U2 *>(f.zw);
    a.betal = f.betal;
    a.beta = f.beta;
    a.qt = f.qt;
    a.anc = f.anc;
    a.flin = f.flin;
    a.glo = f.glo;
    a.lorder = f.lorder;
    a.loff = f.loff;
    a.hord = f.hord;
    a.nslow = f.nslow;
    a.cnt = f.cnt;
    const size_t sm = fused_sweep_lds(f.d);
    const uint32_t hoff = hord_offset(f.n - kFB, h);
#define BN_FSWEEP(np)                                                                     \
    do {                                                                                  \
        if (forward)                                                                      \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fsweep<true, np>), dim3(tiles), dim3(kT), sm, \
                               st, a, h, hoff, X);                                        \
        else                                                                              \
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fsweep<false, np>), dim3(tiles), dim3(kT),    \
                               sm, st, a, h, hoff, X);                                    \
    } while (0)
    switch (npre_of(f.d)) {
        case 3: BN_FSWEEP(3); break;
        case 4: BN_FSWEEP(4); break;
        default: BN_FSWEEP(8); break;
    }
#undef BN_FSWEEP
    return hipGetLastError();
}

}  // namespace bnk
