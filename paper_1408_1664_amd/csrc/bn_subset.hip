// Subset transforms on device arrays (bn_subset_transform on doubles,
// bn_subset_transform_x32 on the library's FP32-scaled storage): the
// truncated upward zeta transform (Def. 1), the downward zeta transform
// (Def. 2; its truncation only limits which outputs are required) and, on
// doubles, the inverses of the untruncated forms (Moebius), in place on
// 2^nbits values x[S], S a bit mask. Every kernel is written once over an
// array policy: F64 (doubles, signed steps) or X32F (an FP32 significand
// plane and an exponent-byte plane; aligned FP32 adds in registers and LDS,
// renormalised at the store).
//
// Layout of the work (nbits > 12): three passes over the array at 30 bits,
// each one read and one write of every entry.
//   k_subset_tile      the low 12 bits of each 4096-entry tile, in registers
//                      in three layouts with two LDS transposes (256 threads
//                      x 16 entries); an upward truncated transform first
//                      clears every input with more than d ones;
//   k_subset_group     the remaining bits in passes of at most 9 (split
//                      evenly), 32 columns x 2^B patterns per workgroup, two
//                      register layouts joined through LDS;
//   k_subset_bits<B>   a remainder of B <= 4 bits (nbits 13..16), entirely
//                      in registers.
// nbits <= 12: one workgroup in LDS (k_subset_small).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <type_traits>

#include "../../include/bn.h"
#include "bn_device.h"

namespace bnk {

namespace {

constexpr int kT = 256;

__device__ inline uint32_t padx16(uint32_t x) { return x + (x >> 4); }

// Array policies: load / store an entry, the zero, and one zeta step
// a + sign * b (sign -1: the Moebius step, doubles only).
struct F64 {
    using V = double;
    double *x;
    __device__ V load(uint64_t i) const { return x[i]; }
    __device__ void store(uint64_t i, V v) const { x[i] = v; }
    __device__ static V zero() { return 0.0; }
    __device__ static V step(V a, V b, double sign) { return a + sign * b; }
};
struct X32F {
    using V = X32;
    PolX32::Store s;
    unsigned long long *cnt;   // [0] saturated, [1] flushed (null: not counted)
    __device__ V load(uint64_t i) const { return PolX32::load(s, i); }
    __device__ void store(uint64_t i, V v) const { PolX32::store(s, i, v, cnt); }
    __device__ static V zero() { return PolX32::zero(); }
    __device__ static V step(V a, V b, double) { return PolX32::add(a, b); }
};

// One zeta step over register bit q of NR registers: up adds the entry
// without the bit into the entry with it, down the other way.
template <class F, bool UP, int NR>
__device__ inline void reg_step(typename F::V *v, int q, double sign) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (UP && ((r >> q) & 1)) v[r] = F::step(v[r], v[r ^ (1 << q)], sign);
        if (!UP && !((r >> q) & 1)) v[r] = F::step(v[r], v[r | (1 << q)], sign);
    }
}

template <class F, bool UP>
__global__ void __launch_bounds__(kT)
k_subset_tile(F x, double sign, int trunc_d) {
    using V = typename F::V;
    __shared__ V gb[4096 + 256];
    const int t = threadIdx.x;
    const uint64_t base = (uint64_t)blockIdx.x << 12;
    V v[16];
    // layout A: y = t * 16 + r, bits 0..3 in registers
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = x.load(base + ((uint32_t)t << 4) + r);
    if (trunc_d >= 0) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            if (__popcll(base | ((uint32_t)t << 4) | r) > trunc_d) v[r] = F::zero();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) reg_step<F, UP, 16>(v, q, sign);
#pragma unroll
    for (int r = 0; r < 16; ++r) gb[padx16(((uint32_t)t << 4) | r)] = v[r];
    __syncthreads();
    // layout B: y = thi * 256 + r * 16 + tlo, bits 4..7
    const uint32_t tlo = t & 15, thi = t >> 4;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = gb[padx16((thi << 8) | (r << 4) | tlo)];
#pragma unroll
    for (int q = 0; q < 4; ++q) reg_step<F, UP, 16>(v, q, sign);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) gb[padx16((thi << 8) | (r << 4) | tlo)] = v[r];
    __syncthreads();
    // layout C: y = r * 256 + t, bits 8..11
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = gb[padx16((r << 8) | t)];
#pragma unroll
    for (int q = 0; q < 4; ++q) reg_step<F, UP, 16>(v, q, sign);
#pragma unroll
    for (int r = 0; r < 16; ++r) x.store(base + (r << 8) + t, v[r]);
}

// Bits j0 .. j0+B-1 (j0 >= 12, B <= 4). Thread column col = blockIdx * 256
// + t splits into lo (the low j0 bits) and hi (the bits above the group);
// its registers hold the 2^B entries hi | r << j0 | lo. Consecutive threads
// take consecutive lo, so every register load and store is one 2 KB run.
template <class F, bool UP, int B>
__global__ void __launch_bounds__(kT)
k_subset_bits(F x, int j0, double sign) {
    constexpr int NR = 1 << B;
    const uint64_t col = (uint64_t)blockIdx.x * kT + threadIdx.x;
    const uint64_t lo = col & ((1ull << j0) - 1);
    const uint64_t hi = (col >> j0) << (j0 + B);
    typename F::V v[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) v[r] = x.load(hi | ((uint64_t)r << j0) | lo);
#pragma unroll
    for (int q = 0; q < B; ++q) reg_step<F, UP, NR>(v, q, sign);
#pragma unroll
    for (int r = 0; r < NR; ++r) x.store(hi | ((uint64_t)r << j0) | lo, v[r]);
}

// Bits j0 .. j0+B-1 (j0 >= 12, 5 <= B <= 9) over W = 2^LW consecutive low
// indices per workgroup, 32 entries per thread, NT = 2^(B+LW-5) threads.
// Entry (column c, pattern p) is x[hi | p << j0 | lo0 + c]. First layout:
// the registers hold pattern bits 0..4, the thread index the column and
// pattern bits 5..B-1 (TP = B-5 bits). Second layout: the registers hold
// pattern bits TP..TP+4, the thread index the column and pattern bits
// 0..TP-1. Bit 4 is a register bit in both, so the exchange runs in two
// rounds (bit 4 = 0, then 1) through half the entries' worth of LDS. Global
// accesses are runs of W doubles.
template <class F, bool UP, int B, int LW>
__global__ void __launch_bounds__(1 << (B + LW - 5))
k_subset_group(F x, int j0, double sign) {
    using V = typename F::V;
    constexpr int W = 1 << LW;
    constexpr int TP = B - 5;
    constexpr int NH = (1 << (B - 1)) * W;             // entries per exchange round
    constexpr int NPAD = (1 << (B - 1)) / 16 * 16;
    __shared__ V sb[TP > 0 ? NH + NPAD : 1];
    const uint32_t t = threadIdx.x;
    const uint32_t c = t & (W - 1);
    const uint32_t tp = t >> LW;
    const uint64_t w = blockIdx.x;
    const int cb = j0 - LW;                            // bits of the column-chunk index
    const uint64_t lo = ((w & ((1ull << cb) - 1)) << LW) | c;
    const uint64_t hi = (w >> cb) << (j0 + B);
    const uint64_t xb = hi | lo;
    V v[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) v[r] = x.load(xb + ((uint64_t)((tp << 5) | r) << j0));
#pragma unroll
    for (int q = 0; q < 5; ++q) reg_step<F, UP, 32>(v, q, sign);
    if constexpr (TP > 0) {
        // LDS slot of pattern p (bit 4 dropped) and column col
        auto at = [](uint32_t p, uint32_t col) {
            const uint32_t q = (p & 15) | ((p >> 5) << 4);
            return q * W + col + (q >> 4) * 16;
        };
        V u[32];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h) __syncthreads();
#pragma unroll
            for (int r = 16 * h; r < 16 * h + 16; ++r) sb[at((tp << 5) | r, c)] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 32; ++r) {
                const uint32_t p = ((uint32_t)r << TP) | tp;
                if (((p >> 4) & 1) == (uint32_t)h) u[r] = sb[at(p, c)];
            }
        }
        // register bit q is pattern bit TP + q; bits 5..B-1 remain
#pragma unroll
        for (int q = 5 - TP; q < 5; ++q) reg_step<F, UP, 32>(u, q, sign);
#pragma unroll
        for (int r = 0; r < 32; ++r) x.store(xb + ((uint64_t)(((uint32_t)r << TP) | tp) << j0), u[r]);
    } else {
#pragma unroll
        for (int r = 0; r < 32; ++r) x.store(xb + ((uint64_t)((tp << 5) | r) << j0), v[r]);
    }
}

template <class F, bool UP, int LW>
void launch_group(int B, int nbits, F x, int j0, double sign, hipStream_t st) {
    const dim3 grid((unsigned)(1ull << (nbits - B - LW)));
    switch (B) {
        case 5: hipLaunchKernelGGL((k_subset_group<F, UP, 5, LW>), grid, dim3(1 << LW), 0, st, x, j0, sign); break;
        case 6: hipLaunchKernelGGL((k_subset_group<F, UP, 6, LW>), grid, dim3(1 << (1 + LW)), 0, st, x, j0, sign); break;
        case 7: hipLaunchKernelGGL((k_subset_group<F, UP, 7, LW>), grid, dim3(1 << (2 + LW)), 0, st, x, j0, sign); break;
        case 8: hipLaunchKernelGGL((k_subset_group<F, UP, 8, LW>), grid, dim3(1 << (3 + LW)), 0, st, x, j0, sign); break;
        default: hipLaunchKernelGGL((k_subset_group<F, UP, 9, LW>), grid, dim3(1 << (4 + LW)), 0, st, x, j0, sign); break;
    }
}

// nbits <= 12: the whole array in LDS, one step per bit.
template <class F, bool UP>
__global__ void __launch_bounds__(kT)
k_subset_small(F x, int nbits, double sign, int trunc_d) {
    __shared__ typename F::V s[4096];
    const uint32_t N = 1u << nbits;
    for (uint32_t i = threadIdx.x; i < N; i += kT)
        s[i] = (trunc_d >= 0 && __popc(i) > trunc_d) ? F::zero() : x.load(i);
    __syncthreads();
    for (int j = 0; j < nbits; ++j) {
        for (uint32_t i = threadIdx.x; i < N; i += kT) {
            if (UP && ((i >> j) & 1)) s[i] = F::step(s[i], s[i ^ (1u << j)], sign);
            if (!UP && !((i >> j) & 1)) s[i] = F::step(s[i], s[i | (1u << j)], sign);
        }
        __syncthreads();
    }
    for (uint32_t i = threadIdx.x; i < N; i += kT) x.store(i, s[i]);
}

template <class F, bool UP>
hipError_t run(F x, int nbits, double sign, int trunc_d, hipStream_t st) {
    if (nbits <= 12) {
        hipLaunchKernelGGL((k_subset_small<F, UP>), dim3(1), dim3(kT), 0, st, x, nbits, sign,
                           trunc_d);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_subset_tile<F, UP>), dim3((unsigned)(1ull << (nbits - 12))), dim3(kT), 0,
                       st, x, sign, trunc_d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int rem = nbits - 12;
    const int npass = (rem + 8) / 9;          // at most 9 bits per pass, split evenly
    for (int i = 0, j0 = 12; i < npass; ++i) {
        const int B = rem / npass + (i < rem % npass ? 1 : 0);
        if (B >= 5) {
            // runs of 32 doubles (256 B); in the FP32-scaled form runs of 64
            // entries, so that the byte plane too moves whole 64-byte segments
            launch_group<F, UP, std::is_same<F, X32F>::value ? 6 : 5>(B, nbits, x, j0, sign, st);
        } else {
            // 2^(nbits - B) columns, 256 per workgroup (nbits - B >= 12)
            const dim3 grid((unsigned)(1ull << (nbits - B - 8)));
            switch (B) {
                case 1: hipLaunchKernelGGL((k_subset_bits<F, UP, 1>), grid, dim3(kT), 0, st, x, j0, sign); break;
                case 2: hipLaunchKernelGGL((k_subset_bits<F, UP, 2>), grid, dim3(kT), 0, st, x, j0, sign); break;
                case 3: hipLaunchKernelGGL((k_subset_bits<F, UP, 3>), grid, dim3(kT), 0, st, x, j0, sign); break;
                default: hipLaunchKernelGGL((k_subset_bits<F, UP, 4>), grid, dim3(kT), 0, st, x, j0, sign); break;
            }
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        j0 += B;
    }
    return hipSuccess;
}

}  // namespace
}  // namespace bnk

extern "C" bn_status bn_subset_transform(double *dev_x, int32_t nbits, bn_subset_kind kind,
                                         int32_t d, void *hip_stream) {
    if (!dev_x || nbits < 1 || nbits > 32) return BN_EINVAL;
    if (kind != BN_ZETA_UP && kind != BN_ZETA_DOWN && kind != BN_MOBIUS_UP &&
        kind != BN_MOBIUS_DOWN)
        return BN_EINVAL;
    const bool mobius = kind == BN_MOBIUS_UP || kind == BN_MOBIUS_DOWN;
    if (mobius && d >= 0 && d < nbits) return BN_EINVAL;   // only the untruncated forms invert
    const int trunc = (kind == BN_ZETA_UP && d >= 0 && d < nbits) ? d : -1;
    const double sign = mobius ? -1.0 : 1.0;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const bool up = kind == BN_ZETA_UP || kind == BN_MOBIUS_UP;
    const bnk::F64 x{dev_x};
    const hipError_t e = up ? bnk::run<bnk::F64, true>(x, nbits, sign, trunc, st)
                            : bnk::run<bnk::F64, false>(x, nbits, sign, trunc, st);
    return e == hipSuccess ? BN_OK : BN_EDEVICE;
}

extern "C" bn_status bn_subset_transform_x32(float *dev_f, uint8_t *dev_b, int32_t nbits,
                                             bn_subset_kind kind, int32_t d,
                                             unsigned long long *dev_counts, void *hip_stream) {
    if (!dev_f || !dev_b || nbits < 1 || nbits > 32) return BN_EINVAL;
    if (kind != BN_ZETA_UP && kind != BN_ZETA_DOWN) return BN_EINVAL;
    const int trunc = (kind == BN_ZETA_UP && d >= 0 && d < nbits) ? d : -1;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    const bnk::X32F x{bnk::PolX32::Store{dev_f, dev_b}, dev_counts};
    const hipError_t e = kind == BN_ZETA_UP ? bnk::run<bnk::X32F, true>(x, nbits, 1.0, trunc, st)
                                            : bnk::run<bnk::X32F, false>(x, nbits, 1.0, trunc, st);
    return e == hipSuccess ? BN_OK : BN_EDEVICE;
}
