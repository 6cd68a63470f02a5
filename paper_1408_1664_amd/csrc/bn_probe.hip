// Measurement of the blocked 0/1 contraction against the register pass (not
// a step of the solve). The in-tile zeta steps of the library (Def. 1 over a
// tile's low bits, Alg. 2) run as add steps on values a lane holds; the
// alternative is to view 16 consecutive entries as a row and multiply the
// row matrix by the 16 x 16 subset-inclusion matrix Z (Z[j][i] = 1 when the
// bits of j are a subset of those of i) on the FP64 matrix cores. Both
// kernels compute t(g, T) = sum_{S subset T} x(g, S) for every 16-entry
// group g, so that their times can be set side by side.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bn.h"

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kThreadsP = 256;

// Sixteen add steps' worth per group: each lane holds one group's 16 values
// and runs four add steps (one per bit), reps times in a row. A wave takes 64
// groups (8 KB) and moves them between HBM and its registers through LDS, so
// that every load and store instruction covers 1 KB of consecutive bytes;
// in LDS a group sits at a 17-double stride, which keeps a half wave's
// 8-byte accesses on distinct banks.
__global__ void __launch_bounds__(kThreadsP)
k_zeta4_valu(const double *__restrict__ x, double *__restrict__ y, uint64_t groups, int reps) {
    __shared__ double buf[kThreadsP / 64][64 * 17];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t g0 = ((uint64_t)blockIdx.x * (kThreadsP / 64) + w) * 64;
    if (g0 >= groups) return;
    const uint32_t ng = groups - g0 < 64 ? (uint32_t)(groups - g0) : 64u;   // a multiple of 16
    double *b = buf[w];
    const double2 *src = reinterpret_cast<const double2 *>(x + g0 * 16);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t e2 = lane + 64 * j;            // double pair e2 of the wave's groups
        const uint32_t gg = e2 >> 3, ent = (e2 & 7) * 2;
        if (gg < ng) {
            const double2 t = src[e2];
            b[gg * 17 + ent] = t.x;
            b[gg * 17 + ent + 1] = t.y;
        }
    }
    __builtin_amdgcn_wave_barrier();
    double v[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) v[e] = b[lane * 17 + e];
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if ((i >> q) & 1) v[i] += v[i ^ (1 << q)];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int e = 0; e < 16; ++e) b[lane * 17 + e] = v[e];
    __builtin_amdgcn_wave_barrier();
    double2 *dst = reinterpret_cast<double2 *>(y + g0 * 16);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t e2 = lane + 64 * j;
        const uint32_t gg = e2 >> 3, ent = (e2 & 7) * 2;
        if (gg < ng) dst[e2] = make_double2(b[gg * 17 + ent], b[gg * 17 + ent + 1]);
    }
}

// Sixteen groups per wave: D (16 x 16, rows = groups, columns = entries) =
// X Z as four 16 x 16 x 4 FP64 products over the column quarters of X.
// Operand layout of the 16 x 16 x 4 FP64 instruction: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; register r of lane l holds
// D[l / 16 + 4 r][l % 16]. reps > 1 accumulates the same product again.
__global__ void __launch_bounds__(kThreadsP)
k_zeta4_mfma(const double *__restrict__ x, double *__restrict__ y, uint64_t groups, int reps) {
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t g0 = (((uint64_t)blockIdx.x * kThreadsP + threadIdx.x) >> 6) * 16;
    if (g0 >= groups) return;          // groups is a multiple of 16: whole waves
    const uint32_t i = lane & 15, k = lane >> 4;
    double a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        a[c] = x[(g0 + i) * 16 + 4 * c + k];
        b[c] = (((uint32_t)(4 * c) + k) & ~i) == 0 ? 1.0 : 0.0;
    }
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c], b[c], acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) y[(g0 + k + 4 * r) * 16 + i] = acc[r];
}

}  // namespace

extern "C" bn_status bn_zeta4_probe(const double *dev_x, double *dev_y, uint64_t groups,
                                    int32_t method, int32_t reps, void *hip_stream, float *ms) {
    if (!dev_x || !dev_y || !ms) return BN_EINVAL;
    if (groups < 16 || groups % 16 != 0 || groups > (1ull << 32)) return BN_EINVAL;
    if (method != 0 && method != 1) return BN_EINVAL;
    if (reps < 1 || reps > 4096) return BN_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return BN_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return BN_EDEVICE;
    }
    bn_status rc = BN_OK;
    // method 0: 64 groups per wave; method 1: 16 groups per wave
    const uint64_t per_block = (kThreadsP / 64) * (method == 0 ? 64 : 16);
    const dim3 grid((unsigned)((groups + per_block - 1) / per_block));
    if (hipEventRecord(e0, st) != hipSuccess) rc = BN_EDEVICE;
    if (rc == BN_OK) {
        if (method == 0)
            hipLaunchKernelGGL(k_zeta4_valu, grid, dim3(kThreadsP), 0, st, dev_x, dev_y, groups,
                               (int)reps);
        else
            hipLaunchKernelGGL(k_zeta4_mfma, grid, dim3(kThreadsP), 0, st, dev_x, dev_y, groups,
                               (int)reps);
        if (hipGetLastError() != hipSuccess) rc = BN_EDEVICE;
    }
    if (rc == BN_OK && hipEventRecord(e1, st) != hipSuccess) rc = BN_EDEVICE;
    if (rc == BN_OK && hipEventSynchronize(e1) != hipSuccess) rc = BN_EDEVICE;
    if (rc == BN_OK && hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = BN_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}
