// Device-side numeric policies and subset combinatorics for the lattice kernels.
//
// Two number systems share one set of kernels (templates on the policy):
//
//  PolLog  -- plain FP64 natural-log values; "add" is log(e^a + e^b),
//             "mul" is a + b.
//  PolX32  -- a positive value is f * 2^(64 e): f an FP32 significand kept in
//             [2^-32, 2^32) after normalisation, e an int. Stored in HBM as an
//             FP32 word plus one byte b = e + kX32Bias (b = 0 means zero), so
//             the reach is 2^(64*(1-kX32Bias)) .. 2^(64*(255-kX32Bias)):
//             about 8,800 nats below the gauge and 2,400 nats above it.
//             The kernels run on gauged inputs: B_i is divided by an exact
//             power of two 2^E_i per node and q(k) by 2^F_k per layer. Every
//             order's weight then changes by the same constant factor
//             2^(sum E_i + sum F_k), so all posteriors are unchanged.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bnk {

constexpr int kX32Bias = 200;
constexpr int kEZero = -(1 << 26);   // exponent carried by an exact zero

// ---------------------------------------------------------------- FP64 log
struct PolLog {
    using V = double;                 // value in registers and LDS
    struct Store {                    // value in HBM
        double *p;
    };
    static constexpr int kBytes = 8;
    __device__ static inline V zero() { return -__builtin_huge_val(); }
    __device__ static inline V one() { return 0.0; }
    __device__ static inline V mul(V a, V b) { return a + b; }
    __device__ static inline V add(V a, V b) {
        V hi = fmax(a, b), lo = fmin(a, b);
        if (lo == -__builtin_huge_val()) return hi;
        return hi + log1p(exp(lo - hi));
    }
    __device__ static inline V mul_raw(V a, V b) { return a + b; }
    __device__ static inline V norm_v(V a) { return a; }
    // Running sum of many terms: s * e^m, rescaled when a larger term comes
    // in. One exp per term (add() takes an exp and a log1p); the log is
    // taken once, by acc_value.
    struct Acc {
        double m, s;
    };
    __device__ static inline Acc acc_of(V x) {
        return x > -1e300 ? Acc{x, 1.0} : Acc{-__builtin_huge_val(), 0.0};
    }
    __device__ static inline void acc_add(Acc &a, V t) {
        if (!(t > -1e300)) return;
        const double dlt = t - a.m;            // +inf while a is empty
        const double e = exp(-fabs(dlt));
        if (dlt > 0.0) {
            a.s = a.s * e + 1.0;
            a.m = t;
        } else {
            a.s += e;
        }
    }
    __device__ static inline V acc_value(const Acc &a) {
        return a.s > 0.0 ? a.m + log(a.s) : -__builtin_huge_val();
    }
    // Undecoded HBM value: lets loads be issued long before their use.
    using Raw = double;
    __device__ static inline Raw load_raw(const Store &s, uint64_t i) { return s.p[i]; }
    __device__ static inline V decode_raw(Raw r) { return r; }
    struct Raw4 {
        double2 a, b;
    };
    __device__ static inline Raw4 load4_raw(const Store &s, uint64_t i) {
        return Raw4{*reinterpret_cast<const double2 *>(s.p + i),
                    *reinterpret_cast<const double2 *>(s.p + i + 2)};
    }
    __device__ static inline void decode4(const Raw4 &r, V *o) {
        o[0] = r.a.x;
        o[1] = r.a.y;
        o[2] = r.b.x;
        o[3] = r.b.y;
    }
    __device__ static inline void decode4_nz(const Raw4 &r, V *o) { decode4(r, o); }
    __device__ static inline V from_log(double x) { return x; }
    __device__ static inline double to_log(V v) { return v; }
    // log(a / b) in FP64, a, b > 0
    __device__ static inline double log_ratio(V a, V b) { return a - b; }
    __device__ static inline V load(const Store &s, uint64_t i) { return s.p[i]; }
    __device__ static inline void store(const Store &s, uint64_t i, V v,
                                        unsigned long long *) {
        s.p[i] = v;
    }
    // four consecutive entries, i a multiple of 4
    __device__ static inline void load4(const Store &s, uint64_t i, V *o) {
        const double2 a = *reinterpret_cast<const double2 *>(s.p + i);
        const double2 b = *reinterpret_cast<const double2 *>(s.p + i + 2);
        o[0] = a.x;
        o[1] = a.y;
        o[2] = b.x;
        o[3] = b.y;
    }
    __device__ static inline void store4(const Store &s, uint64_t i, const V *v,
                                         unsigned long long *) {
        *reinterpret_cast<double2 *>(s.p + i) = make_double2(v[0], v[1]);
        *reinterpret_cast<double2 *>(s.p + i + 2) = make_double2(v[2], v[3]);
    }
    // Sixteen consecutive entries (i a multiple of 16), undecoded; at16
    // picks entry k (a compile-time constant after unrolling).
    struct Raw16 {
        double2 p[8];
    };
    __device__ static inline Raw16 load16_raw(const Store &s, uint64_t i) {
        Raw16 r;
        const double2 *src = reinterpret_cast<const double2 *>(s.p + i);
#pragma unroll
        for (int k = 0; k < 8; ++k) r.p[k] = src[k];
        return r;
    }
    __device__ static inline V at16(const Raw16 &r, int k) {
        return (k & 1) ? r.p[k >> 1].y : r.p[k >> 1].x;
    }
    __device__ static inline V at16_nz(const Raw16 &r, int k) { return at16(r, k); }
    // Linear tiles: a value x is held as the plain double x * 2^-T (T a
    // natural-log offset here) so that a zeta over the tile costs one FP64
    // add per step. anchor_of places the reference value a at 2^-1000,
    // leaving about 2,000 binary orders of headroom above it.
    using Anchor = double;
    __device__ static inline bool anchor_of(V a, Anchor *T) {
        if (!(a > -1e300)) return false;
        *T = a + 1000.0 * 0.69314718055994530942;
        return true;
    }
    __device__ static inline double to_lin(V x, Anchor T) {
        return x > -1e300 ? exp(x - T) : 0.0;
    }
    // a scale that puts the value 2^e2 at 2^940 (room for 4096 such terms)
    __device__ static inline Anchor anchor_high(int e2) {
        return (double)(e2 - 940) * 0.69314718055994530942;
    }
    __device__ static inline double prod_lin(V a, V b, V c, Anchor T) {
        const double s = a + b + c;
        return s > -1e300 ? exp(s - T) : 0.0;
    }
    // prod_lin with the first two factors already multiplied (mul_raw)
    __device__ static inline double prod2_lin(V ab, V c, Anchor T) {
        const double s = ab + c;
        return s > -1e300 ? exp(s - T) : 0.0;
    }
    __device__ static inline V from_lin(double y, Anchor T) {
        return y > 0.0 ? log(y) + T : zero();
    }
    // from_lin(y) * q
    __device__ static inline V from_lin_q(double y, V q, Anchor T) {
        return q > -1e300 ? from_lin(y, T) + q : zero();
    }
    // binary logarithm (a very negative number for zero)
    __device__ static inline double log2_of(V x) {
        return x > -1e300 ? x * 1.4426950408889634074 : -1e300;
    }
    // store from_lin(y) * q
    __device__ static inline void store_lin_q(const Store &s, uint64_t i, double y, V q,
                                              Anchor T, uint32_t &, uint32_t &) {
        s.p[i] = from_lin_q(y, q, T);
    }
};

// ------------------------------------------------------- FP32 + exponent
// In registers and LDS the exponent is kept in binary orders (a multiple of
// 64): value = f * 2^E. HBM holds the byte b = E/64 + kX32Bias.
struct X32 {
    float f;
    int e;  // E, a multiple of 64
};

struct PolX32 {
    using V = X32;
    struct Store {
        float *f;
        uint8_t *b;
    };
    static constexpr int kBytes = 5;
    __device__ static inline V zero() { return X32{0.0f, kEZero}; }
    __device__ static inline V one() { return X32{1.0f, 0}; }
#ifdef BN_X32_LITERAL
    // Measurement build of the literal block-only FP32 form: the exponent
    // stays 0, so every value is a plain float and only the per-node and
    // per-layer gauges (applied in FP64 to the log scores) set its range;
    // values beyond the FP32 range become inf or 0. Used with the linear
    // tiles off (they would keep the range in doubles).
    __device__ static inline V norm(V x) {
        if (!(x.f > 0.0f)) return zero();
        return X32{ldexpf(x.f, x.e), 0};
    }
#else
    // Bring f back into [2^-32, 2^32) (f >= 0, normal or zero).
    __device__ static inline V norm(V x) {
        if (!(x.f > 0.0f)) return zero();
        const int bits = __float_as_int(x.f);
        const int k = ((bits >> 23) & 0xff) - 127;
        const int s = (k + 32) >> 6;  // floor((k + 32) / 64)
        x.f = __int_as_float(bits - (s << 29));
        x.e += s << 6;
        return x;
    }
#endif
    __device__ static inline V mul(V a, V b) { return norm(X32{a.f * b.f, a.e + b.e}); }
    // Product without renormalisation (f may leave [2^-32, 2^32); add() stays
    // exact as long as f stays within the FP32 range).
    __device__ static inline V mul_raw(V a, V b) { return X32{a.f * b.f, a.e + b.e}; }
    __device__ static inline V norm_v(V a) { return norm(a); }
    // Exact alignment to the larger exponent; the smaller operand is scaled
    // by an exact power of two (it underflows to zero only when it is below
    // FP32 resolution of the result).
    __device__ static inline V add(V a, V b) {
        const int em = max(a.e, b.e);
        return X32{ldexpf(a.f, a.e - em) + ldexpf(b.f, b.e - em), em};
    }
    // Running sum of many terms: the aligned add itself.
    using Acc = X32;
    __device__ static inline Acc acc_of(V x) { return x; }
    __device__ static inline void acc_add(Acc &a, V t) { a = add(a, t); }
    __device__ static inline V acc_value(const Acc &a) { return a; }
    __device__ static inline V from_log(double x) {
        if (!(x > -1e300)) return zero();
#ifdef BN_X32_LITERAL
        return norm(X32{(float)exp(x), 0});
#endif
        const double t = x * 1.4426950408889634074;  // log2
        const int e = (int)floor((t + 32.0) / 64.0);
        const float f = (float)exp(x - (double)e * 64.0 * 0.69314718055994530942);
        return norm(X32{f, e * 64});
    }
    __device__ static inline double to_log(V v) {
        if (!(v.f > 0.0f)) return -__builtin_huge_val();
        return log((double)v.f) + (double)v.e * 0.69314718055994530942;
    }
    __device__ static inline double log_ratio(V a, V b) { return to_log(a) - to_log(b); }
    __device__ static inline V decode(float f, int b) {
        return b ? X32{f, (b - kX32Bias) << 6} : zero();
    }
    __device__ static inline V load(const Store &s, uint64_t i) {
        return decode(s.f[i], s.b[i]);
    }
    // Undecoded HBM value: lets loads be issued long before their use.
    struct Raw {
        float f;
        uint32_t b;
    };
    __device__ static inline Raw load_raw(const Store &s, uint64_t i) {
        return Raw{s.f[i], (uint32_t)s.b[i]};
    }
    __device__ static inline V decode_raw(Raw r) { return decode(r.f, (int)r.b); }
    struct Raw4 {
        float4 f;
        uint32_t b;
    };
    __device__ static inline Raw4 load4_raw(const Store &s, uint64_t i) {
        return Raw4{*reinterpret_cast<const float4 *>(s.f + i),
                    *reinterpret_cast<const uint32_t *>(s.b + i)};
    }
    __device__ static inline void decode4(const Raw4 &r, V *o) {
        o[0] = decode(r.f.x, r.b & 0xff);
        o[1] = decode(r.f.y, (r.b >> 8) & 0xff);
        o[2] = decode(r.f.z, (r.b >> 16) & 0xff);
        o[3] = decode(r.f.w, r.b >> 24);
    }
    // decode4 without the zero test, for factors of a product only: a stored
    // zero has significand 0, so the product is an exact zero whatever the
    // exponent carried with it.
    __device__ static inline void decode4_nz(const Raw4 &r, V *o) {
        o[0] = X32{r.f.x, (int)((r.b & 0xff) - kX32Bias) << 6};
        o[1] = X32{r.f.y, (int)(((r.b >> 8) & 0xff) - kX32Bias) << 6};
        o[2] = X32{r.f.z, (int)(((r.b >> 16) & 0xff) - kX32Bias) << 6};
        o[3] = X32{r.f.w, (int)((r.b >> 24) - kX32Bias) << 6};
    }
    // Encode one value: returns the byte, writes the significand to *f.
    // cnt[0] counts saturations, cnt[1] flushes of nonzero values.
    __device__ static inline uint32_t encode(V v, float *f, unsigned long long *cnt) {
        v = norm(v);
        const int b = (v.e >> 6) + kX32Bias;
        if (v.f == 0.0f) {
            *f = 0.0f;
            return 0;
        }
        if (b < 1) {
            *f = 0.0f;
            if (cnt) atomicAdd(cnt + 1, 1ull);
            return 0;
        }
        if (b > 255) {
            *f = 4.0e9f;
            if (cnt) atomicAdd(cnt, 1ull);
            return 255;
        }
        *f = v.f;
        return (uint32_t)b;
    }
    __device__ static inline void store(const Store &s, uint64_t i, V v,
                                        unsigned long long *cnt) {
        float f;
        const uint32_t b = encode(v, &f, cnt);
        s.f[i] = f;
        s.b[i] = (uint8_t)b;
    }
    __device__ static inline void load4(const Store &s, uint64_t i, V *o) {
        const float4 f = *reinterpret_cast<const float4 *>(s.f + i);
        const uint32_t b = *reinterpret_cast<const uint32_t *>(s.b + i);
        o[0] = decode(f.x, b & 0xff);
        o[1] = decode(f.y, (b >> 8) & 0xff);
        o[2] = decode(f.z, (b >> 16) & 0xff);
        o[3] = decode(f.w, b >> 24);
    }
    __device__ static inline void store4(const Store &s, uint64_t i, const V *v,
                                         unsigned long long *cnt) {
        float f[4];
        uint32_t b = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) b |= encode(v[k], &f[k], cnt) << (8 * k);
        *reinterpret_cast<float4 *>(s.f + i) = make_float4(f[0], f[1], f[2], f[3]);
        *reinterpret_cast<uint32_t *>(s.b + i) = b;
    }
    // Sixteen consecutive entries (i a multiple of 16), undecoded; at16
    // decodes entry k (a compile-time constant after unrolling). at16_nz
    // skips the zero test: a stored zero keeps f = 0, so it is exact as a
    // factor of a product, but not as an operand of add().
    struct Raw16 {
        float4 f[4];
        uint4 b;
    };
    __device__ static inline Raw16 load16_raw(const Store &s, uint64_t i) {
        Raw16 r;
        const float4 *src = reinterpret_cast<const float4 *>(s.f + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) r.f[k] = src[k];
        r.b = *reinterpret_cast<const uint4 *>(s.b + i);
        return r;
    }
    __device__ static inline V at16_nz(const Raw16 &r, int k) {
        const float4 q = r.f[k >> 2];
        const float f = (k & 3) == 0 ? q.x : (k & 3) == 1 ? q.y : (k & 3) == 2 ? q.z : q.w;
        const uint32_t w = (k >> 2) == 0 ? r.b.x : (k >> 2) == 1 ? r.b.y : (k >> 2) == 2 ? r.b.z : r.b.w;
        return X32{f, (int)(((w >> (8 * (k & 3))) & 0xffu) - kX32Bias) << 6};
    }
    __device__ static inline V at16(const Raw16 &r, int k) {
        const uint32_t w = (k >> 2) == 0 ? r.b.x : (k >> 2) == 1 ? r.b.y : (k >> 2) == 2 ? r.b.z : r.b.w;
        return ((w >> (8 * (k & 3))) & 0xffu) ? at16_nz(r, k) : zero();
    }
    // Linear tiles: a value x is held as the plain double x * 2^-T, T a
    // multiple of 64, so that a zeta over the tile costs one FP64 add per
    // step. anchor_of places the reference value a within 2^-1032 .. 2^-968,
    // leaving at least 1,990 binary orders of headroom above it; values far
    // below the reference fall into the subnormal range or to zero.
    using Anchor = int;
    __device__ static inline bool anchor_of(V a, Anchor *T) {
        if (!(a.f > 0.0f)) return false;
        const int e = a.e + ((__float_as_int(a.f) >> 23) & 0xff) - 127;  // floor(log2 a)
        *T = ((e + 1032) >> 6) << 6;
        return true;
    }
    __device__ static inline double to_lin(V x, Anchor T) {
        return ldexp((double)x.f, max(x.e - T, -2000));
    }
    // a scale (a multiple of 64) that puts the value 2^e2 within 2^888 ..
    // 2^951 (room for 4096 such terms below 2^1000)
    __device__ static inline Anchor anchor_high(int e2) { return ((e2 - 888) >> 6) << 6; }
    __device__ static inline double prod_lin(V a, V b, V c, Anchor T) {
        return ldexp((double)(a.f * b.f * c.f), max(a.e + b.e + c.e - T, -2000));
    }
    // prod_lin with the first two factors already multiplied (mul_raw, f up
    // to 2^64). A zero factor has significand 0, so no exponent clamp is
    // needed: ldexp of 0 is 0 for any exponent.
    __device__ static inline double prod2_lin(V ab, V c, Anchor T) {
        return ldexp((double)(ab.f * c.f), ab.e + c.e - T);
    }
    // Back to a normalised X32 (f in [2^-32, 2^32]); y >= 0 and finite.
    __device__ static inline V from_lin(double y, Anchor T) {
        if (!(y > 0.0)) return zero();
        const int e = __builtin_amdgcn_frexp_exp(y);     // y in [2^(e-1), 2^e)
        const int k = ((e + 31) >> 6) << 6;
        return X32{(float)ldexp(y, -k), T + k};
    }
    // from_lin(y) * q
    __device__ static inline V from_lin_q(double y, V q, Anchor T) {
        return from_lin(y * (double)q.f, T + q.e);
    }
    // binary logarithm, rounded down (a very negative number for zero)
    __device__ static inline double log2_of(V x) {
        if (!(x.f > 0.0f)) return -1e300;
        return (double)(x.e + ((__float_as_int(x.f) >> 23) & 0xff) - 127);
    }
    // Store from_lin(y) * q in the 5-byte form without an intermediate
    // normalisation; same result and the same saturation / flush rules as
    // store(), with the counts accumulated in nsat / nfl.
    __device__ static inline void store_lin_q(const Store &s, uint64_t i, double y, V q,
                                              Anchor T, uint32_t &nsat, uint32_t &nfl) {
        const double z = y * (double)q.f;
        const int k = (__builtin_amdgcn_frexp_exp(z) + 31) >> 6;
        float f = (float)ldexp(z, -(k << 6));
        int b = ((T + q.e) >> 6) + k + kX32Bias;
        const bool zero = !(z > 0.0);
        const bool fl = !zero && b < 1;
        const bool sat = !zero && b > 255;
        nfl += fl ? 1u : 0u;
        nsat += sat ? 1u : 0u;
        if (zero || fl) {
            f = 0.0f;
            b = 0;
        }
        if (sat) {
            f = 4.0e9f;
            b = 255;
        }
        s.f[i] = f;
        s.b[i] = (uint8_t)b;
    }
    // Conversion of many values under one scale: lin_encode gives the
    // significand and the unbiased exponent byte minus T/64 (no range
    // checks); the byte is then b = e + T/64 + bias.
    __device__ static inline float lin_encode(double z, int *e) {
        const int k = (__builtin_amdgcn_frexp_exp(z) + 31) >> 6;
        *e = k;
        return (float)ldexp(z, -(k << 6));
    }
};

// -------------------------------------------------------- combinatorics
// binom points at a (33 x 33) table, binom[a * 33 + b] = C(a, b).
__device__ static inline uint32_t C(const uint32_t *binom, int a, int b) {
    return (b < 0 || a < 0 || b > a || a > 32) ? 0u : binom[a * 33 + b];
}

// Number of subsets of a w-set with at most t elements.
__device__ static inline uint32_t Kcount(const uint32_t *binom, int w, int t) {
    uint32_t s = 0;
    for (int k = 0; k <= t && k <= w; ++k) s += C(binom, w, k);
    return s;
}

// Positions (ascending) of the colex-rank c subset of size k.
__device__ static inline void colex_unrank(const uint32_t *binom, uint32_t c, int k,
                                           int *pos) {
    for (int t = k; t >= 1; --t) {
        int p = t - 1;
        while (p < 31 && C(binom, p + 1, t) <= c) ++p;
        pos[t - 1] = p;
        c -= C(binom, p, t);
    }
}

// Remove bit i from a mask: the compressed index of S (i not in S) in node
// i's lattice over the other n-1 variables.
__device__ static inline uint64_t compress_bit(uint64_t S, int i) {
    return (S & ((1ull << i) - 1)) | ((S >> (i + 1)) << i);
}
__device__ static inline uint64_t expand_bit(uint64_t c, int i) {
    return (c & ((1ull << i) - 1)) | ((c >> i) << (i + 1));
}

}  // namespace bnk
