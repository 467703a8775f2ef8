// Storage types and rounding of the stored populations, shared by the D2Q8
// and D3Q14 kernels (device code only).
//
// Populations are computed in FP32 and stored as FP32, FP16 or BF16 (held as
// raw bits).  Stores round to nearest, or stochastically: the stochastic
// variants take 16 random bits per stored value.
#ifndef PLBM_NUMERIC_H
#define PLBM_NUMERIC_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plbm {

// ------------------------------------------------------------------ storage

struct bf16_bits { uint16_t b; };

template <class S> struct Cvt;
template <> struct Cvt<float> {
    static __device__ __forceinline__ float ld(float v) { return v; }
    static __device__ __forceinline__ float st(float f) { return f; }
};
template <> struct Cvt<_Float16> {
    static __device__ __forceinline__ float ld(_Float16 v) { return (float)v; }
    // Round the FP32 value to FP16, nearest even (default mode); overflow -> Inf.
    // The empty asm pins f as an FP32 register value: without it the backend
    // may fold the producing FMA and this narrowing into one mixed-precision
    // FMA (a single rounding straight to FP16) in some template instances and
    // not in others, and results would then depend on the launch shape.
    static __device__ __forceinline__ _Float16 st(float f) {
        asm volatile("" : "+v"(f));
        return (_Float16)f;
    }
};
template <> struct Cvt<bf16_bits> {
    static __device__ __forceinline__ float ld(bf16_bits v) {
        return __uint_as_float((uint32_t)v.b << 16);
    }
    // round to nearest, ties to even; a NaN becomes a quiet NaN that keeps its
    // sign and top payload bits, overflow -> Inf (gfx950's v_cvt_pk_bf16_f32;
    // the empty asm keeps f an FP32 register value, as for FP16)
    static __device__ __forceinline__ bf16_bits st(float f) {
        asm volatile("" : "+v"(f));
        const __bf16 h = (__bf16)f;
        bf16_bits r;
        r.b = __builtin_bit_cast(uint16_t, h);
        return r;
    }
};

// ------------------------------------------------------------------ stochastic rounding
//
// Round-to-nearest storage stalls on very smooth fields: when the per-step
// change of a population is below half a unit in the last place of the stored
// value, every node rounds the same way and the stored map freezes (a bias,
// not noise).  Stochastic rounding moves to the upper or lower neighbour with
// probabilities proportional to the distance, which is unbiased.  The random
// bits are a counter-based hash of the node's position, the step and the
// direction, so a run is deterministic and independent of the launch shape and
// schedule.

// Integer finaliser "lowbias32" (C. Wellons, hash-prospector): a bijective
// mix of 32 bits with low bias, two multiplies.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// 16 random bits for direction i from 32-bit words r[0], r[1], ... (two per word).
__device__ __forceinline__ uint32_t bits16(const uint32_t* r, int i) {
    return (r[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
}

// FP32 storage: the exact sum a + b (TwoSum, contraction off) rounded to one
// of its two FP32 neighbours; the farther one is chosen with probability
// |error| / gap, resolved with 16 random bits.
__device__ __forceinline__ float sr_add_f32(float a, float b, uint32_t r16) {
    const float s = a + b;
    const float bb = s - a;
    const float err = (a - (s - bb)) + (b - bb);
    if (err == 0.0f || s == 0.0f) return s;
    const uint32_t u = __float_as_uint(s);
    const uint32_t un = ((err > 0.0f) == (s > 0.0f)) ? u + 1u : u - 1u;   // neighbour toward a + b
    const float nb = __uint_as_float(un);
    const float gap = fabsf(nb - s);
    const float p = ((float)r16 + 0.5f) * (1.0f / 65536.0f);
    return fabsf(err) > gap * p ? nb : s;
}

// 16-bit storage: add random bits below the kept mantissa and truncate.  FP16
// keeps 10 of FP32's 23 mantissa bits (exact for values in FP16's normal
// range; the converter then rounds the already short value), BF16 keeps 7.
__device__ __forceinline__ _Float16 sr_f16(float v, uint32_t r16) {
    uint32_t u = __float_as_uint(v);
    u = (u + (r16 >> 3)) & ~0x1fffu;
    float t = __uint_as_float(u);
    asm volatile("" : "+v"(t));
    return (_Float16)t;
}
__device__ __forceinline__ bf16_bits sr_bf16(float v, uint32_t r16) {
    // an infinity's low 16 bits are zero, so the added bits cannot carry out
    // of it; a NaN keeps its sign and top payload bits with the quiet bit set
    // (as in the nearest conversion), selected without a branch
    const uint32_t u = __float_as_uint(v);
    bf16_bits o;
    o.b = (uint16_t)(v != v ? (u >> 16) | 0x0040u : (u + r16) >> 16);
    return o;
}

typedef __fp16 plbm_h2 __attribute__((vector_size(2 * sizeof(__fp16))));   // the SR builtins' pairs
typedef __bf16 plbm_b2 __attribute__((vector_size(2 * sizeof(__bf16))));
typedef __bf16 plbm_bf16x2 __attribute__((ext_vector_type(2)));
typedef float plbm_f32x2 __attribute__((ext_vector_type(2)));

// Stochastic rounding by gfx950's conversion instructions, which add the top
// bits of their 32-bit random operand below the kept bits (measured faster
// than the software forms in the D3Q14 kernels, slower in the D2Q8 fused
// kernel).  BF16: the same bits as sr_bf16, NaNs included.  FP16: the same
// bits as sr_f16 for results in FP16's normal range; below it the instruction
// rounds at the subnormal's own spacing (sr_f16 rounds those twice: to 10
// mantissa bits stochastically, then to the subnormal to nearest).  Each
// instruction writes the low half of its destination and keeps the high half
// of its first operand: v's own bits, never read.  (The form that writes the
// high half is not used: hipcc of ROCm 7.2 then stores the low half for both
// values of a pair.)
__device__ __forceinline__ bf16_bits sr_bf16_hw(float v, uint32_t r16) {
    asm volatile("" : "+v"(v));
    const plbm_b2 t = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(plbm_b2, v), v, r16 << 16, false);
    bf16_bits o;
    o.b = __builtin_bit_cast(uint16_t, t[0]);
    return o;
}
__device__ __forceinline__ _Float16 sr_f16_hw(float v, uint32_t r16) {
    asm volatile("" : "+v"(v));
    const plbm_h2 t = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(plbm_h2, v), v, r16 << 16, false);
    return __builtin_bit_cast(_Float16, t[0]);
}

// Directions 2k and 2k + 1 rounded to S, w the node's random word k (16 bits
// for direction 2k in its low half, for 2k + 1 in its high half; unused
// without SR).  BF16 to nearest takes one packed conversion for the pair
// (gfx950's v_cvt_pk_bf16_f32, the same bits as Cvt<bf16_bits>::st of each
// value); HW selects the instruction forms of stochastic rounding.  FP16 to
// nearest rounds each value on its own (packing the pair measured slower: the
// halves cost register moves).
template <class S, int SR, bool HW = false>
__device__ __forceinline__ void round_pair(float a, float b, uint32_t w, S& oa, S& ob) {
    if constexpr (__is_same(S, float)) {
        oa = a;
        ob = b;
    } else if constexpr (__is_same(S, _Float16)) {
        if constexpr (SR) {
            oa = HW ? sr_f16_hw(a, w & 0xffffu) : sr_f16(a, w & 0xffffu);
            ob = HW ? sr_f16_hw(b, w >> 16) : sr_f16(b, w >> 16);
        } else {
            oa = Cvt<_Float16>::st(a);
            ob = Cvt<_Float16>::st(b);
        }
    } else if constexpr (SR) {
        oa = HW ? sr_bf16_hw(a, w & 0xffffu) : sr_bf16(a, w & 0xffffu);
        ob = HW ? sr_bf16_hw(b, w >> 16) : sr_bf16(b, w >> 16);
    } else {
        asm volatile("" : "+v"(a), "+v"(b));
        const plbm_f32x2 v = {a, b};
        const uint32_t u = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, plbm_bf16x2));
        oa.b = (uint16_t)u;
        ob.b = (uint16_t)(u >> 16);
    }
}

// N values (N even) rounded pairwise as above, word k for values 2k, 2k + 1.
template <class S, int SR, int N, bool HW = false>
__device__ __forceinline__ void round_pairs(const float* v, const uint32_t* r, S* o) {
    static_assert(N % 2 == 0, "pairs");
#pragma unroll
    for (int k = 0; k < N / 2; ++k)
        round_pair<S, SR, HW>(v[2 * k], v[2 * k + 1], SR ? r[k] : 0u, o[2 * k], o[2 * k + 1]);
}

}  // namespace plbm

#endif
