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
    // round to nearest, ties to even; NaN stays a quiet NaN, overflow -> Inf.
    // The NaN case compiles to a vector test and a branch that a wavefront
    // skips when none of its values is a NaN; a branch-free select costs more
    // vector instructions per stored value and measured slower in the
    // VALU-bound fused kernel.
    static __device__ __forceinline__ bf16_bits st(float f) {
        uint32_t u = __float_as_uint(f);
        bf16_bits r;
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
            r.b = (uint16_t)((u >> 16) | 0x0040u);
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            r.b = (uint16_t)(u >> 16);
        }
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

}  // namespace plbm

#endif
