// snn_mfma.h -- operand forms of the reduced-precision contractions and the
// matrix-core kernels of the per-step path.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "snn_dev.h"

namespace snn {

enum Prec { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP8 = 2 };

// The two reduced operand forms, on the conversion instructions of gfx950:
//   bfloat16: round to nearest even (v_cvt_pk_bf16_f32);
//   OCP FP8 E4M3: 4 significant bits, exponent bias 7, subnormal spacing 2^-9
//     below 2^-6, round to nearest even, saturating at +-448 (a clamp, then
//     v_cvt_pk_fp8_f32 / v_cvt_f32_fp8).
// For every finite FP32 input these agree with the same roundings written
// out in integer arithmetic on the FP32 bit pattern (an exhaustive
// comparison over all finite FP32 values found no difference); each takes
// one or two instructions per value.
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// bfloat16 codes of a (low half) and b (high half).
__device__ __forceinline__ uint32_t bf16_codes2(float a, float b)
{
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ uint32_t bf16_code(float x) { return bf16_codes2(x, x) & 0xFFFFu; }
__device__ __forceinline__ float bf16_value(uint32_t c) { return __uint_as_float(c << 16); }

// E4M3 codes of a (byte 0) and b (byte 1).
__device__ __forceinline__ uint32_t e4m3_codes2(float a, float b)
{
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(__builtin_amdgcn_fmed3f(a, -448.f, 448.f),
                                                     __builtin_amdgcn_fmed3f(b, -448.f, 448.f), 0, false);
}
__device__ __forceinline__ uint32_t e4m3_code(float x) { return e4m3_codes2(x, x) & 0xFFu; }

// Values of two operands rounded to a form.
__device__ __forceinline__ f32x2_t bf16_round2(float a, float b)
{
    const f32x2_t v = {a, b};
    return __builtin_convertvector(__builtin_convertvector(v, bf16x2_t), f32x2_t);
}

__device__ __forceinline__ f32x2_t e4m3_round2(float a, float b)
{
    const int q = (int)e4m3_codes2(a, b);
    return f32x2_t{__builtin_amdgcn_cvt_f32_fp8(q, 0), __builtin_amdgcn_cvt_f32_fp8(q, 1)};
}

// Value of x as the contraction sees it in the form `prec` (the gather
// kernels' view of the same operand rounding).
__device__ __forceinline__ float operand_value(int prec, float x)
{
    if (prec == PREC_BF16) return bf16_round2(x, x).x;
    if (prec == PREC_FP8) return e4m3_round2(x, x).x;
    return x;
}

// Two values at a time (one conversion instruction for both).
__device__ __forceinline__ f32x2_t operand_value2(int prec, float a, float b)
{
    if (prec == PREC_BF16) return bf16_round2(a, b);
    if (prec == PREC_FP8) return e4m3_round2(a, b);
    return f32x2_t{a, b};
}

typedef __bf16 bf16x8_t __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x16_t __attribute__((__vector_size__(16 * sizeof(float))));

template <int PREC>
struct Form {
    static constexpr int planes = PREC == PREC_FP32 ? 3 : 1;
    static constexpr int esize = PREC == PREC_FP8 ? 1 : 2;  // bytes per element
    static constexpr int vbytes = 8 * esize;                 // bytes per lane operand
    using vec = typename std::conditional<PREC == PREC_FP8, uint2, uint4>::type;
    static constexpr int batch = PREC == PREC_FP32 ? 2 : 5;   // k-steps whose operands are read ahead
    static constexpr int batch8 = PREC == PREC_FP32 ? 2 : 4;  // the same within 8-step windows
};

// 8 spike bits -> 8 operand elements equal to 1 or 0.
__device__ __forceinline__ uint4 ones_bf16(uint32_t byte)
{
    uint4 r;
    r.x = ((byte & 1u) * 0x3F80u) | (((byte >> 1) & 1u) * 0x3F800000u);
    r.y = (((byte >> 2) & 1u) * 0x3F80u) | (((byte >> 3) & 1u) * 0x3F800000u);
    r.z = (((byte >> 4) & 1u) * 0x3F80u) | (((byte >> 5) & 1u) * 0x3F800000u);
    r.w = (((byte >> 6) & 1u) * 0x3F80u) | (((byte >> 7) & 1u) * 0x3F800000u);
    return r;
}

__device__ __forceinline__ uint2 ones_fp8(uint32_t byte)
{
    // E4M3 1.0 = 0x38
    uint2 r;
    r.x = ((byte & 1u) * 0x38u) | (((byte >> 1) & 1u) * 0x3800u) | (((byte >> 2) & 1u) * 0x380000u) |
          (((byte >> 3) & 1u) * 0x38000000u);
    r.y = (((byte >> 4) & 1u) * 0x38u) | (((byte >> 5) & 1u) * 0x3800u) | (((byte >> 6) & 1u) * 0x380000u) |
          (((byte >> 7) & 1u) * 0x38000000u);
    return r;
}

// One MFMA step on raw operand registers.
template <int PREC>
__device__ __forceinline__ f32x16_t mfma(uint4 a, uint4 b, f32x16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                   0, 0, 0);
}
template <int PREC>
__device__ __forceinline__ f32x16_t mfma8(uint2 a, uint2 b, f32x16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0,
                                                      0, 0);
}

// One MFMA step of the form PREC on raw operand registers.
template <int PREC>
__device__ __forceinline__ f32x16_t mma(uint4 a, uint4 b, f32x16_t c)
{
    return mfma<PREC>(a, b, c);
}
template <int PREC>
__device__ __forceinline__ f32x16_t mma(uint2 a, uint2 b, f32x16_t c)
{
    return mfma8<PREC>(a, b, c);
}

// Operand codes of one value x in the form PREC (plane 0 first).
template <int PREC>
__device__ __forceinline__ void split(float x, uint32_t c[3])
{
    if constexpr (PREC == PREC_FP32) {
        c[0] = bf16_code(x);
        const float r1 = x - bf16_value(c[0]);
        c[1] = bf16_code(r1);
        const float r2 = r1 - bf16_value(c[1]);
        c[2] = bf16_code(r2);
    } else if constexpr (PREC == PREC_BF16) {
        c[0] = bf16_code(x);
    } else {
        c[0] = e4m3_code(x);
    }
}

// Arguments of one step's front-half launch (traces, current, neurons).
struct FrontArgs {
    const float *W;
    const double *theta;
    const uint32_t *bits;   // this step's input spikes, per sample
    const float *xprev;     // x_pre(t-1)
    float *xcur;            // x_pre(t)
    const uint32_t *Cprev;  // inhibitory spike counts of step t-1
    uint32_t *Ccur, *Cnext;
    float *v_exc, *v_inh, *x_post;
    uint16_t *rf;
    int k;                  // step index within the call (outputs)
    Outs o;
};

size_t mfma_front_lds(const Params &p, int prec);
size_t mfma_plastic_lds(const Params &p, int prec);
bool mfma_plastic_fits(const Params &p, int prec);

template <int PREC>
__global__ void k_mfma_front(Params p, FrontArgs a);
template <int PREC>
__global__ void k_mfma_plastic(Params p, float *__restrict__ W, double *__restrict__ theta,
                               const uint16_t *__restrict__ rf, const float *__restrict__ x_post,
                               const float *__restrict__ x_pre, const uint32_t *__restrict__ bitsT_t);

}  // namespace snn
