// snn_mfma.h -- operand forms of the reduced-precision contractions and the
// matrix-core kernels of the per-step path.
#pragma once
#include <hip/hip_runtime.h>

#include "snn_dev.h"

namespace snn {

enum Prec { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP8 = 2 };

// bfloat16 code of x, round to nearest even (finite x).
__device__ __forceinline__ uint32_t bf16_code(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t c) { return __uint_as_float(c << 16); }

// OCP FP8 E4M3 code of x, round to nearest even: 4 significant bits,
// exponent bias 7, subnormal spacing 2^-9 below 2^-6, saturating at 448.
__device__ __forceinline__ uint32_t e4m3_code(float x)
{
    const uint32_t u = __float_as_uint(x);
    const uint32_t sign = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7FFFFFFFu;
    uint32_t c;
    if (a >= 0x3C800000u) {  // |x| >= 2^-6: round the FP32 significand to 3 fraction bits
        const uint32_t r = (a + 0x7FFFFu + ((a >> 20) & 1u)) >> 20;  // exponent(8) | fraction(3)
        c = r - (120u << 3);                                         // rebias 127 -> 7
        if (r < (120u << 3) || c > 0x7Eu) c = 0x7Eu;                 // saturate (largest finite)
    } else {                 // multiples of 2^-9; 8 * 2^-9 = 2^-6 is code 0x08
        c = (uint32_t)rintf(__uint_as_float(a) * 512.f);
    }
    return sign | c;
}
__device__ __forceinline__ float e4m3_value(uint32_t c)
{
    const uint32_t e = (c >> 3) & 15u, m = c & 7u;
    const float v = e ? ldexpf(1.f + 0.125f * (float)m, (int)e - 7) : ldexpf((float)m, -9);
    return (c & 0x80u) ? -v : v;
}

// x rounded to the E4M3 grid, as an FP32 value (the value of e4m3_code(x)):
// 3 fraction bits at or above 2^-6, multiples of 2^-9 below, at most 448.
__device__ __forceinline__ float e4m3_round(float x)
{
    const uint32_t u = __float_as_uint(x);
    const uint32_t a = u & 0x7FFFFFFFu;
    float r;
    if (a >= 0x3C800000u)
        r = fminf(__uint_as_float((a + 0x7FFFFu + ((a >> 20) & 1u)) & 0xFFF00000u), 448.f);
    else
        r = rintf(__uint_as_float(a) * 512.f) * (1.f / 512.f);
    return __uint_as_float(__float_as_uint(r) | (u & 0x80000000u));
}

// Value of x as the contraction sees it in the form `prec` (the gather
// kernels' view of the same operand rounding).
__device__ __forceinline__ float operand_value(int prec, float x)
{
    if (prec == PREC_BF16) return bf16_value(bf16_code(x));
    if (prec == PREC_FP8) return e4m3_round(x);
    return x;
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
