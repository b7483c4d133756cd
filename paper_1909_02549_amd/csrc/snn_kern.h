// snn_kern.h -- device helpers shared by the plain, fused and persistent
// kernels (one definition of each arithmetic step of the method).
#pragma once
#include <hip/hip_runtime.h>

#include "snn_dev.h"

namespace snn {

__host__ __device__ constexpr size_t align16(size_t n) { return (n + 15) & ~(size_t)15; }

// Philox4x64-10: ten rounds; per round two 64x64->128-bit products of the
// counter words 0 and 2 with the round multipliers, mixed with words 1 and 3
// and the key, the key advanced by the two Weyl increments between rounds.
// Full 64 x 64 -> 128-bit product a * b as (hi, lo), from four 32 x 32 ->
// 64-bit multiply-adds (schoolbook on 32-bit halves, each partial sum below
// 2^64), where separate high and low halves would take six multiplies.
__device__ __forceinline__ void mulhilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo)
{
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32), b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t t = (uint64_t)a0 * b0;
    const uint64_t u = (uint64_t)a1 * b0 + (t >> 32);
    const uint64_t v = (uint64_t)a0 * b1 + (uint32_t)u;
    lo = (v << 32) | (uint32_t)t;
    hi = (uint64_t)a1 * b1 + (u >> 32) + (v >> 32);
}

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4])
{
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c0, hi0, lo0);
        mulhilo64(M1, c2, hi1, lo1);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Nearest-spike (or additive) trace: decay by lam, then 1 (or +1) on a spike.
__device__ __forceinline__ float trace_step(float x, float lam, uint32_t spike, int additive)
{
    x *= lam;
    if (spike) x = additive ? x + 1.f : 1.f;
    return x;
}

// Batch reduction step of one term (terms are non-negative traces, the
// accumulator starts at 0, so max over the spiking samples equals the max
// over all B terms).
__device__ __forceinline__ float reduce2(int mode, float acc, float x)
{
    return mode == RED_MAX ? fmaxf(acc, x) : acc + x;
}

// The soft maximum with temperature tau, tau log((1 / B) sum_b exp(z_b / tau)),
// over B terms of which only the spiking samples' are non-zero: a zero term
// adds exp(0) = 1, so with S = sum over the spiking samples of
// exp(z_b / tau) - 1 the reduction is tau log1p(S / B).  soft_term gives one
// summand from k = log2(e) / tau with the hardware base-2 exponential (about
// 1 ulp: an absolute error near 1e-7 per summand, which moves the reduced
// change by about tau 1e-7, far below the weights' FP32 rounding; z = 0
// gives exactly 0); soft_value the reduction of the sum, tau ln(2)
// log2(1 + S / B) with the hardware base-2 logarithm (where S / B is far
// below 1 the rounding of 1 + S / B costs an absolute error near
// tau 6e-8, again far below the weights' rounding; S = 0 gives exactly 0).
__device__ __forceinline__ float soft_term(float x, float k) { return __builtin_amdgcn_exp2f(x * k) - 1.f; }
__device__ __forceinline__ float soft_value(const Params &p, float S)
{
    return p.tau_ln2_r * __builtin_amdgcn_logf(1.f + S * p.inv_B);
}

// One trace value as a summand of the batch reduction (the soft maximum's
// transform, else the value itself).
__device__ __forceinline__ float stdp_term(const Params &p, float x)
{
    return p.reduce == RED_SOFT ? soft_term(x, p.itau2_r) : x;
}

// W <- clamp(W + nu_post P - nu_pre D); mean divides the sums by B, the soft
// maximum maps them through tau log1p(S / B).
__device__ __forceinline__ float stdp_apply(const Params &p, float w, float P, float D)
{
    if (p.reduce == RED_MEAN) {
        P *= p.inv_B;
        D *= p.inv_B;
    } else if (p.reduce == RED_SOFT) {
        P = soft_value(p, P);
        D = soft_value(p, D);
    }
    w = w + p.nu_post * P - p.nu_pre * D;
    return fminf(fmaxf(w, p.w_min), p.w_max);
}

// Threshold offset seen by the excitatory neurons this step: theta decays by
// beta at the start of every learning step; frozen when not learning.
__device__ __forceinline__ float theta_offset(const Params &p, double theta)
{
    if (!p.adaptive) return 0.f;
    return (float)(p.learn ? theta * p.beta : theta);
}

// theta <- theta * beta + theta_plus * R_b(s_exc[b, j]) from the column's
// spike count (sum: count, mean: count / B, max and signed max: any, soft
// maximum: the soft maximum of count ones and B - count zeros, in FP32 like
// the weights' (its relative error near 1e-7 stays far inside the FP64
// accumulation's needs), added to theta in FP64).  The soft branch is
// compiled into the kernels of that reduction kind (RK) only; RK -1: every
// branch, chosen from p.reduce at run time.
template <int RK = -1>
__device__ __forceinline__ double theta_step(const Params &p, double theta, int count)
{
    double r = (double)count;
    if (p.reduce == RED_MEAN) r = (double)count / (double)p.B;
    else if (p.reduce == RED_MAX || p.reduce == RED_MAX_SIGNED) r = count > 0 ? 1.0 : 0.0;
    else if ((RK == -1 || RK == RK_SOFT) && p.reduce == RED_SOFT)
        r = (double)soft_value(p, (float)count * soft_term(1.f, p.itau2_r));
    return theta * p.beta + p.theta_plus * r;
}

struct NeuronState {
    float ve, vi;
    uint32_t rf;
    float xpost;
};

// The parameters of the neuron update and its outputs, copied out of Params
// once per launch by kernels that keep Params in memory, so that the per-neuron
// code reads them from registers (same member names as Params).
struct NeuronK {
    int has_inh, learn, trace_add, n_exc, B, ls, bwords;
    LifP exc, inh;
    float w_ei, w_ie, lam_post;
};

__device__ __forceinline__ NeuronK neuron_consts(const Params &p)
{
    return NeuronK{p.has_inh, p.learn, p.trace_add, p.n_exc, p.B, p.ls, p.bwords, p.exc, p.inh, p.w_ei, p.w_ie,
                   p.lam_post};
}

// The same with the floating-point constants held in vector registers: in
// kernels short of scalar registers they would otherwise be spilled and read
// back lane by lane at every use.  (An empty asm statement with a "+v"
// operand only fixes the register class.)
__device__ __forceinline__ void in_vgpr(float &x) { asm volatile("" : "+v"(x)); }

__device__ __forceinline__ NeuronK neuron_consts_v(const Params &p)
{
    NeuronK k = neuron_consts(p);
    for (LifP *l : {&k.exc, &k.inh}) {
        in_vgpr(l->v_rest);
        in_vgpr(l->v_reset);
        in_vgpr(l->v_th);
        in_vgpr(l->alpha);
    }
    in_vgpr(k.w_ei);
    in_vgpr(k.w_ie);
    in_vgpr(k.lam_post);
    return k;
}

// One step of the excitatory adaptive-LIF neuron j and its inhibitory
// partner for one sample:
//   I_exc = I_ff + w_ie * (C_inh(t-1) - s_inh(t-1)[j])   (all-but-self)
//   I_inh = w_ei * s_exc(t-1)[j]                          (one-to-one)
//   v <- v_rest + (v - v_rest) * alpha; if refractory: count down, input
//   discarded; else v += I, spike when v >= v_th (+ theta), then v_reset and
//   refrac steps.  Post trace decays and is set on an exc spike.
template <class PP>
__device__ __forceinline__ void neuron_update(const PP &p, float I_ff, uint32_t Cprev, float th_off,
                                              NeuronState &st, bool &se, bool &si)
{
    // both outcomes are computed and selected (no branches on per-lane
    // conditions); the arithmetic of the taken outcome is unchanged
    const uint32_t re = st.rf & 0xFFu, ri = (st.rf >> 8) & 0xFFu;
    const bool se_prev = (re & RF_SPIKE) != 0u;
    const bool si_prev = (ri & RF_SPIKE) != 0u;
    const uint32_t ce = re & RF_COUNT, ci = ri & RF_COUNT;
    float Ie = I_ff;
    if (p.has_inh) Ie += p.w_ie * (float)((int)Cprev - (int)si_prev);
    const float ved = p.exc.v_rest + (st.ve - p.exc.v_rest) * p.exc.alpha;
    const float vei = ved + Ie;
    const bool e_free = ce == 0u;
    se = e_free && vei >= p.exc.v_th + th_off;
    st.ve = e_free ? (se ? p.exc.v_reset : vei) : ved;
    const uint32_t ce2 = e_free ? (se ? (uint32_t)p.exc.refrac : 0u) : ce - 1u;
    si = false;
    uint32_t ci2 = ci;
    if (p.has_inh) {
        const float Ii = se_prev ? p.w_ei : 0.f;
        const float vid = p.inh.v_rest + (st.vi - p.inh.v_rest) * p.inh.alpha;
        const float vii = vid + Ii;
        const bool i_free = ci == 0u;
        si = i_free && vii >= p.inh.v_th;
        st.vi = i_free ? (si ? p.inh.v_reset : vii) : vid;
        ci2 = i_free ? (si ? (uint32_t)p.inh.refrac : 0u) : ci - 1u;
    }
    if (p.learn) st.xpost = trace_step(st.xpost, p.lam_post, se, p.trace_add);
    st.rf = (ce2 | (se ? RF_SPIKE : 0u)) | ((ci2 | (si ? RF_SPIKE : 0u)) << 8);
}

// Optional per-call outputs of neuron (b, j) at step k of the call.
__device__ __forceinline__ void write_outputs(const Params &p, const Outs &o, int k, int b, int j, bool se,
                                              bool si, float ve, float vi)
{
    const int words = (p.n_exc + 31) >> 5;
    if (o.counts && se && (!o.until || (uint32_t)k < o.until[b])) o.counts[(size_t)b * p.n_exc + j] += 1u;
    if (o.raster_exc && se)
        atomicOr(&o.raster_exc[((size_t)k * p.B + b) * words + (j >> 5)], 1u << (j & 31));
    if (o.raster_inh && si)
        atomicOr(&o.raster_inh[((size_t)k * p.B + b) * words + (j >> 5)], 1u << (j & 31));
    if (o.v_exc) o.v_exc[((size_t)k * p.B + b) * p.n_exc + j] = ve;
    if (o.v_inh && p.has_inh) o.v_inh[((size_t)k * p.B + b) * p.n_exc + j] = vi;
}

// Outputs of a group of 8 consecutive neurons j0 .. j0+7 of sample b at
// step k; nv of them are real (the rest padding, never set in the masks).
// se_m / si_m hold their exc / inh spikes as bits 0..7.
template <class PP>
__device__ __forceinline__ void write_outputs8(const PP &p, const Outs &o, int k, int b, int j0, int nv,
                                               uint32_t se_m, uint32_t si_m, const float *ve, const float *vi)
{
    const int words = (p.n_exc + 31) >> 5;
    const size_t row = (size_t)k * p.B + b;
    if (o.counts && se_m && (!o.until || (uint32_t)k < o.until[b])) {
        // one owner per entry: a device atomic with its result unused, so the
        // step does not wait for a load of the old count
        uint32_t *cnt = o.counts + (size_t)b * p.n_exc + j0;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if ((se_m >> c) & 1u) (void)__hip_atomic_fetch_add(cnt + c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int w0 = j0 >> 5, sh = j0 & 31;
    if (o.raster_exc && se_m) {
        atomicOr(&o.raster_exc[row * words + w0], se_m << sh);
        if (sh > 24 && (se_m >> (32 - sh))) atomicOr(&o.raster_exc[row * words + w0 + 1], se_m >> (32 - sh));
    }
    if (o.raster_inh && si_m) {
        atomicOr(&o.raster_inh[row * words + w0], si_m << sh);
        if (sh > 24 && (si_m >> (32 - sh))) atomicOr(&o.raster_inh[row * words + w0 + 1], si_m >> (32 - sh));
    }
    if (o.v_exc) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < nv) o.v_exc[row * p.n_exc + j0 + c] = ve[c];
    }
    if (o.v_inh && p.has_inh) {
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < nv) o.v_inh[row * p.n_exc + j0 + c] = vi[c];
    }
}

// kernels (snn_kernels.hip)
__global__ void k_encode(Params p, const uint8_t *img, const uint64_t *ids, const uint32_t *thr_lut,
                         const uint32_t *tl, uint64_t tbase, const uint32_t *forced, uint32_t *bits,
                         uint32_t *bitsT, uint32_t *raster_in, int raster_k0);
__global__ void k_encode_lists(Params p, const uint8_t *img, const uint64_t *ids, const uint32_t *thr_lut,
                               const uint32_t *tl, uint64_t tbase, const uint32_t *forced, uint32_t *bits,
                               uint16_t *lin, uint32_t *cin, uint32_t *raster_in, int raster_k0);
__global__ void k_xpre(Params p, const uint32_t *bits_t, const float *xprev, float *xcur);
__global__ void k_contract(Params p, const float *W, const uint32_t *bits_t, float *I);
__global__ void k_neuron(Params p, const float *I, const double *theta, const uint32_t *Cprev, uint32_t *Ccur,
                         uint32_t *Cnext, float *v_exc, float *v_inh, uint16_t *rf, float *x_post, int k, Outs o);
__global__ void k_plastic(Params p, float *W, double *theta, const uint16_t *rf, const float *x_post,
                          const float *x_pre, const uint32_t *bitsT_t);
__global__ void k_reset(Params p, float *v_exc, float *v_inh, uint16_t *rf, float *x_post, float *x_pre,
                        uint32_t *C, const uint8_t *mask);
__global__ void k_fill_u32(uint32_t *dst, uint32_t value, size_t n);
__global__ void k_slot_init(const uint8_t *mask, uint32_t *tl, uint32_t *counts, int n_exc, int B);
__global__ void k_slot_move(Params p, float *v_exc, float *v_inh, float *x_post, uint16_t *rf, float *xpre_last,
                            uint32_t *C_last, SlotArrays sa, int n_in, const uint32_t *pairs, int n);
// Staging copy of the kept samples' state while the batch is re-formed
// (rows k < nk; block-major neuron arrays [g][k][jbp]).
struct RebatchStage {
    float *v_exc, *v_inh, *x_post;
    uint16_t *rf;
    float *x_pre;  // nk x n_in_pad
    uint32_t *C, *tl;
};
__global__ void k_rebatch_save(Params p, const float *v_exc, const float *v_inh, const float *x_post, const uint16_t *rf,
                               const float *xpre_last, const uint32_t *C_last, const uint32_t *tl, uint32_t t_uniform,
                               const uint32_t *keep, int nk, RebatchStage s);
__global__ void k_rebatch_load(Params p, float *v_exc, float *v_inh, float *x_post, uint16_t *rf, float *xpre_last,
                               uint32_t *C_cur, uint32_t *C_last, uint32_t *tl, int nk, RebatchStage s);
__global__ void k_add_u32(uint32_t *v, uint32_t add, int n);

}  // namespace snn
