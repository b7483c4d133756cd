// snn_fused.hip -- one column-partitioned launch per SNN step, and the
// builder of the sparse spike lists both step kernels read.
//
// Step t in workgroup g (building blocks in snn_fused.h):
//   A  stage the weight block, thresholds, C(t-1)
//   B  task (b, 8 columns), samples in the step's work order: neuron state
//      from HBM; I = sum over the inputs in sample b's spike list (increasing
//      i) of W[i, cols]; recurrent currents; exc adaptive-LIF and inh LIF
//      update; post trace; state back
//   C  (learning) potentiation from the presynaptic traces of the samples
//      whose neurons fired (matrix cores for sum / mean), then per input row
//      (in the step's work order) depression from the post traces of the
//      samples in which input i fired, clamp
//   C3 (learning) FP64 column sums, normalisation scale, theta update
//   E  (learning) x_pre(t+1) for this workgroup's share of the samples, the
//      block back to HBM normalised
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_fused.h"
#include "snn_kern.h"

namespace snn {

size_t fused_lds_bytes(const Params &p) { return FusedLds(p, kFusedThreads, true).total; }

// PREC: the operand form; RK: the reduction kind (RedKind) of the
// plasticity.  For BF16 / FP8 the contraction rounds each weight as it is
// gathered (the block in LDS stays FP32 for the plasticity; it was
// normalised when it was stored, so no scale is pending at this point), the
// post traces in LDS are rounded once after the neurons' state went back to
// HBM in FP32, and the presynaptic traces are rounded as they are read.
template <int PREC, int RK>
__global__ __launch_bounds__(kFusedThreads) void k_fused_step(Params p, FusedArgs a, StepPtrs s)
{
    // the frozen kind (RK_SERVE) runs networks that do not learn: with
    // learn known to be 0 here, every plasticity branch compiles out and the
    // kernel needs fewer registers
    if constexpr (RK == RK_SERVE) p.learn = 0;
    extern __shared__ __align__(16) unsigned char smem[];
    const FusedLds L(p, blockDim.x, true);
    const StepLds S(smem, L);
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int JB = p.jb, JBP = p.jbp, ncg = p.jbp >> 3;
    float *Wg = a.W + (size_t)g * p.n_in_pad * JB;

    load_block(p, S, Wg, a.theta, g, tid, nt);
    __syncthreads();
    step_begin<false>(p, S, s.Cprev, tid, nt);
    __syncthreads();

    // B: one (sample, 8 columns) task at a time, state through registers.
    // Without learning the samples are independent, and the grid's y
    // dimension splits them between workgroups of the same column block
    // (with learning gridDim.y is 1: the plasticity needs every sample)
    const size_t sbase = (size_t)g * p.Bs * JBP;
    const int nv_blk = min(JB, p.n_exc - g * JB);
    for (int q = tid + (int)blockIdx.y * nt; q < p.B * ncg; q += nt * (int)gridDim.y) {
        const int qb = q / ncg;
        const int b = s.ord_s[qb];
        const int c0 = 8 * (q - qb * ncg);
        const size_t n0 = sbase + (size_t)b * JBP + c0;
        float ve[8], vi[8], acc[8];
        uint32_t rw[4];
        const uint32_t cnt = s.cin[b];
        const uint16_t *row = s.lin + (size_t)b * p.n_in_pad;
        uint4 h[kListHead];
        load_heads<kListHead>(row, h);
        load_task_state(p, S, a, n0, b, c0, ve, vi, rw);
        gather_pre<kListHead>(row, (int)cnt, h, S.W, p.ls, c0, p.n_in_pad, RED_SUM, acc, PREC);
        neuron_task(p, S, a.o, s.k, b, c0, g * JB + c0, max(0, min(8, nv_blk - c0)), acc,
                    S.cprev[p.has_inh ? b : 0], ve, vi, rw);
        store_task_state(p, S, a, n0, b, c0, ve, vi, rw);
        if (PREC != PREC_FP32 && p.learn) {
            float *xr = S.xpost + b * p.ls + c0;
#pragma unroll
            for (int c = 0; c < 8; ++c) xr[c] = operand_value(PREC, xr[c]);
        }
    }
    __syncthreads();
    step_publish<false>(p, S, s.Ccur, s.Cnext, g, tid, nt);
    if (!p.learn) return;
    __syncthreads();

    plasticity_all<false, 16, true, kListHead, PREC == PREC_FP32, false, RK>(p, S, s.lt, s.ct, s.ord_in, s.xpre,
                                                                            tid, nt, PREC, 0, s.bits);
    __syncthreads();
    colsums_theta<RK>(p, S, p.norm, tid, nt);
    if (s.bits_next) xpre_next<false>(p, s.bits_next, s.xpre, s.xpre_next, g, gridDim.x, tid, nt);
    store_block(p, S, Wg, a.theta, g, tid, nt);
}

#define SNN_FUSED_INST(PR, RK) template __global__ void k_fused_step<PR, RK>(Params, FusedArgs, StepPtrs);
SNN_FUSED_INST(PREC_FP32, RK_STD)
SNN_FUSED_INST(PREC_BF16, RK_STD)
SNN_FUSED_INST(PREC_FP8, RK_STD)
SNN_FUSED_INST(PREC_FP32, RK_SOFT)
SNN_FUSED_INST(PREC_BF16, RK_SOFT)
SNN_FUSED_INST(PREC_FP8, RK_SOFT)
SNN_FUSED_INST(PREC_FP32, RK_SIGNED)
SNN_FUSED_INST(PREC_BF16, RK_SIGNED)
SNN_FUSED_INST(PREC_FP8, RK_SIGNED)
SNN_FUSED_INST(PREC_FP32, RK_SERVE)
SNN_FUSED_INST(PREC_BF16, RK_SERVE)
SNN_FUSED_INST(PREC_FP8, RK_SERVE)
#undef SNN_FUSED_INST

// Sparse index lists of one chunk of encoded steps:
//   lin[t][b][0 .. cin[t][b])  inputs that spiked in sample b (increasing)
//   lt [t][i][0 .. ct[t][i])   samples in which input i spiked (increasing)
__global__ void k_lists(Params p, const uint32_t *__restrict__ bits, const uint32_t *__restrict__ bitsT,
                        uint16_t *__restrict__ lin, uint32_t *__restrict__ cin, uint16_t *__restrict__ lt,
                        uint32_t *__restrict__ ct, int with_t)
{
    const int t = blockIdx.y;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < p.B) {
        const uint32_t *w = bits + (size_t)t * p.bits_stride + (size_t)q * p.in_words;
        uint16_t *out = lin + ((size_t)t * p.B + q) * p.n_in_pad;
        uint32_t n = 0;
        for (int k = 0; k < p.in_words; ++k) {
            uint32_t m = w[k];
            while (m) {
                out[n++] = (uint16_t)(32 * k + __builtin_ctz(m));
                m &= m - 1;
            }
        }
        cin[(size_t)t * p.B + q] = n;
    }
    if (with_t && q < p.n_in_pad) {
        const uint32_t *w = bitsT + ((size_t)t * p.n_in_pad + q) * p.bwords;
        uint16_t *out = lt + ((size_t)t * p.n_in_pad + q) * p.lt_stride;
        uint32_t n = 0;
        for (int k = 0; k < p.bwords; ++k) {
            uint32_t m = w[k];
            while (m) {
                out[n++] = (uint16_t)(32 * k + __builtin_ctz(m));
                m &= m - 1;
            }
        }
        ct[(size_t)t * p.n_in_pad + q] = n;
    }
}

}  // namespace snn

namespace snn {

// Work order of one step's list walks: the samples by decreasing input-list
// length cin and the inputs by decreasing sample-list length ct (a counting
// sort, lengths above kOrderBins - 2 sharing the first bin; order within a
// bin is arbitrary).  A wave of the step kernels takes consecutive entries,
// so its lanes walk lists of similar length.  Which thread handles which
// sample or input changes nothing in the results.  One workgroup per step.
__global__ __launch_bounds__(kOrderThreads) void k_order(Params p, const uint32_t *__restrict__ cin,
                                                          const uint32_t *__restrict__ ct, uint16_t *__restrict__ ord_s,
                                                          uint16_t *__restrict__ ord_in, int with_t)
{
    __shared__ uint32_t hist[kOrderBins];
    __shared__ uint32_t wsum[kOrderThreads / 64];
    const int t = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    auto bin = [](uint32_t c) { return kOrderBins - 1 - (int)min(c, (uint32_t)(kOrderBins - 1)); };
    for (int pass = 0; pass < (with_t ? 2 : 1); ++pass) {
        const int n = pass == 0 ? p.B : p.n_in;
        const uint32_t *len = pass == 0 ? cin + (size_t)t * p.B : ct + (size_t)t * p.n_in_pad;
        uint16_t *out = pass == 0 ? ord_s + (size_t)t * p.B : ord_in + (size_t)t * p.n_in_pad;
        for (int q = tid; q < kOrderBins; q += kOrderThreads) hist[q] = 0u;
        __syncthreads();
        for (int q = tid; q < n; q += kOrderThreads) atomicAdd(&hist[bin(len[q])], 1u);
        __syncthreads();
        // exclusive prefix sum over the bins (one bin per thread)
        const uint32_t v = hist[tid];
        uint32_t x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        uint32_t base = 0u;
        for (int w = 0; w < wv; ++w) base += wsum[w];
        hist[tid] = base + x - v;
        __syncthreads();
        for (int q = tid; q < n; q += kOrderThreads) out[atomicAdd(&hist[bin(len[q])], 1u)] = (uint16_t)q;
        __syncthreads();
    }
}

}  // namespace snn
