// snn_indep.hip -- all steps of a chunk in one launch, for networks whose
// (sample, column) tasks are independent: no learning and no inhibitory
// layer.
//
// Without the inhibitory layer no neuron's input depends on another neuron
// of its sample, and without learning the weights and thresholds stay fixed,
// so a task's step t + 1 needs only its own state and the sample's input
// spikes of step t + 1 (the minibatch's samples are independent simulations
// of one network, each step a sum of the weight rows of the sample's active
// inputs followed by the LIF update).  The launch therefore needs no grid
// barrier and no exchange between workgroups: workgroup (g, y) holds column
// block g of the weights in LDS, each of its threads keeps one task's state
// in registers for every step of the chunk, and the grid may have any number
// of workgroups (they need not be resident at once).  The arithmetic per
// step is the fused kernel's (same gather order, same neuron update), so the
// results are bit-identical to it.
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_fused.h"
#include "snn_kern.h"

namespace snn {

size_t indep_lds_bytes(const Params &p)
{
    Params q = p;
    q.learn = 0;
    q.has_inh = 0;
    return FusedLds(q, kIndepThreads).total;
}

// grid (nblk, ceil(B * JBP / 8 / kIndepThreads)); task q = tid + nt * y is
// (sample q / ncg, columns 8 * (q % ncg) ...) of column block g.
template <int PREC>
__global__ __launch_bounds__(kIndepThreads) void k_indep(const PersistArgs args)
{
    // the host launches this kernel only for such networks: with both known
    // to be 0 here every learning and inhibition branch compiles out
    Params p = args.p;
    p.learn = 0;
    p.has_inh = 0;
    const FusedArgs &a = args.a;
    const ChunkPtrs &ch = args.ch;
    extern __shared__ __align__(16) unsigned char smem[];
    const FusedLds L(p, blockDim.x);
    const StepLds S(smem, L);
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int JB = p.jb, JBP = p.jbp, ncg = p.jbp >> 3;

    load_block(p, S, a.W + (size_t)g * p.n_in_pad * JB, a.theta, g, tid, nt);
    __syncthreads();
    if (tid < 32) S.th[tid] = theta_offset(p, S.th64[tid]);
    __syncthreads();
    // (no barrier follows: threads without a task may leave)
    const int q = tid + nt * (int)blockIdx.y;
    if (q >= p.B * ncg) return;
    const int b = q / ncg;
    const int c0 = 8 * (q - b * ncg);
    const int nv = max(0, min(8, min(JB, p.n_exc - g * JB) - c0));
    const size_t n0 = (size_t)g * p.Bs * JBP + (size_t)b * JBP + c0;
    float ve[8], vi[8];
    uint32_t rw[4];
    load_task_state(p, S, a, n0, b, c0, ve, vi, rw);

    // the step's list length and first entries are fetched a step ahead
    uint32_t cnt = ch.steps > 0 ? ch.cin[b] : 0u;
    uint4 h[kListHead];
    load_heads<kListHead>(ch.lin + (size_t)b * p.n_in_pad, h);
    for (int k = 0; k < ch.steps; ++k) {
        uint32_t cnt_nx = 0u;
        uint4 h_nx[kListHead];
        if (k + 1 < ch.steps) {
            const size_t r = (size_t)(k + 1) * p.B + b;
            cnt_nx = ch.cin[r];
            load_heads<kListHead>(ch.lin + r * p.n_in_pad, h_nx);
        } else {
#pragma unroll
            for (int w = 0; w < kListHead; ++w) h_nx[w] = make_uint4(0u, 0u, 0u, 0u);
        }
        float acc[8];
        gather_pre<kListHead>(ch.lin + ((size_t)k * p.B + b) * p.n_in_pad, (int)cnt, h, S.W, p.ls, c0, p.n_in_pad,
                              RED_SUM, acc, PREC);
        neuron_task(p, S, a.o, ch.k0 + k, b, c0, g * JB + c0, nv, acc, 0u, ve, vi, rw);
        cnt = cnt_nx;
#pragma unroll
        for (int w = 0; w < kListHead; ++w) h[w] = h_nx[w];
    }
    store_task_state(p, S, a, n0, b, c0, ve, vi, rw);
}

template __global__ void k_indep<PREC_FP32>(const PersistArgs);
template __global__ void k_indep<PREC_BF16>(const PersistArgs);
template __global__ void k_indep<PREC_FP8>(const PersistArgs);

}  // namespace snn
