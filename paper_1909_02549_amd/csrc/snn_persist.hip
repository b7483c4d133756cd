// snn_persist.hip -- all steps of a chunk in one cooperative launch.
//
// Same column partition and step arithmetic as the fused per-step kernel,
// with the per-step round trips to HBM removed: the weight block and the
// post traces stay in LDS and each thread keeps the voltages and refractory
// state of its 8 neurons of one sample in registers for the whole launch
// (so B * JBP / 8 <= threads per block).  The
// only cross-workgroup exchange per step is the per-sample inhibitory spike
// count (device atomics) and the presynaptic traces of the next step; a grid
// barrier separates the steps.  Its wait is bounded: a wait that exceeds the
// bound sets an error flag and ends the launch instead of spinning forever.
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_fused.h"
#include "snn_kern.h"

namespace snn {

constexpr uint32_t kSpinLimit = 1u << 25;  // about a second of s_sleep(1) polls

size_t persist_lds_bytes(const Params &p) { return FusedLds(p, kFusedThreads).total; }

// Grid-wide barrier between steps.  Data another workgroup reads after the
// barrier is written with agent-scope atomic stores or atomic RMWs; every
// wave waits until its memory operations have completed, then one thread per
// workgroup arrives and polls the counter.  Returns false if the wait timed
// out (the launch must end).
__device__ __forceinline__ bool grid_barrier(const PersistSync &sy, uint32_t target, int *abort_lds)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(sy.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        int ok = 1;
        while (__hip_atomic_load(sy.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > kSpinLimit) {
                __hip_atomic_store(sy.err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
        }
        *abort_lds = ok ? 0 : 1;
    }
    __syncthreads();
    return *abort_lds == 0;
}

__global__ __launch_bounds__(kFusedThreads) void k_persist(const PersistArgs *__restrict__ args)
{
    const Params &p = args->p;
    const FusedArgs &a = args->a;
    const ChunkPtrs &ch = args->ch;
    const PersistSync &sy = args->sy;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int abort_lds;
    const FusedLds L(p, blockDim.x);
    const StepLds S(smem, L);
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int JB = p.jb, JBP = p.jbp, ncg = p.jbp >> 3;
    float *Wg = a.W + (size_t)g * p.n_in_pad * JB;

    // prologue: weight block, thresholds, this thread's neuron state
    load_block(p, S, Wg, a.theta, g, tid, nt);
    const bool has_task = tid < p.B * ncg;
    const int b = has_task ? tid / ncg : 0;
    const int c0 = 8 * (tid - b * ncg);
    const size_t n0 = (size_t)g * p.Bs * JBP + (size_t)b * JBP + c0;
    const int nv = max(0, min(8, min(JB, p.n_exc - g * JB) - c0));
    float ve[8], vi[8];
    uint32_t rw[4];
    if (has_task) load_task_state(p, S, a, n0, b, c0, ve, vi, rw);
    // the spike lists are read-only during the launch: the next step's list
    // head is fetched before each barrier
    uint32_t hin_cnt = 0u;
    uint4 hin = make_uint4(0u, 0u, 0u, 0u);
    if (has_task && ch.steps > 0) {
        hin_cnt = ch.cin[b];
        hin = *reinterpret_cast<const uint4 *>(ch.lin + (size_t)b * p.n_in_pad);
    }
    __syncthreads();

    for (int k = 0; k < ch.steps; ++k) {
        const int par = (ch.par0 + k) & 1;
        const int mod = (ch.mod0 + k) % 3;
        const float *xpre = ch.xpre + (size_t)par * p.Bs * p.n_in_pad;
        float *xpre_nx = ch.xpre + (size_t)(par ^ 1) * p.Bs * p.n_in_pad;

        step_begin<true>(p, S, ch.C + (size_t)((mod + 2) % 3) * p.Bs, tid, nt);
        __syncthreads();
        if (has_task) {
            float acc[8];
            const uint16_t *row = ch.lin + ((size_t)k * p.B + b) * p.n_in_pad;
            gather8(row, (int)hin_cnt, make_uint2(hin.x, hin.y), make_uint2(hin.z, hin.w), 8, S.W, JBP, c0,
                    p.n_in_pad, RED_SUM, acc);
            neuron_task(p, S, a.o, ch.k0 + k, b, c0, g * JB + c0, nv, acc, ve, vi, rw);
        }
        __syncthreads();
        step_publish<true>(p, S, ch.C + (size_t)mod * p.Bs, ch.C + (size_t)((mod + 1) % 3) * p.Bs, g, tid, nt);
        if (p.learn) {
            __syncthreads();
            plasticity_all<true>(p, S, ch.lt + (size_t)k * p.n_in_pad * p.lt_stride, ch.ct + (size_t)k * p.n_in_pad, xpre,
                           tid, nt);
            __syncthreads();
            colsums_theta(p, S, tid, nt);
            if (k + 1 < ch.steps || ch.has_next)
                xpre_next<true>(p, ch.bits + (size_t)(k + 1) * p.bits_stride, xpre, xpre_nx, g, gridDim.x, tid, nt);
        }
        if (has_task && k + 1 < ch.steps) {
            hin_cnt = ch.cin[(size_t)(k + 1) * p.B + b];
            hin = *reinterpret_cast<const uint4 *>(ch.lin + ((size_t)(k + 1) * p.B + b) * p.n_in_pad);
        }
        if (!grid_barrier(sy, (uint32_t)(k + 1) * gridDim.x, &abort_lds)) return;
    }

    // epilogue: state, weights (normalised) and thresholds back to HBM
    if (has_task) store_task_state(p, S, a, n0, b, c0, ve, vi, rw);
    if (p.learn) store_block(p, S, Wg, a.theta, g, tid, nt);
}

}  // namespace snn
