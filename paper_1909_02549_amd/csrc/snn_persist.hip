// snn_persist.hip -- all steps of a chunk in one cooperative launch.
//
// Same column partition and step arithmetic as the fused per-step kernel,
// with the per-step round trips to HBM removed: the weight block and the
// post traces stay in LDS and each thread keeps the voltages and refractory
// state of its 8 neurons of one sample in registers for the whole launch
// (so B * JBP / 8 <= threads per block).  The
// only cross-workgroup exchange per step is the per-sample inhibitory spike
// count (device atomics) and the presynaptic traces of the next step.  A
// grid barrier separates the steps, split in two: a workgroup arrives as soon
// as it has published both for step t, then runs step t's plasticity (which
// reads only its own block, its own neurons' traces and x_pre(t), complete
// since the previous barrier) and waits before step t + 1's neuron update.
// So the plasticity hides the barrier's latency and most of the imbalance
// between workgroups.  No workgroup can then be more than one step ahead of
// another, which three x_pre buffers and three count slots cover.  The wait
// is bounded: a wait that exceeds the bound sets an error flag and ends the
// launch instead of spinning forever.
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_fused.h"
#include "snn_mfma.h"
#include "snn_kern.h"

namespace snn {

constexpr uint32_t kSpinLimit = 1u << 25;  // about a second of s_sleep(1) polls

size_t persist_lds_bytes(const Params &p) { return FusedLds(p, kPersistThreads).total; }

// Grid-wide barrier between steps, in two halves.  Arrive: every wave waits
// until its memory operations have completed (data another workgroup reads
// after the barrier is written with agent-scope atomic stores or RMWs), then
// one thread per workgroup increments the counter.  Wait: one thread polls
// until the counter reaches target; returns false if the wait timed out (the
// launch must end).
__device__ __forceinline__ void grid_arrive(const PersistSync &sy)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(sy.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool grid_wait(const PersistSync &sy, uint32_t target, int *abort_lds)
{
    if (threadIdx.x == 0) {
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

template <int PREC, int RK>
__global__ __launch_bounds__(kPersistThreads) void k_persist(const PersistArgs args)
{
    // PREC: the operand form (rounding in the gathers for BF16 / FP8); RK:
    // the reduction kind (RedKind) of the plasticity

    const Params &p = args.p;
    const FusedArgs &a = args.a;
    const ChunkPtrs &ch = args.ch;
    const PersistSync &sy = args.sy;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int abort_lds;
    const FusedLds L(p, blockDim.x);
    const StepLds S(smem, L);
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int JB = p.jb, JBP = p.jbp, ncg = p.jbp >> 3;
    float *Wg = a.W + (size_t)g * p.n_in_pad * JB;

    // prologue: weight block, thresholds, the state of this thread's tasks
    // (task u = (sample, 8 columns) number tid + u * nt)
    load_block(p, S, Wg, a.theta, g, tid, nt);
    bool has_task[kPersistTasks];
    int tb[kPersistTasks], tc0[kPersistTasks], tnv[kPersistTasks];
    float ve[kPersistTasks][8], vi[kPersistTasks][8];
    uint32_t rw[kPersistTasks][4];
    uint32_t hin_cnt[kPersistTasks];
    // list words read ahead (fewer for the reduced forms, whose rounding in
    // the gathers takes the registers: two would spill)
    constexpr int NHP = PREC == PREC_FP32 ? 2 : 1;
    uint4 hin[kPersistTasks][NHP];
#pragma unroll
    for (int u = 0; u < kPersistTasks; ++u) {
        const int q = tid + u * nt;
        has_task[u] = q < p.B * ncg;
        tb[u] = has_task[u] ? q / ncg : 0;
        tc0[u] = 8 * (q - tb[u] * ncg);
        tnv[u] = max(0, min(8, min(JB, p.n_exc - g * JB) - tc0[u]));
        hin_cnt[u] = 0u;
#pragma unroll
        for (int w = 0; w < NHP; ++w) hin[u][w] = make_uint4(0u, 0u, 0u, 0u);
        if (has_task[u]) {
            load_task_state(p, S, a, (size_t)g * p.Bs * JBP + (size_t)tb[u] * JBP + tc0[u], tb[u], tc0[u], ve[u],
                            vi[u], rw[u]);
            // the spike lists are read-only during the launch: the next
            // step's list length and first 8 * NHP entries are fetched
            // before each barrier wait
            if (ch.steps > 0) {
                hin_cnt[u] = ch.cin[tb[u]];
                load_heads<NHP>(ch.lin + (size_t)tb[u] * p.n_in_pad, hin[u]);
            }
        }
    }
    // x_pre(t) of this workgroup's own samples in registers (xpre_next_own)
    constexpr int XC = 2;
    float xc[XC];
    const bool learn = RK != RK_SERVE && p.learn;
    if (learn) xpre_own_load<XC>(p, ch.xpre + (size_t)ch.mod0 * p.Bs * p.n_in_pad, xc, g, gridDim.x, tid, nt);
    __syncthreads();

    // neuron parameters and output pointers in registers for the step loop
    const NeuronK nk = neuron_consts_v(p);
    Outs outs = a.o;
    if (RK != RK_SERVE) outs.until = nullptr;  // (read by the serving kind only)

    // the feed-forward sums of task u at step k (input list of step k, the
    // block in LDS)
    auto gather_task = [&](int k, int u, float *acc) {
        const uint16_t *row = ch.lin + ((size_t)k * p.B + tb[u]) * p.n_in_pad;
        if (PREC == PREC_FP32) {
            gather_pre<NHP>(row, (int)hin_cnt[u], hin[u], S.W, p.ls, tc0[u], p.n_in_pad, RED_SUM, acc, PREC);
        } else {
            // the reduced forms round the normalised weight w * scale
            const float4 slo = *reinterpret_cast<const float4 *>(S.scalef + tc0[u]);
            const float4 shi = *reinterpret_cast<const float4 *>(S.scalef + tc0[u] + 4);
            gather_pre<NHP, true>(row, (int)hin_cnt[u], hin[u], S.W, p.ls, tc0[u], p.n_in_pad, RED_SUM, acc, PREC,
                                  slo, shi);
        }
    };
    // The frozen kind gathers step t + 1's sums between its arrival and its
    // wait: they need only the block, which does not change, and the input
    // lists, so their time hides in the barrier's round trips (which set the
    // step time of small batches).  The learning kinds' block changes in the
    // plasticity that follows the arrival.
    constexpr bool early = RK == RK_SERVE;
    float acc_e[early ? kPersistTasks : 1][8];
    if (early && ch.steps > 0) {
#pragma unroll
        for (int u = 0; u < kPersistTasks; ++u)
            if (has_task[u]) gather_task(0, u, acc_e[u]);
    }
    for (int k = 0; k < ch.steps; ++k) {
        const int mod = (ch.mod0 + k) % 3;
        const float *xpre = ch.xpre + (size_t)mod * p.Bs * p.n_in_pad;
        float *xpre_nx = ch.xpre + (size_t)((mod + 1) % 3) * p.Bs * p.n_in_pad;

        // counts of step t - 1 and x_pre(t) from every workgroup
        if (k > 0 && !grid_wait(sy, (uint32_t)k * gridDim.x, &abort_lds)) return;
        step_begin<true>(p, S, nullptr, tid, nt);
        // C(t - 1) of this thread's samples, in flight during the first gather
        const uint32_t *Cprev = ch.C + (size_t)((mod + 2) % 3) * p.Bs;
        uint32_t cp[kPersistTasks];
#pragma unroll
        for (int u = 0; u < kPersistTasks; ++u) cp[u] = (has_task[u] && p.has_inh) ? ld_u<true>(Cprev + tb[u]) : 0u;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPersistTasks; ++u) {
            if (!has_task[u]) continue;
            float acc[8];
            if (early) {
#pragma unroll
                for (int c = 0; c < 8; ++c) acc[c] = acc_e[early ? u : 0][c];
            } else {
                gather_task(k, u, acc);
            }
            neuron_task(nk, S, outs, ch.k0 + k, tb[u], tc0[u], g * JB + tc0[u], tnv[u], acc, cp[u], ve[u], vi[u],
                        rw[u], PREC != PREC_FP32);
        }
        __syncthreads();
        step_publish<true>(p, S, ch.C + (size_t)mod * p.Bs, ch.C + (size_t)((mod + 1) % 3) * p.Bs, g, tid, nt);
        if (learn && (k + 1 < ch.steps || ch.has_next))
            xpre_next_own<XC>(p, ch.bits + (size_t)(k + 1) * p.bits_stride, xpre, xpre_nx, xc, g, gridDim.x, tid, nt);
        grid_arrive(sy);
        if (learn) {
            plasticity_all<true, 16, true, 2, false, true, RK>(
                p, S, ch.lt + (size_t)k * p.n_in_pad * p.lt_stride, ch.ct + (size_t)k * p.n_in_pad,
                ch.ord_in + (size_t)k * p.n_in_pad, xpre, tid, nt, PREC, PREC, ch.bits + (size_t)k * p.bits_stride);
            __syncthreads();
            colsums_theta<RK>(p, S, k >= ch.norm_from ? p.norm : 0.0, tid, nt);
        }
        if (k + 1 < ch.steps) {
#pragma unroll
            for (int u = 0; u < kPersistTasks; ++u) {
                if (!has_task[u]) continue;
                hin_cnt[u] = ch.cin[(size_t)(k + 1) * p.B + tb[u]];
                load_heads<NHP>(ch.lin + ((size_t)(k + 1) * p.B + tb[u]) * p.n_in_pad, hin[u]);
            }
            if (early) {
#pragma unroll
                for (int u = 0; u < kPersistTasks; ++u)
                    if (has_task[u]) gather_task(k + 1, u, acc_e[early ? u : 0]);
            }
        }
    }

    // epilogue: state, weights (normalised) and thresholds back to HBM
#pragma unroll
    for (int u = 0; u < kPersistTasks; ++u)
        if (has_task[u])
            store_task_state(p, S, a, (size_t)g * p.Bs * JBP + (size_t)tb[u] * JBP + tc0[u], tb[u], tc0[u], ve[u],
                             vi[u], rw[u]);
    if (learn) store_block(p, S, Wg, a.theta, g, tid, nt);
}

#define SNN_PERSIST_INST(PR, RK) template __global__ void k_persist<PR, RK>(const PersistArgs);
SNN_PERSIST_INST(PREC_FP32, RK_STD)
SNN_PERSIST_INST(PREC_BF16, RK_STD)
SNN_PERSIST_INST(PREC_FP8, RK_STD)
SNN_PERSIST_INST(PREC_FP32, RK_SOFT)
SNN_PERSIST_INST(PREC_BF16, RK_SOFT)
SNN_PERSIST_INST(PREC_FP8, RK_SOFT)
SNN_PERSIST_INST(PREC_FP32, RK_SIGNED)
SNN_PERSIST_INST(PREC_BF16, RK_SIGNED)
SNN_PERSIST_INST(PREC_FP8, RK_SIGNED)
SNN_PERSIST_INST(PREC_FP32, RK_SERVE)
SNN_PERSIST_INST(PREC_BF16, RK_SERVE)
SNN_PERSIST_INST(PREC_FP8, RK_SERVE)
#undef SNN_PERSIST_INST

}  // namespace snn
