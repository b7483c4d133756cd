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
// block g of the weights in LDS, its threads keep their tasks' state in
// registers for every step of the chunk, and the grid may have any number
// of workgroups (they need not be resident at once).  A task's 8 columns go
// to one lane (k_indep) or are spread over 2, 4 or 8 lanes (k_indep_narrow,
// 4, 2 or 1 columns each; the host takes 4, or fewer while the grid would
// leave SIMDs without a wave).  The arithmetic per step is the fused
// kernel's (same gather order, same neuron update), so the results are
// bit-identical to it.
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

// The weight block in LDS as JBP / 4 planes of 4 columns: plane u holds
// rows 0 .. n_in_pad (the last all zeros) of columns 4u .. 4u + 3, 16 bytes a
// row.  A lane's two 16-byte reads of a row then fall on any of the 8 groups
// of 4 banks, where the row-major 8-column layout left each read a choice of
// 4, so the random rows of a wave's lanes collide less often.
__device__ __forceinline__ void load_planes(const Params &p, float4 *planes, const float *Wg, int tid, int nt)
{
    const int JB = p.jb, rows = p.n_in_pad + 1, n = (p.jbp >> 2) * rows;
    for (int e = tid; e < n; e += nt) {
        const int u = e / rows, i = e - u * rows;
        float v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = 4 * u + c;
            v[c] = (i < p.n_in_pad && col < JB) ? Wg[(size_t)i * JB + col] : 0.f;
        }
        planes[e] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// acc[0..8) = sum over the first cnt entries of the list (in list order) of
// the operand values of row i, columns c0 .. c0 + 7: the additions of
// gather_pre, from the plane layout (pa: plane of columns c0 .. c0 + 3, pb:
// the next).  The first 8 * NH entries come in h.
template <int NH>
__device__ __forceinline__ void gather_planes(const uint16_t *__restrict__ list, int cnt, const uint4 *h,
                                              const float4 *pa, const float4 *pb, int zero_row, float *acc, int prec)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
    auto four = [&](uint2 q, int k0) {
        const int i0 = (int)(q.x & 0xFFFFu);
        const int i1 = k0 + 1 < cnt ? (int)(q.x >> 16) : zero_row;
        const int i2 = k0 + 2 < cnt ? (int)(q.y & 0xFFFFu) : zero_row;
        const int i3 = k0 + 3 < cnt ? (int)(q.y >> 16) : zero_row;
        const float4 a0 = round4(prec, pa[i0]), b0 = round4(prec, pb[i0]);
        const float4 a1 = round4(prec, pa[i1]), b1 = round4(prec, pb[i1]);
        const float4 a2 = round4(prec, pa[i2]), b2 = round4(prec, pb[i2]);
        const float4 a3 = round4(prec, pa[i3]), b3 = round4(prec, pb[i3]);
        add4(acc, a0), add4(acc + 4, b0);
        add4(acc, a1), add4(acc + 4, b1);
        add4(acc, a2), add4(acc + 4, b2);
        add4(acc, a3), add4(acc + 4, b3);
    };
#pragma unroll
    for (int q = 0; q < NH; ++q) {
        if (8 * q < cnt) four(make_uint2(h[q].x, h[q].y), 8 * q);
        if (8 * q + 4 < cnt) four(make_uint2(h[q].z, h[q].w), 8 * q + 4);
    }
    const uint2 *l4 = reinterpret_cast<const uint2 *>(list);
    for (int k0 = 8 * NH; k0 < cnt; k0 += 8) {
        const uint2 e0 = l4[k0 >> 2];
        const uint2 e1 = k0 + 4 < cnt ? l4[(k0 >> 2) + 1] : make_uint2(0u, 0u);
        four(e0, k0);
        if (k0 + 4 < cnt) four(e1, k0 + 4);
    }
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

    // the block as planes (in the weight region, which holds at least
    // (n_in_pad + 1) x JBP floats) and the thresholds (the weights of a
    // network that does not learn carry no pending normalisation scale)
    float4 *planes = reinterpret_cast<float4 *>(S.W);
    load_planes(p, planes, a.W + (size_t)g * p.n_in_pad * JB, tid, nt);
    if (tid < 32) {
        const int jt = g * JB + tid;
        S.th[tid] = theta_offset(p, (tid < JB && jt < p.n_exc) ? a.theta[jt] : 0.0);
    }
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
    const float4 *pa = planes + (size_t)(c0 >> 2) * (p.n_in_pad + 1);
    const float4 *pb = pa + (p.n_in_pad + 1);

    // Spike counts accumulate in registers (16 bits per neuron, a chunk has
    // at most 512 steps) and reach memory once per chunk: on gfx950 one
    // in-order counter tracks a wave's loads, stores and atomics, so a count
    // atomic issued in step t would hold up the wait for step t + 1's list
    // data.  The other outputs (rasters, voltages) are written per step.
    Outs o = a.o;
    o.counts = nullptr;
    const uint32_t until = a.o.until ? a.o.until[b] : 0xFFFFFFFFu;
    uint32_t cnt16[4] = {0u, 0u, 0u, 0u};

    // each step's list length and first entries are fetched a step ahead,
    // into two slots that alternate between the two halves of the unrolled
    // loop (no register copies, which would wait for the load just issued)
    uint32_t c0s = 0u, c1s = 0u;
    uint4 h0[kListHead], h1[kListHead];
    // (past the chunk's last step the last step's list is read again: the
    // loads stay unconditional, so the wait before a slot's first use counts
    // exactly the loads issued after it)
    auto fetch = [&](int k, uint32_t &c, uint4 *h) {
        const size_t r = (size_t)min(k, max(ch.steps - 1, 0)) * p.B + b;
        c = ch.cin[r];
        load_heads<kListHead>(ch.lin + r * p.n_in_pad, h);
    };
    auto step = [&](int k, uint32_t c, const uint4 *h) {
        float acc[8];
        gather_planes<kListHead>(ch.lin + ((size_t)k * p.B + b) * p.n_in_pad, (int)c, h, pa, pb, p.n_in_pad, acc,
                                 PREC);
        // (scale 1: the sums enter unscaled, as acc * 1 would)
        const uint32_t se = neuron_task(p, S, o, ch.k0 + k, b, c0, g * JB + c0, nv, acc, 0u, ve, vi, rw, true);
        if ((uint32_t)(ch.k0 + k) < until) {
#pragma unroll
            for (int e = 0; e < 8; ++e) cnt16[e >> 1] += ((se >> e) & 1u) << (16 * (e & 1));
        }
    };
    fetch(0, c0s, h0);
    for (int k = 0; k < ch.steps; k += 2) {
        fetch(k + 1, c1s, h1);
        step(k, c0s, h0);
        if (k + 1 >= ch.steps) break;
        fetch(k + 2, c0s, h0);
        step(k + 1, c1s, h1);
    }
    if (a.o.counts) {
        uint32_t *cnt = a.o.counts + (size_t)b * p.n_exc + g * JB + c0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint32_t v = (cnt16[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
            if (v) (void)__hip_atomic_fetch_add(cnt + e, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    store_task_state(p, S, a, n0, b, c0, ve, vi, rw);
}

// NC consecutive floats of a plane row (NC = 1, 2 or 4, the first at a
// multiple of NC within the row's 4 columns).
template <int NC>
__device__ __forceinline__ void load_cols(const float *ptr, float *v)
{
    if constexpr (NC == 4) {
        const float4 x = *reinterpret_cast<const float4 *>(ptr);
        v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
    } else if constexpr (NC == 2) {
        const float2 x = *reinterpret_cast<const float2 *>(ptr);
        v[0] = x.x, v[1] = x.y;
    } else {
        v[0] = *ptr;
    }
}

// The narrow form, for grids too small to fill the GPU (small batches): the
// columns of each 8-column task are spread over 8 / NC lanes (NC = 1, 2 or
// 4 columns each), which walk the same input list, so each lane's chain of
// dependent instructions per step is shorter.  The sums run in the same
// order and the neuron update is the same, so the results are bit-identical
// to k_indep's.  Lane q = tid + nt * y: 8-column task q / (8 / NC), its
// columns NC * (q % (8 / NC)) ...
template <int PREC, int NC>
__global__ __launch_bounds__(kIndepThreads) void k_indep_narrow(const PersistArgs args)
{
    constexpr int L = 8 / NC;
    Params p = args.p;
    p.learn = 0;
    p.has_inh = 0;
    const FusedArgs &a = args.a;
    const ChunkPtrs &ch = args.ch;
    extern __shared__ __align__(16) unsigned char smem[];
    const FusedLds Lds(p, blockDim.x);
    const StepLds S(smem, Lds);
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int JB = p.jb, JBP = p.jbp, ncg = p.jbp >> 3;

    float4 *planes = reinterpret_cast<float4 *>(S.W);
    load_planes(p, planes, a.W + (size_t)g * p.n_in_pad * JB, tid, nt);
    if (tid < 32) {
        const int jt = g * JB + tid;
        S.th[tid] = theta_offset(p, (tid < JB && jt < p.n_exc) ? a.theta[jt] : 0.0);
    }
    __syncthreads();
    // (no barrier follows: threads without a task may leave)
    const int q = tid + nt * (int)blockIdx.y;
    if (q >= p.B * ncg * L) return;
    const int t8 = q / L;
    const int b = t8 / ncg;
    const int c0 = 8 * (t8 - b * ncg) + NC * (q - t8 * L);
    const int nv = max(0, min(NC, min(JB, p.n_exc - g * JB) - c0));
    const size_t n0 = (size_t)g * p.Bs * JBP + (size_t)b * JBP + c0;
    float ve[NC];
    uint32_t rf[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        ve[c] = a.v_exc[n0 + c];
        rf[c] = a.rf[n0 + c];
    }
    // this lane's columns in their plane (4 floats a row)
    const float *pl = reinterpret_cast<const float *>(planes + (size_t)(c0 >> 2) * (p.n_in_pad + 1)) + (c0 & 3);
    const int zero_row = p.n_in_pad;

    // counts in registers as in k_indep (16 bits per neuron), other outputs
    // per step
    Outs o = a.o;
    o.counts = nullptr;
    const uint32_t until = a.o.until ? a.o.until[b] : 0xFFFFFFFFu;
    uint32_t cnt16[(NC + 1) / 2];
#pragma unroll
    for (int e = 0; e < (NC + 1) / 2; ++e) cnt16[e] = 0u;

    // sum over the list in list order, four entries in flight (the additions
    // of gather_planes, column by column)
    auto gather = [&](const uint16_t *__restrict__ list, int cnt, const uint4 *h, float *acc) {
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.f;
        auto four = [&](uint2 e, int k0) {
            const int i0 = (int)(e.x & 0xFFFFu);
            const int i1 = k0 + 1 < cnt ? (int)(e.x >> 16) : zero_row;
            const int i2 = k0 + 2 < cnt ? (int)(e.y & 0xFFFFu) : zero_row;
            const int i3 = k0 + 3 < cnt ? (int)(e.y >> 16) : zero_row;
            float v[4][NC];
            load_cols<NC>(pl + 4 * i0, v[0]);
            load_cols<NC>(pl + 4 * i1, v[1]);
            load_cols<NC>(pl + 4 * i2, v[2]);
            load_cols<NC>(pl + 4 * i3, v[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[c] += operand_value(PREC, v[r][c]);
        };
#pragma unroll
        for (int w = 0; w < kListHead; ++w) {
            if (8 * w < cnt) four(make_uint2(h[w].x, h[w].y), 8 * w);
            if (8 * w + 4 < cnt) four(make_uint2(h[w].z, h[w].w), 8 * w + 4);
        }
        const uint2 *l4 = reinterpret_cast<const uint2 *>(list);
        for (int k0 = 8 * kListHead; k0 < cnt; k0 += 8) {
            const uint2 e0 = l4[k0 >> 2];
            const uint2 e1 = k0 + 4 < cnt ? l4[(k0 >> 2) + 1] : make_uint2(0u, 0u);
            four(e0, k0);
            if (k0 + 4 < cnt) four(e1, k0 + 4);
        }
    };

    uint32_t c0s = 0u, c1s = 0u;
    uint4 h0[kListHead], h1[kListHead];
    auto fetch = [&](int k, uint32_t &c, uint4 *h) {
        const size_t r = (size_t)min(k, max(ch.steps - 1, 0)) * p.B + b;
        c = ch.cin[r];
        load_heads<kListHead>(ch.lin + r * p.n_in_pad, h);
    };
    auto step = [&](int k, uint32_t cnt, const uint4 *h) {
        float acc[NC];
        gather(ch.lin + ((size_t)k * p.B + b) * p.n_in_pad, (int)cnt, h, acc);
        const int kk = ch.k0 + k;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            NeuronState st{ve[c], 0.f, rf[c], 0.f};
            bool se, si;
            neuron_update(p, acc[c], 0u, S.th[c0 + c], st, se, si);
            const bool real = c < nv;
            ve[c] = real ? st.ve : ve[c];
            rf[c] = real ? st.rf : rf[c];
            if (real) {
                write_outputs(p, o, kk, b, g * JB + c0 + c, se, false, ve[c], 0.f);
                if (se && (uint32_t)kk < until) cnt16[c >> 1] += 1u << (16 * (c & 1));
            }
        }
    };
    fetch(0, c0s, h0);
    for (int k = 0; k < ch.steps; k += 2) {
        fetch(k + 1, c1s, h1);
        step(k, c0s, h0);
        if (k + 1 >= ch.steps) break;
        fetch(k + 2, c0s, h0);
        step(k + 1, c1s, h1);
    }
    if (a.o.counts) {
        uint32_t *cnt = a.o.counts + (size_t)b * p.n_exc + g * JB + c0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t v = (cnt16[c >> 1] >> (16 * (c & 1))) & 0xFFFFu;
            if (v) (void)__hip_atomic_fetch_add(cnt + c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        a.v_exc[n0 + c] = ve[c];
        a.rf[n0 + c] = (uint16_t)rf[c];
    }
}

#define SNN_NARROW_INST(PR)                                                  \
    template __global__ void k_indep_narrow<PR, 1>(const PersistArgs);   \
    template __global__ void k_indep_narrow<PR, 2>(const PersistArgs);   \
    template __global__ void k_indep_narrow<PR, 4>(const PersistArgs);
SNN_NARROW_INST(PREC_FP32)
SNN_NARROW_INST(PREC_BF16)
SNN_NARROW_INST(PREC_FP8)
#undef SNN_NARROW_INST

template __global__ void k_indep<PREC_FP32>(const PersistArgs);
template __global__ void k_indep<PREC_BF16>(const PersistArgs);
template __global__ void k_indep<PREC_FP8>(const PersistArgs);

}  // namespace snn
