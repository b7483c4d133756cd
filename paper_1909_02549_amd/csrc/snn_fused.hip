// snn_fused.hip -- one column-partitioned launch per SNN step.
//
// Workgroup g owns the JB post-synaptic columns [g*JB, g*JB+JB) for every
// sample of the batch: their weight block W[:, cols] (staged in LDS), their
// neuron state and their adaptive thresholds.  What the method couples across
// columns is small: the per-sample inhibitory spike count C[b] (all-but-self
// inhibition) and the presynaptic traces x_pre (read by every column); both
// are exchanged through global memory between steps.
//
// In LDS the block is stored with JBP = JB rounded up to 8 columns per row
// plus one all-zero row, so a thread owning 8 consecutive columns reads a row
// with two 16-byte loads, and padding slots of an index list point at the
// zero row (adding +0 leaves a sum unchanged).
//
// Step t in workgroup g:
//   A  stage the weight block, thresholds and C(t-1)
//   B  task (b, 8 columns): I = sum over the inputs i in sample b's spike
//      list (increasing i) of W[i, cols]; recurrent currents; exc
//      adaptive-LIF and inh LIF update; post trace.  Exc spikes set per-column
//      sample masks, inh spikes add to C(t)
//   C1 (learning) potentiation: for each column with post spikes, all
//      threads sweep the rows with P = R over its spiking samples of x_pre
//   C2 (learning) task (i, 8 columns): D = R over the samples in input i's
//      spike list of x_post[b, cols]; W = clamp(W + nu_post P - nu_pre D)
//   C3 (learning) FP64 column sums, scale to the target sum, theta update,
//      block written back scaled
//   E  (learning) x_pre(t+1) for this workgroup's share of the samples
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_fused.h"

namespace snn {

// LDS carve-up shared by host (size) and device (offsets).
struct FusedLds {
    size_t w, xpost, cprev, cinh, spk, part, scale, theta, total;
    __host__ __device__ FusedLds(const Params &p, int nthreads)
    {
        size_t o = 0;
        w = o;
        o += align16((size_t)(p.n_in_pad + 1) * p.jbp * 4);
        xpost = o;
        o += p.learn ? align16((size_t)(p.B + 1) * p.jbp * 4) : 0;
        cprev = o;
        o += align16((size_t)p.B * 4);
        cinh = o;
        o += align16((size_t)p.B * 4);
        spk = o;
        o += align16((size_t)p.jb * p.bwords * 4);
        part = o;
        o += align16((size_t)(nthreads / 32) * 32 * 8);
        scale = o;
        o += 32 * 8;
        theta = o;
        o += 32 * 4;
        total = o;
    }
};

size_t fused_lds_bytes(const Params &p) { return FusedLds(p, kFusedThreads).total; }

__device__ __forceinline__ void add4(float *acc, const float4 v)
{
    acc[0] += v.x;
    acc[1] += v.y;
    acc[2] += v.z;
    acc[3] += v.w;
}

__device__ __forceinline__ void red4(int mode, float *acc, const float4 v)
{
    acc[0] = reduce2(mode, acc[0], v.x);
    acc[1] = reduce2(mode, acc[1], v.y);
    acc[2] = reduce2(mode, acc[2], v.z);
    acc[3] = reduce2(mode, acc[3], v.w);
}

// acc[0..8) = R over the first `cnt` entries of `list` (u16 row indices, in
// list order) of rows[idx * jbp + c0 .. + 8), four rows in flight at a time;
// slots past cnt read row `zero_row` (all zeros).
__device__ __forceinline__ void gather8(const uint16_t *__restrict__ list, int cnt, const float *rows, int jbp,
                                        int c0, int zero_row, int mode, float *acc)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
    const uint2 *l4 = reinterpret_cast<const uint2 *>(list);
    for (int k0 = 0; k0 < cnt; k0 += 4) {
        const uint2 q = l4[k0 >> 2];
        const int i0 = (int)(q.x & 0xFFFFu);
        const int i1 = k0 + 1 < cnt ? (int)(q.x >> 16) : zero_row;
        const int i2 = k0 + 2 < cnt ? (int)(q.y & 0xFFFFu) : zero_row;
        const int i3 = k0 + 3 < cnt ? (int)(q.y >> 16) : zero_row;
        const float4 *r0 = reinterpret_cast<const float4 *>(rows + i0 * jbp + c0);
        const float4 *r1 = reinterpret_cast<const float4 *>(rows + i1 * jbp + c0);
        const float4 *r2 = reinterpret_cast<const float4 *>(rows + i2 * jbp + c0);
        const float4 *r3 = reinterpret_cast<const float4 *>(rows + i3 * jbp + c0);
        const float4 a0 = r0[0], b0 = r0[1], a1 = r1[0], b1 = r1[1];
        const float4 a2 = r2[0], b2 = r2[1], a3 = r3[0], b3 = r3[1];
        if (mode == RED_MAX) {
            red4(mode, acc, a0), red4(mode, acc + 4, b0);
            red4(mode, acc, a1), red4(mode, acc + 4, b1);
            red4(mode, acc, a2), red4(mode, acc + 4, b2);
            red4(mode, acc, a3), red4(mode, acc + 4, b3);
        } else {
            add4(acc, a0), add4(acc + 4, b0);
            add4(acc, a1), add4(acc + 4, b1);
            add4(acc, a2), add4(acc + 4, b2);
            add4(acc, a3), add4(acc + 4, b3);
        }
    }
}

__global__ __launch_bounds__(kFusedThreads) void k_fused_step(Params p, FusedArgs a, StepPtrs s)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const FusedLds L(p, blockDim.x);
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int JB = p.jb, JBP = p.jbp, ncg = p.jbp >> 3;
    const int jj = tid & 31;
    const int rg = tid >> 5;
    const int nrg = nt >> 5;

    float *W_lds = reinterpret_cast<float *>(smem + L.w);
    float *xpost_lds = reinterpret_cast<float *>(smem + L.xpost);
    uint32_t *cprev_lds = reinterpret_cast<uint32_t *>(smem + L.cprev);
    uint32_t *cinh_lds = reinterpret_cast<uint32_t *>(smem + L.cinh);
    uint32_t *spk = reinterpret_cast<uint32_t *>(smem + L.spk);
    double *part = reinterpret_cast<double *>(smem + L.part);
    double *scale = reinterpret_cast<double *>(smem + L.scale);
    float *th_lds = reinterpret_cast<float *>(smem + L.theta);
    float *Wg = a.W + (size_t)g * p.n_in_pad * JB;

    // A: weight block (row-padded to JBP, plus the zero row), small inputs
    if (jj < JBP) {
        int i = rg;
        for (; i + 3 * nrg < p.n_in_pad; i += 4 * nrg) {
            float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f;
            if (jj < JB) {
                v0 = Wg[(size_t)i * JB + jj];
                v1 = Wg[(size_t)(i + nrg) * JB + jj];
                v2 = Wg[(size_t)(i + 2 * nrg) * JB + jj];
                v3 = Wg[(size_t)(i + 3 * nrg) * JB + jj];
            }
            W_lds[i * JBP + jj] = v0;
            W_lds[(i + nrg) * JBP + jj] = v1;
            W_lds[(i + 2 * nrg) * JBP + jj] = v2;
            W_lds[(i + 3 * nrg) * JBP + jj] = v3;
        }
        for (; i < p.n_in_pad; i += nrg) W_lds[i * JBP + jj] = jj < JB ? Wg[(size_t)i * JB + jj] : 0.f;
        if (rg == 0) {
            W_lds[p.n_in_pad * JBP + jj] = 0.f;
            if (p.learn) xpost_lds[p.B * JBP + jj] = 0.f;
        }
    }
    for (int b = tid; b < p.B; b += nt) {
        cprev_lds[b] = p.has_inh ? s.Cprev[b] : 0u;
        cinh_lds[b] = 0u;
    }
    for (int q = tid; q < JB * p.bwords; q += nt) spk[q] = 0u;
    if (tid < 32) {
        const int jt = g * JB + tid;
        th_lds[tid] = (tid < JB && jt < p.n_exc) ? theta_offset(p, a.theta[jt]) : 0.f;
    }
    __syncthreads();

    // B: contraction + neuron update, task (b, column group)
    const size_t sbase = (size_t)g * p.B * JB;
    for (int q = tid; q < p.B * ncg; q += nt) {
        const int b = q / ncg;
        const int c0 = 8 * (q - b * ncg);
        NeuronState st[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int jl = c0 + c;
            st[c] = NeuronState{0.f, 0.f, 0u, 0.f};
            if (jl < JB && g * JB + jl < p.n_exc) {
                const size_t n = sbase + (size_t)b * JB + jl;
                st[c].ve = a.v_exc[n];
                st[c].vi = p.has_inh ? a.v_inh[n] : 0.f;
                st[c].rf = a.rf[n];
                st[c].xpost = p.learn ? a.x_post[n] : 0.f;
            }
        }
        float acc[8];
        gather8(s.lin + (size_t)b * p.n_in_pad, (int)s.cin[b], W_lds, JBP, c0, p.n_in_pad, RED_SUM, acc);
        uint32_t cnt_inh = 0u;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int jl = c0 + c;
            const int j = g * JB + jl;
            if (jl < JB && j < p.n_exc) {
                const size_t n = sbase + (size_t)b * JB + jl;
                bool se, si;
                neuron_update(p, acc[c], cprev_lds[b], th_lds[jl], st[c], se, si);
                a.v_exc[n] = st[c].ve;
                if (p.has_inh) a.v_inh[n] = st[c].vi;
                a.rf[n] = (uint16_t)st[c].rf;
                if (p.learn) {
                    a.x_post[n] = st[c].xpost;
                    xpost_lds[b * JBP + jl] = st[c].xpost;
                    if (se) atomicOr(&spk[jl * p.bwords + (b >> 5)], 1u << (b & 31));
                }
                cnt_inh += si ? 1u : 0u;
                write_outputs(p, a.o, s.k, b, j, se, si, st[c].ve, st[c].vi);
            } else if (p.learn && jl < JBP) {
                xpost_lds[b * JBP + jl] = 0.f;
            }
        }
        if (cnt_inh) atomicAdd(&cinh_lds[b], cnt_inh);
    }
    __syncthreads();
    for (int b = tid; b < p.B; b += nt) {
        const uint32_t c = cinh_lds[b];
        if (c) atomicAdd(&s.Ccur[b], c);
        if (g == 0 && s.Cnext) s.Cnext[b] = 0u;
    }
    if (!p.learn) return;

    // C1: potentiation, W[i, c] += nu_post * R_{b spiking in c} x_pre[b, i]
    for (int c = 0; c < JB; ++c) {
        const uint32_t *sp = spk + c * p.bwords;
        uint32_t any = 0u;
        for (int bw = 0; bw < p.bwords; ++bw) any |= sp[bw];
        if (!any) continue;
        for (int i = tid; i < p.n_in; i += nt) {
            float P = 0.f;
            for (int bw = 0; bw < p.bwords; ++bw) {
                uint32_t m = sp[bw];
                while (m) {
                    const int b = 32 * bw + __builtin_ctz(m);
                    m &= m - 1;
                    P = reduce2(p.reduce, P, s.xpre[(size_t)b * p.n_in_pad + i]);
                }
            }
            if (p.reduce == RED_MEAN) P *= p.inv_B;
            W_lds[i * JBP + c] = W_lds[i * JBP + c] + p.nu_post * P;
        }
    }
    __syncthreads();

    // C2: depression and clamp, task (i, column group)
    for (int q = tid; q < p.n_in * ncg; q += nt) {
        const int i = q / ncg;
        const int c0 = 8 * (q - i * ncg);
        float D[8];
        gather8(s.lt + (size_t)i * p.lt_stride, (int)s.ct[i], xpost_lds, JBP, c0, p.B, p.reduce, D);
        float4 *wr = reinterpret_cast<float4 *>(W_lds + i * JBP + c0);
        const float4 w0 = wr[0], w1 = wr[1];
        float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float d = D[c];
            if (p.reduce == RED_MEAN) d *= p.inv_B;
            w[c] = fminf(fmaxf(w[c] - p.nu_pre * d, p.w_min), p.w_max);
        }
        wr[0] = make_float4(w[0], w[1], w[2], w[3]);
        wr[1] = make_float4(w[4], w[5], w[6], w[7]);
    }
    __syncthreads();

    // C3: column sums (FP64), normalisation factor, theta, write-back
    double cs = 0.0;
    if (jj < JB)
        for (int i = rg; i < p.n_in; i += nrg) cs += (double)W_lds[i * JBP + jj];
    part[rg * 32 + jj] = cs;
    __syncthreads();
    if (tid < 32) {
        double c = 0.0;
        for (int r = 0; r < nrg; ++r) c += part[r * 32 + tid];
        scale[tid] = (p.norm > 0.0 && c > 0.0) ? p.norm / c : 1.0;
        const int jt = g * JB + tid;
        if (tid < JB && jt < p.n_exc && p.adaptive) {
            int cnt = 0;
            for (int bw = 0; bw < p.bwords; ++bw) cnt += __builtin_popcount(spk[tid * p.bwords + bw]);
            a.theta[jt] = theta_step(p, a.theta[jt], cnt);
        }
    }

    // E: presynaptic traces of the next step for this workgroup's samples
    if (s.bits_next) {
        for (int b = g; b < p.B; b += gridDim.x) {
            const uint32_t *sb = s.bits_next + (size_t)b * p.in_words;
            const float *xc = s.xpre + (size_t)b * p.n_in_pad;
            float *xn = s.xpre_next + (size_t)b * p.n_in_pad;
            for (int i = tid; i < p.n_in_pad; i += nt)
                xn[i] = trace_step(xc[i], p.lam_pre, (sb[i >> 5] >> (i & 31)) & 1u, p.trace_add);
        }
    }
    __syncthreads();
    if (jj < JB) {
        const bool do_scale = p.norm > 0.0;
        const double sc = scale[jj];
        for (int i = rg; i < p.n_in_pad; i += nrg) {
            float w = W_lds[i * JBP + jj];
            if (do_scale && i < p.n_in) w = (float)((double)w * sc);
            Wg[(size_t)i * JB + jj] = w;
        }
    }
}

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
