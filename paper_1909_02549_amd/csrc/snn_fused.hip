// snn_fused.hip -- one column-partitioned launch per SNN step, and the same
// step body run for all T steps by one cooperative (persistent) launch.
//
// Workgroup g owns the JB post-synaptic columns [g*JB, g*JB+JB) for every
// sample of the batch: their weight block W[:, cols] (staged in LDS), their
// neuron state, their adaptive thresholds.  Everything the method couples
// across columns is small: the per-sample inhibitory spike count C[b] (all-
// but-self inhibition) and the presynaptic traces x_pre (shared by all
// columns); both are exchanged through global memory between steps.
//
// Step t in workgroup g:
//   A  stage W block in LDS, thresholds and C(t-1) in LDS
//   B  per (b, j): I = sum of W[i, j] over inputs i that spiked in sample b
//      (gather from LDS), recurrent currents, exc adaptive-LIF + inh LIF
//      update, post trace; exc spikes -> per-column sample masks in LDS,
//      inh spikes -> per-sample counts -> C(t)
//   C  (learning) per (i, j): D = R_b over samples where input i spiked of
//      x_post[b, j]; P = R_b over samples where j spiked of x_pre[b, i];
//      W = clamp(W + nu_post P - nu_pre D); FP64 column sums; scale to norm;
//      theta update; W block back to HBM
//   E  (learning) x_pre(t+1) for this workgroup's share of the samples
// Thread mapping: lane = (bs, jj), bs = lane / 32 picks one of two samples a
// wave handles per round, jj = lane % 32 the column (JB <= 32).
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_fused.h"

namespace snn {

// LDS carve-up shared by host (size) and device (offsets).
struct FusedLds {
    size_t w, xpost, bits, cprev, cinh, spk, part, scale, theta, total;
    __host__ __device__ FusedLds(const Params &p, int nthreads)
    {
        size_t o = 0;
        w = o;
        o += align16((size_t)p.n_in_pad * p.jb * 4);
        xpost = o;
        o += p.learn ? align16((size_t)p.B * p.jb * 4) : 0;
        // input spikes of the step: B x in_words for the contraction, then
        // reused for the transpose n_in_pad x bwords during plasticity
        bits = o;
        {
            const size_t a1 = (size_t)p.B * p.in_words * 4;
            const size_t a2 = p.learn ? (size_t)p.n_in_pad * p.bwords * 4 : 0;
            o += align16(a1 > a2 ? a1 : a2);
        }
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

// Bulk copy with four 16-byte loads in flight per thread (all four loads
// are issued before the first store).
__device__ __forceinline__ void copy_u4(void *dst_, const void *__restrict__ src_, size_t n_words, int tid, int nt)
{
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src_);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst_);
    const size_t n4 = n_words / 4;
    const size_t st = (size_t)nt;
    size_t q = tid;
    for (; q + 3 * st < n4; q += 4 * st) {
        const uint4 r0 = s4[q], r1 = s4[q + st], r2 = s4[q + 2 * st], r3 = s4[q + 3 * st];
        d4[q] = r0;
        d4[q + st] = r1;
        d4[q + 2 * st] = r2;
        d4[q + 3 * st] = r3;
    }
    for (; q < n4; q += st) d4[q] = s4[q];
    const uint32_t *s1 = reinterpret_cast<const uint32_t *>(src_);
    uint32_t *d1 = reinterpret_cast<uint32_t *>(dst_);
    for (size_t e = n4 * 4 + tid; e < n_words; e += st) d1[e] = s1[e];
}

// R over the set bits k (in increasing order) of words[0..nwords) of
// src[k * stride]; words are fetched four at a time and the next element's
// load is issued before the previous one is accumulated.
__device__ __forceinline__ float gather_bits(const uint32_t *words, int nwords, const float *src, int stride,
                                             int mode)
{
    float acc = 0.f, pend = 0.f;
    bool hp = false;
    auto word = [&](uint32_t mm, int base) {
        while (mm) {
            const int k = base + __builtin_ctz(mm);
            mm &= mm - 1;
            const float v = src[k * stride];
            if (hp) acc = reduce2(mode, acc, pend);
            pend = v;
            hp = true;
        }
    };
    int w0 = 0;
    for (; w0 + 4 <= nwords; w0 += 4) {
        const uint32_t m0 = words[w0], m1 = words[w0 + 1], m2 = words[w0 + 2], m3 = words[w0 + 3];
        word(m0, 32 * w0);
        word(m1, 32 * w0 + 32);
        word(m2, 32 * w0 + 64);
        word(m3, 32 * w0 + 96);
    }
    for (; w0 < nwords; ++w0) word(words[w0], 32 * w0);
    if (hp) acc = reduce2(mode, acc, pend);
    return acc;
}

// One step of workgroup g.  W_lds holds the column block on entry (and the
// updated block on exit when learning).
__device__ __forceinline__ void fused_step_body(const Params &p, const FusedArgs &a, const StepPtrs &s, int g,
                                                unsigned char *smem, const FusedLds &L)
{
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwaves = nt >> 6;
    const int JB = p.jb;
    const int jj = lane & 31;
    const int bs = lane >> 5;
    const int j = g * JB + jj;
    const bool col_ok = jj < JB && j < p.n_exc;

    float *W_lds = reinterpret_cast<float *>(smem + L.w);
    float *xpost_lds = reinterpret_cast<float *>(smem + L.xpost);
    uint32_t *bits_lds = reinterpret_cast<uint32_t *>(smem + L.bits);
    uint32_t *cprev_lds = reinterpret_cast<uint32_t *>(smem + L.cprev);
    uint32_t *cinh_lds = reinterpret_cast<uint32_t *>(smem + L.cinh);
    uint32_t *spk = reinterpret_cast<uint32_t *>(smem + L.spk);
    double *part = reinterpret_cast<double *>(smem + L.part);
    double *scale = reinterpret_cast<double *>(smem + L.scale);
    float *th_lds = reinterpret_cast<float *>(smem + L.theta);

    // A: per-step inputs
    copy_u4(bits_lds, s.bits, (size_t)p.B * p.in_words, tid, nt);
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

    // B: contraction + neuron update, two samples per wave per round
    const int spr = 2 * nwaves;
    const size_t sbase = (size_t)g * p.B * JB;
    for (int b0 = 0; b0 < p.B; b0 += spr) {
        const int b = b0 + 2 * wave + bs;
        if (b < p.B) {
            const size_t n = sbase + (size_t)b * JB + jj;
            NeuronState st{0.f, 0.f, 0u, 0.f};
            if (col_ok) {
                st.ve = a.v_exc[n];
                st.vi = p.has_inh ? a.v_inh[n] : 0.f;
                st.rf = a.rf[n];
                st.xpost = p.learn ? a.x_post[n] : 0.f;
            }
            const float acc = gather_bits(bits_lds + b * p.in_words, p.in_words, W_lds + (jj < JB ? jj : 0), JB,
                                          RED_SUM);
            if (col_ok) {
                bool se, si;
                neuron_update(p, acc, cprev_lds[b], th_lds[jj], st, se, si);
                a.v_exc[n] = st.ve;
                if (p.has_inh) a.v_inh[n] = st.vi;
                a.rf[n] = (uint16_t)st.rf;
                if (p.learn) {
                    a.x_post[n] = st.xpost;
                    xpost_lds[b * JB + jj] = st.xpost;
                    if (se) atomicOr(&spk[jj * p.bwords + (b >> 5)], 1u << (b & 31));
                }
                if (si) atomicAdd(&cinh_lds[b], 1u);
                write_outputs(p, a.o, s.k, b, j, se, si, st.ve, st.vi);
            }
        }
    }
    __syncthreads();
    for (int b = tid; b < p.B; b += nt) {
        const uint32_t c = cinh_lds[b];
        if (c) atomicAdd(&s.Ccur[b], c);
        if (g == 0 && s.Cnext) s.Cnext[b] = 0u;
    }
    if (!p.learn) return;
    // the transposed input spikes replace the per-sample ones in LDS
    copy_u4(bits_lds, s.bitsT, (size_t)p.n_in_pad * p.bwords, tid, nt);

    // C1: potentiation.  For every column with post spikes this step, all
    // threads sweep the rows: P[i] = R over the spiking samples b of
    // x_pre[b, i] (coalesced over i), then W[i, j] += nu_post * P.
    for (int c = 0; c < JB; ++c) {
        const uint32_t *sp = spk + c * p.bwords;
        uint32_t any = 0u;
        for (int bw = 0; bw < p.bwords; ++bw) any |= sp[bw];
        if (!any) continue;
        for (int i = tid; i < p.n_in; i += nt) {
            float P = gather_bits(sp, p.bwords, s.xpre + i, p.n_in_pad, p.reduce);
            if (p.reduce == RED_MEAN) P *= p.inv_B;
            W_lds[i * JB + c] = W_lds[i * JB + c] + p.nu_post * P;
        }
    }
    __syncthreads();

    // C2: depression, clamp and column partial sums.  D[i, j] = R over the
    // samples b in which input i spiked of x_post[b, j] (LDS gather).
    const int rg = tid >> 5;
    const int nrg = nt >> 5;
    double cs = 0.0;
    if (col_ok) {
        for (int i = rg; i < p.n_in; i += nrg) {
            float D = gather_bits(bits_lds + i * p.bwords, p.bwords, xpost_lds + jj, JB, p.reduce);
            if (p.reduce == RED_MEAN) D *= p.inv_B;
            const float w = fminf(fmaxf(W_lds[i * JB + jj] - p.nu_pre * D, p.w_min), p.w_max);
            W_lds[i * JB + jj] = w;
            cs += (double)w;
        }
    }
    part[rg * 32 + jj] = cs;
    __syncthreads();
    if (tid < 32) {
        double c = 0.0;
        for (int q = 0; q < nrg; ++q) c += part[q * 32 + tid];
        scale[tid] = (p.norm > 0.0 && c > 0.0) ? p.norm / c : 1.0;
        const int jt = g * JB + tid;
        if (tid < JB && jt < p.n_exc && p.adaptive) {
            int cnt = 0;
            for (int bw = 0; bw < p.bwords; ++bw) cnt += __builtin_popcount(spk[tid * p.bwords + bw]);
            a.theta[jt] = theta_step(p, a.theta[jt], cnt);
        }
    }
    __syncthreads();
    if (p.norm > 0.0 && col_ok) {
        const double sc = scale[jj];
        for (int i = rg; i < p.n_in; i += nrg) W_lds[i * JB + jj] = (float)((double)W_lds[i * JB + jj] * sc);
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
}

__global__ __launch_bounds__(kFusedThreads) void k_fused_step(Params p, FusedArgs a, StepPtrs s)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const FusedLds L(p, blockDim.x);
    const int g = blockIdx.x;
    float *W_lds = reinterpret_cast<float *>(smem + L.w);
    float *Wg = a.W + (size_t)g * p.n_in_pad * p.jb;
    const size_t nw = (size_t)p.n_in_pad * p.jb;
    copy_u4(W_lds, Wg, nw, threadIdx.x, blockDim.x);
    __syncthreads();
    fused_step_body(p, a, s, g, smem, L);
    if (p.learn) copy_u4(Wg, W_lds, nw, threadIdx.x, blockDim.x);
}

}  // namespace snn
