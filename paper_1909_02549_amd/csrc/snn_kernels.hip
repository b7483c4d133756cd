// snn_kernels.hip -- gfx950 kernels of one minibatched SNN timestep.
//
// One step (Implementation and Unsupervised Learning sections of Saunders et
// al., AAAI-20): Poisson input encoding; feed-forward current from the
// input spikes and the shared weights; recurrent inhibition from the previous
// step's inhibitory spikes; the excitatory adaptive-LIF and inhibitory LIF
// updates; STDP traces; the batch-reduced weight change with clamp and
// column normalisation; the shared threshold update.
//
// This file holds the building blocks and the plain per-step kernels.  The
// fused and persistent step kernels live in snn_fused.hip.
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_mfma.h"

namespace snn {

// ---------------------------------------------------------------------------
// Encoder: Philox4x64-10 counter-based generator (Salmon et al., SC'11).
// Counter (i / 8, t, id, 0), key (seed, 0); the four 64-bit outputs give eight
// 32-bit uniforms, low half first; input i spikes when its uniform is below
// the rate threshold thr[pixel] (thr / 2^32 = rate * dt).
// One 64-lane wave encodes one 32-input word for 64 consecutive samples and,
// if bitsT is given (learning runs), transposes the 32x64 bit tile with
// ballots for the per-input layout.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_encode(Params p, const uint8_t *__restrict__ img,
                                               const uint64_t *__restrict__ ids,
                                               const uint32_t *__restrict__ thr_lut,
                                               const uint32_t *__restrict__ tl, uint64_t tbase,
                                               const uint32_t *__restrict__ forced,
                                               uint32_t *__restrict__ bits, uint32_t *__restrict__ bitsT,
                                               uint32_t *__restrict__ raster_in, int raster_k0)
{
    const int lane = threadIdx.x;
    const int b = blockIdx.x * 64 + lane;
    const int w = blockIdx.y;
    const int k = blockIdx.z;
    uint32_t word = 0;
    if (b < p.B) {
        const int i_base = 32 * w;
        if (forced) {
            word = forced[((size_t)k * p.B + b) * p.in_words + w];
        } else {
            const uint64_t t = tbase + (uint64_t)k + (tl ? (uint64_t)tl[b] : 0ull);
            const uint64_t id = ids[b];
            for (int q = 0; q < 4; ++q) {
                const int i0 = i_base + 8 * q;
                if (i0 >= p.n_in) break;
                uint64_t r[4];
                philox4x64_10((uint64_t)(i0 >> 3), t, id, 0ull, p.seed, 0ull, r);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int i = i0 + e;
                    if (i < p.n_in) {
                        const uint32_t u = (e & 1) ? (uint32_t)(r[e >> 1] >> 32) : (uint32_t)r[e >> 1];
                        const uint32_t thr = p.uniform_rate ? p.thr_uniform : thr_lut[img[(size_t)b * p.n_in + i]];
                        word |= (uint32_t)(u < thr) << (8 * q + e);
                    }
                }
            }
        }
        const int valid = p.n_in - i_base;
        if (valid < 32) word &= valid <= 0 ? 0u : ((1u << valid) - 1u);
        bits[(size_t)k * p.bits_stride + (size_t)b * p.in_words + w] = word;
        if (raster_in) raster_in[((size_t)(raster_k0 + k) * p.B + b) * p.in_words + w] = word;
    }
    // (the per-input layout feeds the plasticity only)
    if (!bitsT) return;
    uint64_t mine = 0;
#pragma unroll
    for (int e = 0; e < 32; ++e) {
        const uint64_t m = __ballot((word >> e) & 1u);
        if (lane == e) mine = m;
    }
    if (lane < 32) {
        const size_t base = ((size_t)k * p.n_in_pad + (size_t)(32 * w + lane)) * p.bwords + 2 * blockIdx.x;
        bitsT[base] = (uint32_t)mine;
        if (2 * (int)blockIdx.x + 1 < p.bwords) bitsT[base + 1] = (uint32_t)(mine >> 32);
    }
}

// Encoder of the runs that need no transposed input spikes (no learning):
// the same draws as k_encode (input i: counter (i / 8, t, id, 0), uniform
// i mod 8 of the block), and besides the per-sample words it writes each
// sample's input spike list (increasing i) and its length, which the
// column-block kernels walk.  One 64-lane wave per (sample, step); a lane
// draws 16 consecutive inputs (two generator calls), so one pass covers
// 1024 inputs; an exclusive scan of the lanes' spike counts places each
// lane's entries in the list.  grid (ceil(B / 4), steps), 256 threads.
__global__ __launch_bounds__(256) void k_encode_lists(Params p, const uint8_t *__restrict__ img,
                                                      const uint64_t *__restrict__ ids,
                                                      const uint32_t *__restrict__ thr_lut,
                                                      const uint32_t *__restrict__ tl, uint64_t tbase,
                                                      const uint32_t *__restrict__ forced,
                                                      uint32_t *__restrict__ bits, uint16_t *__restrict__ lin,
                                                      uint32_t *__restrict__ cin, uint32_t *__restrict__ raster_in,
                                                      int raster_k0)
{
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.y;
    if (b >= p.B) return;  // (whole waves: no barrier below)
    const uint64_t t = tbase + (uint64_t)k + (tl ? (uint64_t)tl[b] : 0ull);
    const uint64_t id = forced ? 0ull : ids[b];
    uint16_t *out = lin + ((size_t)k * p.B + b) * p.n_in_pad;
    uint32_t base = 0;
    for (int i_pass = 0; i_pass < p.n_in; i_pass += 1024) {
        const int i0 = i_pass + 16 * lane;
        uint32_t m = 0;
        if (i0 < p.n_in) {
            if (forced) {
                m = forced[((size_t)k * p.B + b) * p.in_words + (i0 >> 5)] >> (i0 & 16);
            } else {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int ib = i0 + 8 * h;
                    if (ib >= p.n_in) break;
                    uint64_t r[4];
                    philox4x64_10((uint64_t)(ib >> 3), t, id, 0ull, p.seed, 0ull, r);
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int i = ib + e;
                        if (i < p.n_in) {
                            const uint32_t u = (e & 1) ? (uint32_t)(r[e >> 1] >> 32) : (uint32_t)r[e >> 1];
                            const uint32_t thr =
                                p.uniform_rate ? p.thr_uniform : thr_lut[img[(size_t)b * p.n_in + i]];
                            m |= (uint32_t)(u < thr) << (8 * h + e);
                        }
                    }
                }
            }
            const int valid = p.n_in - i0;
            m &= valid >= 16 ? 0xFFFFu : (1u << valid) - 1u;
        }
        // the 32-input words: lanes 2w and 2w + 1 hold its halves
        const uint32_t hi = __shfl_down(m, 1, 64);
        const int w = (i_pass >> 5) + (lane >> 1);
        if (!(lane & 1) && w < p.in_words) {
            const uint32_t word = m | (hi << 16);
            bits[(size_t)k * p.bits_stride + (size_t)b * p.in_words + w] = word;
            if (raster_in) raster_in[((size_t)(raster_k0 + k) * p.B + b) * p.in_words + w] = word;
        }
        // exclusive scan of the lanes' spike counts
        const uint32_t c = (uint32_t)__builtin_popcount(m);
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        uint32_t pos = base + incl - c;
        for (uint32_t mm = m; mm; mm &= mm - 1u) out[pos++] = (uint16_t)(i0 + __builtin_ctz(mm));
        base += __shfl(incl, 63, 64);
    }
    if (lane == 0) cin[(size_t)k * p.B + b] = base;
}

// Presynaptic traces of one step: x <- lam * x, then 1 (or x + 1) on a spike.
__global__ void k_xpre(Params p, const uint32_t *__restrict__ bits_t, const float *__restrict__ xprev,
                       float *__restrict__ xcur)
{
    const size_t n = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (size_t)p.B * p.n_in_pad) return;
    const int b = (int)(n / p.n_in_pad), i = (int)(n % p.n_in_pad);
    const uint32_t s = (bits_t[(size_t)b * p.in_words + (i >> 5)] >> (i & 31)) & 1u;
    xcur[n] = trace_step(xprev[n], p.lam_pre, s, p.trace_add);
}

// Plain feed-forward contraction: I[b, j] = sum over inputs i that spiked in
// sample b of q(W[i, j]), summed in increasing i, q the operand form of the
// precision (identity for FP32).  One thread per (b, j).
__global__ void k_contract(Params p, const float *__restrict__ W, const uint32_t *__restrict__ bits_t,
                           float *__restrict__ I)
{
    const size_t tix = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)p.nblk * p.B * p.jbp;
    if (tix >= total) return;
    const int jj = (int)(tix % p.jbp);
    const size_t gb = tix / p.jbp;
    const int b = (int)(gb % p.B);
    const int g = (int)(gb / p.B);
    const size_t ns = ((size_t)g * p.Bs + b) * p.jbp + jj;
    if (jj >= p.jb) {
        I[ns] = 0.f;
        return;
    }
    const float *Wg = W + (size_t)g * p.n_in_pad * p.jb + jj;
    const uint32_t *sb = bits_t + (size_t)b * p.in_words;
    float acc = 0.f;
    for (int w = 0; w < p.in_words; ++w) {
        uint32_t m = sb[w];
        while (m) {
            const int i = 32 * w + __builtin_ctz(m);
            m &= m - 1;
            acc += operand_value(p.prec, Wg[(size_t)i * p.jb]);
        }
    }
    I[ns] = acc;
}

// Per-step neuron update, one thread per group of 8 consecutive neurons of
// one sample (16-byte state loads and stores): recurrent currents, both
// layers, post trace, spike outputs.
__global__ void k_neuron(Params p, const float *__restrict__ I, const double *__restrict__ theta,
                         const uint32_t *__restrict__ Cprev, uint32_t *__restrict__ Ccur,
                         uint32_t *__restrict__ Cnext, float *__restrict__ v_exc, float *__restrict__ v_inh,
                         uint16_t *__restrict__ rf, float *__restrict__ x_post, int k, Outs o)
{
    const int ncg = p.jbp >> 3;
    const size_t tix = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tix >= (size_t)p.nblk * p.B * ncg) return;
    const int cg = (int)(tix % ncg);
    const size_t gb = tix / ncg;
    const int b = (int)(gb % p.B);
    const int g = (int)(gb / p.B);
    const int c0 = 8 * cg, j0 = g * p.jb + c0;
    if (j0 == 0 && Cnext) Cnext[b] = 0u;
    const int nv = max(0, min(8, min(p.jb - c0, p.n_exc - j0)));
    if (nv == 0) return;
    const size_t n0 = ((size_t)g * p.Bs + b) * p.jbp + c0;
    float ve[8], vi[8], xp[8], cur[8];
    uint32_t rw[4];
    {
        const float4 a0 = *reinterpret_cast<const float4 *>(v_exc + n0);
        const float4 a1 = *reinterpret_cast<const float4 *>(v_exc + n0 + 4);
        ve[0] = a0.x, ve[1] = a0.y, ve[2] = a0.z, ve[3] = a0.w, ve[4] = a1.x, ve[5] = a1.y, ve[6] = a1.z, ve[7] = a1.w;
        const float4 i0 = *reinterpret_cast<const float4 *>(I + n0);
        const float4 i1 = *reinterpret_cast<const float4 *>(I + n0 + 4);
        cur[0] = i0.x, cur[1] = i0.y, cur[2] = i0.z, cur[3] = i0.w;
        cur[4] = i1.x, cur[5] = i1.y, cur[6] = i1.z, cur[7] = i1.w;
        const uint4 r = *reinterpret_cast<const uint4 *>(rf + n0);
        rw[0] = r.x, rw[1] = r.y, rw[2] = r.z, rw[3] = r.w;
    }
    if (p.has_inh) {
        const float4 a0 = *reinterpret_cast<const float4 *>(v_inh + n0);
        const float4 a1 = *reinterpret_cast<const float4 *>(v_inh + n0 + 4);
        vi[0] = a0.x, vi[1] = a0.y, vi[2] = a0.z, vi[3] = a0.w, vi[4] = a1.x, vi[5] = a1.y, vi[6] = a1.z, vi[7] = a1.w;
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) vi[c] = 0.f;
    }
    if (p.learn) {
        const float4 a0 = *reinterpret_cast<const float4 *>(x_post + n0);
        const float4 a1 = *reinterpret_cast<const float4 *>(x_post + n0 + 4);
        xp[0] = a0.x, xp[1] = a0.y, xp[2] = a0.z, xp[3] = a0.w, xp[4] = a1.x, xp[5] = a1.y, xp[6] = a1.z, xp[7] = a1.w;
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) xp[c] = 0.f;
    }
    const uint32_t cp = p.has_inh ? Cprev[b] : 0u;
    uint32_t se_m = 0u, si_m = 0u;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (c < nv) {
            const uint32_t r16 = (rw[c >> 1] >> (16 * (c & 1))) & 0xFFFFu;
            NeuronState st{ve[c], vi[c], r16, xp[c]};
            bool se, si;
            neuron_update(p, cur[c], cp, theta_offset(p, theta[j0 + c]), st, se, si);
            ve[c] = st.ve;
            vi[c] = st.vi;
            xp[c] = st.xpost;
            rw[c >> 1] = (rw[c >> 1] & ~(0xFFFFu << (16 * (c & 1)))) | (st.rf << (16 * (c & 1)));
            se_m |= (se ? 1u : 0u) << c;
            si_m |= (si ? 1u : 0u) << c;
        }
    }
    *reinterpret_cast<float4 *>(v_exc + n0) = make_float4(ve[0], ve[1], ve[2], ve[3]);
    *reinterpret_cast<float4 *>(v_exc + n0 + 4) = make_float4(ve[4], ve[5], ve[6], ve[7]);
    if (p.has_inh) {
        *reinterpret_cast<float4 *>(v_inh + n0) = make_float4(vi[0], vi[1], vi[2], vi[3]);
        *reinterpret_cast<float4 *>(v_inh + n0 + 4) = make_float4(vi[4], vi[5], vi[6], vi[7]);
    }
    if (p.learn) {
        *reinterpret_cast<float4 *>(x_post + n0) = make_float4(xp[0], xp[1], xp[2], xp[3]);
        *reinterpret_cast<float4 *>(x_post + n0 + 4) = make_float4(xp[4], xp[5], xp[6], xp[7]);
    }
    *reinterpret_cast<uint4 *>(rf + n0) = make_uint4(rw[0], rw[1], rw[2], rw[3]);
    if (si_m) atomicAdd(&Ccur[b], (uint32_t)__builtin_popcount(si_m));
    write_outputs8(p, o, k, b, j0, nv, se_m, si_m, ve, vi);
}

// Plain plasticity, one workgroup per column block:
//   P[i, j] = R_b x_pre[b, i] s_exc[b, j]   (potentiation on a post spike)
//   D[i, j] = R_b s_in[b, i] x_post[b, j]   (depression on a pre spike)
//   W <- clamp(W + nu_post P - nu_pre D), column sums in FP64, W[:, j] *=
//   norm / c_j; theta <- theta * beta + theta_plus * R_b s_exc[b, j].
// R is sum, mean (sum / B), max or the soft maximum, applied to P and D
// separately; the traces enter in the operand form of the precision
// (unrounded for FP32).  The
// signed max instead adds max_b (nu_post P_b - nu_pre D_b), the largest
// per-sample change, 0 for a sample with neither spike on the synapse.
__global__ __launch_bounds__(256) void k_plastic(Params p, float *__restrict__ W, double *__restrict__ theta,
                                                 const uint16_t *__restrict__ rf,
                                                 const float *__restrict__ x_post,
                                                 const float *__restrict__ x_pre,
                                                 const uint32_t *__restrict__ bitsT_t)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int g = blockIdx.x;
    const int JB = p.jb;
    const int tid = threadIdx.x;
    uint32_t *spk = reinterpret_cast<uint32_t *>(smem);                      // JB * bwords
    double *part = reinterpret_cast<double *>(smem + align16((size_t)JB * p.bwords * 4)); // R * JB
    double *scale = part + (size_t)(blockDim.x / JB) * JB;                  // JB

    for (int q = tid; q < JB * p.bwords; q += blockDim.x) spk[q] = 0u;
    __syncthreads();
    const size_t sbase = (size_t)g * p.Bs * p.jbp;
    for (int q = tid; q < p.B * JB; q += blockDim.x) {
        const int b = q / JB, jj = q % JB;
        if (rf[sbase + (size_t)b * p.jbp + jj] & RF_SPIKE)
            atomicOr(&spk[jj * p.bwords + (b >> 5)], 1u << (b & 31));
    }
    __syncthreads();

    const int R = blockDim.x / JB;
    const int jj = tid % JB;
    const int r0 = tid / JB;
    const int j = g * JB + jj;
    const bool col_ok = r0 < R && j < p.n_exc;
    float *Wg = W + (size_t)g * p.n_in_pad * JB;
    double cs = 0.0;
    if (col_ok && p.reduce == RED_MAX_SIGNED) {
        for (int i = r0; i < p.n_in; i += R) {
            // walk the samples in which input i or post neuron j spiked
            const uint32_t *bt = bitsT_t + (size_t)i * p.bwords;
            const uint32_t *sp = spk + jj * p.bwords;
            float best = -INFINITY;
            int events = 0;
            for (int bw = 0; bw < p.bwords; ++bw) {
                const uint32_t mi = bt[bw], ms = sp[bw];
                uint32_t m = mi | ms;
                events += __builtin_popcount(m);
                while (m) {
                    const int bit = __builtin_ctz(m);
                    const int b = 32 * bw + bit;
                    m &= m - 1;
                    const float pot = (ms >> bit) & 1u
                                          ? p.nu_post * operand_value(p.prec, x_pre[(size_t)b * p.n_in_pad + i])
                                          : 0.f;
                    const float dep = (mi >> bit) & 1u
                                          ? p.nu_pre * operand_value(p.prec, x_post[sbase + (size_t)b * p.jbp + jj])
                                          : 0.f;
                    best = fmaxf(best, pot - dep);
                }
            }
            if (events < p.B) best = fmaxf(best, 0.f);
            const float w = fminf(fmaxf(Wg[(size_t)i * JB + jj] + best, p.w_min), p.w_max);
            Wg[(size_t)i * JB + jj] = w;
            cs += (double)w;
        }
    } else if (col_ok) {
        for (int i = r0; i < p.n_in; i += R) {
            float D = 0.f, P = 0.f;
            const uint32_t *bt = bitsT_t + (size_t)i * p.bwords;
            for (int bw = 0; bw < p.bwords; ++bw) {
                uint32_t m = bt[bw];
                while (m) {
                    const int b = 32 * bw + __builtin_ctz(m);
                    m &= m - 1;
                    D = reduce2(p.reduce, D,
                                stdp_term(p, operand_value(p.prec, x_post[sbase + (size_t)b * p.jbp + jj])));
                }
            }
            const uint32_t *sp = spk + jj * p.bwords;
            for (int bw = 0; bw < p.bwords; ++bw) {
                uint32_t m = sp[bw];
                while (m) {
                    const int b = 32 * bw + __builtin_ctz(m);
                    m &= m - 1;
                    P = reduce2(p.reduce, P, stdp_term(p, operand_value(p.prec, x_pre[(size_t)b * p.n_in_pad + i])));
                }
            }
            const float w = stdp_apply(p, Wg[(size_t)i * JB + jj], P, D);
            Wg[(size_t)i * JB + jj] = w;
            cs += (double)w;
        }
    }
    if (r0 < R) part[r0 * JB + jj] = cs;
    __syncthreads();
    if (r0 == 0) {
        double c = 0.0;
        for (int q = 0; q < R; ++q) c += part[q * JB + jj];
        scale[jj] = (p.norm > 0.0 && c > 0.0) ? p.norm / c : 1.0;
        if (j < p.n_exc && p.adaptive) {
            int cnt = 0;
            for (int bw = 0; bw < p.bwords; ++bw) cnt += __builtin_popcount(spk[jj * p.bwords + bw]);
            theta[j] = theta_step(p, theta[j], cnt);
        }
    }
    __syncthreads();
    if (col_ok && p.norm > 0.0) {
        const double s = scale[jj];
        for (int i = r0; i < p.n_in; i += R) {
            const size_t q = (size_t)i * JB + jj;
            Wg[q] = (float)((double)Wg[q] * s);
        }
    }
}

// Episodic reset of per-sample state (all samples b < B, or those with
// mask[b] set).
__global__ void k_reset(Params p, float *__restrict__ v_exc, float *__restrict__ v_inh, uint16_t *__restrict__ rf,
                        float *__restrict__ x_post, float *__restrict__ x_pre, uint32_t *__restrict__ C,
                        const uint8_t *__restrict__ mask)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t ns = (size_t)p.nblk * p.B * p.jbp;
    if (t < ns) {
        const int jj = (int)(t % p.jbp);
        const size_t gb = t / p.jbp;
        const int b = (int)(gb % p.B);
        const int g = (int)(gb / p.B);
        if (!mask || mask[b]) {
            const size_t n = ((size_t)g * p.Bs + b) * p.jbp + jj;
            v_exc[n] = p.exc.v_rest;
            v_inh[n] = p.inh.v_rest;
            rf[n] = 0;
            x_post[n] = 0.f;
        }
    }
    const size_t nx = (size_t)p.B * p.n_in_pad;
    if (t < nx) {
        const int b = (int)(t / p.n_in_pad);
        if (!mask || mask[b]) {
            x_pre[t] = 0.f;
            x_pre[(size_t)p.Bs * p.n_in_pad + t] = 0.f;
            x_pre[2 * (size_t)p.Bs * p.n_in_pad + t] = 0.f;
        }
    }
    if (t < (size_t)p.B) {
        if (!mask || mask[t]) {
            C[t] = 0u;
            C[p.Bs + t] = 0u;
            C[2 * p.Bs + t] = 0u;
        }
    }
}

// Serving: new slots (mask[b] set) start at local step 0 with zero counts.
__global__ void k_slot_init(const uint8_t *__restrict__ mask, uint32_t *__restrict__ tl, uint32_t *__restrict__ counts,
                            int n_exc, int B)
{
    const int b = blockIdx.x;
    if (b >= B || !mask[b]) return;
    if (threadIdx.x == 0) tl[b] = 0u;
    for (int j = threadIdx.x; j < n_exc; j += blockDim.x) counts[(size_t)b * n_exc + j] = 0u;
}

// Re-forming the batch without a reset.  k_rebatch_save gathers the
// per-sample state of the kept samples (old slot keep[k] -> staging row k):
// the neurons' v_exc, v_inh, x_post and flags, the presynaptic traces and
// the inhibitory spike count of the last step, the local step (from tl, or
// t_uniform when every slot shares one).  k_rebatch_load then writes slot
// b < nk from staging row b and puts slots nk .. B-1 in the initial state at
// local step 0; it also clears the current step's count slot.  Launched
// over max(nblk * B * jbp, B * n_in_pad) threads of the layout in question.
__global__ void k_rebatch_save(Params p, const float *__restrict__ v_exc, const float *__restrict__ v_inh,
                               const float *__restrict__ x_post, const uint16_t *__restrict__ rf,
                               const float *__restrict__ xpre_last, const uint32_t *__restrict__ C_last,
                               const uint32_t *__restrict__ tl, uint32_t t_uniform, const uint32_t *__restrict__ keep,
                               int nk, RebatchStage s)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (size_t)p.nblk * nk * p.jbp) {
        const int jj = (int)(t % p.jbp);
        const size_t gk = t / p.jbp;
        const int k = (int)(gk % nk);
        const int g = (int)(gk / nk);
        const size_t src = ((size_t)g * p.Bs + keep[k]) * p.jbp + jj;
        s.v_exc[t] = v_exc[src];
        s.v_inh[t] = v_inh[src];
        s.x_post[t] = x_post[src];
        s.rf[t] = rf[src];
    }
    if (t < (size_t)nk * p.n_in_pad) {
        const int k = (int)(t / p.n_in_pad);
        s.x_pre[t] = xpre_last[(size_t)keep[k] * p.n_in_pad + t % p.n_in_pad];
    }
    if (t < (size_t)nk) {
        s.C[t] = C_last[keep[t]];
        s.tl[t] = tl ? tl[keep[t]] : t_uniform;
    }
}

__global__ void k_rebatch_load(Params p, float *__restrict__ v_exc, float *__restrict__ v_inh,
                               float *__restrict__ x_post, uint16_t *__restrict__ rf, float *__restrict__ xpre_last,
                               uint32_t *__restrict__ C_cur, uint32_t *__restrict__ C_last, uint32_t *__restrict__ tl,
                               int nk, RebatchStage s)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (size_t)p.nblk * p.B * p.jbp) {
        const int jj = (int)(t % p.jbp);
        const size_t gb = t / p.jbp;
        const int b = (int)(gb % p.B);
        const int g = (int)(gb / p.B);
        const size_t n = ((size_t)g * p.Bs + b) * p.jbp + jj;
        if (b < nk) {
            const size_t q = ((size_t)g * nk + b) * p.jbp + jj;
            v_exc[n] = s.v_exc[q];
            v_inh[n] = s.v_inh[q];
            x_post[n] = s.x_post[q];
            rf[n] = s.rf[q];
        } else {
            v_exc[n] = p.exc.v_rest;
            v_inh[n] = p.inh.v_rest;
            x_post[n] = 0.f;
            rf[n] = 0;
        }
    }
    if (t < (size_t)p.B * p.n_in_pad) xpre_last[t] = t < (size_t)nk * p.n_in_pad ? s.x_pre[t] : 0.f;
    if (t < (size_t)p.B) {
        C_cur[t] = 0u;
        C_last[t] = (int)t < nk ? s.C[t] : 0u;
        tl[t] = (int)t < nk ? s.tl[t] : 0u;
    }
}

// Serving: move slot pairs[2q] to slot pairs[2q + 1], q < n (grid y = q).
// Every destination is a free slot below every source and no slot is both,
// so the copies do not overlap.  Carries the network's per-sample state (the
// neurons' v_exc, v_inh, x_post and flags, the last step's presynaptic
// traces and inhibitory count) and the server's image, id, local step and
// counts.  The destination's current-step count slot is zero already (it
// was an idle slot below the active width).
__global__ void k_slot_move(Params p, float *__restrict__ v_exc, float *__restrict__ v_inh,
                            float *__restrict__ x_post, uint16_t *__restrict__ rf, float *__restrict__ xpre_last,
                            uint32_t *__restrict__ C_last, SlotArrays sa, int n_in, const uint32_t *__restrict__ pairs,
                            int n)
{
    const int q = blockIdx.y;
    if (q >= n) return;
    const uint32_t src = pairs[2 * q], dst = pairs[2 * q + 1];
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (size_t)p.nblk * p.jbp) {
        const size_t g = t / p.jbp, jj = t % p.jbp;
        const size_t s = (g * p.Bs + src) * p.jbp + jj, d = (g * p.Bs + dst) * p.jbp + jj;
        v_exc[d] = v_exc[s];
        v_inh[d] = v_inh[s];
        x_post[d] = x_post[s];
        rf[d] = rf[s];
    }
    if (t < (size_t)p.n_in_pad) xpre_last[(size_t)dst * p.n_in_pad + t] = xpre_last[(size_t)src * p.n_in_pad + t];
    if (t < (size_t)p.n_exc) sa.counts[(size_t)dst * p.n_exc + t] = sa.counts[(size_t)src * p.n_exc + t];
    if (t < (size_t)n_in) sa.img[(size_t)dst * n_in + t] = sa.img[(size_t)src * n_in + t];
    if (t == 0) {
        sa.ids[dst] = sa.ids[src];
        sa.tl[dst] = sa.tl[src];
        C_last[dst] = C_last[src];
    }
}

// Serving: every slot's local step advances by the steps just run.
__global__ void k_add_u32(uint32_t *__restrict__ v, uint32_t add, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) v[q] += add;
}

__global__ void k_fill_u32(uint32_t *__restrict__ dst, uint32_t value, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        dst[q] = value;
}

}  // namespace snn
