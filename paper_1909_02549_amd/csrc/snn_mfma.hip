// snn_mfma.hip -- matrix-core (MFMA) form of the two contractions of one
// step, used by the per-step path:
//   synaptic current   I[b, j] = sum_i  s_in[b, i]   q(W[i, j])
//   STDP potentiation  P[i, j] = sum_b  q(x_pre[b, i]) s_exc[b, j]
//   STDP depression    D[i, j] = sum_b  s_in[b, i]   q(x_post[b, j])
// (Implementation and Reduction methods sections: a spike-input product for
// the current, batch-summed outer products for the weight change).  Spikes
// are exact 0/1 operands; q is the operand form of the precision:
//   FP32  three bfloat16 planes hi + mid + lo whose sum is exactly the FP32
//         value (8 + 8 + 8 significant bits), so the products are exact;
//   BF16  one bfloat16 plane, round to nearest even;
//   FP8   one OCP E4M3 plane, round to nearest even;
// the matrix cores accumulate in FP32.  Mean divides the sums by B, max has
// no matrix form and stays on the gather kernel.
//
// v_mfma_f32_32x32x16_{bf16,fp8_fp8} operand layout (one 64-lane wave):
//   A (32 x 16, M x K): lane l holds row l % 32, K elements 8 (l / 32) + e
//   B (16 x 32, K x N): lane l holds column l % 32, K elements 8 (l / 32) + e
//   C (32 x 32): lane l holds column l % 32, rows 8 (r / 4) + 4 (l / 32) + r % 4
//                in accumulator r = 0 .. 15
#include <hip/hip_runtime.h>

#include <type_traits>

#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_mfma.h"

namespace snn {

// ---------------------------------------------------------------------------
// one step's front half: presynaptic traces, synaptic current, neurons
// ---------------------------------------------------------------------------
//
// One workgroup (8 waves) per column block g (JB <= 32 columns, padded to 32
// with zero weights).  The block's FP32 weights (one contiguous span) are
// loaded into LDS in one burst; in chunks of kFrontRows rows they are
// converted to operand planes laid out as the B operand wants them:
//   plane[ks][half][n][e] = q(W[16 ks + 8 half + e, n])
// so each lane reads one contiguous 16-byte (8-byte for FP8) operand.  The
// samples are taken in rounds of 256 (32 per wave); their input spike words
// are staged in LDS per round, and a 256-entry table turns a spike byte into
// the lane's A operand (eight 0/1 elements) with one LDS read.  The neuron
// state of a round is loaded into registers before its matrix work, so
// those loads stream while the weights are converted and multiplied.
//
// The current is consumed in place: each lane of the accumulator owns column
// n of 16 samples, which is exactly the state it needs to advance those
// neurons (the loads of one accumulator row are 128-byte rows of the
// block-major state).  The workgroups also advance the presynaptic traces
// x_pre(t) = trace(x_pre(t-1), s_in(t)) in equal slices and clear the next
// step's inhibitory counts, so a learning step is this launch and the STDP
// launch.
constexpr int kFrontRows = 160;
constexpr int kFrontWaves = 8;
constexpr int kFrontThreads = 64 * kFrontWaves;
constexpr int kFrontSamples = 32 * kFrontWaves;  // samples per round
constexpr int kFrontConv = kFrontRows * 32 / kFrontThreads;  // weights converted per thread per chunk

struct FrontLds {
    size_t wf, planes, sbits, lut, total;
    size_t plane_bytes;
    __host__ __device__ FrontLds(const Params &p, int prec)
    {
        const int np = prec == PREC_FP32 ? 3 : 1;
        const int esize = prec == PREC_FP8 ? 1 : 2;
        plane_bytes = (size_t)kFrontRows * 32 * esize;
        wf = 0;
        planes = align16((size_t)p.n_in_pad * p.jb * 4);
        sbits = planes + np * plane_bytes;
        lut = align16(sbits + (size_t)kFrontSamples * p.in_words * 4);
        total = lut + 256 * 8 * esize;
    }
};

size_t mfma_front_lds(const Params &p, int prec) { return FrontLds(p, prec).total; }

template <int PREC>
__global__ __launch_bounds__(kFrontThreads) void k_mfma_front(Params p, FrontArgs a)
{
    using F = Form<PREC>;
    extern __shared__ __align__(16) unsigned char smem[];
    const FrontLds L(p, PREC);
    float *wf = reinterpret_cast<float *>(smem + L.wf);
    unsigned char *planes = smem + L.planes;
    uint32_t *sbits = reinterpret_cast<uint32_t *>(smem + L.sbits);
    unsigned char *lut = smem + L.lut;
    const size_t plane_bytes = L.plane_bytes;
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int n = lane & 31, half = lane >> 5;
    const int JB = p.jb, IW = p.in_words;

    const int j = g * JB + n;
    const bool col = n < JB && j < p.n_exc;
    const size_t base = (size_t)g * p.Bs * p.jbp + n;
    // neuron state of this lane's 16 samples in the first round
    float ve[16], vi[16], xp[16];
    uint32_t rw[16], cp[16];
    auto load_state = [&](int b0) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int bb = b0 + 8 * (r >> 2) + 4 * half + (r & 3);
            const bool ok = col && bb < p.B;
            const size_t s = base + (size_t)bb * p.jbp;
            ve[r] = ok ? a.v_exc[s] : 0.f;
            vi[r] = ok && p.has_inh ? a.v_inh[s] : 0.f;
            xp[r] = ok && p.learn ? a.x_post[s] : 0.f;
            rw[r] = ok ? (uint32_t)a.rf[s] : 0u;
            cp[r] = ok && p.has_inh ? a.Cprev[bb] : 0u;
        }
    };
    load_state(wave * 32);
    const float th_off = col ? theta_offset(p, a.theta[j]) : 0.f;
    // spike byte -> eight 0/1 operand elements
    if (tid < 256) {
        if constexpr (F::esize == 2)
            reinterpret_cast<uint4 *>(lut)[tid] = ones_bf16((uint32_t)tid);
        else
            reinterpret_cast<uint2 *>(lut)[tid] = ones_fp8((uint32_t)tid);
    }

    // the weight block into LDS: one burst of 16-byte loads (the span is
    // n_in_pad * JB floats, n_in_pad a multiple of 32)
    {
        const float4 *src = reinterpret_cast<const float4 *>(a.W + (size_t)g * p.n_in_pad * JB);
        float4 *dst = reinterpret_cast<float4 *>(wf);
        const int nf4 = p.n_in_pad * JB / 4;
        for (int q0 = 0; q0 < nf4; q0 += 8 * kFrontThreads) {
            float4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + u * kFrontThreads + tid;
                v[u] = q < nf4 ? src[q] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int q = q0 + u * kFrontThreads + tid;
                if (q < nf4) dst[q] = v[u];
            }
        }
    }
    // columns JB .. 31 of the planes are never written: zero them once
    for (int q = tid; q < (int)(F::planes * plane_bytes / 16); q += kFrontThreads)
        reinterpret_cast<uint4 *>(planes)[q] = make_uint4(0u, 0u, 0u, 0u);
    if (g == 0 && a.Cnext)
        for (int b = tid; b < p.B; b += kFrontThreads) a.Cnext[b] = 0u;
    if (p.learn) {
        // this workgroup's slice of the B x n_in_pad presynaptic traces
        const size_t total = (size_t)p.B * p.n_in_pad;
        const size_t per = (total + gridDim.x - 1) / gridDim.x;
        const size_t q0 = (size_t)g * per;
        const size_t q1 = min(total, q0 + per);
        for (size_t q = q0 + tid; q < q1; q += kFrontThreads) {
            const int b = (int)(q / p.n_in_pad), i = (int)(q - (size_t)b * p.n_in_pad);
            const uint32_t s = (a.bits[(size_t)b * IW + (i >> 5)] >> (i & 31)) & 1u;
            a.xcur[q] = trace_step(a.xprev[q], p.lam_pre, s, p.trace_add);
        }
    }

    for (int bw0 = 0; bw0 < p.B; bw0 += kFrontSamples) {
        const int b0 = bw0 + wave * 32;
        const bool active = b0 < p.B;
        if (bw0 > 0) load_state(b0);
        __syncthreads();  // previous round done with sbits
        const int nsw = min(kFrontSamples, p.B - bw0) * IW;
        for (int q = tid; q < kFrontSamples * IW; q += kFrontThreads)
            sbits[q] = q < nsw ? a.bits[(size_t)bw0 * IW + q] : 0u;
        const uint32_t *brow = sbits + (size_t)(wave * 32 + n) * IW;
        f32x16_t acc = {};
        for (int k0 = 0; k0 < p.n_in_pad; k0 += kFrontRows) {
            const int kc = min(kFrontRows, p.n_in_pad - k0);
            __syncthreads();  // weights and sbits staged / previous chunk consumed
            {
                // all of this thread's weights of the chunk first, then the stores
                float wv[kFrontConv];
#pragma unroll
                for (int u = 0; u < kFrontConv; ++u) {
                    const int q = tid + u * kFrontThreads;
                    const int k = q >> 5, jj = q & 31;
                    wv[u] = (k < kc && jj < JB) ? wf[(size_t)(k0 + k) * JB + jj] : 0.f;
                }
#pragma unroll
                for (int u = 0; u < kFrontConv; ++u) {
                    const int q = tid + u * kFrontThreads;
                    const int k = q >> 5, jj = q & 31;
                    if (k < kc && jj < JB) {
                        uint32_t c[3];
                        split<PREC>(wv[u], c);
                        const int e = (((k >> 3) * 32 + jj) << 3) + (k & 7);
#pragma unroll
                        for (int pl = 0; pl < F::planes; ++pl) {
                            if constexpr (F::esize == 2)
                                reinterpret_cast<uint16_t *>(planes + pl * plane_bytes)[e] = (uint16_t)c[pl];
                            else
                                (planes + pl * plane_bytes)[e] = (uint8_t)c[pl];
                        }
                    }
                }
            }
            __syncthreads();
            if (active) {
                // the chunk's spike words of this lane's sample, then its k-steps
                // unrolled so the operand reads run ahead of the matrix cores
                uint32_t words[kFrontRows / 32];
#pragma unroll
                for (int w = 0; w < kFrontRows / 32; ++w) words[w] = 32 * w < kc ? brow[(k0 >> 5) + w] : 0u;
#pragma unroll
                for (int g4 = 0; g4 < kFrontRows / 16; g4 += F::batch) {
                    if (16 * g4 >= kc) break;
                    // operands of a batch of k-steps first, then their matrix work
                    typename F::vec av[F::batch], bv[F::batch][F::planes];
#pragma unroll
                    for (int u = 0; u < F::batch; ++u) {
                        const int ks = g4 + u;
                        const bool in = 16 * ks < kc;  // past the chunk: zero operands
                        const uint32_t byte = (words[ks >> 1] >> (8 * (2 * (ks & 1) + half))) & 0xFFu;
                        const size_t off = ((size_t)(ks * 2 + half) * 32 + n) * F::vbytes;
                        av[u] = reinterpret_cast<const typename F::vec *>(lut)[in ? byte : 0u];
#pragma unroll
                        for (int pl = 0; pl < F::planes; ++pl)
                            bv[u][pl] = in ? *reinterpret_cast<const typename F::vec *>(planes + pl * plane_bytes + off)
                                           : typename F::vec{};
                    }
#pragma unroll
                    for (int u = 0; u < F::batch; ++u)
#pragma unroll
                        for (int pl = 0; pl < F::planes; ++pl) acc = mma<PREC>(av[u], bv[u][pl], acc);
                }
            }
        }
        if (!active) continue;

        // neurons (b, j) of this lane: j = g JB + n, b = b0 + 8 (r / 4) + 4 half + r % 4
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int bb = b0 + 8 * (r >> 2) + 4 * half + (r & 3);
            const bool ok = col && bb < p.B;
            bool se = false, si = false;
            if (ok) {
                NeuronState st{ve[r], vi[r], rw[r], xp[r]};
                neuron_update(p, acc[r], cp[r], th_off, st, se, si);
                const size_t s = base + (size_t)bb * p.jbp;
                a.v_exc[s] = st.ve;
                if (p.has_inh) a.v_inh[s] = st.vi;
                if (p.learn) a.x_post[s] = st.xpost;
                a.rf[s] = (uint16_t)st.rf;
                write_outputs(p, a.o, a.k, bb, j, se, si, st.ve, st.vi);
            }
            // inhibitory spikes of one sample row: one atomic per half-wave
            const uint64_t m = __ballot(si);
            const uint32_t cnt = (uint32_t)__popcll(half ? (m >> 32) : (m & 0xFFFFFFFFull));
            if (n == 0 && cnt && bb < p.B) atomicAdd(&a.Ccur[bb], cnt);
        }
    }
}

// ---------------------------------------------------------------------------
// STDP weight change, update, clamp, normalisation, theta
// ---------------------------------------------------------------------------
//
// One workgroup (8 waves) per column block g; wave w owns input tiles
// i0 = 32 (w + 8 t), t < kPlasticTiles, and keeps their updated weights in
// registers until the column sums are known.
//   P tiles: A = q(x_pre) rows of the samples in which some column of the
//            block fired (compacted list, K = that count rounded up to 16,
//            the rows staged in LDS 16 at a time), B = their 0/1 exc spikes;
//   D tiles: A = 0/1 input spikes of the tile's inputs over all samples (the
//            per-input bit rows, staged in LDS), B = q(x_post) of the block,
//            staged in LDS as operand planes.
constexpr int kPlasticWaves = 8;
constexpr int kPlasticThreads = 64 * kPlasticWaves;
constexpr int kPlasticTiles = 4;  // n_in_pad <= 32 * 8 * 4 = 1024

struct PlasticLds {
    size_t smask, slist, cnt, bp, bd, bt, xs, lut, part, scale, total;
    int B16, bt_stride;
    __host__ __device__ PlasticLds(const Params &p, int prec)
    {
        const int planes = prec == PREC_FP32 ? 3 : 1;
        const int esize = prec == PREC_FP8 ? 1 : 2;
        B16 = (p.B + 15) & ~15;
        bt_stride = p.bwords | 1;  // odd row stride: the 32 rows a wave reads hit distinct banks
        size_t o = 0;
        smask = o;
        o = align16(o + (size_t)B16 * 4);
        slist = o;
        o = align16(o + (size_t)B16 * 2 + 16);
        cnt = o;
        o = align16(o + 33 * 4);
        bp = o;
        o = align16(o + (size_t)B16 * 32 * esize);
        bd = o;
        o = align16(o + (size_t)planes * B16 * 32 * esize);
        bt = o;
        o = align16(o + (size_t)p.n_in_pad * bt_stride * 4);
        xs = o;
        o = align16(o + (size_t)16 * p.n_in_pad * 4);
        lut = o;
        o = align16(o + 256 * 8 * esize);
        part = o;
        o = align16(o + (size_t)kPlasticWaves * 32 * 8);
        scale = o;
        o = align16(o + 32 * 8);
        total = o;
    }
};

size_t mfma_plastic_lds(const Params &p, int prec) { return PlasticLds(p, prec).total; }

bool mfma_plastic_fits(const Params &p, int prec)
{
    return p.reduce < RED_MAX && p.jb <= 32 && p.n_in_pad <= 32 * kPlasticWaves * kPlasticTiles &&
           mfma_plastic_lds(p, prec) <= 160 * 1024;
}

template <int PREC>
__global__ __launch_bounds__(kPlasticThreads) void k_mfma_plastic(Params p, float *__restrict__ W,
                                                                  double *__restrict__ theta,
                                                                  const uint16_t *__restrict__ rf,
                                                                  const float *__restrict__ x_post,
                                                                  const float *__restrict__ x_pre,
                                                                  const uint32_t *__restrict__ bitsT_t)
{
    using F = Form<PREC>;
    extern __shared__ __align__(16) unsigned char smem[];
    const PlasticLds L(p, PREC);
    uint32_t *smask = reinterpret_cast<uint32_t *>(smem + L.smask);
    uint16_t *slist = reinterpret_cast<uint16_t *>(smem + L.slist);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(smem + L.cnt);  // [32] column spike counts, [32] list length
    unsigned char *bp = smem + L.bp;
    unsigned char *bd = smem + L.bd;
    uint32_t *bt = reinterpret_cast<uint32_t *>(smem + L.bt);
    float *xs = reinterpret_cast<float *>(smem + L.xs);
    unsigned char *lut = smem + L.lut;
    double *part = reinterpret_cast<double *>(smem + L.part);
    double *scale = reinterpret_cast<double *>(smem + L.scale);
    const size_t bd_plane = (size_t)L.B16 * 32 * F::esize;

    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int n = lane & 31, half = lane >> 5;
    const int JB = p.jb, JBP = p.jbp, B16 = L.B16;
    const size_t sbase = (size_t)g * p.Bs * JBP;

    float *Wg = W + (size_t)g * p.n_in_pad * JB;
    const int ntiles = p.n_in_pad >> 5;
    // wnew[t][r]: first the potentiation term nu_post R(P), then the updated
    // weight of row 32 tile + 8 (r / 4) + 4 half + r % 4, column n
    float wnew[kPlasticTiles][16];
#pragma unroll
    for (int t = 0; t < kPlasticTiles; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) wnew[t][r] = 0.f;

    // 1. the per-input spike rows; exc spikes of the block per sample, column
    //    counts; q(x_post) planes (loads batched 8 deep)
    for (int q = tid; q < B16; q += kPlasticThreads) smask[q] = 0u;
    if (tid < 33) cnt[tid] = 0u;
    // spike byte -> eight 0/1 operand elements
    if (tid < 256) {
        if constexpr (F::esize == 2)
            reinterpret_cast<uint4 *>(lut)[tid] = ones_bf16((uint32_t)tid);
        else
            reinterpret_cast<uint2 *>(lut)[tid] = ones_fp8((uint32_t)tid);
    }
    for (int q0 = 0; q0 < p.n_in_pad * p.bwords; q0 += 8 * kPlasticThreads) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * kPlasticThreads + tid;
            v[u] = q < p.n_in_pad * p.bwords ? bitsT_t[q] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * kPlasticThreads + tid;
            if (q < p.n_in_pad * p.bwords) {
                const int i = q / p.bwords, w = q - i * p.bwords;
                bt[i * L.bt_stride + w] = v[u];
            }
        }
    }
    __syncthreads();
    for (int q0 = 0; q0 < B16 * 32; q0 += 8 * kPlasticThreads) {
        float xv[8];
        uint32_t rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * kPlasticThreads + tid;
            const int b = q >> 5, jj = q & 31;
            const bool ok = b < p.B && jj < JB;
            const size_t s = sbase + (size_t)b * JBP + jj;
            xv[u] = ok ? x_post[s] : 0.f;
            rv[u] = ok ? (uint32_t)rf[s] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * kPlasticThreads + tid;
            if (q >= B16 * 32) break;
            const int b = q >> 5, jj = q & 31;
            if (rv[u] & RF_SPIKE) {
                atomicOr(&smask[b], 1u << jj);
                atomicAdd(&cnt[jj], 1u);
            }
            uint32_t c[3];
            split<PREC>(xv[u], c);
            const int e = (((b >> 3) * 32 + jj) << 3) + (b & 7);
#pragma unroll
            for (int pl = 0; pl < F::planes; ++pl) {
                if constexpr (F::esize == 2)
                    reinterpret_cast<uint16_t *>(bd + pl * bd_plane)[e] = (uint16_t)c[pl];
                else
                    (bd + pl * bd_plane)[e] = (uint8_t)c[pl];
            }
        }
    }
    __syncthreads();
    // 2. compacted list of the samples with a spike in the block (wave 0)
    if (wave == 0) {
        uint32_t base = 0;
        for (int b0 = 0; b0 < B16; b0 += 64) {
            const int b = b0 + lane;
            const bool f = b < B16 && smask[b] != 0u;
            const uint64_t m = __ballot(f);
            if (f) slist[base + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)b;
            base += (uint32_t)__popcll(m);
        }
        const uint32_t k1 = (base + 15) & ~15u;
        for (uint32_t q = base + lane; q < k1; q += 64) slist[q] = 0xFFFFu;
        if (lane == 0) cnt[32] = k1;
    }
    __syncthreads();
    const int K1 = (int)cnt[32];
    // P's B operand: bp[ks][half][n][e] = s_exc[slist[16 ks + 8 half + e], n]
    for (int q = tid; q < K1 * 32; q += kPlasticThreads) {
        const int kk = q >> 5, jj = q & 31;
        const uint32_t sid = slist[kk];
        const uint32_t on = sid != 0xFFFFu ? (smask[sid] >> jj) & 1u : 0u;
        const size_t e = ((size_t)((kk >> 4) * 2 + ((kk >> 3) & 1)) * 32 + jj) * 8 + (kk & 7);
        if constexpr (F::esize == 2)
            reinterpret_cast<uint16_t *>(bp)[e] = (uint16_t)(on * 0x3F80u);
        else
            bp[e] = (uint8_t)(on * 0x38u);
    }

    // the first tile's weights stream in during P
    float wcur[16];
    auto load_w = [&](int t, float *dst) {
        const int tile = wave + kPlasticWaves * t;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * tile + 8 * (r >> 2) + 4 * half + (r & 3);
            dst[r] = (tile < ntiles && n < JB && i < p.n_in) ? Wg[(size_t)i * JB + n] : 0.f;
        }
    };
    load_w(0, wcur);

    // 3. P for all tiles, 16 compacted samples' x_pre rows at a time in LDS,
    //    accumulated as the potentiation term nu_post R(P)
    const float rs = p.reduce == RED_MEAN ? p.inv_B : 1.f;
    const int nrow4 = p.n_in_pad / 4;
    for (int ks = 0; ks < K1 / 16; ++ks) {
        __syncthreads();  // bp written / previous rows consumed
        for (int q0 = 0; q0 < 16 * nrow4; q0 += 4 * kPlasticThreads) {
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kPlasticThreads + tid;
                const int e = q / nrow4, c4 = q - e * nrow4;
                const uint32_t sid = q < 16 * nrow4 ? slist[16 * ks + e] : 0xFFFFu;
                v[u] = sid != 0xFFFFu ? reinterpret_cast<const float4 *>(x_pre + (size_t)sid * p.n_in_pad)[c4]
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kPlasticThreads + tid;
                if (q < 16 * nrow4) reinterpret_cast<float4 *>(xs)[q] = v[u];
            }
        }
        __syncthreads();
        const size_t off = ((size_t)(ks * 2 + half) * 32 + n) * F::vbytes;
#pragma unroll
        for (int t = 0; t < kPlasticTiles; ++t) {
            const int tile = wave + kPlasticWaves * t;
            if (tile >= ntiles) break;
            uint32_t c[8][3];
#pragma unroll
            for (int e = 0; e < 8; ++e) split<PREC>(xs[(8 * half + e) * p.n_in_pad + 32 * tile + n], c[e]);
            f32x16_t accP = {};
            if constexpr (F::esize == 2) {
                const uint4 bo = *reinterpret_cast<const uint4 *>(bp + off);
#pragma unroll
                for (int pl = 0; pl < F::planes; ++pl) {
                    const uint4 av = make_uint4(c[0][pl] | (c[1][pl] << 16), c[2][pl] | (c[3][pl] << 16),
                                                c[4][pl] | (c[5][pl] << 16), c[6][pl] | (c[7][pl] << 16));
                    accP = mfma<PREC>(av, bo, accP);
                }
            } else {
                const uint2 av = make_uint2(c[0][0] | (c[1][0] << 8) | (c[2][0] << 16) | (c[3][0] << 24),
                                            c[4][0] | (c[5][0] << 8) | (c[6][0] << 16) | (c[7][0] << 24));
                accP = mfma8<PREC>(av, *reinterpret_cast<const uint2 *>(bp + off), accP);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) wnew[t][r] += p.nu_post * (accP[r] * rs);
        }
    }
    __syncthreads();  // bp complete for the K1 == 0 case as well

    // 4. D per tile; the next tile's weights load while the matrix cores run;
    //    w <- clamp(w + nu_post R(P) - nu_pre R(D)) in registers
    double cs = 0.0;
#pragma unroll
    for (int t = 0; t < kPlasticTiles; ++t) {
        const int tile = wave + kPlasticWaves * t;
        if (tile >= ntiles) break;
        const int i0 = 32 * tile;
        float w0[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) w0[r] = wcur[r];
        if (t + 1 < kPlasticTiles) load_w(t + 1, wcur);
        f32x16_t accD = {};
        const uint32_t *trow = bt + (size_t)(i0 + n) * L.bt_stride;
        const int nks = B16 / 16;
        for (int ks0 = 0; ks0 < nks; ks0 += 8) {
            // four spike words (8 k-steps), unrolled so the operand reads run
            // ahead of the matrix cores
            uint32_t words[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) words[w] = ks0 + 2 * w < nks ? trow[(ks0 >> 1) + w] : 0u;
#pragma unroll
            for (int g2 = 0; g2 < 8; g2 += F::batch8) {
                if (ks0 + g2 >= nks) break;
                typename F::vec av[F::batch8], bv[F::batch8][F::planes];
#pragma unroll
                for (int u = 0; u < F::batch8; ++u) {
                    const int ks = ks0 + g2 + u;
                    const bool in = ks < nks;  // past the last k-step: zero operands
                    const uint32_t byte = (words[(g2 + u) >> 1] >> (8 * (2 * ((g2 + u) & 1) + half))) & 0xFFu;
                    const size_t off = ((size_t)(ks * 2 + half) * 32 + n) * F::vbytes;
                    av[u] = reinterpret_cast<const typename F::vec *>(lut)[in ? byte : 0u];
#pragma unroll
                    for (int pl = 0; pl < F::planes; ++pl)
                        bv[u][pl] = in ? *reinterpret_cast<const typename F::vec *>(bd + pl * bd_plane + off)
                                       : typename F::vec{};
                }
#pragma unroll
                for (int u = 0; u < F::batch8; ++u)
#pragma unroll
                    for (int pl = 0; pl < F::planes; ++pl) accD = mma<PREC>(av[u], bv[u][pl], accD);
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (n < JB && i < p.n_in) {
                const float w = (w0[r] + wnew[t][r]) - p.nu_pre * (accD[r] * rs);
                wnew[t][r] = fminf(fmaxf(w, p.w_min), p.w_max);
                cs += (double)wnew[t][r];
            }
        }
    }
    // 5. FP64 column sums, normalisation factor, theta
    cs += __shfl_xor(cs, 32);
    if (half == 0) part[wave * 32 + n] = cs;
    __syncthreads();
    if (tid < 32) {
        double c = 0.0;
        for (int w = 0; w < kPlasticWaves; ++w) c += part[w * 32 + tid];
        scale[tid] = (p.norm > 0.0 && c > 0.0) ? p.norm / c : 1.0;
        const int j = g * JB + tid;
        if (tid < JB && j < p.n_exc && p.adaptive) theta[j] = theta_step(p, theta[j], (int)cnt[tid]);
    }
    __syncthreads();
    const double sc = scale[n];
#pragma unroll
    for (int t = 0; t < kPlasticTiles; ++t) {
        const int tile = wave + kPlasticWaves * t;
        if (tile >= ntiles) break;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * tile + 8 * (r >> 2) + 4 * half + (r & 3);
            if (n < JB && i < p.n_in)
                Wg[(size_t)i * JB + n] = p.norm > 0.0 ? (float)((double)wnew[t][r] * sc) : wnew[t][r];
        }
    }
}

template __global__ void k_mfma_front<PREC_FP32>(Params, FrontArgs);
template __global__ void k_mfma_front<PREC_BF16>(Params, FrontArgs);
template __global__ void k_mfma_front<PREC_FP8>(Params, FrontArgs);
template __global__ void k_mfma_plastic<PREC_FP32>(Params, float *, double *, const uint16_t *, const float *,
                                                   const float *, const uint32_t *);
template __global__ void k_mfma_plastic<PREC_BF16>(Params, float *, double *, const uint16_t *, const float *,
                                                   const float *, const uint32_t *);
template __global__ void k_mfma_plastic<PREC_FP8>(Params, float *, double *, const uint16_t *, const float *,
                                                  const float *, const uint32_t *);

}  // namespace snn
