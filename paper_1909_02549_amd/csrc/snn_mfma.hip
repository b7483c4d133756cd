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

#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_mfma.h"

namespace snn {

typedef __bf16 bf16x8_t __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x16_t __attribute__((__vector_size__(16 * sizeof(float))));

template <int PREC>
struct Form {
    static constexpr int planes = PREC == PREC_FP32 ? 3 : 1;
    static constexpr int esize = PREC == PREC_FP8 ? 1 : 2;  // bytes per element
    static constexpr int vbytes = 8 * esize;                 // bytes per lane operand
};

// 8 spike bits -> 8 operand elements equal to 1 or 0.
__device__ __forceinline__ uint4 ones_bf16(uint32_t byte)
{
    uint4 r;
    r.x = ((byte & 1u) * 0x3F80u) | (((byte >> 1) & 1u) * 0x3F800000u);
    r.y = (((byte >> 2) & 1u) * 0x3F80u) | (((byte >> 3) & 1u) * 0x3F800000u);
    r.z = (((byte >> 4) & 1u) * 0x3F80u) | (((byte >> 5) & 1u) * 0x3F800000u);
    r.w = (((byte >> 6) & 1u) * 0x3F80u) | (((byte >> 7) & 1u) * 0x3F800000u);
    return r;
}

__device__ __forceinline__ uint2 ones_fp8(uint32_t byte)
{
    // E4M3 1.0 = 0x38
    uint2 r;
    r.x = ((byte & 1u) * 0x38u) | (((byte >> 1) & 1u) * 0x3800u) | (((byte >> 2) & 1u) * 0x380000u) |
          (((byte >> 3) & 1u) * 0x38000000u);
    r.y = (((byte >> 4) & 1u) * 0x38u) | (((byte >> 5) & 1u) * 0x3800u) | (((byte >> 6) & 1u) * 0x380000u) |
          (((byte >> 7) & 1u) * 0x38000000u);
    return r;
}

// One MFMA step on raw operand registers.
template <int PREC>
__device__ __forceinline__ f32x16_t mfma(uint4 a, uint4 b, f32x16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                   0, 0, 0);
}
template <int PREC>
__device__ __forceinline__ f32x16_t mfma8(uint2 a, uint2 b, f32x16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b), c, 0,
                                                      0, 0);
}

// Operand codes of one value x in the form PREC (plane 0 first).
template <int PREC>
__device__ __forceinline__ void split(float x, uint32_t c[3])
{
    if constexpr (PREC == PREC_FP32) {
        c[0] = bf16_code(x);
        const float r1 = x - bf16_value(c[0]);
        c[1] = bf16_code(r1);
        const float r2 = r1 - bf16_value(c[1]);
        c[2] = bf16_code(r2);
    } else if constexpr (PREC == PREC_BF16) {
        c[0] = bf16_code(x);
    } else {
        c[0] = e4m3_code(x);
    }
}

// ---------------------------------------------------------------------------
// synaptic current
// ---------------------------------------------------------------------------
//
// Workgroup (g, y): column block g (JB <= 32 columns, padded to 32 with zero
// weights), samples 128 y .. 128 y + 127, one 32-sample tile per wave.  The
// block's weights pass through LDS in chunks of kContractRows rows, converted
// once to operand planes laid out as the B operand wants them:
//   plane[ks][half][n][e] = q(W[16 ks + 8 half + e, n])
// so each lane reads one contiguous 16-byte (8-byte for FP8) operand.
constexpr int kContractRows = 160;

size_t mfma_contract_lds(int prec)
{
    const int planes = prec == PREC_FP32 ? 3 : 1;
    const int esize = prec == PREC_FP8 ? 1 : 2;
    return (size_t)planes * kContractRows * 32 * esize;
}

template <int PREC>
__global__ __launch_bounds__(256) void k_mfma_contract(Params p, const float *__restrict__ W,
                                                       const uint32_t *__restrict__ bits_t, float *__restrict__ I)
{
    using F = Form<PREC>;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr size_t plane_bytes = (size_t)kContractRows * 32 * F::esize;
    const int g = blockIdx.x;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int n = lane & 31, half = lane >> 5;
    const int b0 = (blockIdx.y * 4 + wave) * 32;
    const int b = b0 + n;
    const bool active = b0 < p.B;
    const int JB = p.jb;
    const float *Wg = W + (size_t)g * p.n_in_pad * JB;

    // columns JB .. 31 are never written below: zero the whole buffer once
    for (int q = tid; q < (int)(F::planes * plane_bytes / 16); q += blockDim.x)
        reinterpret_cast<uint4 *>(smem)[q] = make_uint4(0u, 0u, 0u, 0u);

    f32x16_t acc = {};
    const uint32_t *brow = bits_t + (size_t)(b < p.B ? b : 0) * p.in_words;
    for (int k0 = 0; k0 < p.n_in_pad; k0 += kContractRows) {
        const int kc = min(kContractRows, p.n_in_pad - k0);
        __syncthreads();
        for (int q = tid; q < kc * JB; q += blockDim.x) {
            const int k = q / JB, jj = q - (q / JB) * JB;
            uint32_t c[3];
            split<PREC>(Wg[(size_t)(k0 + k) * JB + jj], c);
            const size_t e = ((size_t)((k >> 4) * 2 + ((k >> 3) & 1)) * 32 + jj) * 8 + (k & 7);
#pragma unroll
            for (int pl = 0; pl < F::planes; ++pl) {
                if constexpr (F::esize == 2)
                    reinterpret_cast<uint16_t *>(smem + pl * plane_bytes)[e] = (uint16_t)c[pl];
                else
                    (smem + pl * plane_bytes)[e] = (uint8_t)c[pl];
            }
        }
        __syncthreads();
        if (active) {
            uint32_t word = 0;
            for (int ks = 0; ks < kc / 16; ++ks) {
                const int kg = k0 + 16 * ks;
                if ((kg & 31) == 0) word = b < p.B ? brow[kg >> 5] : 0u;
                const uint32_t byte = (word >> (8 * (((kg & 31) >> 3) + half))) & 0xFFu;
                const size_t off = ((size_t)(ks * 2 + half) * 32 + n) * F::vbytes;
                if constexpr (F::esize == 2) {
                    const uint4 a = ones_bf16(byte);
#pragma unroll
                    for (int pl = 0; pl < F::planes; ++pl)
                        acc = mfma<PREC>(a, *reinterpret_cast<const uint4 *>(smem + pl * plane_bytes + off), acc);
                } else {
                    acc = mfma8<PREC>(ones_fp8(byte), *reinterpret_cast<const uint2 *>(smem + off), acc);
                }
            }
        }
    }
    if (!active) return;
    const size_t base = (size_t)g * p.Bs * p.jbp;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int bb = b0 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (bb < p.B && n < p.jbp) I[base + (size_t)bb * p.jbp + n] = acc[r];
    }
}

// ---------------------------------------------------------------------------
// STDP weight change, update, clamp, normalisation, theta
// ---------------------------------------------------------------------------
//
// One workgroup (8 waves) per column block g; wave w owns input tiles
// i0 = 32 (w + 8 t), t < kPlasticTiles, and keeps their updated weights in
// registers until the column sums are known.
//   P tile: A = q(x_pre) rows of the samples in which some column of the
//           block fired (compacted list, K = that count rounded up to 16),
//           B = their 0/1 exc spikes, staged in LDS;
//   D tile: A = 0/1 input spikes of the tile's inputs over all samples (from
//           the per-input bit rows), B = q(x_post) of the block, staged in
//           LDS as operand planes.
constexpr int kPlasticWaves = 8;
constexpr int kPlasticTiles = 4;  // n_in_pad <= 32 * 8 * 4 = 1024

struct PlasticLds {
    size_t smask, slist, cnt, bp, bd, part, scale, total;
    int B16;
    __host__ __device__ PlasticLds(const Params &p, int prec)
    {
        const int planes = prec == PREC_FP32 ? 3 : 1;
        const int esize = prec == PREC_FP8 ? 1 : 2;
        B16 = (p.B + 15) & ~15;
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
    return p.reduce != RED_MAX && p.jb <= 32 && p.n_in_pad <= 32 * kPlasticWaves * kPlasticTiles &&
           mfma_plastic_lds(p, prec) <= 160 * 1024;
}

template <int PREC>
__global__ __launch_bounds__(512) void k_mfma_plastic(Params p, float *__restrict__ W, double *__restrict__ theta,
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
    double *part = reinterpret_cast<double *>(smem + L.part);
    double *scale = reinterpret_cast<double *>(smem + L.scale);
    const size_t bd_plane = (size_t)L.B16 * 32 * F::esize;

    const int g = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int n = lane & 31, half = lane >> 5;
    const int JB = p.jb, JBP = p.jbp, B16 = L.B16;
    const size_t sbase = (size_t)g * p.Bs * JBP;

    // 1. exc spikes of the block per sample, column counts; q(x_post) planes
    for (int q = tid; q < B16; q += nt) smask[q] = 0u;
    if (tid < 33) cnt[tid] = 0u;
    __syncthreads();
    for (int q = tid; q < B16 * 32; q += nt) {
        const int b = q >> 5, jj = q & 31;
        float x = 0.f;
        if (b < p.B && jj < JB) {
            const size_t s = sbase + (size_t)b * JBP + jj;
            if (rf[s] & RF_SPIKE) {
                atomicOr(&smask[b], 1u << jj);
                atomicAdd(&cnt[jj], 1u);
            }
            x = x_post[s];
        }
        uint32_t c[3];
        split<PREC>(x, c);
        const size_t e = ((size_t)((b >> 4) * 2 + ((b >> 3) & 1)) * 32 + jj) * 8 + (b & 7);
#pragma unroll
        for (int pl = 0; pl < F::planes; ++pl) {
            if constexpr (F::esize == 2)
                reinterpret_cast<uint16_t *>(bd + pl * bd_plane)[e] = (uint16_t)c[pl];
            else
                (bd + pl * bd_plane)[e] = (uint8_t)c[pl];
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
    for (int q = tid; q < K1 * 32; q += nt) {
        const int kk = q >> 5, jj = q & 31;
        const uint32_t sid = slist[kk];
        const uint32_t on = sid != 0xFFFFu ? (smask[sid] >> jj) & 1u : 0u;
        const size_t e = ((size_t)((kk >> 4) * 2 + ((kk >> 3) & 1)) * 32 + jj) * 8 + (kk & 7);
        if constexpr (F::esize == 2)
            reinterpret_cast<uint16_t *>(bp)[e] = (uint16_t)(on * 0x3F80u);
        else
            bp[e] = (uint8_t)(on * 0x38u);
    }
    __syncthreads();

    // 3. tiles: P and D on the matrix cores, update and clamp in registers
    float *Wg = W + (size_t)g * p.n_in_pad * JB;
    const int ntiles = p.n_in_pad >> 5;
    float wnew[kPlasticTiles][16];
    double cs = 0.0;
#pragma unroll
    for (int t = 0; t < kPlasticTiles; ++t) {
        const int tile = wave + kPlasticWaves * t;
        if (tile >= ntiles) break;
        const int i0 = 32 * tile;
        f32x16_t accP = {}, accD = {};
        // P: A[i][kk] = q(x_pre[slist[kk], i0 + n])
        for (int ks = 0; ks < K1 / 16; ++ks) {
            uint32_t c[8][3];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t sid = slist[16 * ks + 8 * half + e];
                const float x = sid != 0xFFFFu ? x_pre[(size_t)sid * p.n_in_pad + i0 + n] : 0.f;
                split<PREC>(x, c[e]);
            }
            const size_t off = ((size_t)(ks * 2 + half) * 32 + n) * F::vbytes;
            if constexpr (F::esize == 2) {
                const uint4 bo = *reinterpret_cast<const uint4 *>(bp + off);
#pragma unroll
                for (int pl = 0; pl < F::planes; ++pl) {
                    const uint4 a = make_uint4(c[0][pl] | (c[1][pl] << 16), c[2][pl] | (c[3][pl] << 16),
                                               c[4][pl] | (c[5][pl] << 16), c[6][pl] | (c[7][pl] << 16));
                    accP = mfma<PREC>(a, bo, accP);
                }
            } else {
                const uint2 a = make_uint2(c[0][0] | (c[1][0] << 8) | (c[2][0] << 16) | (c[3][0] << 24),
                                           c[4][0] | (c[5][0] << 8) | (c[6][0] << 16) | (c[7][0] << 24));
                accP = mfma8<PREC>(a, *reinterpret_cast<const uint2 *>(bp + off), accP);
            }
        }
        // D: A[i][b] = s_in[b, i0 + n] from the input's bit row
        const uint32_t *trow = bitsT_t + (size_t)(i0 + n) * p.bwords;
        uint32_t word = 0;
        for (int ks = 0; ks < B16 / 16; ++ks) {
            if ((ks & 1) == 0) word = (16 * ks < p.B) ? trow[ks >> 1] : 0u;
            const uint32_t byte = (word >> (8 * (2 * (ks & 1) + half))) & 0xFFu;
            const size_t off = ((size_t)(ks * 2 + half) * 32 + n) * F::vbytes;
            if constexpr (F::esize == 2) {
                const uint4 a = ones_bf16(byte);
#pragma unroll
                for (int pl = 0; pl < F::planes; ++pl)
                    accD = mfma<PREC>(a, *reinterpret_cast<const uint4 *>(bd + pl * bd_plane + off), accD);
            } else {
                accD = mfma8<PREC>(ones_fp8(byte), *reinterpret_cast<const uint2 *>(bd + off), accD);
            }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = i0 + 8 * (r >> 2) + 4 * half + (r & 3);
            float w = 0.f;
            if (n < JB && i < p.n_in) {
                w = stdp_apply(p, Wg[(size_t)i * JB + n], accP[r], accD[r]);
                cs += (double)w;
            }
            wnew[t][r] = w;
        }
    }
    // 4. FP64 column sums, normalisation factor, theta
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
    const double s = scale[n];
#pragma unroll
    for (int t = 0; t < kPlasticTiles; ++t) {
        const int tile = wave + kPlasticWaves * t;
        if (tile >= ntiles) break;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * tile + 8 * (r >> 2) + 4 * half + (r & 3);
            if (n < JB && i < p.n_in) Wg[(size_t)i * JB + n] = p.norm > 0.0 ? (float)((double)wnew[t][r] * s) : wnew[t][r];
        }
    }
}

template __global__ void k_mfma_contract<PREC_FP32>(Params, const float *, const uint32_t *, float *);
template __global__ void k_mfma_contract<PREC_BF16>(Params, const float *, const uint32_t *, float *);
template __global__ void k_mfma_contract<PREC_FP8>(Params, const float *, const uint32_t *, float *);
template __global__ void k_mfma_plastic<PREC_FP32>(Params, float *, double *, const uint16_t *, const float *,
                                                   const float *, const uint32_t *);
template __global__ void k_mfma_plastic<PREC_BF16>(Params, float *, double *, const uint16_t *, const float *,
                                                   const float *, const uint32_t *);
template __global__ void k_mfma_plastic<PREC_FP8>(Params, float *, double *, const uint16_t *, const float *,
                                                  const float *, const uint32_t *);

}  // namespace snn
