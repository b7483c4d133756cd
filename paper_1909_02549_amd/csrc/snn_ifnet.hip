// snn_ifnet.hip -- the converted feed-forward network of integrate-and-fire
// neurons with reset by subtraction (ANN to SNN conversion section): analog
// input, two hidden IF layers, output-layer input summed over the run.
//
// Three launches per run:
//  k_if_input    the analog input's current I1 = (p / 255) W1 + b1, the same
//                at every step, computed once for the whole batch on a grid
//                of (32-sample tile) x (32-neuron tile) workgroups;
//  k_if_net      one workgroup per (32-sample tile, 32-neuron h2 tile) runs
//                all T steps: voltages in registers, the h1 -> h2 and h2 ->
//                output contractions on the matrix cores, spikes exchanged
//                through LDS, one workgroup barrier per step;
//  k_if_readout  the h2 tiles' shares of the readout added, and the argmax.
// All contractions are v_mfma_f32_32x32x16_bf16 with the FP32 weights split
// into three bfloat16 planes that sum to them exactly; pixels (integers up to
// 255) and spikes are exact bfloat16 operands, so every product is exact and
// only the FP32 accumulation rounds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/snn.h"
#include "snn_mfma.h"
#include "snn_runtime.h"

using namespace snn;

namespace {

constexpr int kMaxH1 = 256, kMaxH2 = 128, kMaxOut = 32;
constexpr int kMaxK2 = kMaxH1 / 16;  // 16-deep chunks of the h1 -> h2 contraction
constexpr int kNetThreads = 768;     // 12 waves: 4 chunk waves (h2), 8 h1 waves (one h1 tile each)
// Spike words of a 32-neuron tile: the ballot of C row r holds the words of
// samples 8 (r / 4) + r % 4 (low half) and that + 4 (high half); stored whole
// at word 2r, sample S's word is at ballot_slot(S) (and is half
// ballot_slot(S) % 2 of the ballot of row ballot_slot(S) / 2).
__device__ __forceinline__ int ballot_slot(int S) { return 8 * (S >> 3) + 2 * (S & 3) + ((S >> 2) & 1); }

struct IfDims {
    int n_in, h1, h2, n_out;
    int k1, n1t;  // layer 1: 16-deep chunks of n_in, 32-wide tiles of h1
    int k2, n2t;  // layer 2: chunks of h1, tiles of h2
    int k3;       // layer 3: chunks of h2 (one tile of outputs)
};

// Weight fragments: for chunk c (rows 16c..16c+15) and tile q (columns
// 32q..32q+31) lane l holds column 32q + l % 32, rows 16c + 8 (l / 32) + e,
// e = 0..7, as 8 bfloat16 codes in a uint4 (element e in half e % 2 of
// dword e / 2): the B operand of v_mfma_f32_32x32x16_bf16.  Plane p of
// fragment (c, q) is at P[((c * Nt + q) * 3 + p) * 64 + lane].
__global__ void k_if_pack(const float *__restrict__ W, int K, int N, int Kc, int Nt, uint4 *__restrict__ P)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= Kc * Nt * 64) return;
    const int lane = idx & 63, cq = idx >> 6;
    const int c = cq / Nt, q = cq % Nt;
    const int col = 32 * q + (lane & 31);
    uint32_t code[3][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int row = 16 * c + 8 * (lane >> 5) + e;
        const float w = (row < K && col < N) ? W[(size_t)row * N + col] : 0.f;
        uint32_t cc[3];
        split<PREC_FP32>(w, cc);
#pragma unroll
        for (int p = 0; p < 3; ++p) code[p][e] = cc[p];
    }
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        uint4 v;
        v.x = code[p][0] | (code[p][1] << 16);
        v.y = code[p][2] | (code[p][3] << 16);
        v.z = code[p][4] | (code[p][5] << 16);
        v.w = code[p][6] | (code[p][7] << 16);
        P[(size_t)(cq * 3 + p) * 64 + lane] = v;
    }
}

__device__ __forceinline__ uint32_t px_bf16(uint32_t p) { return __float_as_uint((float)p) >> 16; }

struct IfInArgs {
    const uint8_t *img;  // B x n_in
    const uint4 *P1;     // layer-1 fragments
    const float *b1;     // n1t * 32, zero padded
    float *I1;           // B x n1t * 32
    int B;
    IfDims d;
};

// First-layer current of one (32-sample, 32-neuron) tile.  The 16 waves
// take every sixteenth 16-pixel chunk, four chunks' operands loaded before
// their products; the partial sums are added in wave order.
constexpr int kInWaves = 16;  // also the number of row blocks of a C tile

// 8 pixels (bytes) of one sample, raw: one 8-byte load when rows are 8-byte
// aligned (n_in % 8 == 0; k0 < n_in then implies the bytes are in the row).
template <bool VEC8>
__device__ __forceinline__ uint2 pixels_raw(const uint8_t *im, int k0, int n_in)
{
    if constexpr (VEC8) {
        return *reinterpret_cast<const uint2 *>(im + k0);
    } else {
        uint32_t px[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) px[e] = k0 + e < n_in ? im[k0 + e] : 0u;
        return make_uint2(px[0] | (px[1] << 8) | (px[2] << 16) | (px[3] << 24),
                          px[4] | (px[5] << 8) | (px[6] << 16) | (px[7] << 24));
    }
}

// The 8 pixels as bfloat16 operand elements (integers up to 255 are exact).
__device__ __forceinline__ uint4 pixels_bf16(uint2 raw)
{
    uint4 A;
    A.x = px_bf16(raw.x & 0xFFu) | (px_bf16((raw.x >> 8) & 0xFFu) << 16);
    A.y = px_bf16((raw.x >> 16) & 0xFFu) | (px_bf16(raw.x >> 24) << 16);
    A.z = px_bf16(raw.y & 0xFFu) | (px_bf16((raw.y >> 8) & 0xFFu) << 16);
    A.w = px_bf16((raw.y >> 16) & 0xFFu) | (px_bf16(raw.y >> 24) << 16);
    return A;
}

// Loads are unconditional (addresses clamped into range) and issued for all
// four chunks before any product, so that they are in flight together; the
// operand of a chunk past the end or of a sample past the batch is zeroed
// instead.  The 16 partial sums are added in wave order, wave r adding row
// block r of the tile.
template <bool VEC8>
__global__ __launch_bounds__(64 * kInWaves) void k_if_input(IfInArgs a)
{
    __shared__ float red[kInWaves][16][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int s0 = blockIdx.x * 32, q = blockIdx.y;
    const int srow = s0 + (lane & 31);
    const bool rv = srow < a.B;
    const uint8_t *im = a.img + (size_t)(rv ? srow : s0) * a.d.n_in;
    const int k1 = a.d.k1, n1t = a.d.n1t;
    f32x16_t acc = {};
    for (int base = w; base < k1; base += 4 * kInWaves) {
        uint2 raw[4];
        uint4 Bh[4], Bm[4], Bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = base + j * kInWaves;
            const int cc = c < k1 ? c : base;
            raw[j] = pixels_raw<VEC8>(im, 16 * cc + 8 * (lane >> 5), a.d.n_in);
            const uint4 *pb = a.P1 + (size_t)((cc * n1t + q) * 3) * 64 + lane;
            Bh[j] = pb[0];
            Bm[j] = pb[64];
            Bl[j] = pb[128];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint4 A = pixels_bf16(raw[j]);
            if (!(rv && base + j * kInWaves < k1)) A = make_uint4(0, 0, 0, 0);
            acc = mfma<PREC_FP32>(A, Bh[j], acc);
            acc = mfma<PREC_FP32>(A, Bm[j], acc);
            acc = mfma<PREC_FP32>(A, Bl[j], acc);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) red[w][r][lane] = acc[r];
    __syncthreads();
    const int r = w;  // kInWaves == 16 row blocks
    float sum = red[0][r][lane];
#pragma unroll
    for (int v = 1; v < kInWaves; ++v) sum += red[v][r][lane];
    const int n1p = 32 * n1t;
    const int col = 32 * q + (lane & 31);
    const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (s0 + row < a.B) a.I1[(size_t)(s0 + row) * n1p + col] = sum * (1.f / 255.f) + a.b1[col];
}

struct IfNetArgs {
    const float *I1;  // B x n1t * 32
    const uint4 *P2, *P3;
    const float *b2, *b3;  // padded to 32-wide tiles
    float *rpart;          // n2t x B x 32 partial readouts (one per h2 tile)
    float th1, th2;
    int B, T;
    IfDims d;
    snn_ifnet_outputs o;
};

// LDS of k_if_net: the h2 operand fragments of two steps' h1 spikes, the h2
// partial sums of two steps (4 chunk groups) and two steps' h2 spike words
// (one tile).
constexpr size_t kAbufBytes = 2 * kMaxK2 * 64 * sizeof(uint4);
constexpr size_t kPartBytes = 2 * 4 * 16 * 64 * sizeof(float);
constexpr size_t kNetLds = kAbufBytes + kPartBytes + 2 * 32 * sizeof(uint32_t);
constexpr int kOutWave = 3;  // the chunk wave that runs the output layer

// One workgroup per (32-sample tile, h2 tile y) runs all T steps as a
// four-stage pipeline of 12 waves; in iteration i:
//   waves 4..11 ("h1 waves") integrate step i of h1 tile w - 4 (every h2
//     tile's workgroup integrates all of h1) and publish the h2 operand
//     fragments of its two chunks in buffer i % 2;
//   waves 0..3 ("chunk waves"), wave p:
//     multiplies step i - 1's fragments of chunks 4p..4p + 3 by h2 tile y's
//       weights (three planes, held in registers) and stores the partial
//       sum in buffer (i - 1) % 2;
//     finishes step i - 2 for C rows 4p..4p + 3 of the tile: adds the four
//       partial sums in wave order plus the bias, integrates, and stores the
//       rows' ballot words of the tile in buffer (i - 2) % 2;
//     (wave kOutWave only) multiplies step i - 3's spike words of the tile
//       by the output weights of chunks 2y and 2y + 1, accumulating this
//       tile's share of the readout over the run;
// one workgroup barrier ends the iteration.  C layout of a tile: lane l
// holds neuron 32q + l % 32 of samples 8 (r / 4) + 4 (l / 32) + r % 4,
// r = 0..15.  REC: also record voltages and rasters (the parity outputs).
template <bool REC>
__global__ __launch_bounds__(kNetThreads) void k_if_net(IfNetArgs a)
{
    extern __shared__ uint4 lds_if[];
    const IfDims d = a.d;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w & 3;
    const bool h1wave = w >= 4;
    const int q1 = w - 4;  // h1 wave's tile
    const int s0 = blockIdx.x * 32, y = blockIdx.y;
    const bool lead = y == 0;  // the workgroup that records h1 outputs
    uint4 *abuf = lds_if;
    float *part = reinterpret_cast<float *>(reinterpret_cast<char *>(lds_if) + kAbufBytes);
    uint32_t *mask2 = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(part) + kPartBytes);  // two steps' h2 words

    // operand fragments of the chunks no h1 tile writes (c >= 2 n1t) stay zero
    const int nz = (kMaxK2 - 2 * d.n1t) * 64;
    for (int k = tid; k < 2 * nz; k += kNetThreads) {
        const int bf = k / nz, rest = k - bf * nz;
        abuf[bf * kMaxK2 * 64 + 2 * d.n1t * 64 + rest] = make_uint4(0, 0, 0, 0);
    }
    const int col_in = lane & 31;
    const int slot = ballot_slot(col_in);
    const int h1w = (d.h1 + 31) >> 5, h2w = (d.h2 + 31) >> 5;
    const uint4 zero = make_uint4(0, 0, 0, 0);

    // Each role runs its own loop with one barrier per iteration (T + 3 in
    // both), so that only its own state is live in registers.
    if (h1wave) {
        const int n1p = 32 * d.n1t;
        const bool has1 = q1 < d.n1t;
        const int col = 32 * q1 + col_in;
        float I1[16], v1[16];
        uint32_t cnt1[8];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int s = s0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const bool ok = has1 && s < a.B;
            const float x = a.I1[(size_t)(ok ? s : s0) * n1p + (has1 ? col : col_in)];
            I1[r] = ok ? x : 0.f;
            v1[r] = 0.f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) cnt1[j] = 0;
        __syncthreads();
        for (int i = 0; i <= a.T + 2; ++i) {
            if (i < a.T && has1) {
                const int t = i;
                uint4 *ab = abuf + (t & 1) * kMaxK2 * 64;
                // the ballot of row r holds samples row0 (low half) and
                // row0 + 4 (high half), stored whole at word 2r
                uint64_t mb[16];
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const float u = v1[r] + I1[r];
                    const bool s = u >= a.th1;
                    v1[r] = s ? u - a.th1 : u;
                    cnt1[r >> 1] += (uint32_t)s << (16 * (r & 1));
                    mb[r] = __builtin_amdgcn_ballot_w64(s);
                    if (REC && lead && a.o.v_h1) {
                        const int s_ = s0 + 8 * (r >> 2) + (r & 3) + 4 * (lane >> 5);
                        if (s_ < a.B && col < d.h1) a.o.v_h1[((size_t)t * a.B + s_) * d.h1 + col] = v1[r];
                    }
                }
                // the word of sample S = l % 32 is half h(S) of the ballot of
                // row r(S) (slot(S) = 2 r(S) + h(S)): picked per lane from the
                // wave-uniform ballots (lane: sample l % 32, units
                // 8 (l / 32)..+7 of each chunk); then the h2 operand fragments
                // of chunks 2 q1 and 2 q1 + 1 are published
                uint64_t sel = 0;
#pragma unroll
                for (int r = 0; r < 16; ++r) sel = (slot >> 1) == r ? mb[r] : sel;
                const uint32_t word = (slot & 1) ? (uint32_t)(sel >> 32) : (uint32_t)sel;
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    ab[(2 * q1 + j) * 64 + lane] = ones_bf16((word >> (16 * j + 8 * (lane >> 5))) & 0xFFu);
                if (REC && lead && a.o.raster_h1 && lane < 32 && s0 + lane < a.B)
                    a.o.raster_h1[((size_t)t * a.B + s0 + lane) * h1w + q1] = word;
            }
            __syncthreads();
        }
        if (lead && a.o.counts_h1 && has1 && col < d.h1) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int s = s0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (s < a.B) a.o.counts_h1[(size_t)s * d.h1 + col] = (cnt1[r >> 1] >> (16 * (r & 1))) & 0xFFFFu;
            }
        }
    } else {
        // chunk wave p = wr: h2 tile y's weights of chunks 4p..4p + 3
        const int p = wr;
        uint4 wp[4][3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * p + j;
            const uint4 *pw = a.P2 + (size_t)(((c < d.k2 ? c : 0) * d.n2t + y) * 3) * 64 + lane;
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const uint4 x = pw[64 * pl];
                wp[j][pl] = c < d.k2 ? x : zero;
            }
        }
        // wave p also integrates C rows 4p..4p + 3 of the h2 tile; wave
        // kOutWave runs the output chunks 2y and 2y + 1
        uint4 w3[2][3];
        const bool outw = p == kOutWave;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c3 = 2 * y + j;
#pragma unroll
            for (int pl = 0; pl < 3; ++pl) {
                const uint4 x = a.P3[(size_t)((c3 < d.k3 ? c3 : 0) * 3 + pl) * 64 + lane];
                w3[j][pl] = (outw && c3 < d.k3) ? x : zero;
            }
        }
        const float bias2 = a.b2[32 * y + col_in];
        float v2[4] = {0.f, 0.f, 0.f, 0.f};
        uint32_t cnt2[2] = {0u, 0u};
        f32x16_t acc3 = {};
        __syncthreads();
        for (int i = 0; i <= a.T + 2; ++i) {
            if (outw && i >= 3) {
                // output layer for step t = i - 3 from the tile's spike words
                const int t = i - 3;
                const uint32_t word2 = mask2[(t & 1) * 32 + slot];
                if (REC && a.o.raster_h2 && lane < 32 && s0 + lane < a.B)
                    a.o.raster_h2[((size_t)t * a.B + s0 + lane) * h2w + y] = word2;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint4 A = ones_bf16((word2 >> (16 * j + 8 * (lane >> 5))) & 0xFFu);
                    acc3 = mfma<PREC_FP32>(A, w3[j][0], acc3);
                    acc3 = mfma<PREC_FP32>(A, w3[j][1], acc3);
                    acc3 = mfma<PREC_FP32>(A, w3[j][2], acc3);
                }
            }
            if (i >= 2 && i <= a.T + 1) {
                // finish step t = i - 2 for C rows 4p..4p + 3: add the four
                // partial sums in wave order plus the bias, integrate, publish
                // the rows' ballot words
                const int t = i - 2;
                const float *pt = part + (t & 1) * 4 * 16 * 64;
                const int col2 = 32 * y + col_in;
                uint64_t mb[4];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int r = 4 * p + rr;
                    const float sum = ((pt[r * 64 + lane] + pt[(16 + r) * 64 + lane]) + pt[(32 + r) * 64 + lane]) +
                                      pt[(48 + r) * 64 + lane];
                    const float u = v2[rr] + (sum + bias2);
                    const bool s = u >= a.th2;
                    v2[rr] = s ? u - a.th2 : u;
                    cnt2[rr >> 1] += (uint32_t)s << (16 * (rr & 1));
                    mb[rr] = __builtin_amdgcn_ballot_w64(s);
                    if (REC && a.o.v_h2) {
                        const int s_ = s0 + 8 * (r >> 2) + (r & 3) + 4 * (lane >> 5);
                        if (s_ < a.B && col2 < d.h2) a.o.v_h2[((size_t)t * a.B + s_) * d.h2 + col2] = v2[rr];
                    }
                }
                uint64_t *mq = reinterpret_cast<uint64_t *>(mask2 + (t & 1) * 32);
                if (lane == 0) {
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) mq[4 * p + rr] = mb[rr];
                }
            }
            if (i >= 1 && i <= a.T) {
                // partial h2 current of step t = i - 1 over chunks 4p..4p + 3
                const int t = i - 1;
                const uint4 *ab = abuf + (t & 1) * kMaxK2 * 64;
                f32x16_t acc = {};
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint4 A = ab[(4 * p + j) * 64 + lane];
                    acc = mfma<PREC_FP32>(A, wp[j][0], acc);
                    acc = mfma<PREC_FP32>(A, wp[j][1], acc);
                    acc = mfma<PREC_FP32>(A, wp[j][2], acc);
                }
                float *pt = part + (t & 1) * 4 * 16 * 64 + p * 16 * 64;
#pragma unroll
                for (int r = 0; r < 16; ++r) pt[r * 64 + lane] = acc[r];
            }
            __syncthreads();
        }
        if (a.o.counts_h2 && 32 * y + col_in < d.h2) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int r = 4 * p + rr;
                const int s = s0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (s < a.B)
                    a.o.counts_h2[(size_t)s * d.h2 + 32 * y + col_in] = (cnt2[rr >> 1] >> (16 * (rr & 1))) & 0xFFFFu;
            }
        }
        if (outw) {
            // this tile's share of the readout
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int s = s0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (s < a.B) a.rpart[((size_t)y * a.B + s) * 32 + col_in] = acc3[r];
            }
        }
    }
}

// Readout: the h2 tiles' shares added in tile order, plus T * b3, and the
// argmax (first maximum on ties).  32 lanes per sample, lane o = output o.
__global__ __launch_bounds__(256) void k_if_readout(const float *__restrict__ rpart, const float *__restrict__ b3,
                                                     int B, int T, int n2t, int n_out, float *__restrict__ out_sum,
                                                     int32_t *__restrict__ pred)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = g >> 5, o = g & 31;
    const bool ok = s < B && o < n_out;
    const int sc = s < B ? s : 0;
    float part[4];
#pragma unroll
    for (int y = 0; y < 4; ++y) part[y] = rpart[((size_t)(y < n2t ? y : 0) * B + sc) * 32 + o];
    float sum = part[0];
#pragma unroll
    for (int y = 1; y < 4; ++y)
        if (y < n2t) sum += part[y];
    const float val = sum + (float)T * b3[o];
    if (ok && out_sum) out_sum[(size_t)s * n_out + o] = val;
    // argmax over the 32 lanes of the sample: larger value, or equal value
    // and smaller index
    float bv = ok ? val : -INFINITY;
    int bi = o;
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) {
        const float ov = __shfl_xor(bv, m, 32);
        const int oi = __shfl_xor(bi, m, 32);
        if (ov > bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (pred && o == 0 && s < B) pred[s] = bi;
}

// Scratch of snn_ifnet_run_noalloc: the first-layer current I1 (B x n1t *
// 32 floats) followed by the partial readouts (n2t x B x 32 floats), for
// callers that cannot allocate.  Each GPU holds one copy until the process
// ends; every call on a GPU uses that GPU's copy.
constexpr size_t kNoallocScratchBytes = size_t(6) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

// Device addresses of `scratch`, one per GPU, looked up with that GPU current
// when the first handle on it is created (the host-side name of the array is
// not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int device, void **ptr)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = q;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

struct snn_ifnet {
    snn_ifnet_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    IfDims d{};
    uint4 *P[3] = {nullptr, nullptr, nullptr};
    float *b[3] = {nullptr, nullptr, nullptr};
    float *I1 = nullptr;
    float *rpart = nullptr;  // n2t x max_batch x 32 partial readouts
    void *scratch = nullptr; // this device's copy of `scratch` (snn_ifnet_run_noalloc)
    float *wtmp = nullptr;
    size_t wtmp_n = 0;
    bool set[3] = {false, false, false};
    size_t lds = 0;
    ~snn_ifnet()
    {
        if (stream) (void)hipStreamSynchronize(stream);
        else (void)hipDeviceSynchronize();
        for (int l = 0; l < 3; ++l) {
            if (P[l]) (void)hipFree(P[l]);
            if (b[l]) (void)hipFree(b[l]);
        }
        if (I1) (void)hipFree(I1);
        if (rpart) (void)hipFree(rpart);
        if (wtmp) (void)hipFree(wtmp);
    }
    // rows K, columns N, 16-deep chunks, 32-wide tiles of layer l (0-based)
    void shape(int l, int &K, int &N, int &Kc, int &Nt) const
    {
        K = l == 0 ? d.n_in : l == 1 ? d.h1 : d.h2;
        N = l == 0 ? d.h1 : l == 1 ? d.h2 : d.n_out;
        Kc = (K + 15) / 16;
        Nt = (N + 31) / 32;
    }
};

#define IF_TRY(call)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return snn_net::error(SNN_EDEVICE, (std::string(#call) + ": " + hipGetErrorString(e_)).c_str()); \
    } while (0)

extern "C" snn_status snn_ifnet_create(const snn_ifnet_config *cfg, void *stream, snn_ifnet **out)
{
    if (!out) return snn_net::error(SNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cfg) return snn_net::error(SNN_EINVAL, "snn_ifnet_config is NULL");
    if (cfg->abi_version != SNN_ABI_VERSION) return snn_net::error(SNN_EINVAL, "abi_version mismatch");
    if (cfg->n_in < 1 || cfg->n_in > 65536) return snn_net::error(SNN_EINVAL, "n_in must be in [1, 65536]");
    if (cfg->n_h1 < 1 || cfg->n_h1 > (uint32_t)kMaxH1) return snn_net::error(SNN_EINVAL, "n_h1 must be in [1, 256]");
    if (cfg->n_h2 < 1 || cfg->n_h2 > (uint32_t)kMaxH2) return snn_net::error(SNN_EINVAL, "n_h2 must be in [1, 128]");
    if (cfg->n_out < 1 || cfg->n_out > (uint32_t)kMaxOut) return snn_net::error(SNN_EINVAL, "n_out must be in [1, 32]");
    if (!(cfg->theta_h1 > 0.0) || !(cfg->theta_h2 > 0.0) || cfg->theta_h1 > 1e30 || cfg->theta_h2 > 1e30)
        return snn_net::error(SNN_EINVAL, "thresholds must be finite and > 0");
    if (cfg->max_batch < 1 || cfg->max_batch > (1u << 24)) return snn_net::error(SNN_EINVAL, "max_batch must be in [1, 2^24]");
    snn_ifnet *n = new (std::nothrow) snn_ifnet();
    if (!n) return snn_net::error(SNN_ENOMEM, "host allocation failed");
    n->cfg = *cfg;
    n->stream = static_cast<hipStream_t>(stream);
    IfDims &d = n->d;
    d.n_in = cfg->n_in;
    d.h1 = cfg->n_h1;
    d.h2 = cfg->n_h2;
    d.n_out = cfg->n_out;
    d.k1 = (d.n_in + 15) / 16;
    d.n1t = (d.h1 + 31) / 32;
    d.k2 = (d.h1 + 15) / 16;
    d.n2t = (d.h2 + 31) / 32;
    d.k3 = (d.h2 + 15) / 16;
    n->lds = kNetLds;
    auto bail = [&](hipError_t e, const char *what) {
        delete n;
        return snn_net::error(e == hipErrorOutOfMemory ? SNN_ENOMEM : SNN_EDEVICE,
                              (std::string(what) + ": " + hipGetErrorString(e)).c_str());
    };
    hipError_t e = hipGetDevice(&n->device);
    if (e != hipSuccess) return bail(e, "hipGetDevice");
    if ((e = scratch_address(n->device, &n->scratch)) != hipSuccess) return bail(e, "hipGetSymbolAddress(scratch)");
    size_t wmax = 0;
    for (int l = 0; l < 3; ++l) {
        int K, N, Kc, Nt;
        n->shape(l, K, N, Kc, Nt);
        wmax = std::max(wmax, (size_t)K * N);
        if ((e = hipMalloc(&n->P[l], (size_t)Kc * Nt * 3 * 64 * sizeof(uint4))) != hipSuccess) return bail(e, "hipMalloc");
        if ((e = hipMalloc(&n->b[l], (size_t)Nt * 32 * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc");
    }
    n->wtmp_n = wmax;
    if ((e = hipMalloc(&n->wtmp, wmax * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc");
    if ((e = hipMalloc(&n->I1, (size_t)cfg->max_batch * 32 * d.n1t * sizeof(float))) != hipSuccess)
        return bail(e, "hipMalloc");
    if ((e = hipMalloc(&n->rpart, (size_t)cfg->max_batch * 32 * d.n2t * sizeof(float))) != hipSuccess)
        return bail(e, "hipMalloc");
    if ((e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_if_net<false>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)n->lds)) != hipSuccess ||
        (e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_if_net<true>),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)n->lds)) != hipSuccess)
        return bail(e, "hipFuncSetAttribute");
    *out = n;
    return SNN_OK;
}

extern "C" void snn_ifnet_destroy(snn_ifnet *net) { delete net; }

extern "C" snn_status snn_ifnet_set_layer(snn_ifnet *net, uint32_t layer, const float *w_host, size_t n_w,
                                          const float *b_host, size_t n_b)
{
    if (!net) return snn_net::error(SNN_EINVAL, "net is NULL");
    if (layer < 1 || layer > 3) return snn_net::error(SNN_EINVAL, "layer must be 1, 2 or 3");
    if (!w_host || !b_host) return snn_net::error(SNN_EINVAL, "weights or biases are NULL");
    const int l = (int)layer - 1;
    int K, N, Kc, Nt;
    net->shape(l, K, N, Kc, Nt);
    if (n_w != (size_t)K * N) return snn_net::error(SNN_EINVAL, "weight count does not match the layer sizes");
    if (n_b != (size_t)N) return snn_net::error(SNN_EINVAL, "bias count does not match the layer size");
    std::vector<float> bp((size_t)Nt * 32, 0.f);
    std::memcpy(bp.data(), b_host, n_b * sizeof(float));
    IF_TRY(hipMemcpyAsync(net->wtmp, w_host, n_w * sizeof(float), hipMemcpyHostToDevice, net->stream));
    IF_TRY(hipMemcpyAsync(net->b[l], bp.data(), bp.size() * sizeof(float), hipMemcpyHostToDevice, net->stream));
    const int items = Kc * Nt * 64;
    hipLaunchKernelGGL(k_if_pack, dim3((items + 255) / 256), dim3(256), 0, net->stream, net->wtmp, K, N, Kc, Nt,
                       net->P[l]);
    IF_TRY(hipGetLastError());
    IF_TRY(hipStreamSynchronize(net->stream));
    net->set[l] = true;
    return SNN_OK;
}

// Argument checks shared by snn_ifnet_run and snn_ifnet_run_noalloc.
static snn_status ifnet_check(const snn_ifnet *net, const uint8_t *images_dev, uint32_t batch, uint32_t T)
{
    if (!net) return snn_net::error(SNN_EINVAL, "net is NULL");
    if (!images_dev) return snn_net::error(SNN_EINVAL, "images_dev is NULL");
    if (batch == 0) return snn_net::error(SNN_EINVAL, "batch must be > 0");
    if (T == 0 || T > 65535) return snn_net::error(SNN_EINVAL, "T must be in [1, 65535]");
    if (!net->set[0] || !net->set[1] || !net->set[2]) return snn_net::error(SNN_EINVAL, "every layer must be set first");
    return SNN_OK;
}

// The three launches of a run, with the first-layer current in I1 (batch x
// n1t * 32 floats) and the partial readouts in rpart (n2t x batch x 32).
static snn_status ifnet_launch(snn_ifnet *net, const uint8_t *images_dev, uint32_t batch, uint32_t T,
                               const snn_ifnet_outputs *out, float *I1, float *rpart)
{
    snn_ifnet_outputs o{};
    if (out) o = *out;
    const int tiles = (int)((batch + 31) / 32);
    const bool vec8 = net->d.n_in % 8 == 0 && (reinterpret_cast<uintptr_t>(images_dev) & 7) == 0;
    IfInArgs ia{images_dev, net->P[0], net->b[0], I1, (int)batch, net->d};
    if (vec8)
        hipLaunchKernelGGL(k_if_input<true>, dim3(tiles, net->d.n1t), dim3(64 * kInWaves), 0, net->stream, ia);
    else
        hipLaunchKernelGGL(k_if_input<false>, dim3(tiles, net->d.n1t), dim3(64 * kInWaves), 0, net->stream, ia);
    IF_TRY(hipGetLastError());
    IfNetArgs na{I1, net->P[1], net->P[2], net->b[1], net->b[2], rpart, (float)net->cfg.theta_h1,
                 (float)net->cfg.theta_h2, (int)batch, (int)T, net->d, o};
    const dim3 grid(tiles, net->d.n2t);
    if (o.raster_h1 || o.raster_h2 || o.v_h1 || o.v_h2)
        hipLaunchKernelGGL(k_if_net<true>, grid, dim3(kNetThreads), net->lds, net->stream, na);
    else
        hipLaunchKernelGGL(k_if_net<false>, grid, dim3(kNetThreads), net->lds, net->stream, na);
    IF_TRY(hipGetLastError());
    if (o.out_sum || o.pred)
        hipLaunchKernelGGL(k_if_readout, dim3((batch + 7) / 8), dim3(256), 0, net->stream, rpart, net->b[2],
                           (int)batch, (int)T, net->d.n2t, net->d.n_out, o.out_sum, o.pred);
    IF_TRY(hipGetLastError());
    return SNN_OK;
}

extern "C" snn_status snn_ifnet_run(snn_ifnet *net, const uint8_t *images_dev, uint32_t batch, uint32_t T,
                                    const snn_ifnet_outputs *out)
{
    const snn_status st = ifnet_check(net, images_dev, batch, T);
    if (st != SNN_OK) return st;
    if (batch > net->cfg.max_batch) return snn_net::error(SNN_ENOMEM, "batch exceeds max_batch");
    return ifnet_launch(net, images_dev, batch, T, out, net->I1, net->rpart);
}

extern "C" snn_status snn_ifnet_run_noalloc(snn_ifnet *net, const uint8_t *images_dev, uint32_t batch, uint32_t T,
                                            const snn_ifnet_outputs *out)
{
    const snn_status st = ifnet_check(net, images_dev, batch, T);
    if (st != SNN_OK) return st;
    const size_t i1_floats = (size_t)batch * 32 * net->d.n1t;
    const size_t need = (i1_floats + (size_t)batch * 32 * net->d.n2t) * sizeof(float);
    if (need > kNoallocScratchBytes)
        return snn_net::error(SNN_ENOMEM, ("batch needs " + std::to_string(need) + " scratch bytes, more than the " +
                                           std::to_string(kNoallocScratchBytes) + " of snn_ifnet_run_noalloc")
                                              .c_str());
    float *base = static_cast<float *>(net->scratch);
    return ifnet_launch(net, images_dev, batch, T, out, base, base + i1_floats);
}

extern "C" snn_status snn_ifnet_sync(snn_ifnet *net)
{
    if (!net) return snn_net::error(SNN_EINVAL, "net is NULL");
    IF_TRY(hipStreamSynchronize(net->stream));
    return SNN_OK;
}
