// snn_fused.h -- the column-block step shared by the fused (one launch per
// step) and persistent (one cooperative launch per chunk of steps) kernels.
//
// Workgroup g owns the JB post-synaptic columns [g*JB, g*JB+JB) for every
// sample of the batch: their weight block W[:, cols] (in LDS), their neuron
// state and their adaptive thresholds.  What the method couples across
// columns is small: the per-sample inhibitory spike count C[b] (all-but-self
// inhibition) and the presynaptic traces x_pre (read by every column).
//
// In LDS the weight block and the post traces are stored with row stride
// p.ls (JBP, or JBP + 4 when JBP is 16 or 32 so that rows read by
// different lanes start on different banks); JBP = JB
// rounded up to 8 columns per row plus one all-zero row, so a thread owning 8
// consecutive columns reads a row with two 16-byte loads, and the padding
// slots of an index list point at the zero row (adding +0 changes no sum).
//
// Column normalisation is kept lazily: after a learning step the block holds
// the clamped, not yet normalised weights and scale[c] = norm / sum_i W[i, c]
// (FP64 sum and quotient, also kept rounded to FP32); the next step applies
// the FP32 scale (w <- w * scale, within one rounding of the FP64 product)
// when it updates the weight, the contraction multiplies its column sum by it,
// and the block is written back to HBM normalised with the FP64 scale.
#pragma once
#include <hip/hip_runtime.h>

#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_mfma.h"

namespace snn {

constexpr int kFusedThreads = 1024;   // fused per-step kernel: 16 waves
constexpr int kPersistThreads = 512;  // persistent kernel: 8 waves, with
constexpr int kPersistTasks = 2;      //   two (sample, 8 columns) tasks each
constexpr int kListHead = 4;          // 16-byte words of a spike list read ahead
constexpr int kIndepThreads = 256;    // chunk kernel of independent tasks: 4 waves
constexpr int kMfmaPotentiation = 0;  // spiking samples above which potentiation runs on the matrix cores
static_assert(kFusedThreads % 128 == 0 && kPersistThreads % 128 == 0, "split-row plasticity needs nt % 128 == 0");

// Per-network pointers (state and parameters owned by the handle).
struct FusedArgs {
    float *W;
    double *theta;
    float *v_exc, *v_inh, *x_post;
    uint16_t *rf;
    Outs o;
};

// Per-step pointers.
struct StepPtrs {
    const uint32_t *bits;       // input spikes of step t, B x in_words
    const uint32_t *bits_next;  // input spikes of step t + 1 (nullptr: none)
    const uint16_t *lin;        // per-sample input spike lists of step t
    const uint32_t *cin;        //   and their lengths
    const uint16_t *lt;         // per-input sample spike lists of step t
    const uint32_t *ct;         //   and their lengths
    const uint16_t *ord_s;      // samples by decreasing list length (step t)
    const uint16_t *ord_in;     // inputs by decreasing list length (step t)
    const float *xpre;          // x_pre(t), B x n_in_pad
    float *xpre_next;           // x_pre(t + 1)
    const uint32_t *Cprev;      // inhibitory spike counts of step t - 1
    uint32_t *Ccur;             // counts of step t (accumulated)
    uint32_t *Cnext;            // cleared for step t + 1
    int k;                      // step index within the call (outputs)
};

// Pointers of one chunk of steps run by a persistent launch.
struct ChunkPtrs {
    const uint32_t *bits;  // input spikes of the chunk's steps (+1 if has_next)
    const uint16_t *lin;
    const uint32_t *cin;
    const uint16_t *lt;
    const uint32_t *ct;
    const uint16_t *ord_in;  // per step: inputs by decreasing list length
    float *xpre;           // 3 x B x n_in_pad, x_pre(s) in buffer s % 3
    uint32_t *C;           // 3 x B, inhibitory counts of step s in slot s % 3
    int steps;             // steps to run
    int has_next;          // inputs of step `steps` are encoded (x_pre ahead)
    int mod0;              // s % 3 of the first step
    int k0;                // output index of the first step
    int norm_from;         // first step (within the chunk) that normalises
};

// Cross-workgroup state of one persistent launch.
struct PersistSync {
    uint32_t *bar;  // arrival counter, zeroed before the launch
    uint32_t *err;  // set to 1 if a barrier wait timed out
};

// Arguments of a persistent launch, passed by value (the kernel argument
// segment), so that the compiler knows every pointer in them addresses global
// memory and uses global rather than flat memory instructions: a flat access
// also counts against the LDS wait counter, so any wait for an LDS read would
// drain the outstanding global loads too.
struct PersistArgs {
    Params p;
    FusedArgs a;
    ChunkPtrs ch;
    PersistSync sy;
};

size_t fused_lds_bytes(const Params &p);
size_t persist_lds_bytes(const Params &p);
template <int PREC, int RK>
__global__ void k_fused_step(Params p, FusedArgs a, StepPtrs s);
template <int PREC, int RK>
__global__ void k_persist(const PersistArgs args);
// no learning and no inhibitory layer: every task on its own, no barrier
size_t indep_lds_bytes(const Params &p);
template <int PREC>
__global__ void k_indep(const PersistArgs args);
template <int PREC, int NC>
__global__ void k_indep_narrow(const PersistArgs args);
__global__ void k_lists(Params p, const uint32_t *bits, const uint32_t *bitsT, uint16_t *lin, uint32_t *cin,
                        uint16_t *lt, uint32_t *ct, int with_t);
constexpr int kOrderThreads = 1024;
constexpr int kOrderBins = 1024;
__global__ void k_order(Params p, const uint32_t *cin, const uint32_t *ct, uint16_t *ord_s, uint16_t *ord_in,
                        int with_t);

// ---------------------------------------------------------------------------
// device building blocks
// ---------------------------------------------------------------------------

// Accesses to data another workgroup of the same persistent launch writes
// (next-step presynaptic traces, inhibitory counts) are agent-scope atomic
// loads / stores: they are coherent across the XCDs' separate L2 caches, so
// the grid barrier needs no cache write-back or invalidation and read-only
// data stays cached.  The fused per-step kernel passes Coherent = false
// (kernel boundaries order its exchanges).
template <bool Coherent>
__device__ __forceinline__ float ld_x(const float *ptr)
{
    if (Coherent) return __hip_atomic_load(ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *ptr;
}

template <bool Coherent>
__device__ __forceinline__ uint32_t ld_u(const uint32_t *ptr)
{
    if (Coherent) return __hip_atomic_load(ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *ptr;
}

template <bool Coherent, typename T>
__device__ __forceinline__ void st_x(T *ptr, T v)
{
    if (Coherent) __hip_atomic_store(ptr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *ptr = v;
}

// LDS carve-up shared by host (size) and device (offsets).
struct FusedLds {
    size_t w, xpost, cprev, cinh, spk, colmask, ulist, part, scale, scalef, theta, theta64, total;
    // share_part: the column-sum partials reuse the post-trace rows (the
    // fused kernel, whose post traces are dead by then)
    __host__ __device__ FusedLds(const Params &p, int nthreads, bool share_part = false)
    {
        size_t o = 0;
        w = o;
        o += align16((size_t)(p.n_in_pad + 1) * p.ls * 4);
        scale = o;
        o += 32 * 8;
        scalef = o;
        o += 32 * 4;
        theta = o;
        o += 32 * 4;
        theta64 = o;
        o += 32 * 8;
        // per-sample regions last: a network without inhibitory layer or
        // without learning leaves the tail it does not use unallocated
        const size_t fixed_end = o;
        cprev = o;
        o += align16((size_t)p.B * 4);
        cinh = o;
        o += align16((size_t)p.B * 4);
        const size_t inh_end = o;
        xpost = o;
        o += p.learn ? align16((size_t)(p.B + 1) * p.ls * 4) : 0;
        spk = o;
        o += align16((size_t)p.jb * p.bwords * 4);
        colmask = o;
        o += align16((size_t)p.B * 4);
        ulist = o;
        o += align16((size_t)(p.B + 1) * 4);
        const size_t part_bytes = (size_t)(nthreads / 32) * 32 * 8;
        if (share_part && p.learn && (size_t)(p.B + 1) * p.ls * 4 >= part_bytes) {
            part = xpost;
        } else {
            part = o;
            o += align16(part_bytes);
        }
        // (without inhibitory layer the neuron tasks read cprev[0] and ignore
        // it, so one entry stays allocated)
        total = p.learn ? o : p.has_inh ? inh_end : fixed_end + 16;
    }
};

// Named views of the LDS regions.
struct StepLds {
    float *W, *xpost, *th, *scalef;
    uint32_t *cprev, *cinh, *spk, *colmask, *ulist;
    double *part, *scale, *th64;
    __device__ StepLds(unsigned char *smem, const FusedLds &L)
        : W(reinterpret_cast<float *>(smem + L.w)), xpost(reinterpret_cast<float *>(smem + L.xpost)),
          th(reinterpret_cast<float *>(smem + L.theta)), scalef(reinterpret_cast<float *>(smem + L.scalef)),
          cprev(reinterpret_cast<uint32_t *>(smem + L.cprev)),
          cinh(reinterpret_cast<uint32_t *>(smem + L.cinh)), spk(reinterpret_cast<uint32_t *>(smem + L.spk)),
          colmask(reinterpret_cast<uint32_t *>(smem + L.colmask)),
          ulist(reinterpret_cast<uint32_t *>(smem + L.ulist)), part(reinterpret_cast<double *>(smem + L.part)),
          scale(reinterpret_cast<double *>(smem + L.scale)), th64(reinterpret_cast<double *>(smem + L.theta64))
    {
    }
};

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

// Four list entries (two u32 words of u16 indices) -> acc[0..8) R= rows.
// Operand rounding of the reduced-precision forms on four loaded values.
__device__ __forceinline__ float4 round4(int prec, float4 v)
{
    if (!prec) return v;
    const f32x2_t lo = operand_value2(prec, v.x, v.y), hi = operand_value2(prec, v.z, v.w);
    return make_float4(lo.x, lo.y, hi.x, hi.y);
}

// A trace value as a summand of the reduction of kind RK (the soft maximum's
// exp(x / tau) - 1, else x), and the reduced sum S as the change it makes
// (tau log1p(S / B) for the soft maximum, S / B for the mean, else S).
template <int RK>
__device__ __forceinline__ float red_in(float x, float k)
{
    return RK == RK_SOFT ? soft_term(x, k) : x;
}

template <int RK>
__device__ __forceinline__ float4 red_in4(float4 v, float k)
{
    if (RK != RK_SOFT) return v;
    return make_float4(soft_term(v.x, k), soft_term(v.y, k), soft_term(v.z, k), soft_term(v.w, k));
}

template <int RK>
__device__ __forceinline__ float red_out(const Params &p, float S)
{
    if (RK == RK_SOFT) return soft_value(p, S);
    return p.reduce == RED_MEAN ? S * p.inv_B : S;
}

__device__ __forceinline__ float4 mul4(float4 a, float4 b) { return make_float4(a.x * b.x, a.y * b.y, a.z * b.z, a.w * b.w); }

// Scale: each row value is first multiplied by the column's pending
// normalisation scale (slo: columns c0 .. c0 + 3, shi: c0 + 4 .. c0 + 7), so
// that the operand rounding sees the normalised FP32 weight.
template <int RK = RK_STD, bool Scale = false>
__device__ __forceinline__ void gather4rows(uint2 q, int k0, int cnt, const float *rows, int jbp, int c0, int zero_row,
                                            int mode, float *acc, int prec, float ksoft = 0.f,
                                            float4 slo = float4{}, float4 shi = float4{})
{
    const int i0 = (int)(q.x & 0xFFFFu);
    const int i1 = k0 + 1 < cnt ? (int)(q.x >> 16) : zero_row;
    const int i2 = k0 + 2 < cnt ? (int)(q.y & 0xFFFFu) : zero_row;
    const int i3 = k0 + 3 < cnt ? (int)(q.y >> 16) : zero_row;
    // row offsets with the 24-bit multiply (full rate; indices and strides
    // are far below 2^24)
    const float4 *r0 = reinterpret_cast<const float4 *>(rows + __mul24(i0, jbp) + c0);
    const float4 *r1 = reinterpret_cast<const float4 *>(rows + __mul24(i1, jbp) + c0);
    const float4 *r2 = reinterpret_cast<const float4 *>(rows + __mul24(i2, jbp) + c0);
    const float4 *r3 = reinterpret_cast<const float4 *>(rows + __mul24(i3, jbp) + c0);
    auto val = [&](float4 v, float4 sc) { return red_in4<RK>(round4(prec, Scale ? mul4(v, sc) : v), ksoft); };
    const float4 a0 = val(r0[0], slo), b0 = val(r0[1], shi);
    const float4 a1 = val(r1[0], slo), b1 = val(r1[1], shi);
    const float4 a2 = val(r2[0], slo), b2 = val(r2[1], shi);
    const float4 a3 = val(r3[0], slo), b3 = val(r3[1], shi);
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

// The entries k0 .. cnt of a list (k0 a multiple of 4), 4 * NW at a time:
// the NW 8-byte list words of a batch are loaded together, then gathered in
// list order (the additions are those of a one-word-at-a-time walk).
template <int NW = 4, int RK = RK_STD, bool Scale = false>
__device__ __forceinline__ void gather_tail(const uint2 *__restrict__ l4, int k0, int cnt, const float *rows, int jbp,
                                            int c0, int zero_row, int mode, float *acc, int prec, float ksoft = 0.f,
                                            float4 slo = float4{}, float4 shi = float4{})
{
    for (; k0 < cnt; k0 += 4 * NW) {
        uint2 e[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) e[q] = k0 + 4 * q < cnt ? l4[(k0 >> 2) + q] : make_uint2(0u, 0u);
#pragma unroll
        for (int q = 0; q < NW; ++q)
            if (k0 + 4 * q < cnt)
                gather4rows<RK, Scale>(e[q], k0 + 4 * q, cnt, rows, jbp, c0, zero_row, mode, acc, prec, ksoft, slo,
                                       shi);
    }
}

// acc[0..8) = R over the first `cnt` entries of `list` (u16 row indices, in
// list order) of q(rows[idx * jbp + c0 .. + 8)), four rows in flight at a
// time, q the operand rounding of the precision `prec` (none for FP32);
// slots past cnt read row `zero_row` (all zeros).  The first `nhead` (4 or
// 8) entries are passed in registers (head0, head1), loaded ahead of time.
template <int RK = RK_STD>
__device__ __forceinline__ void gather8(const uint16_t *__restrict__ list, int cnt, uint2 head0, uint2 head1,
                                        int nhead, const float *rows, int jbp, int c0, int zero_row, int mode,
                                        float *acc, int prec, float ksoft = 0.f)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
    if (cnt <= 0) return;
    const uint2 *l4 = reinterpret_cast<const uint2 *>(list);
    gather4rows<RK>(head0, 0, cnt, rows, jbp, c0, zero_row, mode, acc, prec, ksoft);
    if (cnt > 4) gather4rows<RK>(nhead == 8 ? head1 : l4[1], 4, cnt, rows, jbp, c0, zero_row, mode, acc, prec, ksoft);
    gather_tail<4, RK>(l4, 8, cnt, rows, jbp, c0, zero_row, mode, acc, prec, ksoft);
}

// The same with the first 8 * NH entries of the list in h[0 .. NH) (16-byte
// words loaded together ahead of time, so a list of up to 8 * NH entries costs
// one memory round trip); entries past those are read from `list`.
template <int NH, bool Scale = false>
__device__ __forceinline__ void gather_pre(const uint16_t *__restrict__ list, int cnt, const uint4 *h, const float *rows,
                                           int jbp, int c0, int zero_row, int mode, float *acc, int prec,
                                           float4 slo = float4{}, float4 shi = float4{})
{
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.f;
#pragma unroll
    for (int q = 0; q < NH; ++q) {
        if (8 * q < cnt)
            gather4rows<RK_STD, Scale>(make_uint2(h[q].x, h[q].y), 8 * q, cnt, rows, jbp, c0, zero_row, mode, acc,
                                       prec, 0.f, slo, shi);
        if (8 * q + 4 < cnt)
            gather4rows<RK_STD, Scale>(make_uint2(h[q].z, h[q].w), 8 * q + 4, cnt, rows, jbp, c0, zero_row, mode, acc,
                                       prec, 0.f, slo, shi);
    }
    gather_tail<2, RK_STD, Scale>(reinterpret_cast<const uint2 *>(list), 8 * NH, cnt, rows, jbp, c0, zero_row, mode,
                                  acc, prec, 0.f, slo, shi);
}

// Load the first 8 * NH entries of a list (NH 16-byte words, all in flight).
template <int NH>
__device__ __forceinline__ void load_heads(const uint16_t *list, uint4 *h)
{
    const uint4 *l = reinterpret_cast<const uint4 *>(list);
#pragma unroll
    for (int q = 0; q < NH; ++q) h[q] = l[q];
}

// Step phase A: C(t-1) (unless Cprev is null: the caller keeps it in
// registers) and per-step scratch in LDS, threshold offsets.  theta64 holds
// the workgroup's thresholds (FP64).
template <bool Coherent>
__device__ __forceinline__ void step_begin(const Params &p, const StepLds &S, const uint32_t *Cprev, int tid, int nt)
{
    const int nb_inh = p.has_inh ? p.B : 0, nb_learn = p.learn ? p.B : 0;
    for (int q = tid; q < nb_inh; q += nt) {
        if (Cprev) S.cprev[q] = ld_u<Coherent>(Cprev + q);
        S.cinh[q] = 0u;
    }
    for (int q = tid; q < nb_learn; q += nt) S.colmask[q] = 0u;
    for (int q = tid; q < (p.learn ? p.jb * p.bwords : 0); q += nt) S.spk[q] = 0u;
    if (tid < 32) S.th[tid] = theta_offset(p, S.th64[tid]);
}

// Step phase B for one task: 8 neurons j0+c of sample b (c < nv real).
// acc: column sums of the sample's input spikes over the LDS block (raw,
// before the pending scale, unless scaled: then each weight was multiplied
// by its column's scale before its operand rounding); cp: the sample's
// inhibitory spike count of step t - 1.  Updates the register state, the post traces in LDS, the spike
// masks and the inhibitory count; writes requested outputs.  Returns the
// excitatory spikes as bits 0..7.
template <class PP>
__device__ __forceinline__ uint32_t neuron_task(const PP &p, const StepLds &S, const Outs &o, int k, int b, int c0,
                                                int j0, int nv, const float *acc, uint32_t cp, float *ve, float *vi,
                                                uint32_t *rw, bool scaled = false)
{
    float xp[8];
    if (p.learn) {
        const float4 x0 = *reinterpret_cast<const float4 *>(S.xpost + b * p.ls + c0);
        const float4 x1 = *reinterpret_cast<const float4 *>(S.xpost + b * p.ls + c0 + 4);
        xp[0] = x0.x, xp[1] = x0.y, xp[2] = x0.z, xp[3] = x0.w;
        xp[4] = x1.x, xp[5] = x1.y, xp[6] = x1.z, xp[7] = x1.w;
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) xp[c] = 0.f;
    }
    // padding columns (c >= nv) keep their state and never spike; per-lane
    // conditions are selects, not branches
    uint32_t se_m = 0u, si_m = 0u;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int jl = c0 + c;
        const float I = scaled ? acc[c] : acc[c] * S.scalef[jl];
        NeuronState st{ve[c], vi[c], (rw[c >> 1] >> (16 * (c & 1))) & 0xFFFFu, xp[c]};
        bool se, si;
        neuron_update(p, I, cp, S.th[jl], st, se, si);
        const bool real = c < nv;
        ve[c] = real ? st.ve : ve[c];
        vi[c] = real ? st.vi : vi[c];
        xp[c] = real ? st.xpost : 0.f;
        const uint32_t sh = 16u * (uint32_t)(c & 1);
        rw[c >> 1] = real ? (rw[c >> 1] & ~(0xFFFFu << sh)) | (st.rf << sh) : rw[c >> 1];
        se_m |= (real && se ? 1u : 0u) << c;
        si_m |= (real && si ? 1u : 0u) << c;
    }
    if (p.learn) {
        *reinterpret_cast<float4 *>(S.xpost + b * p.ls + c0) = make_float4(xp[0], xp[1], xp[2], xp[3]);
        *reinterpret_cast<float4 *>(S.xpost + b * p.ls + c0 + 4) = make_float4(xp[4], xp[5], xp[6], xp[7]);
        if (se_m) {
            atomicOr(&S.colmask[b], se_m << c0);
            for (uint32_t m = se_m; m; m &= m - 1u)
                atomicOr(&S.spk[(c0 + __builtin_ctz(m)) * p.bwords + (b >> 5)], 1u << (b & 31));
        }
    }
    if (si_m) atomicAdd(&S.cinh[b], (uint32_t)__builtin_popcount(si_m));
    write_outputs8(p, o, k, b, j0, nv, se_m, si_m, ve, vi);
    return se_m;
}

// After phase B: publish the inhibitory counts, clear the next step's slot
// (workgroup 0), and list the samples with any post spike in this block in
// increasing order (wave 0, ballots).  ulist[B] holds their number.
template <bool Coherent>
__device__ __forceinline__ void step_publish(const Params &p, const StepLds &S, uint32_t *Ccur, uint32_t *Cnext, int g,
                                             int tid, int nt)
{
    for (int q = tid; q < (p.has_inh ? p.B : 0); q += nt) {
        const uint32_t c = S.cinh[q];
        if (c) atomicAdd(&Ccur[q], c);
        if (g == 0 && Cnext) st_x<Coherent>(Cnext + q, 0u);
    }
    if (p.learn && tid < 64) {
        uint32_t base = 0;
        for (int b0 = 0; b0 < p.B; b0 += 64) {
            const int b = b0 + tid;
            const bool hit = b < p.B && S.colmask[b] != 0u;
            const uint64_t m = __ballot(hit);
            if (hit) S.ulist[base + __popcll(m & ((1ull << tid) - 1ull))] = (uint32_t)b;
            base += (uint32_t)__popcll(m);
        }
        if (tid == 0) S.ulist[p.B] = base;
    }
}

// Step phase C for input row i (one thread, all column groups):
//   P[c] = R over listed spiking samples b with neuron c fired of x_pre[b, i]
//   D[c] = R over the samples in input i's spike list of x_post[b, c]
//   w = clamp(float(w * scale[c]) + nu_post * P[c] - nu_pre * D[c])
// The x_pre values of the first XR spiking samples are loaded once into
// registers (all in flight together) and reused by every column group; each
// group walks the sample list for its depression sums.
template <bool Coherent, int XR, int RK = RK_STD>
__device__ __forceinline__ void plasticity_row_cg(const Params &p, const StepLds &S, int i, int cnt, uint4 head,
                                                  const uint16_t *ltrow, const float *xpre, int ucnt, uint32_t colany,
                                                  int prec, int prec_d)
{
    const int ncg = p.jbp >> 3;
    float x[XR];
    uint32_t cm[XR];
#pragma unroll
    for (int v = 0; v < XR; ++v) {
        cm[v] = 0u;
        x[v] = 0.f;
        if (v < ucnt) {
            const int b = (int)S.ulist[v];
            cm[v] = S.colmask[b];
            if (cm[v]) x[v] = red_in<RK>(operand_value(prec, ld_x<Coherent>(xpre + (size_t)b * p.n_in_pad + i)), p.itau2_r);
        }
    }
    for (int cg = 0; cg < ncg; ++cg) {
        const int c0 = 8 * cg;
        float P[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) P[c] = 0.f;
        const uint32_t grp = (colany >> c0) & 0xFFu;
        if (grp) {
            // the spike masks are the same in every lane: scalar branches skip
            // the samples and columns that did not fire
#pragma unroll
            for (int v = 0; v < XR; ++v) {
                const uint32_t m = __builtin_amdgcn_readfirstlane((cm[v] >> c0) & 0xFFu);
                if (m) {
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        if ((m >> c) & 1u) P[c] = reduce2(p.reduce, P[c], x[v]);
                }
            }
            for (int u = XR; u < ucnt; ++u) {
                const int b = (int)S.ulist[u];
                const uint32_t m = (S.colmask[b] >> c0) & 0xFFu;
                if (!m) continue;
                const float xv = red_in<RK>(operand_value(prec, ld_x<Coherent>(xpre + (size_t)b * p.n_in_pad + i)),
                                            p.itau2_r);
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    if ((m >> c) & 1u) P[c] = reduce2(p.reduce, P[c], xv);
            }
        }
        float D[8];
        gather8<RK>(ltrow, cnt, make_uint2(head.x, head.y), make_uint2(head.z, head.w), 8, S.xpost, p.ls, c0, p.B,
                    p.reduce, D, prec_d, p.itau2_r);
        float4 *wr = reinterpret_cast<float4 *>(S.W + i * p.ls + c0);
        const float4 w0 = wr[0], w1 = wr[1];
        float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float xw = w[c] * S.scalef[c0 + c];
            if ((grp >> c) & 1u) xw = xw + p.nu_post * red_out<RK>(p, P[c]);
            const float d = red_out<RK>(p, D[c]);
            w[c] = fminf(fmaxf(xw - p.nu_pre * d, p.w_min), p.w_max);
        }
        wr[0] = make_float4(w[0], w[1], w[2], w[3]);
        wr[1] = make_float4(w[4], w[5], w[6], w[7]);
    }
}

// Plasticity of column groups [cg0, cg0 + ng) of row i (ng <= 2; cg0 the
// same in every lane of the wave): one walk over the input's sample list for
// both groups (the row split over two threads).  The potentiation terms are
// taken 8 listed spiking samples at a time: sample numbers and column masks
// are the same in every lane (scalar branches); the 8 x_pre loads go out
// together, the first 8 before the depression walk, which hides them.
template <bool Coherent, int NH, int RK = RK_STD>
__device__ __forceinline__ void plasticity_row_half(const Params &p, const StepLds &S, int i, int cg0, int ng,
                                                    int cnt, const uint4 *h, const uint16_t *ltrow, const float *xpre,
                                                    int ucnt, uint32_t pdone, int prec, int prec_d)
{
    // pdone: columns whose weights already hold w * scale + potentiation
    // (the matrix-core pass); then ucnt is 0 here
    float P[2][8], D[2][8];
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int c = 0; c < 8; ++c) P[g][c] = 0.f, D[g][c] = 0.f;
    uint32_t m8[8];
    float x8[8];
    // masks of this thread's 16 columns and x_pre values of listed samples
    // u0 .. u0 + 8 (loads only for samples that fired in these columns)
    auto fetch = [&](int u0) {
        uint32_t b8[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int u = u0 + v;
            b8[v] = u < ucnt ? S.ulist[u] : 0u;
            m8[v] = __builtin_amdgcn_readfirstlane(u < ucnt ? (S.colmask[b8[v]] >> (8 * cg0)) & 0xFFFFu : 0u);
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            x8[v] = 0.f;
            if (m8[v]) x8[v] = ld_x<Coherent>(xpre + (size_t)b8[v] * p.n_in_pad + i);
        }
    };
    auto accumulate = [&]() {
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const uint32_t m = m8[v];
            if (m) {
                const float xv = red_in<RK>(operand_value(prec, x8[v]), p.itau2_r);
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    if ((m >> c) & 1u) P[c >> 3][c & 7] = reduce2(p.reduce, P[c >> 3][c & 7], xv);
            }
        }
    };
    if (ucnt > 0) fetch(0);
#pragma unroll
    for (int q = 0; q < 2 * NH; ++q) {
        if (4 * q < cnt) {
            const uint2 e = (q & 1) ? make_uint2(h[q >> 1].z, h[q >> 1].w) : make_uint2(h[q >> 1].x, h[q >> 1].y);
#pragma unroll
            for (int g = 0; g < 2; ++g)
                if (g < ng)
                    gather4rows<RK>(e, 4 * q, cnt, S.xpost, p.ls, 8 * (cg0 + g), p.B, p.reduce, D[g], prec_d,
                                    p.itau2_r);
        }
    }
    // list entries past the head, 8 at a time (two list words loaded
    // together), in list order
    const uint2 *l4 = reinterpret_cast<const uint2 *>(ltrow);
    for (int k0 = 8 * NH; k0 < cnt; k0 += 8) {
        uint2 e[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) e[q] = k0 + 4 * q < cnt ? l4[(k0 >> 2) + q] : make_uint2(0u, 0u);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (k0 + 4 * q >= cnt) break;
#pragma unroll
            for (int g = 0; g < 2; ++g)
                if (g < ng)
                    gather4rows<RK>(e[q], k0 + 4 * q, cnt, S.xpost, p.ls, 8 * (cg0 + g), p.B, p.reduce, D[g],
                                    prec_d, p.itau2_r);
        }
    }
    if (ucnt > 0) {
        accumulate();
        for (int u0 = 8; u0 < ucnt; u0 += 8) {
            fetch(u0);
            accumulate();
        }
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (g >= ng) break;
        const int c0 = 8 * (cg0 + g);
        float4 *wr = reinterpret_cast<float4 *>(S.W + i * p.ls + c0);
        const float4 w0 = wr[0], w1 = wr[1];
        float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float xw = ((pdone >> (c0 + c)) & 1u) ? w[c] : w[c] * S.scalef[c0 + c];
            xw = xw + p.nu_post * red_out<RK>(p, P[g][c]);
            const float d = red_out<RK>(p, D[g][c]);
            w[c] = fminf(fmaxf(xw - p.nu_pre * d, p.w_min), p.w_max);
        }
        wr[0] = make_float4(w[0], w[1], w[2], w[3]);
        wr[1] = make_float4(w[4], w[5], w[6], w[7]);
    }
}

// Potentiation on the matrix cores, for the sum and mean reductions:
//   P[i, c] = sum over the listed spiking samples b of q(x_pre[b, i]) s[b, c]
// as a 32 x 32 tile product per 32 input rows, K = the listed samples in
// chunks of 16 (x_pre operands straight from memory, the FP32 form in three
// exact bfloat16 planes, BF16 / FP8 in one; the spike masks are exact 0 / 1).
// Writes w <- w * scale[c] + nu_post * P[i, c] (P / B for mean) for the fired
// columns (colany); the depression pass then leaves their scale alone.  Its
// cost grows with the number of spiking samples over 16, not with the
// samples times the row items, which keeps blocks whose neurons fire in many
// samples of a step from holding up the others.
// One 32-row tile rt of the potentiation product (one wave; lane = lane index).
// With Pre, x0 holds this lane's x_pre operands of the first 32 listed
// samples, loaded ahead of time (tile_loads); later chunks are loaded here.
template <bool Coherent, bool Pre = false, int RK = RK_STD>
__device__ __forceinline__ void potentiation_tile(const Params &p, const StepLds &S, const float *xpre, int ucnt,
                                                  uint32_t colany, int prec, int rt, int lane,
                                                  const float (*x0)[8] = nullptr)
{
    const int col = lane & 31, kh = lane >> 5;
    const bool fired_col = ((colany >> col) & 1u) != 0u && col < p.jb;
    const int row = rt * 32 + col;  // this lane's A row (the A layout puts row lane % 32)
    f32x16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    // two K chunks (32 listed samples) per pass: 16 loads in flight
    for (int k0 = 0; k0 < ucnt; k0 += 32) {
        float x[2][8];
        uint32_t bits[2] = {0u, 0u};
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int u = k0 + 16 * h + 8 * kh + e;
                const uint32_t b = u < ucnt ? S.ulist[u] : 0u;
                if (Pre && k0 == 0)
                    x[h][e] = x0[h][e];
                else
                    x[h][e] = (u < ucnt && row < p.n_in) ? ld_x<Coherent>(xpre + (size_t)b * p.n_in_pad + row) : 0.f;
                bits[h] |= (u < ucnt ? (S.colmask[b] >> col) & 1u : 0u) << e;
            }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (k0 + 16 * h >= ucnt) break;
            const uint4 bop = ones_bf16(bits[h]);
            uint32_t c0[8], c1[8], c2[8];
            // the soft maximum's summands are FP32 values off the forms' grids:
            // three exact bfloat16 parts in every form
            const bool three = prec == PREC_FP32 || RK == RK_SOFT;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                if (three) {
                    uint32_t c[3];
                    split<PREC_FP32>(red_in<RK>(operand_value(prec, x[h][e]), p.itau2_r), c);
                    c0[e] = c[0], c1[e] = c[1], c2[e] = c[2];
                } else {
                    c0[e] = bf16_code(operand_value(prec, x[h][e]));  // exact: the form's grid fits bfloat16
                    c1[e] = c2[e] = 0u;
                }
            }
            const uint4 a0 = make_uint4(c0[0] | (c0[1] << 16), c0[2] | (c0[3] << 16), c0[4] | (c0[5] << 16),
                                        c0[6] | (c0[7] << 16));
            acc = mfma<PREC_BF16>(a0, bop, acc);
            if (three) {
                const uint4 a1 = make_uint4(c1[0] | (c1[1] << 16), c1[2] | (c1[3] << 16),
                                            c1[4] | (c1[5] << 16), c1[6] | (c1[7] << 16));
                const uint4 a2 = make_uint4(c2[0] | (c2[1] << 16), c2[2] | (c2[3] << 16),
                                            c2[4] | (c2[5] << 16), c2[6] | (c2[7] << 16));
                acc = mfma<PREC_BF16>(a1, bop, acc);
                acc = mfma<PREC_BF16>(a2, bop, acc);
            }
        }
    }
    // accumulator r: row 8 (r / 4) + 4 kh + r % 4 of the tile, column col
    if (fired_col) {
        const float sc = S.scalef[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = rt * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
            if (i < p.n_in) {
                float *w = S.W + i * p.ls + col;
                *w = *w * sc + p.nu_post * red_out<RK>(p, acc[r]);
            }
        }
    }
}

// w <- w * scale + nu_post * P for the fired column of this lane in tile rt
// (accumulator r: row 8 (r / 4) + 4 (lane / 32) + r % 4 of the tile).
template <int RK = RK_STD>
__device__ __forceinline__ void potentiation_write(const Params &p, const StepLds &S, const f32x16_t &acc, int rt,
                                                   int lane, bool fired_col)
{
    const int col = lane & 31, kh = lane >> 5;
    if (!fired_col) return;
    const float sc = S.scalef[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = rt * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        if (i < p.n_in) {
            float *w = S.W + i * p.ls + col;
            *w = *w * sc + p.nu_post * red_out<RK>(p, acc[r]);
        }
    }
}

// The potentiation pass of all tiles (sum and mean), software-pipelined per
// wave, on the FP32 matrix instruction (v_mfma_f32_32x32x2_f32: operand A
// lane l = row l % 32 of the tile, K element l / 32; B lane l = column
// l % 32, K element l / 32; the accumulator layout of the other 32 x 32
// forms).  The x_pre operands enter as FP32 values (rounded first in the
// BF16 / FP8 forms), the spikes as exact 0 / 1, so every product is exact and
// the sums accumulate in FP32.  Work items are (tile, chunk of 16 listed
// samples) in order; the x_pre operands of the next item are loaded before
// the current item's matrix products, so a tile's global-memory latency
// overlaps the previous one's work.  Lane l takes the listed samples of
// parity l / 32 of a chunk (8 per chunk); the samples of the first chunk
// and their spike bits at the lane's column are read from LDS once.
template <bool Coherent, int RK = RK_STD>
__device__ __forceinline__ void potentiation_pipe(const Params &p, const StepLds &S, const float *xpre, int ucnt,
                                                  uint32_t colany, int prec, int tid, int nt)
{
    const int lane = tid & 63, col = lane & 31, kh = lane >> 5;
    const int nrt = (p.n_in + 31) >> 5, nw = nt >> 6;
    int rt = tid >> 6;
    if (rt >= nrt || ucnt <= 0) return;
    const bool fired_col = ((colany >> col) & 1u) != 0u && col < p.jb;
    const int nch = (ucnt + 15) >> 4;
    // listed sample u = 16 c + 2 j + kh of chunk c, j < 8: its x_pre row
    // offset (0xFFFFFFFF past the list) and, in bit j, its spike at `col`
    auto samples = [&](int c, uint32_t (&off)[8], uint32_t &bits) {
        bits = 0u;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int u = 16 * c + 2 * j + kh;
            const uint32_t b = u < ucnt ? S.ulist[u] : 0u;
            off[j] = u < ucnt ? b * (uint32_t)p.n_in_pad : 0xFFFFFFFFu;
            bits |= (u < ucnt ? (S.colmask[b] >> col) & 1u : 0u) << j;
        }
    };
    // eight loads at valid addresses whatever the lanes' samples, so that
    // the loop body issues a fixed number of loads and the next item's stay
    // in flight during this one's products.  No select follows them: a
    // sample past the list has spike bit 0 (its x_pre, a finite trace value
    // of some sample, times 0 adds nothing), and rows past n_in are never
    // written back.
    auto load = [&](int t, const uint32_t (&off)[8], float (&x)[8]) {
        const int row = t * 32 + col;
        const bool rok = row < p.n_in;
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = ld_x<Coherent>(xpre + (off[j] != 0xFFFFFFFFu && rok ? off[j] + row : 0u));
    };
    uint32_t off0[8], bits0;
    samples(0, off0, bits0);
    float xa[8], xb[8];
    load(rt, off0, xa);
    uint32_t bits = bits0;
    f32x16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    int c = 0;
    // one item: the next item's loads into nxt, then the products of cur;
    // returns false after the last item (the loop alternates the two
    // buffers, so no copy waits for loads in flight)
    auto item = [&](const float (&cur)[8], float (&nxt)[8]) {
        int rn = rt, cn = c + 1;
        if (cn == nch) {
            cn = 0;
            rn = rt + nw;
        }
        const bool more = rn < nrt;
        // the next item's samples (chunk 0's are kept) and x_pre operands;
        // after the last item the current tile is loaded again, unused
        uint32_t offn[8], bitsn = bits0;
#pragma unroll
        for (int j = 0; j < 8; ++j) offn[j] = off0[j];
        if (cn > 0) samples(cn, offn, bitsn);
        load(more ? rn : rt, offn, nxt);
        // K pairs (2 j, 2 j + 1) holding listed samples of this chunk
        const int npair = min(8, (ucnt - 16 * c + 1) >> 1);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (j >= npair) break;
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(red_in<RK>(operand_value(prec, cur[j]), p.itau2_r),
                                                       (bits >> j) & 1u ? 1.f : 0.f, acc, 0, 0, 0);
        }
        if (cn == 0 || !more) {
            potentiation_write<RK>(p, S, acc, rt, lane, fired_col);
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] = 0.f;
        }
        bits = bitsn;
        rt = rn;
        c = cn;
        return more;
    };
    while (item(xa, xb) && item(xb, xa)) {
    }
}

template <bool Coherent, int RK = RK_STD>
__device__ __forceinline__ void potentiation_mfma(const Params &p, const StepLds &S, const float *xpre, int ucnt,
                                                  uint32_t colany, int prec, int tid, int nt)
{
    const int nrt = (p.n_in + 31) >> 5;
    for (int rt = tid >> 6; rt < nrt; rt += nt >> 6)
        potentiation_tile<Coherent, false, RK>(p, S, xpre, ucnt, colany, prec, rt, tid & 63);
}

// The loads one 32-row tile's depression items start from (lane l: row
// rt * 32 + l % 32): the row's sample list length and first 8 * NH entries.
// plasticity_tiles issues them one tile ahead.
template <int NH>
struct TileLoads {
    uint32_t cnt;
    uint4 h[NH];
};

template <int NH>
__device__ __forceinline__ void tile_loads(const Params &p, const uint16_t *lt, const uint32_t *ct, int rt, int lane,
                                           bool item, TileLoads<NH> &T)
{
    const int row = rt * 32 + (lane & 31);
    T.cnt = 0u;
#pragma unroll
    for (int q = 0; q < NH; ++q) T.h[q] = make_uint4(0u, 0u, 0u, 0u);
    if (item) {
        T.cnt = ct[row];
        load_heads<NH>(lt + (size_t)row * p.lt_stride, T.h);
    }
}

// Phase C for sum and mean, blocks of two or more column groups: per 32-row
// tile one wave takes the potentiation tile product and then the depression
// items of the same rows (lane l: row l % 32, column groups 2 (l / 32) and
// 2 (l / 32) + 1), so the two need no workgroup barrier between them.  The
// next tile's list loads (tile_loads) are issued before the current tile's
// work (Pipe; otherwise after it), so their latency overlaps the current
// tile's potentiation (whose own x_pre loads go out at its start) and
// depression.
template <bool Coherent, int NH, bool Pipe, int RK = RK_STD>
__device__ __forceinline__ void plasticity_tiles(const Params &p, const StepLds &S, const uint16_t *lt,
                                                 const uint32_t *ct, const float *xpre, int ucnt, uint32_t colany,
                                                 int tid, int nt, int prec, int prec_d)
{
    const int ncg = p.jbp >> 3;
    const int lane = tid & 63, nrt = (p.n_in + 31) >> 5, nw = nt >> 6;
    const int hf = lane >> 5, cg0 = 2 * hf, ng = min(2, ncg - cg0);
    int rt = tid >> 6;
    if (rt >= nrt) return;
    TileLoads<NH> cur, nxt;
    tile_loads<NH>(p, lt, ct, rt, lane, rt * 32 + (lane & 31) < p.n_in && ng > 0, cur);
    for (; rt < nrt; rt += nw) {
        const int i = rt * 32 + (lane & 31);
        const bool item = i < p.n_in && ng > 0;
        const int rn = rt + nw;
        if (Pipe && rn < nrt) tile_loads<NH>(p, lt, ct, rn, lane, rn * 32 + (lane & 31) < p.n_in && ng > 0, nxt);
        if (ucnt > 0) {
            potentiation_tile<Coherent, false, RK>(p, S, xpre, ucnt, colany, prec, rt, lane);
            // the tile's weights, written by other lanes of this wave
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (item)
            plasticity_row_half<Coherent, NH, RK>(p, S, i, cg0, ng, (int)cur.cnt, cur.h,
                                                  lt + (size_t)i * p.lt_stride, xpre, 0, colany, prec, prec_d);
        if (Pipe)
            cur = nxt;
        else if (rn < nrt)
            tile_loads<NH>(p, lt, ct, rn, lane, rn * 32 + (lane & 31) < p.n_in && ng > 0, cur);
    }
}

// Rank of the input row of row item q (column-group half (q / 64) % 2): the
// 64-row blocks of the step's input order (rows by decreasing sample-list
// length) go to consecutive 128-item groups, in reverse order within every
// other full set of four groups, so that the workgroup's waves (one group
// per wave pair in a 512-thread workgroup) each get a mix of long and short
// lists; a bijection on the items of nrow rows.
__device__ __forceinline__ int item_rank(int q, int nrow)
{
    const int g = q >> 7, s4 = g >> 2;
    const bool full = 4 * s4 + 3 < (nrow >> 6);
    const int blk = (full && (s4 & 1)) ? 4 * s4 + 3 - (g & 3) : g;
    return (blk << 6) | (q & 63);
}

// Phase C for the signed maximum, row i, column groups [cg0, cg0 + ng):
// per synapse the largest per-sample change
//   M[i, c] = max over b of nu_post q(x_pre[b, i]) s_post[b, c]
//                           - nu_pre q(x_post[b, c]) s_pre[b, i],
// 0 for a sample with neither spike, then w <- clamp(w * scale[c] + M[i, c]).
// The samples fall in three sets: those whose neuron c fired (among the
// listed samples; their terms are taken one by one, with the pre spike bit
// of (b, i)), those in which only input i fired (depression-only terms, never
// positive when nu_pre >= 0), and the rest, which give the zero term unless
// the first two sets cover the batch.  Input i's sample list is walked only
// when they might (its length plus the listed samples reach B) or when a
// depression-only term can be positive (nu_pre < 0); otherwise the zero term
// stands for all of them.  The listed samples and their column masks are
// the same in every lane (cg0 is uniform per wave): scalar branches.
template <bool Coherent>
__device__ __forceinline__ void plasticity_signed_row(const Params &p, const StepLds &S, int i, int cg0, int ng,
                                                      int cnt, const uint16_t *ltrow, const uint32_t *bits_t,
                                                      const float *xpre, int ucnt, int prec, int prec_d)
{
    float M[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) M[c] = -INFINITY;
    const uint32_t *brow = bits_t + (i >> 5);
    const uint32_t ib = 1u << (i & 31);
    for (int u0 = 0; u0 < ucnt; u0 += 8) {
        uint32_t b8[8], m8[8], w8[8];
        float x8[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const int u = u0 + v;
            b8[v] = u < ucnt ? S.ulist[u] : 0u;
            m8[v] = __builtin_amdgcn_readfirstlane(u < ucnt ? (S.colmask[b8[v]] >> (8 * cg0)) & 0xFFFFu : 0u);
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            x8[v] = 0.f;
            w8[v] = 0u;
            if (m8[v]) {
                x8[v] = ld_x<Coherent>(xpre + (size_t)b8[v] * p.n_in_pad + i);
                w8[v] = brow[(size_t)b8[v] * p.in_words];
            }
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const uint32_t m = m8[v];
            if (!m) continue;
            const float pot = p.nu_post * operand_value(prec, x8[v]);
            const bool pre = (w8[v] & ib) != 0u;
            const float *xq = S.xpost + b8[v] * p.ls + 8 * cg0;
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if ((m >> c) & 1u) M[c] = fmaxf(M[c], pre ? pot - p.nu_pre * operand_value(prec_d, xq[c]) : pot);
        }
    }
    const bool walk = cnt + ucnt >= p.B || (p.nu_pre < 0.f && cnt > 0);
    if (walk) {
        // per column: the samples with a spike at input i or neuron col, and
        // the depression-only terms, exactly (rare: a loop, not unrolled)
        for (int c = 0; c < 8 * ng; ++c) {
            const int col = 8 * cg0 + c;
            const uint32_t *sp = S.spk + col * p.bwords;
            int both = 0, qc = 0;
            for (int w = 0; w < p.bwords; ++w) qc += __builtin_popcount(sp[w]);
            float dn = -INFINITY;
            for (int k = 0; k < cnt; ++k) {
                const int b = ltrow[k];
                if ((sp[b >> 5] >> (b & 31)) & 1u)
                    ++both;
                else
                    dn = fmaxf(dn, -p.nu_pre * operand_value(prec_d, S.xpost[b * p.ls + col]));
            }
            const float z = cnt + qc - both < p.B ? fmaxf(dn, 0.f) : dn;
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                if (cc == c) M[cc] = fmaxf(M[cc], z);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 16; ++c) M[c] = fmaxf(M[c], 0.f);
    }
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        if (g >= ng) break;
        const int c0 = 8 * (cg0 + g);
        float4 *wr = reinterpret_cast<float4 *>(S.W + i * p.ls + c0);
        const float4 w0 = wr[0], w1 = wr[1];
        float w[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) w[c] = fminf(fmaxf(w[c] * S.scalef[c0 + c] + M[8 * g + c], p.w_min), p.w_max);
        wr[0] = make_float4(w[0], w[1], w[2], w[3]);
        wr[1] = make_float4(w[4], w[5], w[6], w[7]);
    }
}

// Phase C for the signed maximum over all input rows of the block.  Item q:
// row 64 (q / 128) + q % 64 and column groups 2 ((q / 64) % 2) and the next,
// for blocks of more than two groups (nt a multiple of 128, so the groups
// are uniform per wave); row q and groups 0, 1 otherwise.  bits_t: the
// step's input spikes per sample.
template <bool Coherent>
__device__ __forceinline__ void plasticity_signed(const Params &p, const StepLds &S, const uint16_t *lt,
                                                  const uint32_t *ct, const uint32_t *bits_t, const float *xpre,
                                                  int tid, int nt, int prec, int prec_d)
{
    const int ucnt = (int)S.ulist[p.B];
    const int ncg = p.jbp >> 3;
    const int npair = ncg > 2 ? 2 : 1;
    const int nrow = (p.n_in + 63) & ~63;
    for (int q = tid; q < npair * nrow; q += nt) {
        const int hf = npair == 2 ? (q >> 6) & 1 : 0;
        const int i = npair == 2 ? ((q >> 7) << 6) | (q & 63) : q;
        if (i >= p.n_in) continue;
        const int cg0 = 2 * hf;
        plasticity_signed_row<Coherent>(p, S, i, cg0, min(2, ncg - cg0), (int)ct[i], lt + (size_t)i * p.lt_stride,
                                        bits_t, xpre, ucnt, prec, prec_d);
    }
}

// Phase C over all input rows of the block: split rows (Halves, blocks of
// two or more column groups) or whole rows per thread; a thread loads its
// next row's list head before working on the current row.  Rows are taken in
// the order `ord` (inputs by decreasing sample-list length), so the lanes of
// a wave walk lists of similar length.
template <bool Coherent, int XR, bool Halves, int NH = kListHead, bool Interleave = true, bool Pipe = false,
          int RK = RK_STD>
__device__ __forceinline__ void plasticity_all(const Params &p, const StepLds &S, const uint16_t *lt,
                                               const uint32_t *ct, const uint16_t *ord, const float *xpre, int tid,
                                               int nt, int prec, int prec_d, const uint32_t *bits_t)
{
    if constexpr (RK == RK_SIGNED) {
        plasticity_signed<Coherent>(p, S, lt, ct, bits_t, xpre, tid, nt, prec, prec_d);
        return;
    }
    const int ucnt = (int)S.ulist[p.B];
    const int ncg = p.jbp >> 3;
    if (Interleave && Halves && ncg >= 2 && p.reduce != RED_MAX) {
        uint32_t colany = 0u;
        for (int u = 0; u < ucnt; ++u) colany |= S.colmask[S.ulist[u]];
        colany = __builtin_amdgcn_readfirstlane(colany);
        plasticity_tiles<Coherent, NH, Pipe, RK>(p, S, lt, ct, xpre, ucnt, colany, tid, nt, prec, prec_d);
        return;
    }
    if (Halves && ncg >= 2) {
        uint32_t pdone = 0u;
        int ucnt_items = ucnt;
        // many spiking samples: potentiation on the matrix cores first (few:
        // in the row items, no extra pass)
        if (p.reduce != RED_MAX && ucnt > kMfmaPotentiation) {
            uint32_t colany = 0u;
            for (int u = 0; u < ucnt; ++u) colany |= S.colmask[S.ulist[u]];
            colany = __builtin_amdgcn_readfirstlane(colany);
            if (Pipe)
                potentiation_pipe<Coherent, RK>(p, S, xpre, ucnt, colany, prec, tid, nt);
            else
                potentiation_mfma<Coherent, RK>(p, S, xpre, ucnt, colany, prec, tid, nt);
            __syncthreads();
            pdone = colany;
            ucnt_items = 0;
        }
        // item q: row ord[item_rank(q)], column groups 2 hf and 2 hf + 1 with
        // hf = (q / 64) % 2, the same in every lane of a wave (nt is a
        // multiple of 128)
        const int nrow = (p.n_in + 63) & ~63;
        if (Pipe && ucnt_items == 0) {
            // the next item's row, list length and list head are loaded
            // before the current item's walk
            auto fetch = [&](int q, int &i, TileLoads<NH> &T) {
                const int hf = (q >> 6) & 1;
                const int r = item_rank(q, nrow);
                const bool ok = q < 2 * nrow && r < p.n_in && min(2, ncg - 2 * hf) > 0;
                i = ok ? (int)ord[r] : -1;
                T.cnt = 0u;
#pragma unroll
                for (int w = 0; w < NH; ++w) T.h[w] = make_uint4(0u, 0u, 0u, 0u);
                if (ok) {
                    T.cnt = ct[i];
                    load_heads<NH>(lt + (size_t)i * p.lt_stride, T.h);
                }
            };
            TileLoads<NH> cur, nxt;
            int i_cur, i_nxt;
            fetch(tid, i_cur, cur);
            for (int q = tid; q < 2 * nrow; q += nt) {
                const bool more = q + nt < 2 * nrow;
                if (more) fetch(q + nt, i_nxt, nxt);
                if (i_cur >= 0) {
                    const int cg0 = 2 * ((q >> 6) & 1);
                    plasticity_row_half<Coherent, NH, RK>(p, S, i_cur, cg0, min(2, ncg - cg0), (int)cur.cnt, cur.h,
                                                      lt + (size_t)i_cur * p.lt_stride, xpre, 0, pdone, prec,
                                                      prec_d);
                }
                if (!more) break;
                cur = nxt;
                i_cur = i_nxt;
            }
            return;
        }
        for (int q = tid; q < 2 * nrow; q += nt) {
            const int hf = (q >> 6) & 1;
            const int r = item_rank(q, nrow);
            const int cg0 = 2 * hf;
            const int ng = min(2, ncg - cg0);
            if (r >= p.n_in || ng <= 0) continue;
            const int i = ord[r];
            const uint32_t cnt = ct[i];
            uint4 h[NH];
            load_heads<NH>(lt + (size_t)i * p.lt_stride, h);
            plasticity_row_half<Coherent, NH, RK>(p, S, i, cg0, ng, (int)cnt, h, lt + (size_t)i * p.lt_stride, xpre,
                                              ucnt_items, pdone, prec, prec_d);
        }
        return;
    }
    uint32_t colany = 0u;
    for (int u = 0; u < ucnt; ++u) colany |= S.colmask[S.ulist[u]];
    int r = tid;
    uint32_t cnt_n = 0u;
    uint4 head_n = make_uint4(0u, 0u, 0u, 0u);
    int i_n = 0;
    if (r < p.n_in) {
        i_n = ord[r];
        cnt_n = ct[i_n];
        head_n = *reinterpret_cast<const uint4 *>(lt + (size_t)i_n * p.lt_stride);
    }
    while (r < p.n_in) {
        const int i = i_n;
        const uint32_t cnt = cnt_n;
        const uint4 head = head_n;
        const int rn = r + nt;
        if (rn < p.n_in) {
            i_n = ord[rn];
            cnt_n = ct[i_n];
            head_n = *reinterpret_cast<const uint4 *>(lt + (size_t)i_n * p.lt_stride);
        }
        plasticity_row_cg<Coherent, XR, RK>(p, S, i, (int)cnt, head, lt + (size_t)i * p.lt_stride, xpre, ucnt, colany,
                                        prec, prec_d);
        r = rn;
    }
}

// Phase C3: FP64 column sums of the updated block, the pending
// normalisation scale (norm / column sum; 1 when norm is 0, as on the steps
// before the last of a run under per-run normalisation), the threshold
// update.  Two workgroup barriers.  Both sums issue four LDS loads before
// their additions (a loop of one load and one dependent add per row would
// pay the LDS latency on every row); the order of the additions is the
// row order either way.
template <int RK = RK_STD>
__device__ __forceinline__ void colsums_theta(const Params &p, const StepLds &S, double norm, int tid, int nt)
{
    const int jj = tid & 31, rg = tid >> 5, nrg = nt >> 5;
    double cs = 0.0;
    if (jj < p.jb) {
        int i = rg;
        for (; i + 3 * nrg < p.n_in; i += 4 * nrg) {
            const float w0 = S.W[i * p.ls + jj], w1 = S.W[(i + nrg) * p.ls + jj];
            const float w2 = S.W[(i + 2 * nrg) * p.ls + jj], w3 = S.W[(i + 3 * nrg) * p.ls + jj];
            cs += (double)w0;
            cs += (double)w1;
            cs += (double)w2;
            cs += (double)w3;
        }
        for (; i < p.n_in; i += nrg) cs += (double)S.W[i * p.ls + jj];
    }
    S.part[rg * 32 + jj] = cs;
    __syncthreads();
    if (tid < 32) {
        double c = 0.0;
        int r = 0;
        for (; r + 3 < nrg; r += 4) {
            const double q0 = S.part[r * 32 + tid], q1 = S.part[(r + 1) * 32 + tid];
            const double q2 = S.part[(r + 2) * 32 + tid], q3 = S.part[(r + 3) * 32 + tid];
            c += q0;
            c += q1;
            c += q2;
            c += q3;
        }
        for (; r < nrg; ++r) c += S.part[r * 32 + tid];
        S.scale[tid] = (norm > 0.0 && c > 0.0 && tid < p.jb) ? norm / c : 1.0;
        S.scalef[tid] = (float)S.scale[tid];
        if (p.adaptive && tid < p.jb) {
            int cnt = 0;
            for (int bw = 0; bw < p.bwords; ++bw) cnt += __builtin_popcount(S.spk[tid * p.bwords + bw]);
            S.th64[tid] = theta_step<RK>(p, S.th64[tid], cnt);
        }
    }
    __syncthreads();
}

// Phase E: x_pre(t+1) for this workgroup's share of the samples.
template <bool Coherent>
__device__ __forceinline__ void xpre_next(const Params &p, const uint32_t *bits_next, const float *xpre, float *xn_all,
                                          int g, int ng, int tid, int nt)
{
    for (int b = g; b < p.B; b += ng) {
        const uint32_t *sb = bits_next + (size_t)b * p.in_words;
        const float *xc = xpre + (size_t)b * p.n_in_pad;
        float *xn = xn_all + (size_t)b * p.n_in_pad;
        for (int i = tid; i < p.n_in_pad; i += nt)
            st_x<Coherent>(xn + i, trace_step(ld_x<Coherent>(xc + i), p.lam_pre, (sb[i >> 5] >> (i & 31)) & 1u,
                                              p.trace_add));
    }
}

// The workgroup's share of x_pre: samples g, g + ng, ... (the samples whose
// next-step traces xpre_next writes), as one flat range f of
// own_samples * n_in_pad entries (sample g + (f / n_in_pad) * ng, input
// f % n_in_pad).  Entry f = tid + j * nt (j < XC) of that range is kept in
// register xc[j] across the steps of a persistent launch.
__device__ __forceinline__ int own_entries(const Params &p, int g, int ng)
{
    return g < p.B ? ((p.B - 1 - g) / ng + 1) * p.n_in_pad : 0;
}

__device__ __forceinline__ size_t own_offset(const Params &p, int f, int g, int ng, int &i)
{
    const int sq = f / p.n_in_pad;
    i = f - sq * p.n_in_pad;
    return (size_t)(g + sq * ng) * p.n_in_pad + i;
}

// Fill the register copy from x_pre(t) (buffer xpre).
template <int XC>
__device__ __forceinline__ void xpre_own_load(const Params &p, const float *xpre, float *xc, int g, int ng, int tid,
                                              int nt)
{
    const int total = own_entries(p, g, ng);
#pragma unroll
    for (int j = 0; j < XC; ++j) {
        const int f = tid + j * nt;
        int i;
        xc[j] = f < total ? ld_x<true>(xpre + own_offset(p, f, g, ng, i)) : 0.f;
    }
}

// Phase E of the persistent kernel: x_pre(t+1) of the workgroup's share from
// the register copy of x_pre(t) (entries past XC * nt from xpre), written to
// xn_all for the other workgroups; the register copy becomes x_pre(t+1).
template <int XC>
__device__ __forceinline__ void xpre_next_own(const Params &p, const uint32_t *bits_next, const float *xpre,
                                              float *xn_all, float *xc, int g, int ng, int tid, int nt)
{
    const int total = own_entries(p, g, ng);
#pragma unroll
    for (int j = 0; j < XC; ++j) {
        const int f = tid + j * nt;
        if (f < total) {
            int i;
            const size_t o = own_offset(p, f, g, ng, i);
            const size_t b = o / (size_t)p.n_in_pad;
            const uint32_t bit = (bits_next[b * p.in_words + (i >> 5)] >> (i & 31)) & 1u;
            xc[j] = trace_step(xc[j], p.lam_pre, bit, p.trace_add);
            st_x<true>(xn_all + o, xc[j]);
        }
    }
    for (int f = tid + XC * nt; f < total; f += nt) {
        int i;
        const size_t o = own_offset(p, f, g, ng, i);
        const size_t b = o / (size_t)p.n_in_pad;
        const uint32_t bit = (bits_next[b * p.in_words + (i >> 5)] >> (i & 31)) & 1u;
        st_x<true>(xn_all + o, trace_step(ld_x<true>(xpre + o), p.lam_pre, bit, p.trace_add));
    }
}

// Prologue of both kernels: weight block (row-padded, zero row), thresholds,
// pending scale 1.
__device__ __forceinline__ void load_block(const Params &p, const StepLds &S, const float *Wg, const double *theta,
                                           int g, int tid, int nt)
{
    const int JB = p.jb, JBP = p.jbp, LS = p.ls;
    const int jj = tid & 31, rg = tid >> 5, nrg = nt >> 5;
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
            S.W[i * LS + jj] = v0;
            S.W[(i + nrg) * LS + jj] = v1;
            S.W[(i + 2 * nrg) * LS + jj] = v2;
            S.W[(i + 3 * nrg) * LS + jj] = v3;
        }
        for (; i < p.n_in_pad; i += nrg) S.W[i * LS + jj] = jj < JB ? Wg[(size_t)i * JB + jj] : 0.f;
        if (rg == 0) {
            S.W[p.n_in_pad * LS + jj] = 0.f;
            if (p.learn) S.xpost[p.B * LS + jj] = 0.f;
        }
    }
    if (tid < 32) {
        const int jt = g * JB + tid;
        S.th64[tid] = (tid < JB && jt < p.n_exc) ? theta[jt] : 0.0;
        S.scale[tid] = 1.0;
        S.scalef[tid] = 1.f;
    }
}

// Epilogue of a learning launch: the block, normalised, and the thresholds.
__device__ __forceinline__ void store_block(const Params &p, const StepLds &S, float *Wg, double *theta, int g,
                                            int tid, int nt)
{
    const int JB = p.jb, LS = p.ls;
    const int jj = tid & 31, rg = tid >> 5, nrg = nt >> 5;
    if (jj < JB) {
        const double sc = S.scale[jj];
        for (int i = rg; i < p.n_in_pad; i += nrg) {
            float w = S.W[i * LS + jj];
            if (i < p.n_in) w = (float)((double)w * sc);
            Wg[(size_t)i * JB + jj] = w;
        }
    }
    if (tid < JB && g * JB + tid < p.n_exc) theta[g * JB + tid] = S.th64[tid];
}

// State of the 8 neurons of task (b, c0): voltages, packed refractory words,
// post traces (into LDS), from / to the HBM arrays.
__device__ __forceinline__ void load_task_state(const Params &p, const StepLds &S, const FusedArgs &a, size_t n0, int b,
                                                int c0, float *ve, float *vi, uint32_t *rw)
{
    const float4 e0 = *reinterpret_cast<const float4 *>(a.v_exc + n0);
    const float4 e1 = *reinterpret_cast<const float4 *>(a.v_exc + n0 + 4);
    ve[0] = e0.x, ve[1] = e0.y, ve[2] = e0.z, ve[3] = e0.w, ve[4] = e1.x, ve[5] = e1.y, ve[6] = e1.z, ve[7] = e1.w;
    if (p.has_inh) {
        const float4 i0 = *reinterpret_cast<const float4 *>(a.v_inh + n0);
        const float4 i1 = *reinterpret_cast<const float4 *>(a.v_inh + n0 + 4);
        vi[0] = i0.x, vi[1] = i0.y, vi[2] = i0.z, vi[3] = i0.w, vi[4] = i1.x, vi[5] = i1.y, vi[6] = i1.z, vi[7] = i1.w;
    } else {
#pragma unroll
        for (int c = 0; c < 8; ++c) vi[c] = 0.f;
    }
    if (p.learn) {
        *reinterpret_cast<float4 *>(S.xpost + b * p.ls + c0) = *reinterpret_cast<const float4 *>(a.x_post + n0);
        *reinterpret_cast<float4 *>(S.xpost + b * p.ls + c0 + 4) =
            *reinterpret_cast<const float4 *>(a.x_post + n0 + 4);
    }
    const uint4 r = *reinterpret_cast<const uint4 *>(a.rf + n0);
    rw[0] = r.x, rw[1] = r.y, rw[2] = r.z, rw[3] = r.w;
}

__device__ __forceinline__ void store_task_state(const Params &p, const StepLds &S, const FusedArgs &a, size_t n0,
                                                 int b, int c0, const float *ve, const float *vi, const uint32_t *rw)
{
    *reinterpret_cast<float4 *>(a.v_exc + n0) = make_float4(ve[0], ve[1], ve[2], ve[3]);
    *reinterpret_cast<float4 *>(a.v_exc + n0 + 4) = make_float4(ve[4], ve[5], ve[6], ve[7]);
    if (p.has_inh) {
        *reinterpret_cast<float4 *>(a.v_inh + n0) = make_float4(vi[0], vi[1], vi[2], vi[3]);
        *reinterpret_cast<float4 *>(a.v_inh + n0 + 4) = make_float4(vi[4], vi[5], vi[6], vi[7]);
    }
    if (p.learn) {
        *reinterpret_cast<float4 *>(a.x_post + n0) = *reinterpret_cast<const float4 *>(S.xpost + b * p.ls + c0);
        *reinterpret_cast<float4 *>(a.x_post + n0 + 4) =
            *reinterpret_cast<const float4 *>(S.xpost + b * p.ls + c0 + 4);
    }
    *reinterpret_cast<uint4 *>(a.rf + n0) = make_uint4(rw[0], rw[1], rw[2], rw[3]);
}

}  // namespace snn
