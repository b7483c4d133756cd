// snn_dev.h -- shared definitions of the gfx950 kernels and the host runtime.
//
// Data layout in HBM (one network, batch B):
//   columns j are grouped in blocks of JB consecutive post-synaptic neurons,
//   g = j / JB, jj = j % JB; every per-neuron array and the weight matrix are
//   block-major, so one column block (the unit a fused or plasticity
//   workgroup owns) is one contiguous span:
//     state(b, j)  at (g * Bs + b) * JBP + jj      (v_exc, v_inh, x_post, rf)
//                  (JBP = JB rounded up to 8: 32-byte aligned 8-neuron groups)
//     W(i, j)      at (g * n_in_pad + i) * JB + jj (FP32 master)
//   inputs are padded to n_in_pad = 32 * in_words; pad inputs never spike
//   and their weights stay 0.
//   input spikes of step t: bits[t * bits_stride + b * in_words + w] (bit
//   i % 32 of word i / 32) and the transpose bitsT[t][i][bw] (bit b % 32 of
//   word b / 32).
//   presynaptic traces x_pre[t % 3][b][i] (buffer stride Bs rows);
//   inhibitory spike counts per sample C[t % 3][b] (slot stride Bs).
#pragma once
#include <stdint.h>

namespace snn {

struct LifP {
    float v_rest, v_reset, v_th, alpha;  // alpha = exp(-dt / tau), rounded to f32
    int refrac;                          // refractory steps (<= 127)
};

struct Params {
    int n_in, n_in_pad, in_words;
    int n_exc, n_pad, jb, nblk;
    int jbp;                  // jb rounded up to a multiple of 8 (state rows)
    int ls;                   // LDS row stride of a column block (jbp, + 4 at 16 / 32)
    int lt_stride;            // entries per per-input sample list (B rounded to 8)
    int has_inh;
    int B, bwords;            // batch, ceil(B / 32)
    int Bs;                   // sample stride of the per-neuron state arrays
                              // (allocated capacity; B <= Bs may vary)
    int bits_stride;          // words per step of the per-sample input spikes
                              // (B * in_words rounded up to 4: 16-byte rows)
    int learn, adaptive, trace_add, reduce;
    int prec;                 // operand form of the contractions (Prec)
    int uniform_rate;
    uint32_t thr_uniform;
    LifP exc, inh;
    float w_ei, w_ie;
    float lam_pre, lam_post, nu_pre, nu_post, w_min, w_max;
    float inv_B;
    float itau2_r, tau_ln2_r; // soft-maximum reduction: log2(e) / temperature, temperature * ln(2)
    double norm, beta, theta_plus, inv_Bd;
    uint64_t seed;
};

// Per-neuron packed flags (u16): low byte excitatory, high byte inhibitory;
// in each byte bits 0..6 hold the refractory count, bit 7 the spike of the
// previous step.
constexpr uint32_t RF_SPIKE = 0x80u;
constexpr uint32_t RF_COUNT = 0x7Fu;

// Output pointers of one run (device; nullptr = not recorded).
struct Outs {
    uint32_t *counts;      // B x n_exc
    uint32_t *raster_in;   // T x B x in_words
    uint32_t *raster_exc;  // T x B x exc_words
    uint32_t *raster_inh;  // T x B x exc_words
    float *v_exc;          // T x B x n_exc
    float *v_inh;          // T x B x n_exc
    const uint32_t *until; // B: spikes of sample b are counted at call step k
                           // only while k < until[b] (serving; nullptr: always)
};

// Serving: the per-slot arrays a slot move carries besides the network state.
struct SlotArrays {
    uint8_t *img;           // slots x n_in
    uint64_t *ids;
    uint32_t *tl, *counts;  // local step; slots x n_exc spike counts
};

enum Reduce { RED_SUM = 0, RED_MEAN = 1, RED_MAX = 2, RED_MAX_SIGNED = 3, RED_SOFT = 4 };

// Reduction kind a plasticity kernel is compiled for: sum, mean and max
// (chosen at run time from Params::reduce), the soft maximum (the traces
// enter as exp(x / tau) - 1, the reduced sums leave through tau log1p(S / B)),
// or the signed maximum of the per-sample changes.  RK_SERVE: a frozen
// network with per-slot count limits (Outs::until), the serving loop's
// launches; no plasticity is compiled in, and only this kind reads the limits.
enum RedKind { RK_STD = 0, RK_SOFT = 1, RK_SIGNED = 2, RK_SERVE = 3 };

__host__ __device__ constexpr int red_kind(int reduce)
{
    return reduce == RED_SOFT ? RK_SOFT : reduce == RED_MAX_SIGNED ? RK_SIGNED : RK_STD;
}

}  // namespace snn
