// snn_fused.h -- argument blocks of the fused / persistent step kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "snn_dev.h"

namespace snn {

constexpr int kFusedThreads = 1024;  // 16 waves; two samples per wave per round

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
    const uint32_t *bitsT;      // the same, n_in_pad x bwords
    const uint32_t *bits_next;  // input spikes of step t + 1 (nullptr: none)
    const uint16_t *lin;        // per-sample input spike lists of step t
    const uint32_t *cin;        //   and their lengths
    const uint16_t *lt;         // per-input sample spike lists of step t
    const uint32_t *ct;         //   and their lengths
    const float *xpre;          // x_pre(t), B x n_in_pad
    float *xpre_next;           // x_pre(t + 1)
    const uint32_t *Cprev;      // inhibitory spike counts of step t - 1
    uint32_t *Ccur;             // counts of step t (accumulated)
    uint32_t *Cnext;            // cleared for step t + 1
    int k;                      // step index within the call (outputs)
};

size_t fused_lds_bytes(const Params &p);
__global__ void k_fused_step(Params p, FusedArgs a, StepPtrs s);
__global__ void k_lists(Params p, const uint32_t *bits, const uint32_t *bitsT, uint16_t *lin, uint32_t *cin,
                        uint16_t *lt, uint32_t *ct, int with_t);

}  // namespace snn
