/*
 * snn.h -- C ABI of the MI355X (gfx950) minibatched spiking-network library.
 *
 * The library advances a batch of B independent clock-driven simulations of
 * one network for T steps (Saunders et al., "Minibatch Processing in Spiking
 * Neural Networks", AAAI-20, Implementation section): per-sample state is
 * duplicated B times, weights and adaptive thresholds exist once and receive
 * batch-reduced updates.  One step is: Poisson input encoding, the
 * feed-forward synaptic contraction, recurrent inhibition, the fused
 * adaptive-LIF / LIF update, STDP traces, the batch-reduced weight change with
 * clamp and per-column normalisation, and the threshold update.
 *
 * Conventions
 *  - Every call returns an snn_status; on failure snn_last_error() returns a
 *    message (thread-local, valid until the next call on the same thread).
 *  - Pointers named *_host are host memory, *_dev are device memory of the
 *    device the handle was created on.  The caller owns every pointer passed
 *    in; the library copies what it keeps.  The handle owns all simulation
 *    state (weights, thresholds, voltages, traces).
 *  - snn_run is stream-ordered and asynchronous on the handle's stream;
 *    outputs are valid after snn_sync() or after the stream is synchronised.
 *  - Handles are not thread-safe, except that snn_serve_submit and
 *    snn_serve_poll may be called from any thread.
 *  - No call allocates device memory except snn_create, snn_run when the batch
 *    size grows beyond what was allocated or when path AUTO measures its
 *    candidates (scratch copies of the network, once per shape), snn_rebatch
 *    (a staging copy of the kept samples), snn_serve_create and
 *    snn_ifnet_create.
 */
#ifndef SNN_H
#define SNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SNN_ABI_VERSION 2u

typedef struct snn_net snn_net;       /* opaque network + state handle */
typedef struct snn_server snn_server; /* opaque serving loop handle    */

typedef enum {
    SNN_OK = 0,
    SNN_EINVAL = -1,    /* invalid argument or configuration                */
    SNN_ENOMEM = -2,    /* batch above max_batch or above the HBM budget    */
    SNN_EDEVICE = -3,   /* a HIP call failed; the message names it          */
    SNN_EAGAIN = -4,    /* serving: request not finished yet                */
    SNN_ENOTFOUND = -5, /* serving: unknown or already returned request id  */
    SNN_ESTATE = -6     /* call not valid in the handle's current state     */
} snn_status;

/* Batch reduction of per-sample parameter updates (Reduction methods
 * section: averaging by default, summation, per-synapse maximum per step as
 * in the unsupervised-learning experiment; the section leaves the choice of
 * reduction to the user).  Each reduces, per synapse, the B per-sample
 * potentiation terms P_b = s_post[b] x_pre[b] and, separately, the B
 * depression terms D_b = s_pre[b] x_post[b], then
 * w <- clamp(w + nu_post R(P) - nu_pre R(D)).
 *   SUM, MEAN   sum over b, and the sum / B;
 *   MAX         the largest term;
 *   SOFT_MAX    a family between MEAN and MAX: the log-mean-exp with
 *               temperature tau, R(z) = tau log((1/B) sum_b exp(z_b / tau)),
 *               which tends to the mean as tau grows and to the maximum as
 *               tau tends to 0 (tau from snn_config.reduce_tau or
 *               snn_stdp_reduce_soft);
 *   MAX_SIGNED  (a variant) w <- clamp(w + max_b (nu_post P_b - nu_pre D_b)),
 *               the largest per-sample change, 0 for a sample with no spike
 *               on the synapse.
 * Theta's increment is reduced the same way over the spike indicators
 * (MAX_SIGNED: the maximum).  Every path computes every reduction. */
typedef enum {
    SNN_REDUCE_SUM = 0,
    SNN_REDUCE_MEAN = 1,
    SNN_REDUCE_MAX = 2,
    SNN_REDUCE_MAX_SIGNED = 3,
    SNN_REDUCE_SOFT_MAX = 4
} snn_reduce;

/* Operand form of the two contractions of a step (the synaptic current and
 * the STDP products).  Spikes are exact 0/1 operands; the weight (current)
 * and the traces (STDP) enter
 *   SNN_FP32      unrounded (the matrix-core route splits each FP32 value
 *                 into three bfloat16 parts that sum to it exactly),
 *   SNN_BF16      rounded to bfloat16, nearest even,
 *   SNN_FP8_E4M3  rounded to OCP FP8 E4M3, nearest even (saturating at 448),
 * each from its FP32 value.  Sums accumulate in FP32; the master weights stay
 * FP32, theta and the column sums FP64.  Every path computes every form. */
typedef enum { SNN_FP32 = 0, SNN_BF16 = 1, SNN_FP8_E4M3 = 2 } snn_precision;

/* How the T-step loop is executed.
 *   PLAIN      one launch per kernel per step (encoder, contraction, neuron
 *              update, plasticity), gathers over the spiking inputs and
 *              samples: the straightforward per-step path;
 *   FUSED      one column-partitioned launch per step carrying contraction,
 *              neuron update and plasticity, encoder hoisted over all T;
 *   PERSISTENT one cooperative launch for all T steps, state kept on chip;
 *              a network without learning and without inhibitory layer
 *              (no neuron's input depends on another neuron) runs each
 *              encoder chunk in one launch of independent tasks instead:
 *              no grid barrier, any batch size;
 *   AUTO       chosen by the library's autotuner for (batch, T, precision);
 *   MFMA       per-step launches with the synaptic current and the STDP
 *              outer products over the batch on the matrix cores (sum and
 *              mean; the other reductions keep the gather plasticity
 *              kernel of PLAIN). */
typedef enum {
    SNN_PATH_PLAIN = 0,
    SNN_PATH_FUSED = 1,
    SNN_PATH_PERSISTENT = 2,
    SNN_PATH_AUTO = 3,
    SNN_PATH_MFMA = 4
} snn_path;

/* One LIF population (Scaling and Unsupervised Learning sections).
 * Voltages in mV, times in ms.  adaptive != 0 adds the shared threshold
 * offset theta (+theta_plus per spike, decays with tau_theta_ms). */
typedef struct {
    double v_rest, v_reset, v_thresh, tau_ms;
    int32_t refrac_steps, adaptive;
    double theta_plus, tau_theta_ms;
} snn_lif;

typedef struct {
    uint32_t abi_version;          /* must be SNN_ABI_VERSION                      */
    uint32_t n_in, n_exc, n_inh;   /* n_inh = 0: no inhibitory layer; else = n_exc */
    int32_t uniform_rate;          /* 1: every input fires at max_rate_hz          */
    int32_t learn;                 /* 1: STDP, normalisation and theta active      */
    int32_t trace_additive;        /* 0: trace set to 1 on a spike; 1: += 1        */
    int32_t reduce;                /* snn_reduce                                   */
    int32_t precision;             /* snn_precision                                */
    int32_t path;                  /* snn_path                                     */
    double dt_ms, max_rate_hz;     /* pixel p fires at p/255 * max_rate_hz          */
    snn_lif exc, inh;
    double w_ei;                   /* exc -> inh, one-to-one                        */
    double w_ie;                   /* inh -> exc, to all but the partner            */
    double nu_pre, nu_post;        /* depression on pre spike, potentiation on post */
    double tau_pre_ms, tau_post_ms;
    double w_min, w_max;           /* clamp after every update                      */
    double norm;                   /* column sum target; <= 0 disables              */
    uint64_t seed;                 /* Philox key of the Poisson encoder             */
    uint32_t max_batch;            /* largest batch snn_run will accept             */
    uint32_t norm_per_run;         /* 1: normalise once, after the last step of
                                      each snn_run / snn_run_spikes call (a
                                      cheaper variant, on every path);
                                      0: after every learning step            */
    uint64_t hbm_budget_bytes;     /* 0: no limit                                   */
    double reduce_tau;             /* temperature of SNN_REDUCE_SOFT_MAX: finite and
                                      at least x_max / 64, x_max the largest trace
                                      value (1 for nearest-spike traces,
                                      1 / (1 - lambda) for additive ones, lambda the
                                      slower of the two trace decays per step);
                                      ignored by the other reductions          */
} snn_config;

/* Device outputs of snn_run; any NULL pointer is skipped.
 * Bit rasters hold bit (k % 32) of word k / 32 for neuron / input k.
 *   counts     batch x n_exc u32, exc spike counts of this call (overwritten)
 *   raster_in  T x batch x ceil(n_in/32) u32 input spikes
 *   raster_exc T x batch x ceil(n_exc/32) u32, raster_inh likewise
 *   v_exc      T x batch x n_exc f32 voltage after each step, v_inh likewise */
typedef struct {
    uint32_t *counts;
    uint32_t *raster_in;
    uint32_t *raster_exc;
    uint32_t *raster_inh;
    float *v_exc;
    float *v_inh;
} snn_outputs;

#define SNN_RUN_RESET 1u /* episodic: reset per-sample state before step 0
                            (Episodic vs. continuing simulation section) */

/* Library ABI version (SNN_ABI_VERSION of the build). */
uint32_t snn_abi_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *snn_last_error(void);

/* Create a network on the current HIP device.  `stream` is a hipStream_t
 * (NULL = the default stream) on which all work is ordered.  Weights start
 * at zero and theta at zero; call snn_set_weights before running.
 * Errors: SNN_EINVAL (bad config or ABI version), SNN_ENOMEM, SNN_EDEVICE. */
snn_status snn_create(const snn_config *cfg, void *stream, snn_net **out);

/* Wait for outstanding work and release every resource of the handle. */
void snn_destroy(snn_net *net);

/* Change the stream later work is ordered on. */
snn_status snn_set_stream(snn_net *net, void *stream);

/* Weights, host memory, row-major n_in x n_exc f32 (n = n_in * n_exc).
 * The FP32 master copy is replaced; contraction copies are refreshed. */
snn_status snn_set_weights(snn_net *net, const float *w_host, size_t n);
snn_status snn_get_weights(snn_net *net, float *w_host, size_t n);

/* Shared adaptive thresholds, host memory, n_exc f64 (kept in FP64). */
snn_status snn_set_theta(snn_net *net, const double *theta_host, size_t n);
snn_status snn_get_theta(snn_net *net, double *theta_host, size_t n);

/* Select the batch reduction of weight and threshold updates (Reduction
 * methods section), a snn_reduce value.  Takes effect at the next step.
 * SNN_REDUCE_SOFT_MAX keeps the handle's temperature (snn_config.reduce_tau
 * or the last snn_stdp_reduce_soft).  SNN_EINVAL for a NULL handle, a mode
 * outside snn_reduce, or SOFT_MAX with a temperature out of range. */
snn_status snn_stdp_reduce(snn_net *net, int32_t mode);

/* Select the soft-maximum reduction (SNN_REDUCE_SOFT_MAX) with temperature
 * tau (Reduction methods section: a user-chosen reduction of the batch
 * dimension; this family spans the mean and the maximum the section
 * compares).  Takes effect at the next step.  SNN_EINVAL for a NULL handle
 * or a tau that is not finite or below x_max / 64 (snn_config.reduce_tau). */
snn_status snn_stdp_reduce_soft(snn_net *net, double tau);

/* Re-form the batch without a reset (an extension of the Dynamic minibatch
 * size section, which re-initialises every sample's state when the batch
 * size changes, for continuing simulation as in the Episodic vs. continuing
 * simulation section).  New slot k < n_keep takes every per-sample variable
 * of current slot keep_host[k]: voltages, refractory counts and previous
 * spikes, traces, the last step's inhibitory count and its local step
 * number (the Poisson encoder's step counter); slots n_keep .. batch - 1
 * start from the initial state at local step 0.  Weights and theta are
 * untouched.  The next snn_run / snn_run_spikes without SNN_RUN_RESET at
 * this batch size continues every slot from there (its images and ids give
 * slot b's inputs); a run with SNN_RUN_RESET or another batch size resets
 * as usual.  keep_host: host memory, n_keep distinct entries below the
 * current batch (0 before any run); may reorder.  Synchronises the handle's
 * stream and allocates a staging copy of the kept samples' state for the
 * call.  SNN_EINVAL for a NULL handle, batch 0, n_keep > batch, n_keep above
 * the current batch, a NULL or invalid list; SNN_ENOMEM for batch above
 * max_batch or the HBM budget, or a failed allocation (the per-sample state
 * is then lost and the next run resets). */
snn_status snn_rebatch(snn_net *net, const uint32_t *keep_host, uint32_t n_keep, uint32_t batch);

/* Select the execution path (snn_path) and the operand form of the
 * contractions (snn_precision).  SNN_EINVAL for values out of range. */
snn_status snn_set_path(snn_net *net, int32_t path, int32_t precision);

/* Replay repeated episodic runs from captured HIP graphs (on = 1) or launch
 * every kernel (on = 0, the default).  With graphs on, an snn_run /
 * snn_run_spikes with SNN_RUN_RESET (or a new batch size) is captured the
 * first time its arguments occur (path, batch, T, buffers, reduction,
 * precision) and replayed with a single launch afterwards; results are those
 * of the launched kernels.  On the PERSISTENT path the captured kernel is an
 * ordinary (not cooperative) launch: its workgroups must all be resident at
 * once, which holds when no other work occupies the GPU's CUs; otherwise its
 * bounded grid barrier times out and snn_sync reports SNN_EDEVICE.
 * Profiling (snn_profile_enable) always launches directly.  Captured graphs
 * are dropped when the batch capacity, path, precision or reduction changes.
 * SNN_EINVAL for a NULL handle or on not in {0, 1}. */
snn_status snn_set_graphs(snn_net *net, int32_t on);

/* The execution path the most recent snn_run / snn_run_spikes used (the
 * autotuner's choice when the handle's path is SNN_PATH_AUTO, or the fallback
 * when the requested path does not fit the batch). */
snn_status snn_last_path(snn_net *net, int32_t *path);

/* Advance `batch` samples by T steps (Implementation section).
 *   images_dev batch x n_in u8 pixels (ignored when uniform_rate)
 *   ids_dev    batch u64 sample ids; the encoder is keyed by (seed, id,
 *              local step), never by the batch slot
 *   flags      SNN_RUN_RESET for an episodic trial; a batch size different
 *              from the previous call re-initialises state as well (Dynamic
 *              minibatch size section)
 * Errors: SNN_EINVAL (T = 0, batch = 0, NULL images without uniform_rate),
 *         SNN_ENOMEM (batch > max_batch or over the HBM budget; nothing runs),
 *         SNN_EDEVICE. */
snn_status snn_run(snn_net *net, const uint8_t *images_dev, const uint64_t *ids_dev,
                   uint32_t batch, uint32_t T, uint32_t flags, const snn_outputs *out);

/* As snn_run, with the input spikes given instead of the Poisson encoder:
 * in_bits_dev is T x batch x ceil(n_in/32) u32 (bit layout of raster_in). */
snn_status snn_run_spikes(snn_net *net, const uint32_t *in_bits_dev, uint32_t batch, uint32_t T,
                          uint32_t flags, const snn_outputs *out);

/* Block until all work queued on the handle's stream has finished. */
snn_status snn_sync(snn_net *net);

/* Per-kernel timing: with profiling on, each run of consecutive launches of
 * one kernel on the handle's stream is bracketed by two HIP events recorded
 * on that stream (no events between the launches of a run), and the elapsed
 * times and launch counts are accumulated per kernel name (cleared when
 * profiling is turned on); a kernel's average is thus the run time per
 * launch, back-to-back gaps included.  snn_profile_get returns entry idx (SNN_ENOTFOUND past the last one):
 * its name (copied into name[name_len]), launch count and total milliseconds.
 * Reading synchronises the stream. */
snn_status snn_profile_enable(snn_net *net, int32_t on);
snn_status snn_profile_get(snn_net *net, uint32_t idx, char *name, size_t name_len, uint64_t *launches,
                           double *total_ms);

/* Device bytes the handle would hold for `batch` samples (state, weights,
 * scratch), the quantity compared with hbm_budget_bytes. */
size_t snn_state_bytes(const snn_config *cfg, uint32_t batch);

/* Continuous-batching inference server over a frozen network (learn must be
 * 0).  Single-sample requests (Dynamic minibatch size section: queries one at
 * a time) join a device-resident batch while slots and the HBM budget allow.
 * The batch advances in chunks of chunk_steps steps; a slot counts spikes
 * only up to its own request's T, so chunks always run in full.  Between
 * chunks finished requests leave, the remaining slots are compacted to the
 * lowest indices (state and all) and queued requests join above them; the
 * worker keeps one chunk queued ahead of the one running.  A request's
 * result does not depend on which other requests share the batch.  With
 * path AUTO the execution path is tuned here for every power-of-two width.
 *   max_slots   largest device batch; hbm_budget 0 = no limit
 * snn_serve_create takes the network's weights, path and operand form at
 * call time. */
snn_status snn_serve_create(snn_net *frozen, uint32_t max_slots, uint64_t hbm_budget,
                            uint32_t chunk_steps, snn_server **out);

/* Queue one request: image_host n_in u8 (copied), T steps, sample id `id`.
 * Returns its request id.  SNN_ENOMEM if one slot does not fit the budget. */
snn_status snn_serve_submit(snn_server *srv, const uint8_t *image_host, uint64_t id, uint32_t T,
                            uint64_t *req_id);

/* Result of a finished request: counts_host n_exc u32 spike counts and the
 * submit-to-completion latency in seconds.  SNN_EAGAIN while queued or
 * running; SNN_ENOTFOUND for an unknown id or one already returned. */
snn_status snn_serve_poll(snn_server *srv, uint64_t req_id, uint32_t *counts_host, double *latency_s);

/* Serving statistics: requests completed, slot-steps executed, peak active
 * slots, and the device time spent in launches (seconds). */
snn_status snn_serve_stats(snn_server *srv, uint64_t *completed, uint64_t *slot_steps,
                           uint32_t *peak_active, double *busy_s);

/* Drain queued and running requests, then stop; later polls are invalid. */
snn_status snn_serve_destroy(snn_server *srv);

/* ------------------------------------------------------------------------
 * Converted feed-forward network of integrate-and-fire neurons (ANN to SNN
 * conversion section): a ReLU multi-layer perceptron whose non-linearities are
 * replaced by the firing rates of non-leaky IF neurons with reset by
 * subtraction.
 *   - The image is a constant analog input: pixel p enters as p / 255 at
 *     every step.
 *   - Hidden layers h1 and h2: at each step a neuron's voltage gains
 *     I = a W + b (a = the previous layer's output of the same step: the
 *     analog input for h1, the 0/1 spikes of h1 for h2); a neuron whose
 *     voltage reaches its layer's threshold spikes and has the threshold
 *     subtracted (at most one spike per step; no leak, no lower bound).
 *   - Readout: the output layer's input s_h2 W_3 + b_3 summed over the run;
 *     the predicted class is its argmax (the first maximum on ties).
 * Every run starts from zero voltages; samples are independent.  Sums are
 * FP32: the matrix cores take each FP32 weight as three bfloat16 parts that
 * add up to it exactly, and pixels and spikes are exact operands.
 * Sizes: 1 <= n_h1 <= 256, 1 <= n_h2 <= 128, 1 <= n_out <= 32,
 * 1 <= n_in <= 65536. */
typedef struct snn_ifnet snn_ifnet; /* opaque converted-network handle */

typedef struct {
    uint32_t abi_version;            /* must be SNN_ABI_VERSION            */
    uint32_t n_in, n_h1, n_h2, n_out;
    uint32_t max_batch;              /* largest batch snn_ifnet_run takes  */
    double theta_h1, theta_h2;       /* thresholds, > 0                    */
} snn_ifnet_config;

/* Device outputs of snn_ifnet_run; any NULL pointer is skipped.
 *   out_sum    batch x n_out f32, output-layer input summed over the run
 *   pred       batch i32, argmax of out_sum
 *   counts_h1  batch x n_h1 u32 spike counts of the run, counts_h2 likewise
 *   raster_h1  T x batch x ceil(n_h1/32) u32 spikes (bit layout of
 *              snn_outputs), raster_h2 likewise
 *   v_h1       T x batch x n_h1 f32 voltage after each step, v_h2 likewise */
typedef struct {
    float *out_sum;
    int32_t *pred;
    uint32_t *counts_h1;
    uint32_t *counts_h2;
    uint32_t *raster_h1;
    uint32_t *raster_h2;
    float *v_h1;
    float *v_h2;
} snn_ifnet_outputs;

/* Create a converted network on the current HIP device, work ordered on
 * `stream` (a hipStream_t, NULL = default stream).  Every layer must be set
 * with snn_ifnet_set_layer before the first run.
 * Errors: SNN_EINVAL (sizes out of range, thresholds not > 0, ABI version),
 *         SNN_ENOMEM, SNN_EDEVICE. */
snn_status snn_ifnet_create(const snn_ifnet_config *cfg, void *stream, snn_ifnet **out);

/* Wait for outstanding work and release the handle. */
void snn_ifnet_destroy(snn_ifnet *net);

/* Weights and biases of layer 1 (input -> h1), 2 (h1 -> h2) or 3 (h2 ->
 * output), host memory: w_host n_prev x n_this row-major f32 (n_w elements),
 * b_host n_this f32 (n_b elements).  Copied; returns when the copy is done.
 * Errors: SNN_EINVAL (NULL handle or pointer, layer out of range, wrong
 *         element counts), SNN_EDEVICE. */
snn_status snn_ifnet_set_layer(snn_ifnet *net, uint32_t layer, const float *w_host, size_t n_w,
                               const float *b_host, size_t n_b);

/* Simulate `batch` images_dev (batch x n_in u8, device) for T steps from zero
 * voltages; stream-ordered and asynchronous like snn_run.
 * Errors: SNN_EINVAL (NULL handle or images, batch = 0, T = 0 or T > 65535,
 *         a layer not set), SNN_ENOMEM (batch > max_batch; nothing runs),
 *         SNN_EDEVICE. */
snn_status snn_ifnet_run(snn_ifnet *net, const uint8_t *images_dev, uint32_t batch, uint32_t T,
                         const snn_ifnet_outputs *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * run as snn_ifnet_run, with the same outputs, but its scratch (the
 * first-layer current and the partial readouts, (32 ceil(n_h1/32) +
 * 32 ceil(n_h2/32)) * 4 bytes per sample) lives in a fixed 6 MiB array of
 * device memory inside the library instead of the handle's buffers.  Each GPU
 * holds one copy of that array from its first snn_ifnet_create until the
 * process ends.  The call allocates nothing and reads nothing the previous
 * call left in the array (every scratch entry is written before it is read).
 * All calls on one GPU share its array: calls whose work overlaps on the
 * device (different streams, or different handles without ordering between
 * them) race and give undefined results; calls ordered on one stream are
 * safe.  batch is not limited by max_batch, only by the array.
 * Errors: as snn_ifnet_run, and SNN_ENOMEM when batch needs more than 6 MiB
 *         of scratch (batch > 4096 for 256 h1 and 128 h2 neurons; nothing
 *         runs). */
snn_status snn_ifnet_run_noalloc(snn_ifnet *net, const uint8_t *images_dev, uint32_t batch, uint32_t T,
                                 const snn_ifnet_outputs *out);

/* Block until the handle's stream has finished its queued work. */
snn_status snn_ifnet_sync(snn_ifnet *net);

#ifdef __cplusplus
}
#endif

#endif /* SNN_H */
