// snn_runtime.h -- the network handle behind the opaque snn_net of snn.h.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/snn.h"
#include "snn_dev.h"

// Steps encoded per encoder launch (bounds the input-spike buffers; one extra
// step is encoded so the last step of a chunk sees its successor's inputs).
constexpr uint32_t kChunk = 512;
// LDS a workgroup may use on gfx950 (160 KiB per CU).
constexpr size_t kMaxLds = 160 * 1024;

struct snn_net {
    snn_config cfg{};
    snn::Params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 256;
    int path = 0;
    int precision = 0;
    int last_path = -1;

    // shared parameters
    float *W = nullptr;          // FP32 master, block layout
    double *theta = nullptr;     // n_pad, FP64
    uint32_t *thr_lut = nullptr; // 256 spike thresholds

    // per-sample state, capacity cap_B
    uint32_t cap_B = 0, cur_B = 0;
    float *v_exc = nullptr, *v_inh = nullptr, *x_post = nullptr, *I = nullptr;
    uint16_t *rf = nullptr;
    float *x_pre = nullptr;      // 3 x B x n_in_pad (x_pre of step s in buffer s % 3)
    uint32_t *C = nullptr;       // 3 x B
    uint32_t *bits = nullptr;    // (chunk + 1) steps of input spikes, per sample
    uint32_t *bitsT = nullptr;   //   and per input
    uint16_t *lin = nullptr;     // (chunk + 1) x B x n_in_pad input spike lists
    uint32_t *cin = nullptr;
    uint16_t *lt = nullptr;      // (chunk + 1) x n_in_pad x lt_stride sample lists
    uint32_t *ct = nullptr;
    uint16_t *ord_s = nullptr;   // (chunk + 1) x B samples by decreasing cin
    uint16_t *ord_in = nullptr;  // (chunk + 1) x n_in_pad inputs by decreasing ct
    uint32_t chunk = kChunk;     // steps per encoder launch for the current batch
    uint32_t run_T = 0;          // steps of the current snn_run call (per-run normalisation)
    uint32_t cap_chunk = kChunk; // steps the buffers hold at capacity
    uint8_t *flags_mask = nullptr;
    // per-slot local steps of a batch re-formed by snn_rebatch (per_slot:
    // continuing runs encode slot b at slot_t[b] + k; else every slot at tloc)
    uint32_t *slot_t = nullptr;
    bool per_slot = false;

    // optional per-kernel timing with HIP events on the handle's stream: one
    // event pair brackets each run of consecutive launches of one kernel (a
    // span), so the events add nothing between those launches
    struct KStat {
        std::string name;
        uint64_t launches = 0;
        double total_ms = 0.0;
    };
    struct Span {
        int kid = -1;  // kernel of the open span, -1: none open
        std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
        uint64_t launches = 0;
    };
    bool prof = false;
    std::vector<KStat> kstats;
    Span span;
    std::vector<Span> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> evpool;
    int kstat_id(const char *name);
    void prof_open(int kid);  // before a launch of kernel kid
    void prof_close();        // before stream work that is not such a launch
    snn_status prof_flush();

    uint64_t gstep = 0;  // steps since the state was initialised
    uint64_t tloc = 0;   // local step of the current samples (encoder counter)
    // the C ABI's error helper for other translation units
    static snn_status error(snn_status st, const char *msg);

    ~snn_net();
    void free_state();
    snn_status ensure_state(uint32_t B);
    void set_batch(uint32_t B);
    snn_status reset_state(const uint8_t *mask_dev);
    // captured episodic runs of the per-step paths (snn_graph.hip)
    struct Graph {
        hipGraphExec_t exec = nullptr;
        int last_path = 0;
    };
    static constexpr size_t kMaxGraphs = 16;
    bool use_graphs = false;
    bool capturing = false;  // an episode is being captured (persistent: ordinary launch)
    hipStream_t cap_stream = nullptr;
    std::map<std::string, Graph> graphs;
    void graphs_invalidate();
    snn_status episode(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced, uint32_t batch,
                       uint32_t T, const snn::Outs &o);
    snn_status episode_body(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                            uint32_t batch, uint32_t T, const snn::Outs &o, const uint32_t *tl = nullptr);
    snn_status rebatch(const uint32_t *keep_dev, uint32_t n_keep, uint32_t B);
    snn_status run_graph(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                         uint32_t batch, uint32_t T, const snn::Outs &o);
    snn_status encode_chunk(const uint8_t *img, const uint64_t *ids, const uint32_t *tl, uint64_t tbase, int steps,
                            const uint32_t *forced, uint32_t *raster_in, int raster_k0);
    snn_status plain_step(int kk, int k, const snn::Outs &o, bool mfma);
    size_t mfma_attr_bytes[3] = {64 * 1024, 64 * 1024, 64 * 1024};    // STDP kernel, per precision
    size_t mfma_c_attr_bytes[3] = {64 * 1024, 64 * 1024, 64 * 1024};  // current kernel, per precision
    snn_status xpre_first(const uint32_t *bits_t);
    bool fused_ok() const;
    size_t fused_attr_bytes[3][4] = {};  // per operand form and reduction kind
    snn_status fused_step(int kk, int k, bool has_next, const snn::Outs &o);

    // persistent path: grid barrier counter / error flag
    uint32_t *bar = nullptr, *err = nullptr;
    size_t persist_attr_bytes[3][4] = {};
    int coop_ok = -1;
    bool persist_ok();
    // no learning and no inhibitory layer: the persistent path's chunk
    // kernel needs no grid barrier (k_indep)
    bool indep() const { return !p.learn && !p.has_inh; }
    size_t indep_attr_bytes[3][4] = {};  // per form and columns per lane (1, 2, 4, 8)
    snn_status persist_chunk(int steps, bool has_next, int k0, const snn::Outs &o);
    snn_status check_device_error();
    snn_status run(const uint8_t *images, const uint64_t *ids, const uint32_t *forced, uint32_t batch, uint32_t T,
                   uint32_t flags, const snn_outputs *out);
    snn_status run_steps(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced, uint32_t T,
                         const snn::Outs &o, const uint32_t *tl = nullptr);
    // serving: `steps` more steps of the first B slots, encoder keyed by the
    // per-slot local steps tl, exc spike counts added into counts while the
    // call's step is below until[b]
    snn_status serve_steps(const uint8_t *images, const uint64_t *ids, const uint32_t *tl, uint32_t B, uint32_t steps,
                           uint32_t *counts, const uint8_t *new_mask, const uint32_t *until);
    uint32_t serve_tune_T = 0;  // serving: the chunk length the path choice is tuned for
    // serving: move slots (pairs_dev: n (from, to) pairs) with the server's
    // per-slot arrays
    snn_status move_slots(const uint32_t *pairs_dev, int n, const snn::SlotArrays &sa, int n_in);
    friend struct snn_server;
    // AUTO: the fastest available execution path for this batch, measured
    // once on scratch copies of the network (snn_autotune.hip); with jb
    // non-null also over column block widths (*jb receives the winner's)
    int choose_path(uint32_t batch, uint32_t T, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                    int *jb = nullptr);
    static int default_jb(uint32_t n_exc, int cus);
    static snn_status create(const snn_config *cfg, void *stream, int jb, snn_net **out);
    snn_status relayout(int jb);
};
