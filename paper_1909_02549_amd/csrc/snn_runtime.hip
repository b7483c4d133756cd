// snn_runtime.hip -- host side of the C ABI declared in include/snn.h:
// handle, device buffers, batch (re)initialisation, the T-step drivers of the
// plain, fused and persistent paths, weights / theta transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/snn.h"
#include "snn_dev.h"
#include "snn_fused.h"
#include "snn_kern.h"
#include "snn_mfma.h"
#include "snn_runtime.h"

using namespace snn;

static thread_local std::string g_err;

static snn_status fail(snn_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(call)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (call);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            return fail(SNN_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

// Launch a kernel on the handle's stream; with profiling on, account it under
// `name` (the launch joins the open span of that kernel or opens a new one).
#define SNN_LAUNCH(kname_, kern, grid, block, shmem, ...)                                                  \
    do {                                                                                                \
        if (this->prof) {                                                                               \
            static thread_local int kid_ = -1;                                                          \
            if (kid_ < 0 || kid_ >= (int)this->kstats.size() || this->kstats[kid_].name != (kname_))      \
                kid_ = this->kstat_id(kname_);                                                            \
            this->prof_open(kid_);                                                                      \
            hipLaunchKernelGGL(kern, grid, block, shmem, this->stream, __VA_ARGS__);                    \
            this->span.launches += 1;                                                                   \
        } else {                                                                                        \
            hipLaunchKernelGGL(kern, grid, block, shmem, this->stream, __VA_ARGS__);                    \
        }                                                                                               \
    } while (0)

extern "C" uint32_t snn_abi_version(void) { return SNN_ABI_VERSION; }
extern "C" const char *snn_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------

static int device_cu_count()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    }
    return cus;
}

// Column block width: one block per CU when the layer is large (at most 32
// columns, the fused kernel's limit), at least 8 columns otherwise.
static int choose_jb(uint32_t n_exc, int cus)
{
    int jb = (int)((n_exc + (uint32_t)cus - 1) / (uint32_t)cus);
    if (jb < 8) jb = 8;
    if (jb > 32) jb = 32;
    return jb;
}

// Steps per encoder chunk: the sparse lists take B * n_in_pad and
// n_in_pad * round8(B) u16 per step; keep one chunk under 1 GiB.
static uint32_t chunk_steps(const Params &p, uint32_t B)
{
    const size_t per = ((size_t)B * p.n_in_pad + (size_t)p.n_in_pad * ((B + 7) & ~7u)) * 2 + 16 * (size_t)B;
    size_t c = ((size_t)1 << 30) / std::max<size_t>(per, 1);
    c = std::min<size_t>(std::max<size_t>(c, 8), kChunk);
    return (uint32_t)c;
}

static void fill_dims(Params &p, const snn_config &c, int jb)
{
    p.n_in = (int)c.n_in;
    p.in_words = (int)((c.n_in + 31) / 32);
    p.n_in_pad = 32 * p.in_words;
    p.n_exc = (int)c.n_exc;
    p.jb = jb;
    p.jbp = (jb + 7) & ~7;
    // LDS rows of 16 or 32 floats would start on only 2 or 4 banks
    p.ls = (p.jbp == 16 || p.jbp == 32) ? p.jbp + 4 : p.jbp;
    p.nblk = (int)((c.n_exc + jb - 1) / jb);
    p.n_pad = p.nblk * jb;
    p.has_inh = c.n_inh > 0;
}

static size_t state_bytes(const Params &p, uint32_t B)
{
    const uint32_t chunk = chunk_steps(p, B);
    const size_t ns = (size_t)p.nblk * p.jbp * B;
    const size_t bw = (B + 31) / 32;
    size_t s = 0;
    s += (size_t)(chunk + 1) * ((size_t)B * p.n_in_pad + (size_t)p.n_in_pad * ((B + 7) & ~7u)) * 2;  // lists
    s += (size_t)(chunk + 1) * ((size_t)B + p.n_in_pad) * 4;                                       // lengths
    s += (size_t)(chunk + 1) * ((size_t)B + p.n_in_pad) * 2;                                       // orders
    s += ns * (4 + 4 + 4 + 4 + 2);                 // v_exc, v_inh, x_post, I, rf
    s += 3 * (size_t)B * p.n_in_pad * 4;            // x_pre (three steps)
    s += 3 * (size_t)B * 4;                         // C
    s += (size_t)(chunk + 1) * (B * p.in_words + 3) * 4;  // bits
    s += (size_t)(chunk + 1) * p.n_in_pad * bw * 4; // bitsT
    return s;
}

static size_t param_bytes(const Params &p)
{
    return (size_t)p.n_in_pad * p.n_pad * (4 + 2 + 1) + (size_t)p.n_pad * 8 + 1024;
}

// Smallest temperature of the soft-maximum reduction: every summand
// expm1(x / tau) stays below e^64 (x at most 1 for nearest-spike traces, at
// most 1 / (1 - lambda) for additive ones), so sums over any batch stay far
// from the FP32 range limit.
static double soft_tau_min(const snn_config &c)
{
    double xmax = 1.0;  // nearest-spike traces
    if (c.trace_additive) {
        // additive traces stay below 1 / (1 - lambda), lambda the slower decay
        const double lam = std::max(std::exp(-c.dt_ms / c.tau_pre_ms), std::exp(-c.dt_ms / c.tau_post_ms));
        xmax = lam < 1.0 ? 1.0 / (1.0 - lam) : HUGE_VAL;
    }
    return xmax / 64.0;
}

static bool soft_tau_ok(const snn_config &c, double tau)
{
    return std::isfinite(tau) && tau >= soft_tau_min(c);
}

static snn_status validate(const snn_config *c)
{
    if (!c) return fail(SNN_EINVAL, "snn_config is NULL");
    if (c->abi_version != SNN_ABI_VERSION) return fail(SNN_EINVAL, "abi_version mismatch");
    if (c->n_in == 0 || c->n_exc == 0) return fail(SNN_EINVAL, "n_in and n_exc must be > 0");
    if (c->n_in > (1u << 20) || c->n_exc > (1u << 22)) return fail(SNN_EINVAL, "layer size too large");
    if (c->n_inh != 0 && c->n_inh != c->n_exc)
        return fail(SNN_EINVAL, "n_inh must be 0 or equal to n_exc (one-to-one exc->inh)");
    if (!(c->dt_ms > 0) || !(c->exc.tau_ms > 0) || (c->n_inh && !(c->inh.tau_ms > 0)))
        return fail(SNN_EINVAL, "dt and time constants must be > 0");
    if (c->exc.refrac_steps < 0 || c->exc.refrac_steps > 127 || c->inh.refrac_steps < 0 ||
        c->inh.refrac_steps > 127)
        return fail(SNN_EINVAL, "refrac_steps must be in [0, 127]");
    if (c->reduce < 0 || c->reduce > 4)
        return fail(SNN_EINVAL, "reduce must be 0 (sum), 1 (mean), 2 (max), 3 (signed max) or 4 (soft max)");
    if (c->precision < 0 || c->precision > 2) return fail(SNN_EINVAL, "precision must be 0, 1 or 2");
    if (c->path < 0 || c->path > 4) return fail(SNN_EINVAL, "path must be 0..4");
    if (c->learn && (!(c->tau_pre_ms > 0) || !(c->tau_post_ms > 0)))
        return fail(SNN_EINVAL, "trace time constants must be > 0");
    if (c->learn && c->exc.adaptive && !(c->exc.tau_theta_ms > 0))
        return fail(SNN_EINVAL, "tau_theta_ms must be > 0");
    if (c->learn && c->reduce == SNN_REDUCE_SOFT_MAX && !soft_tau_ok(*c, c->reduce_tau))
        return fail(SNN_EINVAL, "reduce_tau must be finite and at least the largest trace value / 64");
    if (c->w_min > c->w_max) return fail(SNN_EINVAL, "w_min > w_max");
    if (c->max_batch == 0) return fail(SNN_EINVAL, "max_batch must be > 0");
    if (c->norm_per_run > 1) return fail(SNN_EINVAL, "norm_per_run must be 0 or 1");
    double prob = c->max_rate_hz * c->dt_ms / 1000.0;
    if (!(prob >= 0.0) || prob > 1.0) return fail(SNN_EINVAL, "max_rate_hz * dt must be a probability");
    return SNN_OK;
}

// Spike threshold of pixel value `pixel`: floor(rate * dt * 2^32) with
// rate = pixel / 255 * max_rate (or max_rate for uniform inputs).
static uint32_t rate_threshold(const snn_config &c, int pixel, bool uniform)
{
    const double prob = uniform ? c.max_rate_hz * c.dt_ms / 1000.0
                                : (double)pixel * c.max_rate_hz * c.dt_ms / (255.0 * 1000.0);
    double thr = std::floor(prob * 4294967296.0);
    thr = std::min(std::max(thr, 0.0), 4294967295.0);
    return (uint32_t)thr;
}

static void fill_params(Params &p, const snn_config &c)
{
    auto lif = [&](const snn_lif &l) {
        LifP q;
        q.v_rest = (float)l.v_rest;
        q.v_reset = (float)l.v_reset;
        q.v_th = (float)l.v_thresh;
        q.alpha = (float)std::exp(-c.dt_ms / l.tau_ms);
        q.refrac = l.refrac_steps;
        return q;
    };
    p.exc = lif(c.exc);
    p.inh = c.n_inh ? lif(c.inh) : LifP{0.f, 0.f, 0.f, 0.f, 0};
    p.learn = c.learn != 0;
    p.adaptive = c.exc.adaptive != 0;
    p.trace_add = c.trace_additive != 0;
    p.reduce = c.reduce;
    const double tau = c.reduce == SNN_REDUCE_SOFT_MAX ? c.reduce_tau : 1.0;
    p.itau2_r = (float)(M_LOG2E / tau);
    p.tau_ln2_r = (float)(tau * M_LN2);
    p.prec = c.precision;
    p.uniform_rate = c.uniform_rate != 0;
    p.thr_uniform = rate_threshold(c, 0, true);
    p.w_ei = (float)c.w_ei;
    p.w_ie = (float)c.w_ie;
    p.lam_pre = c.learn ? (float)std::exp(-c.dt_ms / c.tau_pre_ms) : 0.f;
    p.lam_post = c.learn ? (float)std::exp(-c.dt_ms / c.tau_post_ms) : 0.f;
    p.nu_pre = (float)c.nu_pre;
    p.nu_post = (float)c.nu_post;
    p.w_min = (float)c.w_min;
    p.w_max = (float)c.w_max;
    p.norm = c.norm;
    p.beta = (c.learn && c.exc.adaptive) ? std::exp(-c.dt_ms / c.exc.tau_theta_ms) : 1.0;
    p.theta_plus = c.exc.theta_plus;
    p.seed = c.seed;
    p.B = 0;
    p.bwords = 0;
    p.inv_B = 0.f;
    p.inv_Bd = 0.0;
}

// ---------------------------------------------------------------------------
// handle lifetime
// ---------------------------------------------------------------------------

int snn_net::kstat_id(const char *name)
{
    for (size_t q = 0; q < kstats.size(); ++q)
        if (kstats[q].name == name) return (int)q;
    kstats.push_back(KStat{name, 0, 0.0});
    return (int)kstats.size() - 1;
}

void snn_net::prof_open(int kid)
{
    if (span.kid == kid) return;
    prof_close();
    if (evpool.empty() && pending.size() >= 4096) prof_flush();
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (!evpool.empty()) {
        ev = evpool.back();
        evpool.pop_back();
    } else {
        (void)hipEventCreate(&ev.first);
        (void)hipEventCreate(&ev.second);
    }
    (void)hipEventRecord(ev.first, stream);
    span.kid = kid;
    span.ev = ev;
    span.launches = 0;
}

void snn_net::prof_close()
{
    if (span.kid < 0) return;
    (void)hipEventRecord(span.ev.second, stream);
    pending.push_back(span);
    span.kid = -1;
}

snn_status snn_net::prof_flush()
{
    prof_close();
    if (pending.empty()) return SNN_OK;
    HIP_TRY(hipStreamSynchronize(stream));
    for (auto &sp : pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, sp.ev.first, sp.ev.second) == hipSuccess) {
            kstats[sp.kid].launches += sp.launches;
            kstats[sp.kid].total_ms += ms;
        }
        evpool.push_back(sp.ev);
    }
    pending.clear();
    return SNN_OK;
}

snn_net::~snn_net()
{
    prof_flush();
    graphs_invalidate();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto &e : evpool) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    (void)hipFree(bar);
    (void)hipFree(err);
    free_state();
    (void)hipFree(W);
    (void)hipFree(theta);
    (void)hipFree(thr_lut);
}

void snn_net::free_state()
{
    for (void *q : {(void *)v_exc, (void *)v_inh, (void *)x_post, (void *)I, (void *)rf, (void *)x_pre, (void *)C,
                    (void *)bits, (void *)bitsT, (void *)flags_mask, (void *)lin, (void *)cin, (void *)lt, (void *)ct,
                    (void *)ord_s, (void *)ord_in, (void *)slot_t})
        if (q) (void)hipFree(q);
    v_exc = v_inh = x_post = I = x_pre = nullptr;
    rf = nullptr;
    lin = lt = ord_s = ord_in = nullptr;
    C = bits = bitsT = cin = ct = slot_t = nullptr;
    flags_mask = nullptr;
    cap_B = 0;
    cur_B = 0;
    per_slot = false;
}

// The column block width a new handle starts with: one block per CU when the
// layer is large (choose_jb), or the SNN_JB environment override.
int snn_net::default_jb(uint32_t n_exc, int cus)
{
    int jb = choose_jb(n_exc, cus);
    if (const char *e = std::getenv("SNN_JB")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 32) jb = v;
    }
    return jb;
}

extern "C" snn_status snn_create(const snn_config *cfg, void *stream, snn_net **out)
{
    return snn_net::create(cfg, stream, 0, out);
}

// snn_create with the column block width jb (0: default_jb).
snn_status snn_net::create(const snn_config *cfg, void *stream, int jb, snn_net **out)
{
    if (!out) return fail(SNN_EINVAL, "out is NULL");
    *out = nullptr;
    snn_status st = validate(cfg);
    if (st != SNN_OK) return st;
    snn_net *n = new (std::nothrow) snn_net();
    if (!n) return fail(SNN_ENOMEM, "host allocation failed");
    n->cfg = *cfg;
    n->stream = (hipStream_t)stream;
    HIP_TRY(hipGetDevice(&n->device));
    n->cus = device_cu_count();
    if (jb <= 0) jb = default_jb(cfg->n_exc, n->cus);
    fill_dims(n->p, *cfg, jb);
    fill_params(n->p, *cfg);
    n->path = cfg->path;
    n->precision = cfg->precision;
    if (cfg->hbm_budget_bytes && param_bytes(n->p) > cfg->hbm_budget_bytes) {
        delete n;
        return fail(SNN_ENOMEM, "weights alone exceed hbm_budget_bytes");
    }
    const size_t nw = (size_t)n->p.n_in_pad * n->p.n_pad;
    hipError_t e = hipMalloc(&n->W, nw * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&n->theta, (size_t)n->p.n_pad * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&n->thr_lut, 256 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&n->bar, 64);
    if (e == hipSuccess) e = hipMalloc(&n->err, 64);
    if (e != hipSuccess) {
        delete n;
        return fail(SNN_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    std::vector<uint32_t> lut(256);
    for (int q = 0; q < 256; ++q) lut[q] = rate_threshold(*cfg, q, false);
    e = hipMemcpy(n->thr_lut, lut.data(), 256 * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->W, 0, nw * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->theta, 0, (size_t)n->p.n_pad * sizeof(double));
    if (e == hipSuccess) e = hipMemset(n->err, 0, 64);
    if (e != hipSuccess) {
        delete n;
        return fail(SNN_EDEVICE, std::string("init: ") + hipGetErrorString(e));
    }
    *out = n;
    return SNN_OK;
}

extern "C" void snn_destroy(snn_net *net)
{
    if (!net) return;
    if (net->stream) (void)hipStreamSynchronize(net->stream);
    else (void)hipDeviceSynchronize();
    delete net;
}

extern "C" snn_status snn_set_stream(snn_net *net, void *stream)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    net->stream = (hipStream_t)stream;
    net->graphs_invalidate();
    return SNN_OK;
}

// ---------------------------------------------------------------------------
// weights and thresholds
// ---------------------------------------------------------------------------

extern "C" snn_status snn_set_weights(snn_net *net, const float *w, size_t n)
{
    if (!net || !w) return fail(SNN_EINVAL, "NULL argument");
    const Params &p = net->p;
    if (n != (size_t)p.n_in * p.n_exc) return fail(SNN_EINVAL, "n must equal n_in * n_exc");
    std::vector<float> blk((size_t)p.n_in_pad * p.n_pad, 0.f);
    for (int i = 0; i < p.n_in; ++i)
        for (int j = 0; j < p.n_exc; ++j) {
            const int g = j / p.jb, jj = j % p.jb;
            blk[((size_t)g * p.n_in_pad + i) * p.jb + jj] = w[(size_t)i * p.n_exc + j];
        }
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(hipMemcpy(net->W, blk.data(), blk.size() * sizeof(float), hipMemcpyHostToDevice));
    return SNN_OK;
}

extern "C" snn_status snn_get_weights(snn_net *net, float *w, size_t n)
{
    if (!net || !w) return fail(SNN_EINVAL, "NULL argument");
    const Params &p = net->p;
    if (n != (size_t)p.n_in * p.n_exc) return fail(SNN_EINVAL, "n must equal n_in * n_exc");
    std::vector<float> blk((size_t)p.n_in_pad * p.n_pad);
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(hipMemcpy(blk.data(), net->W, blk.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int i = 0; i < p.n_in; ++i)
        for (int j = 0; j < p.n_exc; ++j) {
            const int g = j / p.jb, jj = j % p.jb;
            w[(size_t)i * p.n_exc + j] = blk[((size_t)g * p.n_in_pad + i) * p.jb + jj];
        }
    return SNN_OK;
}

extern "C" snn_status snn_set_theta(snn_net *net, const double *th, size_t n)
{
    if (!net || !th) return fail(SNN_EINVAL, "NULL argument");
    if (n != net->cfg.n_exc) return fail(SNN_EINVAL, "n must equal n_exc");
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(hipMemcpy(net->theta, th, n * sizeof(double), hipMemcpyHostToDevice));
    return SNN_OK;
}

extern "C" snn_status snn_get_theta(snn_net *net, double *th, size_t n)
{
    if (!net || !th) return fail(SNN_EINVAL, "NULL argument");
    if (n != net->cfg.n_exc) return fail(SNN_EINVAL, "n must equal n_exc");
    HIP_TRY(hipStreamSynchronize(net->stream));
    HIP_TRY(hipMemcpy(th, net->theta, n * sizeof(double), hipMemcpyDeviceToHost));
    return SNN_OK;
}

// Change the column block width to jb: the weights and thresholds keep their
// values in the new block layout; the per-sample state and the captured
// graphs are dropped (the next run starts an episode).
snn_status snn_net::relayout(int jb)
{
    if (jb == p.jb) return SNN_OK;
    std::vector<float> w((size_t)p.n_in * p.n_exc);
    std::vector<double> th(p.n_exc);
    snn_status st = snn_get_weights(this, w.data(), w.size());
    if (st == SNN_OK) st = snn_get_theta(this, th.data(), th.size());
    if (st != SNN_OK) return st;
    graphs_invalidate();
    free_state();
    (void)hipFree(W);
    (void)hipFree(theta);
    W = nullptr;
    theta = nullptr;
    fill_dims(p, cfg, jb);
    const size_t nw = (size_t)p.n_in_pad * p.n_pad;
    HIP_TRY(hipMalloc(&W, nw * sizeof(float)));
    HIP_TRY(hipMalloc(&theta, (size_t)p.n_pad * sizeof(double)));
    HIP_TRY(hipMemset(W, 0, nw * sizeof(float)));
    HIP_TRY(hipMemset(theta, 0, (size_t)p.n_pad * sizeof(double)));
    st = snn_set_weights(this, w.data(), w.size());
    if (st == SNN_OK) st = snn_set_theta(this, th.data(), th.size());
    return st;
}

extern "C" snn_status snn_stdp_reduce(snn_net *net, int32_t mode)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (mode < 0 || mode > 4)
        return fail(SNN_EINVAL, "mode must be 0 (sum), 1 (mean), 2 (max), 3 (signed max) or 4 (soft max)");
    if (mode == SNN_REDUCE_SOFT_MAX) return snn_stdp_reduce_soft(net, net->cfg.reduce_tau);
    net->cfg.reduce = mode;
    net->p.reduce = mode;
    net->graphs_invalidate();
    return SNN_OK;
}

extern "C" snn_status snn_stdp_reduce_soft(snn_net *net, double tau)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (!soft_tau_ok(net->cfg, tau)) return fail(SNN_EINVAL, "tau must be finite and at least the largest trace value / 64");
    net->cfg.reduce = SNN_REDUCE_SOFT_MAX;
    net->cfg.reduce_tau = tau;
    net->p.reduce = RED_SOFT;
    net->p.itau2_r = (float)(M_LOG2E / tau);
    net->p.tau_ln2_r = (float)(tau * M_LN2);
    net->graphs_invalidate();
    return SNN_OK;
}

extern "C" snn_status snn_set_path(snn_net *net, int32_t path, int32_t precision)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (path < 0 || path > 4) return fail(SNN_EINVAL, "path must be 0..4");
    if (precision < 0 || precision > 2) return fail(SNN_EINVAL, "precision must be 0..2");
    net->path = path;
    net->precision = precision;
    net->p.prec = precision;
    net->cfg.path = path;
    net->cfg.precision = precision;
    net->graphs_invalidate();
    return SNN_OK;
}

snn_status snn_net::check_device_error()
{
    uint32_t flag = 0;
    HIP_TRY(hipMemcpy(&flag, err, sizeof flag, hipMemcpyDeviceToHost));
    if (flag) {
        HIP_TRY(hipMemset(err, 0, sizeof flag));
        return fail(SNN_EDEVICE, "persistent kernel: grid barrier wait timed out (launch ended early)");
    }
    return SNN_OK;
}

extern "C" snn_status snn_last_path(snn_net *net, int32_t *path)
{
    if (!net || !path) return fail(SNN_EINVAL, "NULL argument");
    *path = net->last_path;
    return SNN_OK;
}

extern "C" snn_status snn_sync(snn_net *net)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    // with profiling on, the open span ends with the work queued so far (not
    // with whatever the stream runs before the next launch or read-out)
    if (net->prof) net->prof_close();
    HIP_TRY(hipStreamSynchronize(net->stream));
    return net->check_device_error();
}

extern "C" size_t snn_state_bytes(const snn_config *cfg, uint32_t batch)
{
    if (!cfg || validate(cfg) != SNN_OK) return 0;
    Params p{};
    fill_dims(p, *cfg, choose_jb(cfg->n_exc, device_cu_count()));
    return state_bytes(p, batch) + param_bytes(p);
}

// ---------------------------------------------------------------------------
// state management
// ---------------------------------------------------------------------------

snn_status snn_net::ensure_state(uint32_t B)
{
    if (B > cfg.max_batch) return fail(SNN_ENOMEM, "batch exceeds max_batch");
    if (cfg.hbm_budget_bytes && state_bytes(p, B) + param_bytes(p) > cfg.hbm_budget_bytes)
        return fail(SNN_ENOMEM, "batch exceeds hbm_budget_bytes");
    if (B > cap_B) {
        HIP_TRY(hipStreamSynchronize(stream));
        free_state();
        const size_t ns = (size_t)p.nblk * p.jbp * B;
        const size_t bw = (B + 31) / 32;
        hipError_t e = hipSuccess;
        auto A = [&](void **ptr, size_t bytes) {
            if (e == hipSuccess) e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
        };
        A((void **)&v_exc, ns * 4);
        A((void **)&v_inh, ns * 4);
        A((void **)&x_post, ns * 4);
        A((void **)&I, ns * 4);
        A((void **)&rf, ns * 2);
        A((void **)&x_pre, 3 * (size_t)B * p.n_in_pad * 4);
        A((void **)&C, 3 * (size_t)B * 4);
        const uint32_t ch = chunk_steps(p, B);
        const size_t lts = (B + 7) & ~7u;
        A((void **)&bits, (size_t)(ch + 1) * ((size_t)B * p.in_words + 3) * 4);
        A((void **)&bitsT, (size_t)(ch + 1) * p.n_in_pad * bw * 4);
        A((void **)&lin, (size_t)(ch + 1) * B * p.n_in_pad * 2);
        A((void **)&cin, (size_t)(ch + 1) * B * 4);
        // (+64 bytes: list heads are read as 64-byte runs, also from the
        // last list when lists hold fewer than 32 entries)
        A((void **)&lt, (size_t)(ch + 1) * p.n_in_pad * lts * 2 + 64);
        A((void **)&ct, (size_t)(ch + 1) * p.n_in_pad * 4);
        A((void **)&ord_s, (size_t)(ch + 1) * B * 2);
        A((void **)&ord_in, (size_t)(ch + 1) * p.n_in_pad * 2);
        A((void **)&flags_mask, B);
        A((void **)&slot_t, (size_t)B * 4);
        if (e != hipSuccess) {
            free_state();
            return fail(SNN_ENOMEM, std::string("state hipMalloc: ") + hipGetErrorString(e));
        }
        cap_B = B;
        cap_chunk = ch;
        chunk = ch;
        graphs_invalidate();
    }
    return SNN_OK;
}

void snn_net::set_batch(uint32_t B)
{
    p.B = (int)B;
    p.bwords = (int)((B + 31) / 32);
    p.inv_B = 1.f / (float)B;
    p.inv_Bd = 1.0 / (double)B;
    p.Bs = (int)cap_B;
    p.bits_stride = (int)((((size_t)B * p.in_words) + 3) & ~(size_t)3);
    p.lt_stride = (int)((B + 7) & ~7u);
    // never more steps than the buffers were sized for at capacity
    chunk = std::min(chunk_steps(p, B), cap_chunk);
}

snn_status snn_net::reset_state(const uint8_t *mask_dev)
{
    const size_t ns = (size_t)p.nblk * p.jbp * p.B;
    const size_t n = std::max(ns, (size_t)p.B * p.n_in_pad);  // k_reset covers b < B
    const int tpb = 256;
    SNN_LAUNCH("reset", k_reset, dim3((unsigned)((n + tpb - 1) / tpb)), dim3(tpb), 0, p, v_exc, v_inh, rf, x_post,
               x_pre, C, mask_dev);
    HIP_TRY(hipGetLastError());
    if (!mask_dev) {
        gstep = 0;
        tloc = 0;
    }
    return SNN_OK;
}

// ---------------------------------------------------------------------------
// plain per-step path
// ---------------------------------------------------------------------------

static inline unsigned blocks_for(size_t n, int tpb) { return (unsigned)((n + tpb - 1) / tpb); }

snn_status snn_net::encode_chunk(const uint8_t *img, const uint64_t *ids, const uint32_t *tl, uint64_t tbase,
                                 int steps, const uint32_t *forced, uint32_t *raster_in, int raster_k0)
{
    dim3 grid((unsigned)((p.B + 63) / 64), (unsigned)p.in_words, (unsigned)steps);
    SNN_LAUNCH("encode", k_encode, grid, dim3(64), 0, p, img, ids, (const uint32_t *)thr_lut, tl, tbase, forced,
               bits, p.learn ? bitsT : nullptr, raster_in, raster_k0);
    HIP_TRY(hipGetLastError());
    return SNN_OK;
}

snn_status snn_net::plain_step(int kk, int k, const Outs &o, bool mfma)
{
    const uint32_t *bits_t = bits + (size_t)kk * p.bits_stride;
    const uint32_t *bitsT_t = bitsT + (size_t)kk * p.n_in_pad * p.bwords;
    float *xcur = x_pre + (size_t)(gstep % 3) * p.Bs * p.n_in_pad;
    const float *xprev = x_pre + (size_t)((gstep + 2) % 3) * p.Bs * p.n_in_pad;
    uint32_t *Ccur = C + (size_t)(gstep % 3) * p.Bs;
    uint32_t *Cprev = C + (size_t)((gstep + 2) % 3) * p.Bs;
    uint32_t *Cnext = C + (size_t)((gstep + 1) % 3) * p.Bs;
    const size_t ns = (size_t)p.nblk * p.jbp * p.B;
    const int tpb = 256;
    const size_t clds = mfma ? mfma_front_lds(p, p.prec) : 0;
    if (mfma && clds <= kMaxLds) {
        // traces, synaptic current on the matrix cores and neurons in one launch
        const void *fn = p.prec == PREC_FP32   ? (const void *)k_mfma_front<PREC_FP32>
                         : p.prec == PREC_BF16 ? (const void *)k_mfma_front<PREC_BF16>
                                               : (const void *)k_mfma_front<PREC_FP8>;
        if (clds > mfma_c_attr_bytes[p.prec]) {
            HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)clds));
            mfma_c_attr_bytes[p.prec] = clds;
        }
        FrontArgs fa{W, theta, bits_t, xprev, xcur, Cprev, Ccur, Cnext, v_exc, v_inh, x_post, rf, k, o};
        const dim3 grid((unsigned)p.nblk);
        if (p.prec == PREC_FP32)
            SNN_LAUNCH("mfma_front", k_mfma_front<PREC_FP32>, grid, dim3(512), clds, p, fa);
        else if (p.prec == PREC_BF16)
            SNN_LAUNCH("mfma_front", k_mfma_front<PREC_BF16>, grid, dim3(512), clds, p, fa);
        else
            SNN_LAUNCH("mfma_front", k_mfma_front<PREC_FP8>, grid, dim3(512), clds, p, fa);
    } else {
        if (p.learn)
            SNN_LAUNCH("xpre", k_xpre, dim3(blocks_for((size_t)p.B * p.n_in_pad, tpb)), dim3(tpb), 0, p, bits_t,
                       xprev, xcur);
        SNN_LAUNCH("contract", k_contract, dim3(blocks_for(ns, tpb)), dim3(tpb), 0, p, (const float *)W, bits_t, I);
        SNN_LAUNCH("neuron", k_neuron, dim3(blocks_for((size_t)p.nblk * p.B * (p.jbp / 8), tpb)), dim3(tpb), 0, p,
                   (const float *)I, (const double *)theta, (const uint32_t *)Cprev, Ccur, Cnext, v_exc, v_inh, rf,
                   x_post, k, o);
    }
    // per-run normalisation: the plasticity launches of all but the run's
    // last step see norm = 0 (no normalisation)
    Params pp = p;
    if (cfg.norm_per_run && (uint32_t)k + 1 != run_T) pp.norm = 0.0;
    if (p.learn && mfma && mfma_plastic_fits(p, p.prec)) {
        const size_t lds = mfma_plastic_lds(p, p.prec);
        const void *fn = p.prec == PREC_FP32   ? (const void *)k_mfma_plastic<PREC_FP32>
                         : p.prec == PREC_BF16 ? (const void *)k_mfma_plastic<PREC_BF16>
                                               : (const void *)k_mfma_plastic<PREC_FP8>;
        if (lds > mfma_attr_bytes[p.prec]) {
            HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            mfma_attr_bytes[p.prec] = lds;
        }
        const dim3 grid((unsigned)p.nblk);
        if (p.prec == PREC_FP32)
            SNN_LAUNCH("mfma_plastic", k_mfma_plastic<PREC_FP32>, grid, dim3(512), lds, pp, W, theta,
                       (const uint16_t *)rf, (const float *)x_post, (const float *)xcur, bitsT_t);
        else if (p.prec == PREC_BF16)
            SNN_LAUNCH("mfma_plastic", k_mfma_plastic<PREC_BF16>, grid, dim3(512), lds, pp, W, theta,
                       (const uint16_t *)rf, (const float *)x_post, (const float *)xcur, bitsT_t);
        else
            SNN_LAUNCH("mfma_plastic", k_mfma_plastic<PREC_FP8>, grid, dim3(512), lds, pp, W, theta,
                       (const uint16_t *)rf, (const float *)x_post, (const float *)xcur, bitsT_t);
    } else if (p.learn) {
        const int R = 256 / p.jb;
        const size_t sm = align16((size_t)p.jb * p.bwords * 4) + (size_t)(R * p.jb + p.jb) * 8;
        SNN_LAUNCH("plastic", k_plastic, dim3((unsigned)p.nblk), dim3(256), sm, pp, W, theta, (const uint16_t *)rf,
                   (const float *)x_post, (const float *)xcur, bitsT_t);
    }
    HIP_TRY(hipGetLastError());
    ++gstep;
    return SNN_OK;
}

// ---------------------------------------------------------------------------
// snn_run
// ---------------------------------------------------------------------------

snn_status snn_net::run(const uint8_t *images, const uint64_t *ids, const uint32_t *forced, uint32_t batch,
                        uint32_t T, uint32_t flags, const snn_outputs *out)
{
    if (batch == 0 || T == 0) return fail(SNN_EINVAL, "batch and T must be > 0");
    if (!forced) {
        if (!ids) return fail(SNN_EINVAL, "ids_dev is NULL");
        if (!images && !cfg.uniform_rate) return fail(SNN_EINVAL, "images_dev is NULL and uniform_rate is 0");
    }
    snn_status st = ensure_state(batch);
    if (st != SNN_OK) return st;
    Outs o{};
    if (out) {
        o.counts = out->counts;
        o.raster_in = out->raster_in;
        o.raster_exc = out->raster_exc;
        o.raster_inh = out->raster_inh;
        o.v_exc = out->v_exc;
        o.v_inh = out->v_inh;
    }
    bool reset = batch != cur_B || (flags & SNN_RUN_RESET);
    set_batch(batch);
    int path = this->path;
    if (path == SNN_PATH_AUTO) {
        // an episode start may also change the column block width
        int jb = p.jb;
        path = choose_path(batch, T, images, ids, forced, reset ? &jb : nullptr);
        if (jb != p.jb) {
            st = relayout(jb);
            if (st == SNN_OK) st = ensure_state(batch);
            if (st != SNN_OK) return st;
            reset = true;
        }
    }
    set_batch(batch);
    if (reset) per_slot = false;
    if (reset && use_graphs && !prof) return run_graph(path, images, ids, forced, batch, T, o);
    if (reset) {
        st = reset_state(nullptr);
        if (st != SNN_OK) return st;
        cur_B = batch;
    }
    if (!per_slot) return episode_body(path, images, ids, forced, batch, T, o);
    // a batch re-formed by snn_rebatch: every slot at its own local step
    st = episode_body(path, images, ids, forced, batch, T, o, slot_t);
    if (st != SNN_OK) return st;
    SNN_LAUNCH("slot_step", k_add_u32, dim3((batch + 255) / 256), dim3(256), 0, slot_t, T, (int)batch);
    HIP_TRY(hipGetLastError());
    return SNN_OK;
}

// Re-form the batch without a reset: new slot k < n_keep takes the state of
// old slot keep[k] (host list, checked by the caller), the other slots start
// fresh; see snn_rebatch.
snn_status snn_net::rebatch(const uint32_t *keep_host, uint32_t n_keep, uint32_t B)
{
    const int nk = (int)n_keep;
    // staging rows of the kept samples and the list itself, in one allocation
    const size_t ns = (size_t)p.nblk * p.jbp * n_keep;
    const size_t nx = (size_t)n_keep * p.n_in_pad;
    size_t off[8], total = 0;
    const size_t sizes[8] = {ns * 4, ns * 4, ns * 4, ns * 2, nx * 4, (size_t)n_keep * 4, (size_t)n_keep * 4,
                             (size_t)n_keep * 4};
    for (int q = 0; q < 8; ++q) {
        off[q] = total;
        total += align16(std::max<size_t>(sizes[q], 16));
    }
    unsigned char *stage = nullptr;
    const uint32_t *keep_dev = nullptr;
    if (n_keep > 0) {
        hipError_t e = hipMalloc((void **)&stage, total);
        if (e != hipSuccess) return fail(SNN_ENOMEM, std::string("rebatch staging: ") + hipGetErrorString(e));
        keep_dev = reinterpret_cast<const uint32_t *>(stage + off[7]);
        e = hipMemcpyAsync(stage + off[7], keep_host, (size_t)n_keep * 4, hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            (void)hipFree(stage);
            return fail(SNN_EDEVICE, std::string("rebatch list copy: ") + hipGetErrorString(e));
        }
    }
    RebatchStage rs{};  // (no staging when no sample is kept: k_rebatch_load reads none)
    if (stage)
        rs = RebatchStage{reinterpret_cast<float *>(stage + off[0]), reinterpret_cast<float *>(stage + off[1]),
                          reinterpret_cast<float *>(stage + off[2]), reinterpret_cast<uint16_t *>(stage + off[3]),
                          reinterpret_cast<float *>(stage + off[4]), reinterpret_cast<uint32_t *>(stage + off[5]),
                          reinterpret_cast<uint32_t *>(stage + off[6])};
    const int tpb = 256;
    snn_status st = SNN_OK;
    if (n_keep > 0) {
        const size_t n = std::max(ns, nx);
        SNN_LAUNCH("rebatch_save", k_rebatch_save, dim3((unsigned)((n + tpb - 1) / tpb)), dim3(tpb), 0, p,
                   (const float *)v_exc, (const float *)v_inh, (const float *)x_post, (const uint16_t *)rf,
                   (const float *)(x_pre + (size_t)((gstep + 2) % 3) * p.Bs * p.n_in_pad),
                   (const uint32_t *)(C + (size_t)((gstep + 2) % 3) * p.Bs), per_slot ? (const uint32_t *)slot_t : nullptr,
                   (uint32_t)tloc, keep_dev, nk, rs);
        if (hipGetLastError() != hipSuccess) st = fail(SNN_EDEVICE, "k_rebatch_save launch failed");
    }
    // (a larger batch than the capacity reallocates the state; the staging
    // copy is complete first: ensure_state waits for the stream)
    if (st == SNN_OK) st = ensure_state(B);
    if (st == SNN_OK) {
        set_batch(B);
        const size_t n = std::max((size_t)p.nblk * p.jbp * B, (size_t)B * p.n_in_pad);
        SNN_LAUNCH("rebatch_load", k_rebatch_load, dim3((unsigned)((n + tpb - 1) / tpb)), dim3(tpb), 0, p, v_exc,
                   v_inh, x_post, rf, x_pre + (size_t)((gstep + 2) % 3) * p.Bs * p.n_in_pad,
                   C + (size_t)(gstep % 3) * p.Bs, C + (size_t)((gstep + 2) % 3) * p.Bs, slot_t, nk, rs);
        if (hipGetLastError() != hipSuccess) st = fail(SNN_EDEVICE, "k_rebatch_load launch failed");
    }
    if (stage) {
        if (hipStreamSynchronize(stream) != hipSuccess && st == SNN_OK) st = fail(SNN_EDEVICE, "rebatch: stream error");
        (void)hipFree(stage);
    }
    if (st != SNN_OK) return st;
    cur_B = B;
    per_slot = true;
    return SNN_OK;
}

// One episode from a reset state: reset, clear the outputs, run T steps.
snn_status snn_net::episode(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                            uint32_t batch, uint32_t T, const Outs &o)
{
    snn_status st = reset_state(nullptr);
    if (st != SNN_OK) return st;
    cur_B = batch;
    return episode_body(path, images, ids, forced, batch, T, o);
}

// Clear the outputs of a run, then T steps on `path`.
snn_status snn_net::episode_body(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                                 uint32_t batch, uint32_t T, const Outs &o, const uint32_t *tl)
{
    const int words = (p.n_exc + 31) / 32;
    auto zero = [&](uint32_t *ptr, size_t n) {
        if (!ptr) return;
        SNN_LAUNCH("fill", k_fill_u32, dim3((unsigned)std::min<size_t>((n + 255) / 256, 4096)), dim3(256), 0, ptr, 0u,
                   n);
    };
    zero(o.counts, (size_t)batch * p.n_exc);
    zero(o.raster_exc, (size_t)T * batch * words);
    zero(o.raster_inh, (size_t)T * batch * words);
    HIP_TRY(hipGetLastError());
    return run_steps(path, images, ids, forced, T, o, tl);
}

snn_status snn_net::xpre_first(const uint32_t *bits_t)
{
    float *xcur = x_pre + (size_t)(gstep % 3) * p.Bs * p.n_in_pad;
    const float *xprev = x_pre + (size_t)((gstep + 2) % 3) * p.Bs * p.n_in_pad;
    SNN_LAUNCH("xpre", k_xpre, dim3(blocks_for((size_t)p.B * p.n_in_pad, 256)), dim3(256), 0, p, bits_t, xprev, xcur);
    HIP_TRY(hipGetLastError());
    return SNN_OK;
}

// The fused per-step (Persist false) or persistent kernel for an operand
// form and a reduction kind.
template <int PREC, int RK, bool Persist>
static const void *kernel_of()
{
    if constexpr (Persist)
        return (const void *)k_persist<PREC, RK>;
    else
        return (const void *)k_fused_step<PREC, RK>;
}

template <bool Persist>
static const void *step_kernel(int prec, int rk)
{
    // (RK_SERVE: the frozen kind, for every run without learning)
    static const void *const table[3][4] = {
        {kernel_of<PREC_FP32, RK_STD, Persist>(), kernel_of<PREC_FP32, RK_SOFT, Persist>(),
         kernel_of<PREC_FP32, RK_SIGNED, Persist>(), kernel_of<PREC_FP32, RK_SERVE, Persist>()},
        {kernel_of<PREC_BF16, RK_STD, Persist>(), kernel_of<PREC_BF16, RK_SOFT, Persist>(),
         kernel_of<PREC_BF16, RK_SIGNED, Persist>(), kernel_of<PREC_BF16, RK_SERVE, Persist>()},
        {kernel_of<PREC_FP8, RK_STD, Persist>(), kernel_of<PREC_FP8, RK_SOFT, Persist>(),
         kernel_of<PREC_FP8, RK_SIGNED, Persist>(), kernel_of<PREC_FP8, RK_SERVE, Persist>()}};
    return table[prec][rk];
}

bool snn_net::fused_ok() const
{
    return p.jb <= 32 && p.n_in_pad < 65535 && p.B < 65535 && fused_lds_bytes(p) <= kMaxLds;
}

snn_status snn_net::fused_step(int kk, int k, bool has_next, const Outs &o)
{
    StepPtrs s;
    s.bits = bits + (size_t)kk * p.bits_stride;
    s.bits_next = has_next ? bits + (size_t)(kk + 1) * p.bits_stride : nullptr;
    s.lin = lin + (size_t)kk * p.B * p.n_in_pad;
    s.cin = cin + (size_t)kk * p.B;
    s.lt = lt + (size_t)kk * p.n_in_pad * p.lt_stride;
    s.ct = ct + (size_t)kk * p.n_in_pad;
    s.ord_s = ord_s + (size_t)kk * p.B;
    s.ord_in = ord_in + (size_t)kk * p.n_in_pad;
    s.xpre = x_pre + (size_t)(gstep % 3) * p.Bs * p.n_in_pad;
    s.xpre_next = x_pre + (size_t)((gstep + 1) % 3) * p.Bs * p.n_in_pad;
    s.Ccur = C + (size_t)(gstep % 3) * p.Bs;
    s.Cprev = C + (size_t)((gstep + 2) % 3) * p.Bs;
    s.Cnext = C + (size_t)((gstep + 1) % 3) * p.Bs;
    s.k = k;
    // per-run normalisation: only the run's last step normalises
    Params pp = p;
    if (cfg.norm_per_run && (uint32_t)k + 1 != run_T) pp.norm = 0.0;
    FusedArgs a{W, theta, v_exc, v_inh, x_post, rf, o};
    const size_t lds = fused_lds_bytes(p);
    const int rk = p.learn ? red_kind(p.reduce) : RK_SERVE;
    const void *fn = step_kernel<false>(p.prec, rk);
    if (lds > fused_attr_bytes[p.prec][rk]) {
        HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        fused_attr_bytes[p.prec][rk] = lds;
    }
    void *kargs[] = {(void *)&pp, (void *)&a, (void *)&s};
    // without learning: enough workgroups per column block to give every
    // thread about one task and the grid a few workgroups per CU
    unsigned split = 1;
    if (!p.learn) {
        const unsigned tasks = (unsigned)p.B * (unsigned)(p.jbp >> 3);
        const unsigned by_tasks = (tasks + kFusedThreads - 1) / kFusedThreads;
        const unsigned by_cus = std::max(1u, 4u * (unsigned)cus / (unsigned)p.nblk);
        split = std::max(1u, std::min(by_tasks, by_cus));
    }
    if (prof) prof_open(kstat_id("fused_step"));
    HIP_TRY(hipLaunchKernel(fn, dim3((unsigned)p.nblk, split), dim3(kFusedThreads), kargs, (unsigned)lds, stream));
    if (prof) span.launches += 1;
    ++gstep;
    return SNN_OK;
}

bool snn_net::persist_ok()
{
    if (indep()) return p.jb <= 32 && p.n_in_pad < 65535 && p.B < 65535 && indep_lds_bytes(p) <= kMaxLds;
    if (coop_ok < 0) {
        int v = 0;
        coop_ok = (hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, device) == hipSuccess && v) ? 1 : 0;
    }
    return coop_ok == 1 && p.jb <= 32 && p.B * (p.jbp / 8) <= kPersistThreads * kPersistTasks && p.nblk <= cus &&
           p.n_in_pad < 65535 && p.B < 65535 && persist_lds_bytes(p) + 64 <= kMaxLds;
}

snn_status snn_net::persist_chunk(int steps, bool has_next, int k0, const Outs &o)
{
    PersistArgs h;
    h.p = p;
    h.a = FusedArgs{W, theta, v_exc, v_inh, x_post, rf, o};
    ChunkPtrs &c = h.ch;
    if (indep()) {
        // independent tasks: one thread per task, any number of workgroups
        c = ChunkPtrs{};
        c.lin = lin;
        c.cin = cin;
        c.steps = steps;
        c.k0 = k0;
        h.sy = PersistSync{nullptr, nullptr};
        const size_t lds = indep_lds_bytes(p);
        // columns per lane: 4 (two lanes per 8-column task: a wave then walks
        // the lists of 32 samples, not 64, and the kernel holds fewer
        // registers; measured 9 % faster than 8 at the largest batches), or
        // fewer while the grid would not give every SIMD a wave (small
        // batches: a shorter chain of instructions per step)
        const unsigned tasks = (unsigned)p.B * (unsigned)(p.jbp >> 3);
        int cols = 4;
        if (const char *e = std::getenv("SNN_INDEP_COLS")) {
            const int v = std::atoi(e);
            if (v == 1 || v == 2 || v == 4 || v == 8) cols = v;
        } else {
            const size_t fill = (size_t)cus * 4 * 64;
            while (cols > 1 && (size_t)tasks * (size_t)p.nblk * (size_t)(8 / cols) < fill) cols >>= 1;
        }
        static const void *const fns[3][4] = {
            {(const void *)k_indep_narrow<PREC_FP32, 1>, (const void *)k_indep_narrow<PREC_FP32, 2>,
             (const void *)k_indep_narrow<PREC_FP32, 4>, (const void *)k_indep<PREC_FP32>},
            {(const void *)k_indep_narrow<PREC_BF16, 1>, (const void *)k_indep_narrow<PREC_BF16, 2>,
             (const void *)k_indep_narrow<PREC_BF16, 4>, (const void *)k_indep<PREC_BF16>},
            {(const void *)k_indep_narrow<PREC_FP8, 1>, (const void *)k_indep_narrow<PREC_FP8, 2>,
             (const void *)k_indep_narrow<PREC_FP8, 4>, (const void *)k_indep<PREC_FP8>}};
        const int ci = cols == 1 ? 0 : cols == 2 ? 1 : cols == 4 ? 2 : 3;
        const void *fn = fns[p.prec][ci];
        if (lds > indep_attr_bytes[p.prec][ci]) {
            HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            indep_attr_bytes[p.prec][ci] = lds;
        }
        const unsigned lanes = tasks * (unsigned)(8 / cols);
        const dim3 grid((unsigned)p.nblk, (lanes + kIndepThreads - 1) / kIndepThreads);
        void *kargs[] = {(void *)&h};
        if (prof) prof_open(kstat_id("indep"));
        HIP_TRY(hipLaunchKernel(fn, grid, dim3(kIndepThreads), kargs, (unsigned)lds, stream));
        if (prof) span.launches += 1;
        gstep += (uint64_t)steps;
        return SNN_OK;
    }
    c.bits = bits;
    c.lin = lin;
    c.cin = cin;
    c.lt = lt;
    c.ct = ct;
    c.ord_in = ord_in;
    c.xpre = x_pre;
    c.C = C;
    c.steps = steps;
    c.has_next = has_next ? 1 : 0;
    c.mod0 = (int)(gstep % 3);
    c.k0 = k0;
    // every step normalises, or under per-run normalisation only the last
    // step of the run (none if the run continues in a later chunk)
    c.norm_from = !cfg.norm_per_run ? 0 : (uint32_t)(k0 + steps) == run_T ? steps - 1 : steps;
    h.sy = PersistSync{bar, err};
    SNN_LAUNCH("fill", k_fill_u32, dim3(1), dim3(64), 0, bar, 0u, (size_t)1);
    const size_t lds = persist_lds_bytes(p);
    // runs without learning (serving with its count limits among them) have
    // a kind of their own
    const int rk = o.until || !p.learn ? RK_SERVE : red_kind(p.reduce);
    const void *kfn = step_kernel<true>(p.prec, rk);
    if (lds > persist_attr_bytes[p.prec][rk]) {
        HIP_TRY(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        persist_attr_bytes[p.prec][rk] = lds;
    }
    // the arguments go by value: the runtime copies them into the launch.
    // Launched directly, the kernel goes out as a cooperative launch (the
    // runtime checks that every workgroup is resident at once); captured in
    // a graph it is an ordinary kernel node: its nblk <= #CU workgroups each
    // take a whole CU's LDS share, so an otherwise idle GPU holds them all,
    // and the bounded grid barrier turns anything else into SNN_EDEVICE.
    void *kargs[] = {(void *)&h};
    if (prof) prof_open(kstat_id("persistent"));
    if (capturing)
        HIP_TRY(hipLaunchKernel(kfn, dim3((unsigned)p.nblk), dim3(kPersistThreads), kargs, (unsigned)lds, stream));
    else
        HIP_TRY(hipLaunchCooperativeKernel(kfn, dim3((unsigned)p.nblk), dim3(kPersistThreads), kargs,
                                           (unsigned)lds, stream));
    if (prof) span.launches += 1;
    gstep += (uint64_t)steps;
    return SNN_OK;
}

snn_status snn_net::error(snn_status st, const char *msg) { return fail(st, msg); }

snn_status snn_net::move_slots(const uint32_t *pairs_dev, int n, const SlotArrays &sa, int n_in)
{
    if (n <= 0) return SNN_OK;
    const size_t span = std::max({(size_t)p.nblk * p.jbp, (size_t)p.n_in_pad, (size_t)p.n_exc, (size_t)n_in});
    SNN_LAUNCH("slot_move", k_slot_move, dim3((unsigned)((span + 255) / 256), (unsigned)n), dim3(256), 0, p, v_exc,
               v_inh, x_post, rf, x_pre + (size_t)((gstep + 2) % 3) * p.Bs * p.n_in_pad,
               C + (size_t)((gstep + 2) % 3) * p.Bs, sa, n_in, pairs_dev, n);
    HIP_TRY(hipGetLastError());
    return SNN_OK;
}

snn_status snn_net::serve_steps(const uint8_t *images, const uint64_t *ids, const uint32_t *tl_dev, uint32_t B,
                                uint32_t steps, uint32_t *counts, const uint8_t *new_mask, const uint32_t *until)
{
    if (B == 0 || B > cap_B || steps == 0) return fail(SNN_EINVAL, "serve_steps: bad batch or steps");
    set_batch(B);
    cur_B = B;
    if (new_mask) {
        snn_status st = reset_state(new_mask);
        if (st != SNN_OK) return st;
        SNN_LAUNCH("slot_init", k_slot_init, dim3(B), dim3(256), 0, new_mask, const_cast<uint32_t *>(tl_dev), counts,
                   p.n_exc, (int)B);
    }
    Outs o{};
    o.counts = counts;
    o.until = until;
    // the active width changes with every admission: tune per power-of-two
    // width (at most log2(capacity) measurements, on the slot buffers, which
    // hold capacity entries)
    int path = this->path;
    if (path == SNN_PATH_AUTO) {
        uint32_t Bk = 1;
        while (Bk < B) Bk <<= 1;
        Bk = std::min(Bk, cap_B);
        set_batch(Bk);  // (the candidate paths depend on the width)
        path = choose_path(Bk, serve_tune_T ? serve_tune_T : steps, images, ids, nullptr);
        set_batch(B);
    }
    snn_status st = run_steps(path, images, ids, nullptr, steps, o, tl_dev);
    if (st != SNN_OK) return st;
    SNN_LAUNCH("slot_step", k_add_u32, dim3((B + 255) / 256), dim3(256), 0, const_cast<uint32_t *>(tl_dev), steps,
               (int)B);
    HIP_TRY(hipGetLastError());
    return SNN_OK;
}

snn_status snn_net::run_steps(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                              uint32_t T, const Outs &o, const uint32_t *tl)
{
    run_T = T;
    if (path == SNN_PATH_PERSISTENT && !persist_ok()) path = SNN_PATH_FUSED;
    if (path == SNN_PATH_FUSED && !fused_ok()) path = SNN_PATH_PLAIN;
    if (path == SNN_PATH_MFMA && p.jb > 32) path = SNN_PATH_PLAIN;
    last_path = path;
    for (uint32_t k0 = 0; k0 < T; k0 += chunk) {
        const int steps = (int)std::min<uint32_t>(chunk, T - k0);
        const bool more = k0 + (uint32_t)steps < T;
        const int enc_steps = steps + (more ? 1 : 0);
        const uint32_t *fc = forced ? forced + (size_t)k0 * p.B * p.in_words : nullptr;
        const bool col_block = path == SNN_PATH_FUSED || path == SNN_PATH_PERSISTENT;
        snn_status st = SNN_OK;
        if (col_block && !p.learn) {
            // no plasticity: the encoder writes the per-sample spike lists
            // itself (no transposed spikes, no list kernel)
            SNN_LAUNCH("encode", k_encode_lists, dim3((unsigned)((p.B + 3) / 4), (unsigned)enc_steps), dim3(256), 0,
                       p, images, ids, (const uint32_t *)thr_lut, tl, tl ? (uint64_t)k0 : tloc, fc, bits, lin, cin,
                       o.raster_in, (int)k0);
            HIP_TRY(hipGetLastError());
        } else {
            st = tl ? encode_chunk(images, ids, tl, k0, enc_steps, fc, o.raster_in, (int)k0)
                    : encode_chunk(images, ids, nullptr, tloc, enc_steps, fc, o.raster_in, (int)k0);
            if (st != SNN_OK) return st;
        }
        if (col_block) {
            if (p.learn)
                SNN_LAUNCH("lists", k_lists, dim3((unsigned)((std::max(p.B, p.n_in_pad) + 255) / 256),
                                                  (unsigned)enc_steps),
                           dim3(256), 0, p, (const uint32_t *)bits, (const uint32_t *)bitsT, lin, cin, lt, ct, 1);
            // (the independent-task chunk kernel takes no work order)
            if (!(path == SNN_PATH_PERSISTENT && indep()))
                SNN_LAUNCH("order", k_order, dim3((unsigned)enc_steps), dim3(kOrderThreads), 0, p,
                           (const uint32_t *)cin, (const uint32_t *)ct, ord_s, ord_in, p.learn);
            HIP_TRY(hipGetLastError());
            if (k0 == 0 && p.learn) {
                st = xpre_first(bits);
                if (st != SNN_OK) return st;
            }
            if (path == SNN_PATH_PERSISTENT) {
                st = persist_chunk(steps, more, (int)k0, o);
                if (st != SNN_OK) return st;
            } else {
                for (int kk = 0; kk < steps; ++kk) {
                    const bool has_next = (kk + 1 < enc_steps);
                    st = fused_step(kk, (int)k0 + kk, has_next, o);
                    if (st != SNN_OK) return st;
                }
            }
        } else {
            for (int kk = 0; kk < steps; ++kk) {
                st = plain_step(kk, (int)k0 + kk, o, path == SNN_PATH_MFMA);
                if (st != SNN_OK) return st;
            }
        }
        tloc += (uint64_t)steps;
    }
    return SNN_OK;
}


extern "C" snn_status snn_run(snn_net *net, const uint8_t *images_dev, const uint64_t *ids_dev, uint32_t batch,
                              uint32_t T, uint32_t flags, const snn_outputs *out)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    return net->run(images_dev, ids_dev, nullptr, batch, T, flags, out);
}

extern "C" snn_status snn_rebatch(snn_net *net, const uint32_t *keep_host, uint32_t n_keep, uint32_t batch)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (batch == 0) return fail(SNN_EINVAL, "batch must be > 0");
    if (n_keep > batch) return fail(SNN_EINVAL, "n_keep exceeds the new batch");
    if (n_keep > 0 && !keep_host) return fail(SNN_EINVAL, "keep_host is NULL");
    if (n_keep > net->cur_B) return fail(SNN_EINVAL, "n_keep exceeds the current batch");
    std::vector<uint8_t> seen(net->cur_B, 0);
    for (uint32_t k = 0; k < n_keep; ++k) {
        if (keep_host[k] >= net->cur_B) return fail(SNN_EINVAL, "keep entry beyond the current batch");
        if (seen[keep_host[k]]++) return fail(SNN_EINVAL, "keep entries must be distinct");
    }
    if (batch > net->cfg.max_batch) return fail(SNN_ENOMEM, "batch exceeds max_batch");
    return net->rebatch(keep_host, n_keep, batch);
}

extern "C" snn_status snn_run_spikes(snn_net *net, const uint32_t *in_bits_dev, uint32_t batch, uint32_t T,
                                     uint32_t flags, const snn_outputs *out)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    if (!in_bits_dev) return fail(SNN_EINVAL, "in_bits_dev is NULL");
    return net->run(nullptr, nullptr, in_bits_dev, batch, T, flags, out);
}

// ---------------------------------------------------------------------------
// per-kernel timing (HIP events on the handle's stream)
// ---------------------------------------------------------------------------

extern "C" snn_status snn_profile_enable(snn_net *net, int32_t on)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    snn_status st = net->prof_flush();
    if (st != SNN_OK) return st;
    net->prof = on != 0;
    if (on) net->kstats.clear();
    return SNN_OK;
}

extern "C" snn_status snn_profile_get(snn_net *net, uint32_t idx, char *name, size_t name_len, uint64_t *launches,
                                      double *total_ms)
{
    if (!net) return fail(SNN_EINVAL, "net is NULL");
    snn_status st = net->prof_flush();
    if (st != SNN_OK) return st;
    if (idx >= net->kstats.size()) return fail(SNN_ENOTFOUND, "no such kernel entry");
    const auto &k = net->kstats[idx];
    if (name && name_len) {
        std::strncpy(name, k.name.c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    if (launches) *launches = k.launches;
    if (total_ms) *total_ms = k.total_ms;
    return SNN_OK;
}
