// snn_serve.hip -- continuous-batching inference server (host side).
//
// Single-sample requests (the Dynamic minibatch size section's one-at-a-time
// queries) join a device-resident batch of a frozen network.  Slots are
// independent simulations (no learning, the inhibition is per sample) and
// the encoder is keyed by (seed, sample id, local step of the slot), so a
// request's counts do not depend on which other requests share the batch or
// on its slot.
//
// The batch advances in chunks of `chunk_steps` steps.  Every chunk runs in
// full: a slot whose request ends inside the chunk stops counting spikes at
// its own last step (the kernels' per-slot count limit), so requests of
// different lengths never cut a chunk short.  Between chunks the worker
//   - retires the finished requests (their counts are copied out after the
//     chunk in which they end),
//   - compacts the active slots to the lowest indices (the highest active
//     slots move into the holes, state and all), so the batch width is the
//     number of active requests,
//   - admits queued requests into the slots above them (fresh state, local
//     step 0).
// All of this is decided on the host when the chunk is planned, so the worker
// keeps one chunk queued ahead of the one the GPU runs: it plans and enqueues
// chunk k + 1, then waits for chunk k and publishes its results (host staging
// buffers alternate between the two).
//
// One worker thread drives the device; submit and poll only touch the queue
// and the result table under a mutex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/snn.h"
#include "snn_dev.h"
#include "snn_kern.h"
#include "snn_runtime.h"

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t req_id, id;
    uint32_t T;
    double t_submit;
    std::vector<uint8_t> image;
};

struct Result {
    std::vector<uint32_t> counts;
    double latency;
};

struct Slot {
    bool active = false;
    uint64_t req_id = 0;
    uint32_t remaining = 0;
    double t_submit = 0.0;
};

// One planned chunk: what to enqueue, and what to publish when it is done.
struct Chunk {
    bool valid = false;
    uint32_t B = 0, steps = 0, first_new = 0;
    std::vector<uint32_t> moves;      // (from, to) pairs
    std::vector<uint32_t> finishing;  // slots whose request ends in this chunk
    std::vector<uint64_t> req_ids;    // their requests
    std::vector<double> t_submit;
};

}  // namespace

struct snn_server {
    snn_net *net = nullptr;   // internal copy of the frozen network
    hipStream_t stream = nullptr;  // the server's own stream (default priority)
    uint32_t cap = 0;         // slots that fit max_slots and the HBM budget
    uint32_t chunk = 1;
    uint32_t n_in = 0, n_exc = 0;

    // device: per-slot image, id, local step, counts; per-chunk mask, count
    // limits and move pairs
    uint8_t *img_d = nullptr;
    uint64_t *ids_d = nullptr;
    uint32_t *tl_d = nullptr, *counts_d = nullptr, *until_d = nullptr, *pairs_d = nullptr;
    uint8_t *mask_d = nullptr;
    // pinned host staging, two of each (chunk parity)
    uint8_t *img_h[2] = {}, *mask_h[2] = {};
    uint64_t *ids_h[2] = {};
    uint32_t *until_h[2] = {}, *pairs_h[2] = {}, *counts_h[2] = {};
    hipEvent_t ev0[2] = {}, ev1[2] = {};

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Result> done;
    std::unordered_set<uint64_t> retiring;  // ended in an enqueued chunk, not yet published
    std::vector<Slot> slots;
    uint64_t next_req = 1;
    bool stop = false;
    snn_status worker_status = SNN_OK;
    std::thread worker;

    uint64_t completed = 0, slot_steps = 0;
    uint32_t peak_active = 0;
    double busy_s = 0.0;

    Chunk pend[2];

    bool plan(int par);            // under mu
    snn_status enqueue(int par);
    snn_status retire(int par);
    void fail_all(snn_status st);  // under mu
    void loop();
    ~snn_server();
};

snn_server::~snn_server()
{
    (void)hipFree(img_d);
    (void)hipFree(ids_d);
    (void)hipFree(tl_d);
    (void)hipFree(counts_d);
    (void)hipFree(until_d);
    (void)hipFree(pairs_d);
    (void)hipFree(mask_d);
    for (int q = 0; q < 2; ++q) {
        for (void *h : {(void *)img_h[q], (void *)mask_h[q], (void *)ids_h[q], (void *)until_h[q],
                        (void *)pairs_h[q], (void *)counts_h[q]})
            if (h) (void)hipHostFree(h);
        if (ev0[q]) (void)hipEventDestroy(ev0[q]);
        if (ev1[q]) (void)hipEventDestroy(ev1[q]);
    }
    snn_destroy(net);
    if (stream) (void)hipStreamDestroy(stream);
}

// Plan the next chunk into pend[par]: compaction moves, admissions, count
// limits, the requests that end in it.  Returns false if no slot is active.
bool snn_server::plan(int par)
{
    Chunk &c = pend[par];
    c.moves.clear();
    c.finishing.clear();
    c.req_ids.clear();
    c.t_submit.clear();
    uint32_t active = 0;
    for (uint32_t s = 0; s < cap; ++s) active += slots[s].active ? 1u : 0u;
    // compaction: the highest active slots fill the holes below `active`
    uint32_t top = cap;
    for (uint32_t h = 0; h < active; ++h) {
        if (slots[h].active) continue;
        do
            --top;
        while (!slots[top].active);
        slots[h] = slots[top];
        slots[top].active = false;
        c.moves.push_back(top);
        c.moves.push_back(h);
    }
    // admissions above the active slots, staged contiguously
    c.first_new = active;
    uint32_t B = active;
    while (B < cap && !queue.empty()) {
        Request &r = queue.front();
        std::memcpy(img_h[par] + (size_t)(B - c.first_new) * n_in, r.image.data(), n_in);
        ids_h[par][B - c.first_new] = r.id;
        slots[B] = Slot{true, r.req_id, r.T, r.t_submit};
        queue.pop_front();
        ++B;
    }
    if (B == 0) return false;
    c.B = B;
    peak_active = std::max(peak_active, B);
    // a full chunk, or the longest remaining request if all end sooner
    uint32_t longest = 0;
    for (uint32_t s = 0; s < B; ++s) longest = std::max(longest, slots[s].remaining);
    c.steps = std::min(chunk, longest);
    for (uint32_t s = 0; s < B; ++s) {
        mask_h[par][s] = s >= c.first_new ? 1u : 0u;
        const uint32_t n = std::min(slots[s].remaining, c.steps);
        until_h[par][s] = n;
        slot_steps += n;
        slots[s].remaining -= n;
        if (slots[s].remaining == 0) {
            c.finishing.push_back(s);
            c.req_ids.push_back(slots[s].req_id);
            c.t_submit.push_back(slots[s].t_submit);
            retiring.insert(slots[s].req_id);
            slots[s].active = false;
        }
    }
    std::memcpy(pairs_h[par], c.moves.data(), c.moves.size() * sizeof(uint32_t));
    c.valid = true;
    return true;
}

snn_status snn_server::enqueue(int par)
{
    Chunk &c = pend[par];
    hipStream_t st = net->stream;
    auto ok = [](hipError_t e) { return e == hipSuccess; };
    if (!ok(hipEventRecord(ev0[par], st))) return SNN_EDEVICE;
    const int nm = (int)(c.moves.size() / 2);
    if (nm > 0) {
        if (!ok(hipMemcpyAsync(pairs_d, pairs_h[par], c.moves.size() * 4, hipMemcpyHostToDevice, st)))
            return SNN_EDEVICE;
        const snn::SlotArrays sa{img_d, ids_d, tl_d, counts_d};
        const snn_status s = net->move_slots(pairs_d, nm, sa, (int)n_in);
        if (s != SNN_OK) return s;
    }
    const uint32_t nnew = c.B - c.first_new;
    if (nnew > 0) {
        if (!ok(hipMemcpyAsync(img_d + (size_t)c.first_new * n_in, img_h[par], (size_t)nnew * n_in,
                               hipMemcpyHostToDevice, st)) ||
            !ok(hipMemcpyAsync(ids_d + c.first_new, ids_h[par], (size_t)nnew * 8, hipMemcpyHostToDevice, st)) ||
            !ok(hipMemcpyAsync(mask_d, mask_h[par], c.B, hipMemcpyHostToDevice, st)))
            return SNN_EDEVICE;
    }
    if (!ok(hipMemcpyAsync(until_d, until_h[par], (size_t)c.B * 4, hipMemcpyHostToDevice, st))) return SNN_EDEVICE;
    const snn_status s =
        net->serve_steps(img_d, ids_d, tl_d, c.B, c.steps, counts_d, nnew > 0 ? mask_d : nullptr, until_d);
    if (s != SNN_OK) return s;
    for (size_t k = 0; k < c.finishing.size(); ++k)
        if (!ok(hipMemcpyAsync(counts_h[par] + k * n_exc, counts_d + (size_t)c.finishing[k] * n_exc, n_exc * 4,
                               hipMemcpyDeviceToHost, st)))
            return SNN_EDEVICE;
    if (!ok(hipEventRecord(ev1[par], st))) return SNN_EDEVICE;
    return SNN_OK;
}

// Wait for chunk pend[par] and publish the requests that ended in it.
snn_status snn_server::retire(int par)
{
    Chunk &c = pend[par];
    if (!c.valid) return SNN_OK;
    if (hipEventSynchronize(ev1[par]) != hipSuccess) return SNN_EDEVICE;
    const double t1 = now_s();
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev0[par], ev1[par]);
    std::lock_guard<std::mutex> lk(mu);
    busy_s += 1e-3 * ms;
    for (size_t k = 0; k < c.finishing.size(); ++k) {
        Result r;
        r.counts.assign(counts_h[par] + k * n_exc, counts_h[par] + (k + 1) * n_exc);
        r.latency = t1 - c.t_submit[k];
        done.emplace(c.req_ids[k], std::move(r));
        retiring.erase(c.req_ids[k]);
        ++completed;
    }
    c.valid = false;
    return SNN_OK;
}

void snn_server::fail_all(snn_status st)
{
    worker_status = st;
    stop = true;
    queue.clear();
    retiring.clear();
    for (auto &sl : slots) sl.active = false;
}

void snn_server::loop()
{
    if (hipSetDevice(net->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        fail_all(SNN_EDEVICE);
        return;
    }
    int par = 0;
    for (;;) {
        bool have;
        {
            std::lock_guard<std::mutex> lk(mu);
            have = plan(par);
        }
        snn_status st = have ? enqueue(par) : SNN_OK;
        // the chunk before it (the GPU runs it meanwhile)
        if (st == SNN_OK) st = retire(par ^ 1);
        if (st != SNN_OK) {
            (void)hipStreamSynchronize(net->stream);
            std::lock_guard<std::mutex> lk(mu);
            fail_all(st);
            return;
        }
        if (have) {
            par ^= 1;
            continue;
        }
        std::unique_lock<std::mutex> lk(mu);
        if (queue.empty()) {
            if (stop) return;
            cv.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

extern "C" snn_status snn_serve_create(snn_net *frozen, uint32_t max_slots, uint64_t hbm_budget, uint32_t chunk_steps,
                                       snn_server **out)
{
    if (!out) return snn_net::error(SNN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!frozen) return snn_net::error(SNN_EINVAL, "frozen is NULL");
    if (frozen->cfg.learn) return snn_net::error(SNN_EINVAL, "serving needs a frozen network (learn = 0)");
    if (max_slots == 0 || chunk_steps == 0) return snn_net::error(SNN_EINVAL, "max_slots and chunk_steps must be > 0");
    snn_config c = frozen->cfg;
    c.max_batch = max_slots;
    c.hbm_budget_bytes = 0;
    // slots that fit the budget: state and parameter bytes of the device batch
    uint32_t cap = max_slots;
    if (hbm_budget) {
        while (cap > 0 && snn_state_bytes(&c, cap) > hbm_budget) cap = cap > 64 ? cap - cap / 8 : cap - 1;
    }
    snn_server *sv = new (std::nothrow) snn_server();
    if (!sv) return snn_net::error(SNN_ENOMEM, "host allocation failed");
    sv->cap = cap;
    sv->chunk = chunk_steps;
    sv->n_in = c.n_in;
    sv->n_exc = c.n_exc;
    sv->slots.resize(cap);
    if (hipStreamSynchronize(frozen->stream) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking) != hipSuccess) {
        delete sv;
        return snn_net::error(SNN_EDEVICE, "serving stream");
    }
    snn_status st = snn_net::create(&c, sv->stream, frozen->p.jb, &sv->net);
    if (st != SNN_OK) {
        delete sv;
        return st;
    }
    // the frozen handle's current execution path and operand form (either may
    // have been changed with snn_set_path after it was created)
    sv->net->path = frozen->path;
    sv->net->precision = frozen->precision;
    sv->net->p.prec = frozen->p.prec;
    sv->net->cfg.precision = frozen->precision;
    const snn::Params &fp = frozen->p;
    hipError_t e = hipSuccess;
    if (sv->net->p.jb != fp.jb) {
        delete sv;
        return snn_net::error(SNN_EINVAL, "internal network layout differs from the frozen one");
    }
    const size_t nw = (size_t)fp.n_in_pad * fp.n_pad;
    e = hipMemcpyAsync(sv->net->W, frozen->W, nw * sizeof(float), hipMemcpyDeviceToDevice, sv->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sv->net->theta, frozen->theta, (size_t)fp.n_pad * sizeof(double), hipMemcpyDeviceToDevice,
                           sv->stream);
    const uint32_t nb = std::max(cap, 1u);
    auto A = [&](void **ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
    };
    auto H = [&](void **ptr, size_t bytes) {
        if (e == hipSuccess) e = hipHostMalloc(ptr, std::max<size_t>(bytes, 16), hipHostMallocDefault);
    };
    A((void **)&sv->img_d, (size_t)nb * c.n_in);
    A((void **)&sv->ids_d, (size_t)nb * 8);
    A((void **)&sv->tl_d, (size_t)nb * 4);
    A((void **)&sv->counts_d, (size_t)nb * c.n_exc * 4);
    A((void **)&sv->mask_d, nb);
    A((void **)&sv->until_d, (size_t)nb * 4);
    A((void **)&sv->pairs_d, (size_t)nb * 8);
    for (int q = 0; q < 2; ++q) {
        H((void **)&sv->img_h[q], (size_t)nb * c.n_in);
        H((void **)&sv->mask_h[q], nb);
        H((void **)&sv->ids_h[q], (size_t)nb * 8);
        H((void **)&sv->until_h[q], (size_t)nb * 4);
        H((void **)&sv->pairs_h[q], (size_t)nb * 8);
        H((void **)&sv->counts_h[q], (size_t)nb * c.n_exc * 4);
        if (e == hipSuccess) e = hipEventCreate(&sv->ev0[q]);
        if (e == hipSuccess) e = hipEventCreate(&sv->ev1[q]);
    }
    if (e == hipSuccess) e = hipMemsetAsync(sv->img_d, 0, (size_t)nb * c.n_in, sv->stream);
    if (e == hipSuccess) e = hipMemsetAsync(sv->ids_d, 0, (size_t)nb * 8, sv->stream);
    if (e == hipSuccess) e = hipMemsetAsync(sv->tl_d, 0, (size_t)nb * 4, sv->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);
    if (e != hipSuccess) {
        delete sv;
        return snn_net::error(SNN_ENOMEM, "serving buffers");
    }
    if (cap > 0) {
        st = sv->net->ensure_state(cap);
        if (st != SNN_OK) {
            delete sv;
            return st;
        }
    }
    // AUTO: choose the path for every power-of-two width now, so that no
    // request waits behind a measurement; the tuning input is a uniform grey
    // image (about the spike density of the workload's images)
    sv->net->serve_tune_T = chunk_steps;
    if (cap > 0 && sv->net->path == SNN_PATH_AUTO) {
        e = hipMemsetAsync(sv->img_d, 48, (size_t)cap * c.n_in, sv->stream);
        for (uint32_t w = 1; e == hipSuccess; w *= 2) {
            const uint32_t wk = std::min(w, cap);
            sv->net->set_batch(wk);  // (the candidate paths depend on the width)
            (void)sv->net->choose_path(wk, chunk_steps, sv->img_d, sv->ids_d, nullptr);
            if (wk == cap) break;
        }
        if (e == hipSuccess) e = hipMemsetAsync(sv->img_d, 0, (size_t)cap * c.n_in, sv->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(sv->stream);
        if (e != hipSuccess) {
            delete sv;
            return snn_net::error(SNN_EDEVICE, "serving: path tuning");
        }
    }
    sv->worker = std::thread([sv] { sv->loop(); });
    *out = sv;
    return SNN_OK;
}

extern "C" snn_status snn_serve_submit(snn_server *srv, const uint8_t *image_host, uint64_t id, uint32_t T,
                                       uint64_t *req_id)
{
    if (!srv || !image_host || !req_id) return snn_net::error(SNN_EINVAL, "NULL argument");
    if (T == 0) return snn_net::error(SNN_EINVAL, "T must be > 0");
    if (srv->cap == 0) return snn_net::error(SNN_ENOMEM, "hbm_budget holds no serving slot");
    Request r;
    r.id = id;
    r.T = T;
    r.t_submit = now_s();
    r.image.assign(image_host, image_host + srv->n_in);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return snn_net::error(SNN_ESTATE, srv->worker_status != SNN_OK ? "server stopped after a device error"
                                                                                     : "server is shutting down");
        r.req_id = srv->next_req++;
        *req_id = r.req_id;
        srv->queue.push_back(std::move(r));
    }
    srv->cv.notify_one();
    return SNN_OK;
}

extern "C" snn_status snn_serve_poll(snn_server *srv, uint64_t req_id, uint32_t *counts_host, double *latency_s)
{
    if (!srv) return snn_net::error(SNN_EINVAL, "srv is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->done.find(req_id);
    if (it != srv->done.end()) {
        if (counts_host) std::memcpy(counts_host, it->second.counts.data(), it->second.counts.size() * 4);
        if (latency_s) *latency_s = it->second.latency;
        srv->done.erase(it);
        return SNN_OK;
    }
    if (srv->worker_status != SNN_OK) return snn_net::error(srv->worker_status, "server stopped after a device error");
    if (req_id == 0 || req_id >= srv->next_req) return snn_net::error(SNN_ENOTFOUND, "unknown request id");
    if (srv->retiring.count(req_id)) return SNN_EAGAIN;
    for (const Slot &s : srv->slots)
        if (s.active && s.req_id == req_id) return SNN_EAGAIN;
    for (const Request &r : srv->queue)
        if (r.req_id == req_id) return SNN_EAGAIN;
    return snn_net::error(SNN_ENOTFOUND, "request already returned");
}

extern "C" snn_status snn_serve_stats(snn_server *srv, uint64_t *completed, uint64_t *slot_steps,
                                      uint32_t *peak_active, double *busy_s)
{
    if (!srv) return snn_net::error(SNN_EINVAL, "srv is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (completed) *completed = srv->completed;
    if (slot_steps) *slot_steps = srv->slot_steps;
    if (peak_active) *peak_active = srv->peak_active;
    if (busy_s) *busy_s = srv->busy_s;
    return SNN_OK;
}

extern "C" snn_status snn_serve_destroy(snn_server *srv)
{
    if (!srv) return snn_net::error(SNN_EINVAL, "srv is NULL");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_one();
    if (srv->worker.joinable()) srv->worker.join();
    const snn_status st = srv->worker_status;
    delete srv;
    return st;
}
