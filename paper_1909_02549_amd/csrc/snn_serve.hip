// snn_serve.hip -- continuous-batching inference server (host side).
//
// Single-sample requests (the Dynamic minibatch size section's one-at-a-time
// queries) are admitted into free slots of a device-resident batch of a
// frozen network whenever a slot is free; the active slots advance together
// in chunks of steps; a request leaves when its own T is reached and its spike
// counts are copied out.  Slots are independent simulations (no learning, the
// inhibition is per sample) and the encoder is keyed by (seed, sample id,
// local step of the slot), so a request's counts do not depend on which other
// requests share the batch or on its slot.
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
#include <vector>

#include "../../include/snn.h"
#include "snn_dev.h"
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

}  // namespace

struct snn_server {
    snn_net *net = nullptr;   // internal copy of the frozen network
    hipStream_t stream = nullptr;  // the server's own stream (default priority)
    uint32_t cap = 0;         // slots that fit max_slots and the HBM budget
    uint32_t chunk = 1;
    uint32_t n_in = 0, n_exc = 0;

    uint8_t *img_d = nullptr;
    uint64_t *ids_d = nullptr;
    uint32_t *tl_d = nullptr, *counts_d = nullptr;
    uint8_t *mask_d = nullptr;
    uint8_t *img_h = nullptr, *mask_h = nullptr;  // pinned staging
    uint64_t *ids_h = nullptr;
    uint32_t *counts_h = nullptr;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> queue;
    std::unordered_map<uint64_t, Result> done;
    std::vector<Slot> slots;
    uint64_t next_req = 1;
    bool stop = false;
    snn_status worker_status = SNN_OK;
    std::thread worker;

    uint64_t completed = 0, slot_steps = 0;
    uint32_t peak_active = 0;
    double busy_s = 0.0;

    void loop();
    ~snn_server();
};

snn_server::~snn_server()
{
    (void)hipFree(img_d);
    (void)hipFree(ids_d);
    (void)hipFree(tl_d);
    (void)hipFree(counts_d);
    (void)hipFree(mask_d);
    if (img_h) (void)hipHostFree(img_h);
    if (mask_h) (void)hipHostFree(mask_h);
    if (ids_h) (void)hipHostFree(ids_h);
    if (counts_h) (void)hipHostFree(counts_h);
    snn_destroy(net);
    if (stream) (void)hipStreamDestroy(stream);
}

void snn_server::loop()
{
    std::vector<uint32_t> fresh, finishing;
    if (hipSetDevice(net->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        worker_status = SNN_EDEVICE;
        stop = true;
        return;
    }
    for (;;) {
        uint32_t B = 0, steps = 0;
        fresh.clear();
        {
            std::unique_lock<std::mutex> lk(mu);
            // admit queued requests into free slots (lowest index first)
            for (uint32_t s = 0; s < cap && !queue.empty(); ++s) {
                if (slots[s].active) continue;
                Request &r = queue.front();
                std::memcpy(img_h + (size_t)s * n_in, r.image.data(), n_in);
                ids_h[s] = r.id;
                slots[s].active = true;
                slots[s].req_id = r.req_id;
                slots[s].remaining = r.T;
                slots[s].t_submit = r.t_submit;
                fresh.push_back(s);
                queue.pop_front();
            }
            uint32_t active = 0;
            steps = chunk;
            for (uint32_t s = 0; s < cap; ++s)
                if (slots[s].active) {
                    B = s + 1;
                    ++active;
                    steps = std::min(steps, slots[s].remaining);
                }
            peak_active = std::max(peak_active, active);
            if (active == 0) {
                if (stop) return;
                cv.wait_for(lk, std::chrono::milliseconds(1));
                continue;
            }
        }
        const double t0 = now_s();
        hipStream_t st = net->stream;
        snn_status status = SNN_OK;
        for (uint32_t s = 0; s < B; ++s) mask_h[s] = 0;
        for (uint32_t s : fresh) {
            mask_h[s] = 1;
            if (hipMemcpyAsync(img_d + (size_t)s * n_in, img_h + (size_t)s * n_in, n_in, hipMemcpyHostToDevice, st) !=
                    hipSuccess ||
                hipMemcpyAsync(ids_d + s, ids_h + s, sizeof(uint64_t), hipMemcpyHostToDevice, st) != hipSuccess)
                status = SNN_EDEVICE;
        }
        if (!fresh.empty() && hipMemcpyAsync(mask_d, mask_h, B, hipMemcpyHostToDevice, st) != hipSuccess)
            status = SNN_EDEVICE;
        if (status == SNN_OK)
            status = net->serve_steps(img_d, ids_d, tl_d, B, steps, counts_d, fresh.empty() ? nullptr : mask_d);
        finishing.clear();
        {
            std::lock_guard<std::mutex> lk(mu);
            for (uint32_t s = 0; s < B; ++s)
                if (slots[s].active) {
                    slots[s].remaining -= steps;
                    if (slots[s].remaining == 0) finishing.push_back(s);
                }
            slot_steps += (uint64_t)steps * (uint64_t)std::count_if(slots.begin(), slots.begin() + B,
                                                                      [](const Slot &x) { return x.active; });
        }
        for (uint32_t s : finishing)
            if (status == SNN_OK &&
                hipMemcpyAsync(counts_h + (size_t)s * n_exc, counts_d + (size_t)s * n_exc, n_exc * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, st) != hipSuccess)
                status = SNN_EDEVICE;
        if (status == SNN_OK && hipStreamSynchronize(st) != hipSuccess) status = SNN_EDEVICE;
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(mu);
            busy_s += t1 - t0;
            if (status != SNN_OK) {
                worker_status = status;
                stop = true;
                queue.clear();
                for (auto &sl : slots) sl.active = false;
                return;
            }
            for (uint32_t s : finishing) {
                Result r;
                r.counts.assign(counts_h + (size_t)s * n_exc, counts_h + (size_t)(s + 1) * n_exc);
                r.latency = t1 - slots[s].t_submit;
                done.emplace(slots[s].req_id, std::move(r));
                slots[s].active = false;
                ++completed;
            }
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
    H((void **)&sv->img_h, (size_t)nb * c.n_in);
    H((void **)&sv->mask_h, nb);
    H((void **)&sv->ids_h, (size_t)nb * 8);
    H((void **)&sv->counts_h, (size_t)nb * c.n_exc * 4);
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
