// snn_autotune.hip -- choice of the execution path for SNN_PATH_AUTO.
//
// The candidates are the paths whose kernels fit the batch (persistent:
// cooperative launch with every task's state in registers; fused: the
// weight block and post traces fit in LDS; MFMA: matrix-core current and
// STDP; plain: always).  The first AUTO run of
// a given network shape, batch size and precision times each candidate on a
// scratch copy of the network (same weights, thresholds and inputs, so the
// spike activity is representative) for a short warm-up and one timed
// episode, keeps the fastest in a process-wide table, and appends it to the
// file named by SNN_AUTOTUNE_CACHE if set (lines "key path").
// SNN_AUTOTUNE=0 skips the measurement and takes the first available path in
// the order persistent, fused, MFMA, plain; SNN_AUTOTUNE_VERBOSE=1 reports
// each candidate's time on stderr.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/snn.h"
#include "snn_runtime.h"

namespace {

std::mutex g_mu;
std::map<std::string, int> g_table;
bool g_loaded = false;

void load_file_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *fn = std::getenv("SNN_AUTOTUNE_CACHE");
    if (!fn) return;
    std::ifstream f(fn);
    std::string key;
    int path;
    while (f >> key >> path)
        if (path >= 0 && path <= 4 && path != SNN_PATH_AUTO) g_table[key] = path;
}

void append_file(const std::string &key, int path)
{
    const char *fn = std::getenv("SNN_AUTOTUNE_CACHE");
    if (!fn) return;
    std::ofstream f(fn, std::ios::app);
    f << key << ' ' << path << '\n';
}

}  // namespace

int snn_net::choose_path(uint32_t batch, uint32_t T, const uint8_t *images, const uint64_t *ids,
                         const uint32_t *forced)
{
    std::vector<int> cand;
    if (persist_ok()) cand.push_back(SNN_PATH_PERSISTENT);
    if (fused_ok()) cand.push_back(SNN_PATH_FUSED);
    cand.push_back(SNN_PATH_MFMA);
    cand.push_back(SNN_PATH_PLAIN);
    const char *env = std::getenv("SNN_AUTOTUNE");
    const char *venv = std::getenv("SNN_AUTOTUNE_VERBOSE");
    const bool verbose = venv && venv[0] == '1';
    if (cand.size() == 1 || (env && env[0] == '0')) return cand[0];

    std::ostringstream ks;
    ks << cfg.n_in << 'x' << cfg.n_exc << 'x' << cfg.n_inh << "_l" << cfg.learn << "_r" << cfg.reduce << "_p"
       << precision << "_jb" << p.jb << "_B" << batch << "_T" << (T < 512u ? T : 512u) << "_g" << use_graphs
       << "_cu" << cus;
    const std::string key = ks.str();
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_file_locked();
        auto it = g_table.find(key);
        if (it != g_table.end())
            for (int c : cand)
                if (c == it->second) return c;
    }

    // time each candidate on a scratch copy
    snn_config c = cfg;
    c.max_batch = batch;
    c.hbm_budget_bytes = 0;
    c.path = SNN_PATH_PLAIN;
    c.precision = precision;
    snn_net *tmp = nullptr;
    int best = cand[0];
    if (snn_create(&c, stream, &tmp) == SNN_OK && tmp->p.jb == p.jb) {
        tmp->use_graphs = use_graphs;
        const size_t nw = (size_t)p.n_in_pad * p.n_pad;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        bool ok = hipMemcpyAsync(tmp->W, W, nw * sizeof(float), hipMemcpyDeviceToDevice, stream) == hipSuccess &&
                  hipMemcpyAsync(tmp->theta, theta, (size_t)p.n_pad * sizeof(double), hipMemcpyDeviceToDevice,
                                 stream) == hipSuccess &&
                  hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
        // a short warm-up (code loading, LDS limits), then one episode of
        // the requested length (at most 512 steps) from a reset, so the
        // bursty first steps weigh as much as they will in the real run
        const uint32_t warm = T < 8u ? T : 8u;
        const uint32_t steps = T < 512u ? T : 512u;
        float best_ms = 1e30f;
        for (int cnd : cand) {
            if (!ok) break;
            // every candidate starts from the caller's weights and thresholds
            ok = hipMemcpyAsync(tmp->W, W, nw * sizeof(float), hipMemcpyDeviceToDevice, stream) == hipSuccess &&
                 hipMemcpyAsync(tmp->theta, theta, (size_t)p.n_pad * sizeof(double), hipMemcpyDeviceToDevice,
                                stream) == hipSuccess;
            if (!ok) break;
            tmp->path = cnd;
            if (tmp->run(images, ids, forced, batch, warm, SNN_RUN_RESET, nullptr) != SNN_OK) continue;
            // with graph replay on, the timed episode replays a captured graph
            if (tmp->use_graphs && tmp->run(images, ids, forced, batch, steps, SNN_RUN_RESET, nullptr) != SNN_OK)
                continue;
            if (hipEventRecord(e0, stream) != hipSuccess) break;
            if (tmp->run(images, ids, forced, batch, steps, SNN_RUN_RESET, nullptr) != SNN_OK) continue;
            float ms = 0.f;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                break;
            if (tmp->check_device_error() != SNN_OK) continue;
            if (verbose)
                std::fprintf(stderr, "snn autotune %s: path %d (ran %d) %.3f ms for %u steps\n", key.c_str(), cnd,
                             tmp->last_path, ms, steps);
            if (ms < best_ms) {
                best_ms = ms;
                best = cnd;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
    snn_destroy(tmp);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table[key] = best;
    }
    append_file(key, best);
    return best;
}
