// snn_graph.hip -- replay of repeated episodic runs from captured HIP graphs.
//
// An episodic run (SNN_RUN_RESET) on the per-step paths is a fixed sequence
// of launches: state reset, output clearing, then per chunk of steps the
// encoder (and for the fused path the sparse lists) followed by the step
// kernels.  With the same batch, duration, buffers and settings every
// argument of every launch repeats, so the sequence is captured once into a
// HIP graph and later runs replay it with one launch, which removes the host
// launch cost (a few microseconds per kernel, four or more kernels per step)
// that dominates small batches.  The capture records nothing but kernel
// launches (buffers are cleared by fill kernels, never by memset nodes).
// On the persistent path the captured episode is the fill kernels, the
// encoder, the spike lists and orders, the first presynaptic traces and
// one persistent launch per chunk (an ordinary kernel node, its arguments
// by value).
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "../../include/snn.h"
#include "snn_runtime.h"

using namespace snn;

namespace {

template <class T>
void put(std::string &k, const T &v)
{
    k.append(reinterpret_cast<const char *>(&v), sizeof v);
}

}  // namespace

void snn_net::graphs_invalidate()
{
    for (auto &e : graphs) (void)hipGraphExecDestroy(e.second.exec);
    graphs.clear();
}

snn_status snn_net::run_graph(int path, const uint8_t *images, const uint64_t *ids, const uint32_t *forced,
                              uint32_t batch, uint32_t T, const Outs &o)
{
    std::string key;
    put(key, path);
    put(key, batch);
    put(key, T);
    put(key, images);
    put(key, ids);
    put(key, forced);
    put(key, o);
    put(key, p.reduce);
    put(key, p.prec);
    put(key, p.Bs);
    put(key, chunk);
    auto it = graphs.find(key);
    if (it == graphs.end()) {
        if (graphs.size() >= kMaxGraphs) graphs_invalidate();
        if (!cap_stream && hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking) != hipSuccess)
            return error(SNN_EDEVICE, "hipStreamCreateWithFlags failed");
        hipStream_t user = stream;
        stream = cap_stream;
        if (hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
            stream = user;
            return error(SNN_EDEVICE, "hipStreamBeginCapture failed");
        }
        capturing = true;
        snn_status st = episode(path, images, ids, forced, batch, T, o);
        capturing = false;
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(cap_stream, &g);
        stream = user;
        if (st != SNN_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (ec != hipSuccess || !g) return error(SNN_EDEVICE, "hipStreamEndCapture failed");
        Graph gr;
        const hipError_t ei = hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return error(SNN_EDEVICE, "hipGraphInstantiate failed");
        gr.last_path = last_path;
        it = graphs.emplace(key, gr).first;
    }
    if (hipGraphLaunch(it->second.exec, stream) != hipSuccess) return error(SNN_EDEVICE, "hipGraphLaunch failed");
    // host-side counters as the captured episode leaves them
    cur_B = batch;
    gstep = T;
    tloc = T;
    last_path = it->second.last_path;
    return SNN_OK;
}

extern "C" snn_status snn_set_graphs(snn_net *net, int32_t on)
{
    if (!net) return snn_net::error(SNN_EINVAL, "net is NULL");
    if (on != 0 && on != 1) return snn_net::error(SNN_EINVAL, "on must be 0 or 1");
    net->use_graphs = on != 0;
    if (!net->use_graphs) net->graphs_invalidate();
    return SNN_OK;
}
