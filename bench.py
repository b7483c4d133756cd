#!/usr/bin/env python3
"""Throughput benchmark of the minibatched SNN hot path on one MI355X.

One bench step is one episodic trial of the whole hot path: ``snn_run`` of
B = 256 samples for T = 350 clock steps of the 784 -> 6400/6400 Diehl & Cook
style network with STDP on (Poisson encoding, contraction, inhibition, neuron
updates, traces, batch-reduced weight change, clamp, column normalisation,
threshold update, spike-count readout), on the execution path the library's
autotuner picks.  Inputs (images, ids, weights) and the readout buffer are
resident in HBM before the timed region.  value = B * T * steps / elapsed
seconds (sample-steps/s) over the timed trials (default: 3 warm-up trials,
then 10 timed ones); `ms_per_step` is the time of one bench step (a trial),
also given as `ms_per_trial`, and `us_per_clock_step` divides it by T;
`trials` adds the median and the mean +- std of the per-trial times (HIP
events between the trials).

Also reported on the same JSON line:
  paths         the same workload on each execution path (plain per-step
                launches, fused per-step kernel, persistent kernel);
  roofline      the dominant kernel's roofline from its average launch time
                (HIP events on the library's stream over the timed region).
                For the step kernels it uses the per-step bytes of the whole
                learning step (step_bytes: weights, per-neuron state and
                presynaptic traces read and written, 88.5 MB) times the steps
                one launch runs, against the 8 TB/s HBM peak.  The step's
                dense-equivalent flops against the BF16 matrix-core peak
                (step_model) and the kernel's own models (its HBM bytes, its
                sparse vector operations against the 157.3 TFLOP/s vector
                peak) are kept beside it as context;
  serving       frozen 784 -> 1600 network, Poisson arrivals, T in
                {100, 250, 500}: p50 / p99 latency and sample-steps/s at
                5000 requests/s, and (`sweep`) at 2000, 10000 and 20000;
  conversion    the converted 784-256-128-10 IF network (ANN to SNN
                conversion section) at B = 1024 and B = 1, T = 10;
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sample·steps/s (784→6400 D&C, B=256) vs plain path; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1909_02549_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def dims(cfg, B, imgs=None):
    """Sizes of a workload; s_in is the expected number of input spikes per
    step over the batch (rate pixel / 255 x max_rate, or the uniform rate)."""
    n_in = cfg["n_in"]
    n_in_pad = 32 * ((n_in + 31) // 32)
    p = cfg["max_rate_hz"] * cfg["dt_ms"] * 1e-3
    if imgs is not None:
        s_in = float(np.minimum(imgs.astype(np.float64) / 255.0 * p, 1.0).sum())
    else:
        s_in = B * n_in * min(p, 1.0)
    return dict(n_in=n_in, n_in_pad=n_in_pad, n_exc=cfg["n_exc"], B=B, in_words=n_in_pad // 32,
                bwords=(B + 31) // 32, learn=cfg["learn"], has_inh=cfg["n_inh"] > 0, s_in=s_in)


def algorithmic_bytes(kernel: str, d: dict, steps_per_launch: float = 1.0):
    """HBM bytes one launch of `kernel` has to move (read + write), from the
    per-unit figures of the design notes.  None if not modelled."""
    n_in, n_in_pad, N, B = d["n_in"], d["n_in_pad"], d["n_exc"], d["B"]
    w = n_in * N * 4                                   # FP32 weights, one pass
    st = B * N * (4 + 2 + (4 if d["learn"] else 0) + (4 if d["has_inh"] else 0))  # per-neuron state, one pass
    spikes = B * d["in_words"] * 4 + n_in_pad * d["bwords"] * 4  # one step's input spikes, both layouts
    xpre = B * n_in_pad * 4 if d["learn"] else 0        # presynaptic traces of one step
    if kernel == "fused_step":
        return 2 * w * (1 if d["learn"] else 0.5) + 2 * st + 2 * xpre + spikes
    if kernel == "persistent":
        return (2 * w if d["learn"] else w) + 2 * st + steps_per_launch * (2 * xpre + spikes)
    if kernel == "plastic":
        return 2 * w + B * N * (4 + 2) + spikes
    if kernel == "neuron":
        return 2 * st + B * N * 4
    if kernel == "contract":
        return B * N * 4 + spikes
    if kernel == "xpre":
        return 2 * xpre + spikes
    if kernel == "mfma_front":
        return w + 2 * st + 2 * xpre + B * d["in_words"] * 4
    if kernel == "mfma_plastic":
        return 2 * w + B * N * (4 + 2) + B * n_in_pad * 4 + n_in_pad * d["bwords"] * 4
    if kernel == "encode":
        return steps_per_launch * 2 * spikes + B * n_in
    return None


MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp8": 5000.0}
# vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed FP32) x 2.4 GHz
VALU_PEAK_TFLOPS = 157.3
# algorithmic vector operations per unit of the gather kernels (FP32
# equivalents; an FP64 add counts 2, an FMA 2, a compare or min/max 1)
ALU_PER_SPIKE_COL = 1      # contraction: one add per (input spike, column)
ALU_PER_SPIKE_COL_D = 1    # depression sums: one add per (input spike, column)
ALU_PER_NEURON = 11        # exc: decay FMA, input add, inhibition FMA, threshold; inh: decay FMA, add,
                           # threshold; post trace multiply
ALU_PER_WEIGHT = 7         # scale multiply, depression FMA, clamp (2), FP64 column-sum add (2)
# matrix-core operations per algorithmic product: the FP32 form multiplies
# three bfloat16 parts of each operand value
MFMA_PLANES = {"fp32": 3, "bf16": 1, "fp8": 1}


def algorithmic_flops(kernel: str, d: dict):
    """Dense-equivalent flops of one launch of a matrix-core kernel: the
    synaptic current B x n_in x N, the STDP terms P and D as two outer
    products over the batch (the potentiation K is compacted to the samples
    that fired, so fewer products actually run)."""
    if kernel == "mfma_front":
        return 2.0 * d["B"] * d["n_in"] * d["n_exc"]
    if kernel == "mfma_plastic":
        return 4.0 * d["B"] * d["n_in"] * d["n_exc"]
    return None


def alu_ops(kernel: str, d: dict, steps_per_launch: float = 1.0):
    """Algorithmic vector operations of one launch of the gather kernels
    (one step for the fused kernel, a chunk for the persistent one)."""
    if kernel not in ("fused_step", "persistent"):
        return None
    N = d["n_exc"]
    per_step = ALU_PER_SPIKE_COL * d["s_in"] * N + ALU_PER_NEURON * d["B"] * N
    if d["learn"]:
        per_step += ALU_PER_SPIKE_COL_D * d["s_in"] * N + ALU_PER_WEIGHT * d["n_in"] * N
    return per_step * steps_per_launch


def step_bytes(d: dict) -> float:
    """HBM bytes of one learning step of the whole path for a design that
    keeps weights and per-neuron state in HBM: the FP32 weights read and
    written (2 x n_in_pad x N x 4), the per-neuron state read and written
    (v_exc, v_inh, x_post 4 B each, refractory 2 B), the presynaptic traces
    read and written.  88.5 MB for 784 -> 6400 at B = 256."""
    B, n, N = d["B"], d["n_in_pad"], d["n_exc"]
    return 2.0 * n * N * 4 + 2.0 * B * N * 14 + 2.0 * B * n * 4


def step_flops(d: dict) -> float:
    """Dense-equivalent flops of one learning step: the synaptic contraction
    and the two STDP outer products over the batch, 3 x 2 x B x n_in_pad x N.
    7.86 GFLOP for 784 -> 6400 at B = 256."""
    return 6.0 * d["B"] * d["n_in_pad"] * d["n_exc"]


def kernel_roofline(kname: str, d: dict, precision: str, launches: int, total_ms: float, spl: float):
    """Roofline entry of one kernel from its live HIP-event timing: HBM
    fraction from the algorithmic bytes, and for the matrix-core kernels the
    MFMA fraction from the dense-equivalent flops; `bound` is the resource
    with the larger fraction."""
    per = algorithmic_bytes(kname, d, spl)
    if per is None:
        return None
    avg_s = total_ms / 1e3 / max(launches, 1)
    gbs = per / avg_s / 1e9
    r = {"bound": "hbm", "kernel": kname, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": gbs / HBM_PEAK_GBS, "traffic": measured_traffic(kname), "bytes_per_launch": per,
         "avg_launch_us": avg_s * 1e6, "launches": launches, "steps_per_launch": spl}
    fl = algorithmic_flops(kname, d)
    if fl is not None:
        dt = "fp8" if precision == "fp8" else "bf16"
        tf = fl / avg_s / 1e12
        mfrac = tf * MFMA_PLANES[precision] / MFMA_PEAK_TFLOPS[dt]
        r["mfma"] = {"achieved": tf, "peak": MFMA_PEAK_TFLOPS[dt], "unit": "TFLOP/s", "frac": mfrac,
                     "flops_per_launch": fl, "mfma_ops_per_product": MFMA_PLANES[precision], "dtype": dt}
        if mfrac > r["frac"]:
            r.update(bound="mfma", achieved=tf, peak=MFMA_PEAK_TFLOPS[dt], unit="TFLOP/s", frac=mfrac)
    ops = alu_ops(kname, d, spl)
    if ops is not None:
        tf = ops / avg_s / 1e12
        afrac = tf / VALU_PEAK_TFLOPS
        r["alu"] = {"achieved": tf, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": afrac, "ops_per_launch": ops,
                    "hbm_frac": r["frac"]}
        if afrac > r["frac"]:
            r.update(bound="alu", achieved=tf, peak=VALU_PEAK_TFLOPS, unit="TFLOP/s", frac=afrac)
    if kname in ("persistent", "fused_step") and d["learn"]:
        # the per-step figure of the whole learning step (88.5 MB at 784 ->
        # 6400, B = 256: weights, per-neuron state and presynaptic traces read
        # and written) times the steps one launch runs, against the 8 TB/s HBM
        # peak, for both step kernels; the dense-equivalent flops of the step
        # (contraction and both STDP outer products) against the BF16
        # matrix-core peak are kept as context under step_model
        sb, sf = step_bytes(d) * spl, step_flops(d) * spl
        hb, mf = sb / avg_s / 1e9, sf / avg_s / 1e12
        dt = "fp8" if precision == "fp8" else "bf16"
        model = {"bytes_per_step": step_bytes(d), "bytes_per_launch": sb, "hbm_achieved": hb,
                 "hbm_frac": hb / HBM_PEAK_GBS, "flops_per_launch": sf, "mfma_achieved": mf,
                 "mfma_peak": MFMA_PEAK_TFLOPS[dt], "mfma_frac": mf / MFMA_PEAK_TFLOPS[dt]}
        r["kernel_model"] = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
        r["step_model"] = model
        r.update(bound="hbm", achieved=hb, peak=HBM_PEAK_GBS, unit="GB/s", frac=hb / HBM_PEAK_GBS,
                 algorithmic_bytes_per_launch=sb)
    return r


def measured_traffic(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    only if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, imgs, ids, W, target_s: float = 15.0, single_s: float = 6.0) -> dict:
    """Time the FP64 oracle (test infrastructure) on the first steps of one
    trial of the same workload: with all host threads, then single-threaded
    on fewer steps."""
    from oracle import build as obuild
    from oracle import oracle as omod
    if not os.path.exists(omod.LIB_PATH):
        obuild.build()
    cfg, B = wl["cfg"], wl["B"]
    lib = omod.lib()
    cores = int(lib.orc_threads())
    net = omod.OracleNet(cfg, W.astype(np.float64))
    t0 = time.perf_counter()
    net.run(imgs, ids, 2, record=())
    t1 = (time.perf_counter() - t0) / 2
    steps = int(max(2, min(wl["T"], target_s / max(t1, 1e-3))))
    net = omod.OracleNet(cfg, W.astype(np.float64))
    t0 = time.perf_counter()
    net.run(imgs, ids, steps, record=())
    el = time.perf_counter() - t0
    res = {"value": B * steps / el, "unit": "sample·steps/s", "cores": cores, "kind": "oracle",
           "sample": f"first {steps} of the {wl['T']} steps of one B={B} trial, FP64, {el:.1f} s",
           "cpu": cpu_model()}
    # single-threaded, on as many steps as fit single_s at the measured rate
    s1 = int(max(1, min(steps, single_s / max(el / steps * cores, 1e-3))))
    lib.orc_set_threads(1)
    try:
        net = omod.OracleNet(cfg, W.astype(np.float64))
        t0 = time.perf_counter()
        net.run(imgs, ids, s1, record=())
        e1 = time.perf_counter() - t0
    finally:
        lib.orc_set_threads(cores)
    res["single_thread"] = {"value": B * s1 / e1, "sample": f"first {s1} steps, {e1:.1f} s"}
    return res


def time_path(net, imgs_d, ids_d, T, steps, warmup, profile=False):
    """Wall time of `steps` episodic trials after `warmup` untimed ones; every
    trial records the readout (per-sample excitatory spike counts, into one
    preallocated buffer).  With `profile`, the library brackets each run of
    consecutive launches of one kernel in the timed trials with a pair of HIP
    events on its stream (a few events per trial, none between the launches
    of a run), which gives the per-kernel times of the timed region itself."""
    import torch
    out = net.outputs(int(ids_d.shape[0]), T, ("counts",))
    for _ in range(warmup):
        net.snn_run(imgs_d, ids_d, T, reset=True, out=out)
    torch.cuda.synchronize()
    net.snn_sync()
    if profile:
        net.snn_profile_enable(True)
    # one HIP event between consecutive trials on the handle's stream (torch's
    # current stream when the handle was made) gives the per-trial times
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        net.snn_run(imgs_d, ids_d, T, reset=True, out=out)
        ev[k + 1].record()
    torch.cuda.synchronize()
    net.snn_sync()
    el = time.perf_counter() - t0
    time_path.trial_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    prof = {}
    if profile:
        prof = net.snn_profile_get()
        net.snn_profile_enable(False)
    time_path.spikes = int(out["counts"].sum().item())
    return el, prof


def serving_run(n_req: int, rate_hz: float, max_slots: int, chunk: int) -> dict:
    """Frozen 784 -> 1600/1600 network; requests arrive as a Poisson process
    with T drawn from {100, 250, 500}; continuous batching on the device."""
    from paper_1909_02549_amd import inputs
    from paper_1909_02549_amd.snn import Net, Server
    wl = inputs.workload("serve")
    cfg = wl["cfg"]
    W = inputs.frozen_weights(cfg["n_in"], cfg["n_exc"], 78.4, 0)
    net = Net(cfg, max_batch=1, path="auto")
    net.snn_set_weights(W)
    arrivals = inputs.poisson_arrivals(n_req, rate_hz, seed=1)
    Ts = inputs.request_durations(n_req, seed=1)
    imgs = inputs.stroke_images(n_req, 4242, wl["density"])
    srv = Server(net, max_slots=max_slots, chunk_steps=chunk)
    # warm the server (autotune, first launches)
    w = srv.snn_serve_submit(imgs[0], 10 ** 9, 100)
    while srv.snn_serve_poll(w) is None:
        time.sleep(0.001)
    rids = []
    t0 = time.perf_counter()
    for k in range(n_req):
        while time.perf_counter() - t0 < arrivals[k]:
            pass
        rids.append(srv.snn_serve_submit(imgs[k], k, int(Ts[k])))
    lat = {}
    while len(lat) < n_req:
        for r in rids:
            if r in lat:
                continue
            res = srv.snn_serve_poll(r)
            if res is not None:
                lat[r] = res[1]
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    st = srv.snn_serve_stats()
    srv.snn_serve_destroy()
    net.close()
    lv = np.array(list(lat.values()))
    return {"workload": "784->1600/1600 frozen, T in {100,250,500}, Poisson arrivals",
            "rate_req_s": rate_hz, "requests": n_req, "max_slots": max_slots, "chunk_steps": chunk,
            "p50_ms": float(np.percentile(lv, 50) * 1e3), "p99_ms": float(np.percentile(lv, 99) * 1e3),
            "value": float(Ts.astype(np.float64).sum() / wall), "unit": "sample·steps/s",
            "peak_active": st["peak_active"]}


FP32_MATRIX_PEAK_TFLOPS = 157.3


def measured_peaks() -> dict:
    """What this GPU reaches on plain library work, as context for the
    published peaks the rooflines use: a 1 GiB device-to-device copy (read +
    write bytes) and a 8192^3 bfloat16 matrix product (torch / the vendor
    BLAS), each timed with HIP events over 10 repetitions after 3 warm-ups."""
    import torch
    dev = torch.device("cuda")
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    n = 256 * 2 ** 20
    a = torch.empty(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * n * 4 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    m = 8192
    x = torch.randn(m, m, dtype=torch.bfloat16, device=dev)
    y = torch.randn(m, m, dtype=torch.bfloat16, device=dev)
    for _ in range(3):
        z = torch.matmul(x, y)
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(10):
        z = torch.matmul(x, y)
    e1.record()
    torch.cuda.synchronize()
    gemm_tf = 2.0 * m ** 3 * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del x, y, z
    torch.cuda.empty_cache()
    return {"hbm_copy_gbs": copy_gbs, "hbm_copy_frac_of_peak": copy_gbs / HBM_PEAK_GBS,
            "bf16_gemm_tflops": gemm_tf, "bf16_gemm_frac_of_peak": gemm_tf / MFMA_PEAK_TFLOPS["bf16"]}


def conversion_flops(sizes, B: int, T: int) -> float:
    """Algorithmic flops of one converted-network run: the analog input's
    contraction once, the two spike contractions every step."""
    n_in, h1, h2, n_out = sizes
    return 2.0 * B * (n_in * h1 + T * (h1 * h2 + h2 * n_out))


def conversion_issued_flops(sizes, B: int, T: int) -> float:
    """bfloat16 matrix-core flops one run issues: three weight planes, tiles
    padded to 32 samples x 32 neurons x 16-deep chunks, the output layer
    padded to one 32-wide tile."""
    n_in, h1, h2, n_out = sizes
    pad = lambda n, m: m * ((n + m - 1) // m)  # noqa: E731
    return 3 * 2.0 * pad(B, 32) * (pad(n_in, 16) * pad(h1, 32) + T * (pad(h1, 16) * pad(h2, 32) + pad(h2, 16) * 32))


def conversion_run(runs: int = 200, warmup: int = 10, oracle: bool = True) -> dict:
    """The converted feed-forward IF network of the ANN to SNN conversion
    section: 784-256-128-10, analog input, T = 10, B = 1024 (and B = 1, the
    serial case the paper compares against).  Random weights after data-based
    normalisation, synthetic stroke images.  Times whole runs (both kernels)
    with HIP events on the handle's stream."""
    import torch
    from paper_1909_02549_amd import inputs
    from paper_1909_02549_amd.snn import IFNet
    wl = inputs.workload("conv")
    sizes, T, B = wl["sizes"], wl["T"], wl["B"]
    layers = inputs.conversion_mlp(sizes, wl["seed"])
    imgs = inputs.stroke_images(B, 21, wl["density"])
    imgs_d = torch.from_numpy(imgs).cuda()

    def timed(batch):
        net = IFNet(sizes, wl["thresholds"], max_batch=batch)
        net.set_layers(layers)
        x = imgs_d[:batch].contiguous()
        out = None
        for _ in range(warmup):
            out = net.snn_ifnet_run(x, T, record=("pred",))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(runs):
            net.snn_ifnet_run(x, T, record=("pred",))
        e1.record()
        torch.cuda.synchronize()
        net.close()
        return e0.elapsed_time(e1) / runs, out["pred"].cpu().numpy()

    ms, pred = timed(B)
    ms1, _ = timed(1)
    n_in, h1, h2, n_out = sizes
    flops = conversion_flops(sizes, B, T)
    issued = conversion_issued_flops(sizes, B, T)
    res = {"workload": f"converted IF net {n_in}-{h1}-{h2}-{n_out}, analog input, reset by subtraction, T={T}, "
                       f"B={B}, random weights with data-based normalisation, synthetic stroke images",
           "value": B * T / (ms * 1e-3), "unit": "sample·steps/s", "us_per_batch": ms * 1e3,
           "images_per_s": B / (ms * 1e-3), "test_set_10k_ms": 10000 / (B / ms),
           "b1_us_per_image": ms1 * 1e3, "b1_value": T / (ms1 * 1e-3),
           "batch_speedup_b1024_vs_b1": (B / ms) / (1 / ms1),
           # the paper's own figures for this network on its hardware (10 000
           # test images, T = 10: about 0.75 s at B = 1024, over 11 min at
           # B = 1); context, not a target
           "paper_context": {"b1024_value": 1e5 / 0.75, "b1_value": 1e5 / 660.0,
                             "ratio_b1024": (B * T / (ms * 1e-3)) / (1e5 / 0.75),
                             "ratio_b1": (T / (ms1 * 1e-3)) / (1e5 / 660.0)},
           "roofline": {"bound": "mfma", "achieved": flops / (ms * 1e-3) / 1e12,
                        "peak": FP32_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": flops / (ms * 1e-3) / 1e12 / FP32_MATRIX_PEAK_TFLOPS,
                        "flops_per_run": flops,
                        "issued_bf16_frac": issued / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["bf16"]}}
    if oracle:
        from oracle.ifnet import OracleIFNet
        t0 = time.perf_counter()
        ref = OracleIFNet([(W.astype(np.float64), b.astype(np.float64)) for W, b in layers],
                          wl["thresholds"]).run(imgs, T)
        res["oracle_ms_per_batch"] = (time.perf_counter() - t0) * 1e3
        res["pred_agree_with_oracle"] = float((ref["pred"] == pred).mean())
    return res


SCALE_PATHS = ("plain", "plain+graph", "mfma", "mfma+graph", "fused", "fused+graph", "persistent")


def sweep(name: str, trials: int, batches=None, paths=None) -> dict:
    """Throughput sweeps (not part of the default run):
    scale  1000 uniform 20 Hz inputs -> 1000 LIF, no learning, T=1000, over
           B = 1 .. 4096: per-step launches with and without graph replay,
           the matrix-core route, the fused and the persistent kernel
           (`batches` and `paths`, entries of SCALE_PATHS, select a part);
    dc400  784 -> 400/400, T=250, STDP on, over B = 16 .. 1024, each batch
           reduction and operand precision on the autotuned path;
    serve  the serving workload at 2000, 5000, 10000 and 20000 requests/s
           (`trials` x 1000 requests each)."""
    if name == "serve":
        rows = []
        for rate in (2000.0, 5000.0, 10000.0, 20000.0):
            rows.append(serving_run(1000 * trials, rate, max_slots=1024, chunk=25))
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        return {"name": name, "rows": rows}
    import torch
    from paper_1909_02549_amd import inputs
    from paper_1909_02549_amd.snn import Net, SnnError
    wl = inputs.workload(name)
    cfg, T = wl["cfg"], wl["T"]
    if "wlo" in wl:
        W = inputs.uniform_weights(cfg["n_in"], cfg["n_exc"], wl["wlo"], wl["whi"], 0)
    else:
        W = inputs.normal_weights(cfg["n_in"], cfg["n_exc"], wl["wmean"], wl["wstd"], 0)
    dev = torch.device("cuda:0")
    rows = []

    def one(B, path, graphs=False, reduce=None, precision="fp32"):
        c = dict(cfg)
        if reduce is not None:
            c["reduce"] = {"sum": 0, "mean": 1, "max": 2}[reduce]
        imgs = inputs.stroke_images(B, 99, wl["density"]) if wl["density"] is not None else None
        imgs_d = torch.from_numpy(imgs).to(dev) if imgs is not None else None
        ids_d = torch.from_numpy(inputs.sample_ids(B).astype(np.int64)).to(dev)
        try:
            net = Net(c, max_batch=B, path=path, precision=precision)
        except SnnError as e:
            return {"B": B, "path": path, "error": str(e)}
        net.snn_set_weights(W)
        if graphs:
            net.snn_set_graphs(True)
        el, _ = time_path(net, imgs_d, ids_d, T, trials, 1)
        r = {"B": B, "path": path, "graphs": graphs, "used": net.snn_last_path(), "precision": precision,
             "value": B * T * trials / el, "ms_per_clock_step": el * 1e3 / (T * trials)}
        if reduce is not None:
            r["reduce"] = reduce
        net.close()
        return r

    if name == "scale":
        for B in batches or (1, 8, 64, 512, 4096):
            for entry in paths or SCALE_PATHS:
                path, _, g = entry.partition("+")
                rows.append(one(B, path, g == "graph"))
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    else:
        for B in (16, 64, 256, 1024):
            for reduce in ("sum", "mean", "max"):
                for precision in ("fp32", "bf16", "fp8"):
                    rows.append(one(B, "auto", True, reduce, precision))
                    print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"workload": name, "T": T, "trials": trials, "unit": "sample·steps/s", "rows": rows}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed trials (one trial = T clock steps)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dc6400")
    ap.add_argument("--path", default="auto", choices=["plain", "fused", "persistent", "mfma", "auto"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--norm-per-run", action="store_true",
                    help="normalise the columns once per trial instead of after every step")
    ap.add_argument("--no-paths", action="store_true", help="skip the per-path comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--serve-rate", type=float, default=5000.0)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--no-conversion", action="store_true", help="skip the converted IF network run")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy and GEMM peak measurements")
    ap.add_argument("--conversion-only", action="store_true",
                    help="print only the converted IF network's measurement")
    ap.add_argument("--batches", default=None, help="scale sweep: comma-separated batch sizes")
    ap.add_argument("--sweep-paths", default=None,
                    help="scale sweep: comma-separated entries of " + ",".join(SCALE_PATHS))
    ap.add_argument("--sweep", choices=["scale", "dc400", "serve"], default=None,
                    help="print a throughput sweep instead of the benchmark line")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a device copy of this many MiB (profiler calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (the batch or the columns "
              "would be sharded across GPUs); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.sweep:
        batches = [int(x) for x in args.batches.split(",")] if args.batches else None
        paths = args.sweep_paths.split(",") if args.sweep_paths else None
        if paths and any(x not in SCALE_PATHS for x in paths):
            ap.error("--sweep-paths entries must be among " + ",".join(SCALE_PATHS))
        print(json.dumps({"sweep": sweep(args.sweep, args.steps, batches, paths)}), flush=True)
        return
    if args.conversion_only:
        print(json.dumps({"conversion": conversion_run(oracle=not args.no_cpu)}), flush=True)
        return

    import torch
    from paper_1909_02549_amd import inputs
    from paper_1909_02549_amd.snn import Net

    wl = inputs.workload(args.workload)
    cfg, B, T = wl["cfg"], wl["B"], wl["T"]
    if args.norm_per_run:
        cfg = dict(cfg, norm_per_run=1)
    imgs = inputs.stroke_images(B, 1234, wl["density"]) if wl["density"] is not None else None
    ids = inputs.sample_ids(B)
    if "wlo" in wl:
        W = inputs.uniform_weights(cfg["n_in"], cfg["n_exc"], wl["wlo"], wl["whi"], 0)
    else:
        W = inputs.normal_weights(cfg["n_in"], cfg["n_exc"], wl["wmean"], wl["wstd"], 0)
    dev = torch.device("cuda:0")
    imgs_d = torch.from_numpy(imgs).to(dev) if imgs is not None else None
    ids_d = torch.from_numpy(ids.astype(np.int64)).to(dev)

    if args.copy_probe_mb:
        a = torch.empty(args.copy_probe_mb * 2 ** 20 // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    net = Net(cfg, max_batch=B, path=args.path, precision=args.precision)
    net.snn_set_weights(W)
    el, prof = time_path(net, imgs_d, ids_d, T, args.steps, args.warmup, profile=True)
    trial_ms = np.array(time_path.trial_ms)
    trials = {"n": int(len(trial_ms)), "median_ms": float(np.median(trial_ms)), "mean_ms": float(trial_ms.mean()),
              "std_ms": float(trial_ms.std(ddof=1)) if len(trial_ms) > 1 else 0.0,
              "median_value": B * T / (float(np.median(trial_ms)) * 1e-3), "trial_ms": [float(x) for x in trial_ms]}
    used_path = net.snn_last_path()
    value = B * T * args.steps / el

    d = dims(cfg, B, imgs)
    roof = None
    kroofs = {}
    if prof:
        gpu_ms = sum(v[1] for v in prof.values())
        for kn, (ln, ms) in prof.items():
            kr = kernel_roofline(kn, d, args.precision, ln, ms, T * args.steps / max(ln, 1))
            if kr is not None:
                kr["share_of_gpu_time"] = ms / gpu_ms
                kroofs[kn] = kr
        kname = max(prof.items(), key=lambda kv: kv[1][1])[0]
        roof = kroofs.get(kname)
    net.close()

    paths = {}
    if not args.no_paths:
        for pth in ("plain", "mfma", "fused", "persistent"):
            pnet = Net(cfg, max_batch=B, path=pth, precision=args.precision)
            pnet.snn_set_weights(W)
            n = 1 if pth == "plain" else 2
            pel, pprof = time_path(pnet, imgs_d, ids_d, T, n, 1, profile=True)
            entry = {"value": B * T * n / pel, "ms_per_trial": pel * 1e3 / n, "used": pnet.snn_last_path()}
            entry["kernels"] = {}
            for kn, (ln, ms) in pprof.items():
                kr = kernel_roofline(kn, d, args.precision, ln, ms, T * n / max(ln, 1))
                ke = {"launches": ln, "avg_us": ms * 1e3 / max(ln, 1)}
                if kr is not None:
                    ke["hbm_frac"] = kr["bytes_per_launch"] / (kr["avg_launch_us"] / 1e6) / 1e9 / HBM_PEAK_GBS
                    if "mfma" in kr:
                        ke["mfma_frac"] = kr["mfma"]["frac"]
                    if "alu" in kr:
                        ke["alu_frac"] = kr["alu"]["frac"]
                entry["kernels"][kn] = ke
            paths[pth] = entry
            pnet.close()

    serving = None
    if not args.no_serve:
        serving = serving_run(args.serve_requests, args.serve_rate, max_slots=1024, chunk=25)
        # the other arrival rates, the same number of requests each
        serving["sweep"] = [{k: r[k] for k in ("rate_req_s", "requests", "p50_ms", "p99_ms", "value", "peak_active")}
                            for r in (serving_run(args.serve_requests, rate, max_slots=1024, chunk=25)
                                      for rate in (2000.0, 10000.0, 20000.0))]

    conversion = None if args.no_conversion else conversion_run(oracle=not args.no_cpu)
    peaks = None if args.no_peaks else measured_peaks()

    cpu = None if args.no_cpu else cpu_baseline(dict(wl, cfg=cfg), imgs, ids, W)

    line = {
        "metric": METRIC, "value": value, "unit": "sample·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "bench_step": f"one episodic trial: T={T} clock steps of all B={B} samples, spike-count readout recorded",
        "ms_per_trial": el * 1e3 / args.steps, "us_per_clock_step": el * 1e6 / (args.steps * T),
        "readout_spikes_last_trial": time_path.spikes,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[args.precision], "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['n_in']}->{cfg['n_exc']}/{cfg['n_inh']} Diehl&Cook, "
                               f"B={B}, T={T}, STDP {'on' if cfg['learn'] else 'off'}, reduce="
                               f"{['sum', 'mean', 'max', 'max_signed', 'soft_max'][cfg['reduce']]}"
                               f"{', normalisation per trial' if cfg.get('norm_per_run') else ''}, synthetic stroke images",
                   "global_batch": B, "seq_len": T, "parallelism": "single-gpu", "path": used_path,
                   "precision": args.precision},
        "trials": trials, "roofline": roof, "cpu_baseline": cpu, "paths": paths, "serving": serving,
        "conversion": conversion, "measured_peaks": peaks,
        "vs_plain_path": (value / paths["plain"]["value"]) if "plain" in paths else None,
        "kernels": {k: {"launches": v[0], "avg_us": v[1] * 1e3 / max(v[0], 1),
                        **({"roofline": kroofs[k]} if k in kroofs else {})} for k, v in prof.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
