#!/usr/bin/env python3
"""Throughput benchmark of the minibatched SNN hot path on one MI355X.

One bench step is one episodic trial of the whole hot path: ``snn_run`` of
B = 256 samples for T = 350 clock steps of the 784 -> 6400/6400 Diehl & Cook
style network with STDP on (Poisson encoding, contraction, inhibition, neuron
updates, traces, batch-reduced weight change, clamp, column normalisation,
threshold update).  Inputs (images, ids, weights) are resident in HBM before
the timed region.  value = B * T * steps / elapsed seconds (sample-steps/s).

Also reported on the same JSON line:
  plain_path    the same workload on the plain per-step launch path;
  roofline      the dominant kernel's algorithmic bytes per launch divided by
                its average launch time, measured with HIP events recorded on
                the library's stream during the timed region;
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
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


def dims(cfg, B):
    n_in = cfg["n_in"]
    n_in_pad = 32 * ((n_in + 31) // 32)
    return dict(n_in=n_in, n_in_pad=n_in_pad, n_exc=cfg["n_exc"], B=B,
                in_words=n_in_pad // 32, bwords=(B + 31) // 32, learn=cfg["learn"], has_inh=cfg["n_inh"] > 0)


def algorithmic_bytes(kernel: str, d: dict, steps_per_launch: int = 1) -> float | None:
    """HBM bytes one launch of `kernel` must move at minimum (read + write),
    per the per-unit figures in the design notes.  None if not modelled."""
    n_in, n_in_pad, N, B = d["n_in"], d["n_in_pad"], d["n_exc"], d["B"]
    w = n_in * N * 4                     # FP32 weights, one pass
    st_exc = 4 + 2 + (4 if d["learn"] else 0)     # v_exc, packed rf/flags, x_post
    st_inh = 4 if d["has_inh"] else 0             # v_inh
    state = B * N * (st_exc + st_inh)             # one pass over per-neuron state
    bits = B * d["in_words"] * 4 + n_in_pad * d["bwords"] * 4
    xpre = B * n_in_pad * 4
    if kernel == "plastic":
        return 2 * w + B * N * (4 + 2) + bits
    if kernel == "neuron":
        return 2 * state + B * N * 4
    if kernel == "contract":
        return B * N * 4 + bits
    if kernel == "xpre":
        return 2 * xpre
    if kernel == "fused_step":
        return 2 * w + 2 * state + (2 * xpre if d["learn"] else 0) + 2 * bits
    if kernel == "encode":
        return steps_per_launch * 2 * bits + B * n_in
    return None


def cpu_baseline(wl, imgs, ids, W, target_s: float = 15.0) -> dict:
    """Time the FP64 oracle (test infrastructure) on the first steps of one
    trial of the same workload."""
    from oracle.oracle import OracleNet
    from oracle import build as obuild
    from oracle import oracle as omod
    if not os.path.exists(omod.LIB_PATH):
        obuild.build()
    cfg, B = wl["cfg"], wl["B"]
    net = OracleNet(cfg, W.astype(np.float64))
    t0 = time.perf_counter()
    net.run(imgs, ids, 1, record=())
    t1 = time.perf_counter() - t0
    steps = int(max(2, min(wl["T"], target_s / max(t1, 1e-3))))
    net = OracleNet(cfg, W.astype(np.float64))
    t0 = time.perf_counter()
    net.run(imgs, ids, steps, record=())
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": B * steps / el, "unit": "sample·steps/s", "cores": cores, "kind": "oracle",
            "sample": f"first {steps} of the {wl['T']} steps of one B={B} trial, FP64, {el:.1f} s"}


def time_path(net, imgs_d, ids_d, T, steps, warmup, profile=False):
    import torch
    for _ in range(warmup):
        net.snn_run(imgs_d, ids_d, T, reset=True, record=())
    torch.cuda.synchronize()
    if profile:
        net.snn_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.snn_run(imgs_d, ids_d, T, reset=True, record=())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = net.snn_profile_get() if profile else {}
    if profile:
        net.snn_profile_enable(False)
    return el, prof


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed trials (one trial = T clock steps)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dc6400")
    ap.add_argument("--path", default="plain", choices=["plain", "fused", "persistent", "auto"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp8"])
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-path comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a device copy of this many MiB (profiler calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1909_02549_amd import inputs
    from paper_1909_02549_amd.snn import Net

    wl = inputs.workload(args.workload)
    cfg, B, T = wl["cfg"], wl["B"], wl["T"]
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
    value = B * T * args.steps / el

    d = dims(cfg, B)
    roof = None
    if prof:
        kname, (launches, total_ms) = max(prof.items(), key=lambda kv: kv[1][1])
        per = algorithmic_bytes(kname, d)
        avg_s = total_ms / 1e3 / max(launches, 1)
        if per is not None:
            achieved = per / avg_s / 1e9
            roof = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "bytes_per_launch": per, "avg_launch_us": avg_s * 1e6, "launches": launches,
                    "share_of_gpu_time": total_ms / sum(v[1] for v in prof.values())}
    net.close()

    plain = None
    if not args.no_plain and args.path != "plain":
        pnet = Net(cfg, max_batch=B, path="plain", precision="fp32")
        pnet.snn_set_weights(W)
        pel, _ = time_path(pnet, imgs_d, ids_d, T, max(1, args.steps // 2), 1)
        plain = {"value": B * T * max(1, args.steps // 2) / pel,
                 "ms_per_step": pel * 1e3 / max(1, args.steps // 2)}
        pnet.close()

    cpu = None if args.no_cpu else cpu_baseline(wl, imgs, ids, W)

    line = {
        "metric": METRIC, "value": value, "unit": "sample·steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp8": "fp8"}[args.precision], "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['n_in']}->{cfg['n_exc']}/{cfg['n_inh']} Diehl&Cook, "
                               f"B={B}, T={T}, STDP {'on' if cfg['learn'] else 'off'}, reduce="
                               f"{['sum', 'mean', 'max'][cfg['reduce']]}",
                   "global_batch": B, "seq_len": T, "parallelism": "single-gpu", "path": args.path,
                   "precision": args.precision},
        "roofline": roof, "cpu_baseline": cpu, "plain_path": plain,
        "kernels": {k: {"launches": v[0], "avg_us": v[1] * 1e3 / max(v[0], 1)} for k, v in prof.items()},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
