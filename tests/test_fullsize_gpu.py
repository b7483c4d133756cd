"""GPU parity at the full benchmark size: 784 -> 6400/6400, B = 256, stroke
images at 10-30 % density, the launch configuration the benchmark times.

With learning, the shared weights couple the samples, so the oracle runs the
whole batch over the whole 350-step trial (one persistent launch on the GPU):
the early burst of excitatory spikes, where the batch-reduced updates are
largest, and the later regime of grown thresholds.  Voltages are recorded for
the first 30 steps (the oracle continues the same run without them; a
continuing run equals one long run, which the oracle pins show).  The
weights of a column depend only on that column's spikes (its post traces,
its potentiation terms, its normalisation sum) and on the exact input spikes,
so every column whose excitatory raster agrees in every sample and step is
held to the weight bar, and so is its threshold, even if other columns
diverged.  At the first step where a raster differs, every differing neuron
must be an oracle near-tie: the side that did not fire ends the step within
1e-3 mV of its threshold.

Without learning the samples are independent: the GPU runs the whole batch
and the oracle a sample of it (the encoder is keyed by sample id and step, not
by batch position), over 100 steps.
"""
import numpy as np
import pytest

from paper_1909_02549_amd import inputs
from test_parity_gpu import (COL_AGREE, RASTER_AGREE, W_ATOL, W_RTOL, check_voltages, first_divergence,  # noqa: F401
                             torch_cuda)

pytestmark = pytest.mark.gpu


def full_inputs():
    wl = inputs.workload("dc6400")
    B = wl["B"]
    imgs = inputs.stroke_images(B, 1234, wl["density"])
    ids = inputs.sample_ids(B)
    W = inputs.uniform_weights(784, wl["cfg"]["n_exc"], wl["wlo"], wl["whi"], 0)
    return wl, imgs, ids, W


LEARN_T = 350
V_STEPS = 30


@pytest.fixture(scope="module")
def learning_oracle(oracle_mod):
    wl, imgs, ids, W = full_inputs()
    orc = oracle_mod.OracleNet(wl["cfg"], W.astype(np.float64))
    first = orc.run(imgs, ids, V_STEPS, record=("in", "exc", "inh", "v_exc", "theta"))
    rest = orc.run(imgs, ids, LEARN_T - V_STEPS, reset=False, record=("in", "exc", "inh", "counts", "theta"))
    ref = {k: np.concatenate([first[k], rest[k]], axis=1) for k in ("in", "exc", "inh")}
    ref["v_exc"] = first["v_exc"]
    ref["theta_t"] = np.concatenate([first["theta"], rest["theta"]], axis=0)
    ref["W"] = orc.W
    ref["theta"] = orc.theta
    return ref


def gpu_learning_run(torch, path):
    from paper_1909_02549_amd.snn import Net, unpack_bits
    wl, imgs, ids, W = full_inputs()
    cfg = wl["cfg"]
    net = Net(cfg, max_batch=len(ids), path=path)
    net.snn_set_weights(W)
    out = net.snn_run(torch.from_numpy(imgs).cuda(), torch.from_numpy(ids.astype(np.int64)).cuda(), LEARN_T,
                      record=("in", "exc", "inh", "v_exc", "counts"))
    torch.cuda.synchronize()
    g = {"in": unpack_bits(out["in"].cpu().numpy(), cfg["n_in"]).transpose(1, 0, 2),
         "exc": unpack_bits(out["exc"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2),
         "inh": unpack_bits(out["inh"].cpu().numpy(), cfg["n_inh"]).transpose(1, 0, 2),
         "v_exc": out["v_exc"][:V_STEPS].cpu().numpy().transpose(1, 0, 2),
         "counts": out["counts"].cpu().numpy().astype(np.int64),
         "W": net.snn_get_weights(), "theta": net.snn_get_theta(), "path": net.snn_last_path()}
    del out
    net.close()
    return g


def check_near_ties(g, ref, t, cfg):
    """At step t (the first with a differing raster entry, t < V_STEPS) every
    differing excitatory neuron is a near-tie: the side that did not fire ended
    the step within 1e-3 mV of its threshold v_th + theta (the oracle's
    theta after step t-1's update, decayed once)."""
    beta = np.exp(-cfg["dt_ms"] / cfg["exc"]["tau_theta_ms"])
    th_prev = ref["theta_t"][t - 1] if t > 0 else np.zeros(cfg["n_exc"])
    thr = cfg["exc"]["v_thresh"] + th_prev * beta
    b, j = np.nonzero(g["exc"][:, t] != ref["exc"][:, t])
    for bb, jj in zip(b, j):
        v = ref["v_exc"][bb, t, jj] if g["exc"][bb, t, jj] else g["v_exc"][bb, t, jj]
        assert abs(v - thr[jj]) < 1e-3, f"step {t}, sample {bb}, neuron {jj}: v {v} vs threshold {thr[jj]}"


@pytest.mark.parametrize("path", ["auto", "fused", "persistent", "mfma"])
def test_dc6400_learning_full_trial(torch_cuda, learning_oracle, path):
    wl = inputs.workload("dc6400")
    g, ref = gpu_learning_run(torch_cuda, path), learning_oracle
    if path != "auto":
        assert g["path"] == path
    assert np.array_equal(g["in"], ref["in"]), "input spikes not bit-exact"
    assert ref["exc"][:, :20].sum() > 10000, "no burst of excitatory spikes"
    for k in ("exc", "inh"):
        agree = (g[k] == ref[k]).mean()
        assert agree >= RASTER_AGREE, f"{k} raster agreement {agree}"
    t_div = first_divergence(g, ref)
    tv = min(t_div, V_STEPS)
    if tv > 0:
        check_voltages(g["v_exc"][:, :tv], ref["v_exc"][:, :tv], f"before step {tv}: ")
    if t_div < V_STEPS:
        check_near_ties(g, ref, t_div, wl["cfg"])
    same = (g["exc"] == ref["exc"]).all(axis=(0, 1))
    print(f"dc6400 {path}: first divergence at step {t_div}, {same.mean():.4f} of the columns agree "
          f"in all {LEARN_T} steps, exc spikes gpu {int(g['exc'].sum())} oracle {int(ref['exc'].sum())}", flush=True)
    assert same.mean() >= COL_AGREE, f"only {same.mean():.3f} of the columns agree in every entry"
    err = np.abs(g["W"][:, same] - ref["W"][:, same])
    bad = err > W_RTOL * np.abs(ref["W"][:, same]) + W_ATOL
    assert not bad.any(), f"weights of agreeing columns: max err {err.max()}"
    np.testing.assert_allclose(g["theta"][same], ref["theta"][same], rtol=1e-6, atol=1e-12)
    rows = (g["exc"] == ref["exc"]).all(axis=(1, 2))
    assert np.array_equal(g["counts"][rows], ref["exc"][rows].sum(axis=1).astype(np.int64))


@pytest.mark.parametrize("path", ["auto", "fused", "persistent", "mfma"])
def test_dc6400_inference_sampled(torch_cuda, oracle_mod, path):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net, unpack_bits
    wl, imgs, ids, W = full_inputs()
    cfg = inputs.dc_config(wl["cfg"]["n_exc"], learn=False)
    Wn = inputs.frozen_weights(784, wl["cfg"]["n_exc"], 78.4, 0)
    T = 100
    B = len(ids)
    net = Net(cfg, max_batch=B, path=path)
    net.snn_set_weights(Wn)
    out = net.snn_run(torch.from_numpy(imgs).cuda(), torch.from_numpy(ids.astype(np.int64)).cuda(), T,
                      record=("exc", "inh", "v_exc", "counts"))
    torch.cuda.synchronize()
    if path != "auto":
        assert net.snn_last_path() == path
    gexc = unpack_bits(out["exc"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2)
    ginh = unpack_bits(out["inh"].cpu().numpy(), cfg["n_inh"]).transpose(1, 0, 2)
    gv = out["v_exc"].cpu().numpy().transpose(1, 0, 2)
    gcounts = out["counts"].cpu().numpy()
    net.close()
    sel = np.array([0, 1, 37, 128, 200, 255])
    orc = oracle_mod.OracleNet(cfg, Wn.astype(np.float64))
    ref = orc.run(imgs[sel], ids[sel], T, record=("exc", "inh", "v_exc", "counts"))
    assert ref["exc"].sum() > 100
    agree = (gexc[sel] == ref["exc"]).mean()
    assert agree >= RASTER_AGREE, f"exc raster agreement {agree}"
    for r, b in enumerate(sel):
        d = np.nonzero((gexc[b] != ref["exc"][r]).any(axis=1) | (ginh[b] != ref["inh"][r]).any(axis=1))[0]
        t_div = int(d[0]) if len(d) else T
        check_voltages(gv[b, :t_div], ref["v_exc"][r, :t_div], f"sample {b}: ")
        if t_div == T:
            assert np.array_equal(gcounts[b], ref["counts"][r]), f"sample {b}: spike counts differ"
