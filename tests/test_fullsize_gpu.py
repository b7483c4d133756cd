"""GPU parity at the full benchmark size: 784 -> 6400/6400, B = 256, stroke
images at 10-30 % density, the launch configuration the benchmark times.

With learning, the shared weights couple the samples, so the oracle runs the
whole batch, for the first 20 steps (through the first synchronous burst of
excitatory spikes, where the batch-reduced updates are largest).  The weights
of a column depend only on that column's spikes (its post traces, its
potentiation terms, its normalisation sum) and on the exact input spikes, so
every column whose excitatory raster agrees in every sample and step is held
to the weight bar, and so is its threshold, even if other columns diverged.

Without learning the samples are independent: the GPU runs the whole batch
and the oracle a sample of it (the encoder is keyed by sample id and step, not
by batch position), over 100 steps.
"""
import numpy as np
import pytest

from paper_1909_02549_amd import inputs
from test_parity_gpu import RASTER_AGREE, V_RTOL, V_TOL, W_ATOL, W_RTOL, first_divergence, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def full_inputs():
    wl = inputs.workload("dc6400")
    B = wl["B"]
    imgs = inputs.stroke_images(B, 1234, wl["density"])
    ids = inputs.sample_ids(B)
    W = inputs.uniform_weights(784, wl["cfg"]["n_exc"], wl["wlo"], wl["whi"], 0)
    return wl, imgs, ids, W


LEARN_T = 20


@pytest.fixture(scope="module")
def learning_oracle(oracle_mod):
    wl, imgs, ids, W = full_inputs()
    orc = oracle_mod.OracleNet(wl["cfg"], W.astype(np.float64))
    ref = orc.run(imgs, ids, LEARN_T, record=("in", "exc", "inh", "v_exc"))
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
                      record=("in", "exc", "inh", "v_exc"))
    torch.cuda.synchronize()
    g = {"in": unpack_bits(out["in"].cpu().numpy(), cfg["n_in"]).transpose(1, 0, 2),
         "exc": unpack_bits(out["exc"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2),
         "inh": unpack_bits(out["inh"].cpu().numpy(), cfg["n_inh"]).transpose(1, 0, 2),
         "v_exc": out["v_exc"].cpu().numpy().transpose(1, 0, 2),
         "W": net.snn_get_weights(), "theta": net.snn_get_theta(), "path": net.snn_last_path()}
    net.close()
    return g


@pytest.mark.parametrize("path", ["auto", "fused", "persistent", "mfma"])
def test_dc6400_learning_full_batch(torch_cuda, learning_oracle, path):
    g, ref = gpu_learning_run(torch_cuda, path), learning_oracle
    if path != "auto":
        assert g["path"] == path
    assert np.array_equal(g["in"], ref["in"]), "input spikes not bit-exact"
    assert ref["exc"].sum() > 10000, "no burst of excitatory spikes"
    for k in ("exc", "inh"):
        agree = (g[k] == ref[k]).mean()
        assert agree >= RASTER_AGREE, f"{k} raster agreement {agree}"
    t_div = first_divergence(g, ref)
    if t_div > 0:
        vr = ref["v_exc"][:, :t_div]
        dv = np.abs(g["v_exc"][:, :t_div] - vr)
        assert not (dv > V_TOL + V_RTOL * np.abs(vr)).any(), f"voltage error {dv.max()} mV before step {t_div}"
    same = (g["exc"] == ref["exc"]).all(axis=(0, 1))
    assert same.mean() >= 0.9, f"only {same.mean():.3f} of the columns agree in every entry"
    err = np.abs(g["W"][:, same] - ref["W"][:, same])
    bad = err > W_RTOL * np.abs(ref["W"][:, same]) + W_ATOL
    assert not bad.any(), f"weights of agreeing columns: max err {err.max()}"
    np.testing.assert_allclose(g["theta"][same], ref["theta"][same], rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("path", ["auto", "fused", "persistent", "mfma"])
def test_dc6400_inference_sampled(torch_cuda, oracle_mod, path):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net, unpack_bits
    wl, imgs, ids, W = full_inputs()
    cfg = inputs.dc_config(wl["cfg"]["n_exc"], learn=False)
    Wn = inputs.column_scaled(W, 78.4)
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
        vr = ref["v_exc"][r, :t_div]
        dv = np.abs(gv[b, :t_div] - vr)
        assert not (dv > V_TOL + V_RTOL * np.abs(vr)).any(), f"sample {b}: voltage error {dv.max()} mV"
        if t_div == T:
            assert np.array_equal(gcounts[b], ref["counts"][r]), f"sample {b}: spike counts differ"
