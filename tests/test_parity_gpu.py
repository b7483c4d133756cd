"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (FP32 path): input spikes bit-exact; exc/inh rasters agree on at least
99.9 % of (sample, step, neuron) entries; voltages within 1e-3 mV up to the
first raster divergence, or 4e-6 |v| where that is larger (|v| above 250
mV: summed inhibition adds terms of thousands of mV in one step, and FP32
resolves such sums to a few 1e-4 mV; at -1e4 mV one ulp of v is 1e-3 mV);
weights within 1e-4 relative (1e-6 absolute near zero) and theta within 1e-6
relative on every column whose excitatory raster agrees with the oracle in
every sample and step, which must be at least 90 % of the columns.  A
column's weights and threshold depend only on its own spikes, its post
traces and the (bit-exact) input spikes, so agreeing columns are held to the
bar even after another column's spikes diverged.  Samples whose excitatory
rasters agree everywhere have equal spike counts.
"""
import numpy as np
import pytest

from paper_1909_02549_amd import inputs
from paper_1909_02549_amd.inputs import dc_config, sample_ids, stroke_images, uniform_weights

pytestmark = pytest.mark.gpu

RASTER_AGREE = 0.999
V_TOL = 1e-3
V_REL = 4e-6
W_RTOL, W_ATOL = 1e-4, 1e-6
COL_AGREE = 0.9


def v_bar(vr):
    """Voltage bar at oracle voltage vr: 1e-3 mV, or 4e-6 |v| (about 34 FP32
    ulps of v) where that is larger, i.e. for |v| above 250 mV."""
    return np.maximum(V_TOL, V_REL * np.abs(np.asarray(vr, np.float64)))


def check_voltages(gv, vr, what=""):
    dv = np.abs(gv - vr)
    bad = dv > v_bar(vr)
    if bad.any():
        q = np.argmax(np.where(bad, dv, -1.0))
        raise AssertionError(f"{what}voltage error {dv.flat[q]} mV at v={vr.flat[q]} mV")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def run_both(torch, oracle_mod, cfg, W, imgs, ids, T, path="plain", record=("in", "exc", "inh", "v_exc", "counts"),
             reduce=None, forced=None, precision="fp32", oracle_precision=None, before=None):
    """Run the HIP path and the oracle on the same inputs.  The oracle takes
    the same operand form as the GPU unless ``oracle_precision`` says
    otherwise; ``before(net)``, if given, is called on the handle before the
    run.  Returns (gpu, oracle, path the GPU ran)."""
    from paper_1909_02549_amd.snn import Net, pack_bits, unpack_bits
    B = len(ids)
    net = Net(cfg, max_batch=B, path=path, precision=precision)
    net.snn_set_weights(W)
    if before is not None:
        before(net)
    if forced is not None:
        bits = pack_bits(forced.transpose(1, 0, 2))  # T, B, words
        out = net.snn_run_spikes(to_dev(torch, bits.view(np.int32)), T, record=record)
    else:
        out = net.snn_run(to_dev(torch, imgs) if imgs is not None else None,
                          to_dev(torch, ids.astype(np.int64)), T, record=record)
    torch.cuda.synchronize()
    g = {}
    n_in, n_exc = cfg["n_in"], cfg["n_exc"]
    for k, v in out.items():
        a = v.cpu().numpy()
        if k == "in":
            g[k] = unpack_bits(a, n_in).transpose(1, 0, 2)
        elif k in ("exc", "inh"):
            g[k] = unpack_bits(a, n_exc).transpose(1, 0, 2)
        elif k in ("v_exc", "v_inh"):
            g[k] = a.transpose(1, 0, 2)
        else:
            g[k] = a.astype(np.int64)
    g["W"] = net.snn_get_weights()
    g["theta"] = net.snn_get_theta()
    g["path"] = net.snn_last_path()
    net.close()
    orc = oracle_mod.OracleNet(cfg, W.astype(np.float64),
                               precision=precision if oracle_precision is None else oracle_precision)
    ref = orc.run(imgs, ids, T, forced_in=forced, record=tuple(record))
    ref["W"] = orc.W
    ref["theta"] = orc.theta
    return g, ref


def first_divergence(g, ref):
    """First step at which any exc or inh raster entry differs (T if none)."""
    T = ref["exc"].shape[1]
    diff = (g["exc"] != ref["exc"]).any(axis=(0, 2))
    if "inh" in g and "inh" in ref:
        diff |= (g["inh"] != ref["inh"]).any(axis=(0, 2))
    idx = np.nonzero(diff)[0]
    return int(idx[0]) if len(idx) else T


def check_parity(g, ref, learn=True, min_cols=COL_AGREE):
    """Every bar of the module docstring; returns the first divergence step."""
    assert np.array_equal(g["in"], ref["in"]), "input spikes not bit-exact"
    agree_e = (g["exc"] == ref["exc"]).mean()
    assert agree_e >= RASTER_AGREE, f"exc raster agreement {agree_e}"
    if "inh" in g:
        agree_i = (g["inh"] == ref["inh"]).mean()
        assert agree_i >= RASTER_AGREE, f"inh raster agreement {agree_i}"
    t_div = first_divergence(g, ref)
    if "v_exc" in g and t_div > 0:
        check_voltages(g["v_exc"][:, :t_div], ref["v_exc"][:, :t_div], f"before step {t_div}: ")
    if "counts" in g and "counts" in ref:
        rows = (g["exc"] == ref["exc"]).all(axis=(1, 2))
        assert np.array_equal(g["counts"][rows], ref["counts"][rows].astype(np.int64)), "spike counts differ"
    if learn:
        same = (g["exc"] == ref["exc"]).all(axis=(0, 1))
        assert same.mean() >= min_cols, f"only {same.mean():.3f} of the columns agree in every entry"
        err = np.abs(g["W"][:, same] - ref["W"][:, same])
        bad = err > W_RTOL * np.abs(ref["W"][:, same]) + W_ATOL
        assert not bad.any(), f"weights of agreeing columns: max err {err.max()}"
        np.testing.assert_allclose(g["theta"][same], ref["theta"][same], rtol=1e-6, atol=1e-12)
    return t_div


PATHS = ["plain", "fused", "persistent", "mfma"]


@pytest.mark.parametrize("path", PATHS)
def test_dc100_learning_parity(torch_cuda, oracle_mod, path):
    """784 -> 100/100 Diehl & Cook net, B=4, T=100, STDP with mean reduction."""
    w = inputs.workload("dc100")
    cfg = w["cfg"]
    imgs = stroke_images(4, 0, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 0)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(4), 100, path=path)
    assert ref["exc"].sum() > 50
    check_parity(g, ref)
    assert g["path"] == path


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("reduce", ["sum", "max"])
def test_reductions_parity(torch_cuda, oracle_mod, reduce, path):
    cfg = dc_config(100, reduce=reduce)
    imgs = stroke_images(8, 3, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 1)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(8, 10), 60, path=path)
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS + ["auto"])
def test_signed_max_reduction_parity(torch_cuda, oracle_mod, path):
    """Signed max (the largest per-sample change) through the first burst of
    excitatory spikes, on every path (the MFMA route's plasticity is the
    plain gather kernel).  The learned weights follow the signed max, not the
    per-term max, wherever the two differ."""
    cfg = dc_config(100, reduce="max_signed")
    imgs = stroke_images(16, 3, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 1)
    T = 14
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(16, 10), T, path=path)
    assert g["path"] == path or path == "auto"
    assert ref["exc"].sum() > 100
    t_div = check_parity(g, ref)
    assert t_div == T, f"rasters diverged at step {t_div}: weights not compared"
    orc = oracle_mod.OracleNet(dc_config(100, reduce="max"), W.astype(np.float64))
    orc.run(imgs, sample_ids(16, 10), T, record=())
    diff = np.abs(orc.W - ref["W"]) > 1e-5
    assert diff.sum() > 100
    assert (np.abs(g["W"] - ref["W"])[diff] < 0.5 * np.abs(orc.W - ref["W"])[diff]).all()


@pytest.mark.parametrize("path", PATHS + ["auto"])
@pytest.mark.parametrize("tau", [0.03, 0.3, 3.0])
def test_soft_max_reduction_parity(torch_cuda, oracle_mod, tau, path):
    """The soft maximum (log-mean-exp with temperature tau, between the mean
    and the max) on every path, 60 steps of B = 8 through the first bursts.
    At tau = 0.03 it is close to the max reduction, at 3 close to the mean;
    the weights differ from both wherever several samples fire."""
    cfg = dc_config(100, reduce="soft_max", reduce_tau=tau)
    imgs = stroke_images(8, 3, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 1)
    ids = sample_ids(8, 10)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, ids, 60, path=path)
    assert g["path"] == path or path == "auto"
    assert ref["exc"].sum() > 50
    check_parity(g, ref)
    for other in ("mean", "max"):
        orc = oracle_mod.OracleNet(dc_config(100, reduce=other), W.astype(np.float64))
        orc.run(imgs, ids, 60, record=())
        assert np.abs(orc.W - ref["W"]).max() > 1e-4


def test_soft_max_selected_through_the_abi(torch_cuda, oracle_mod):
    """snn_stdp_reduce_soft on a handle created with the mean reduction:
    the next run uses the soft maximum at the new temperature; a temperature
    below the bound is refused and leaves the handle as it was."""
    from paper_1909_02549_amd.snn import SnnError
    cfg = dc_config(100)
    soft = dict(cfg, reduce=4, reduce_tau=0.2)
    imgs = stroke_images(8, 5, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 2)

    def select(net):
        with pytest.raises(SnnError):
            net.snn_stdp_reduce_soft(1e-3)
        net.snn_stdp_reduce_soft(0.2)
    g, _ = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(8, 40), 40, path="persistent",
                    before=select)
    orc = oracle_mod.OracleNet(soft, W.astype(np.float64))
    ref = orc.run(imgs, sample_ids(8, 40), 40, record=("in", "exc", "inh", "v_exc", "counts"))
    ref["W"], ref["theta"] = orc.W, orc.theta
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS + ["auto"])
def test_per_run_normalisation_parity(torch_cuda, oracle_mod, path):
    """Columns normalised once, after the run's last step (the cheaper
    variant), on every path.  Two runs in a row, the second continuing the
    first, so that each call normalises at its own end."""
    from paper_1909_02549_amd.snn import Net
    cfg = dc_config(100, norm_per_run=1)
    imgs = stroke_images(8, 4, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 5)
    ids = sample_ids(8, 30)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, ids, 40, path=path)
    assert path == "auto" or g["path"] == path
    assert ref["exc"].sum() > 50
    check_parity(g, ref)
    np.testing.assert_allclose(g["W"].astype(np.float64).sum(axis=0), 78.4, rtol=1e-5)
    # continuing: a second call of 10 steps on the same handle and oracle,
    # which normalises at its own end
    gc, rc = continuing_pair(torch_cuda, oracle_mod, cfg, W, imgs, ids, path, 40, 10)
    for g_, r_ in zip(gc, rc):
        check_parity(g_, r_)
    np.testing.assert_allclose(gc[1]["W"].astype(np.float64).sum(axis=0), 78.4, rtol=1e-5)


def continuing_pair(torch, oracle_mod, cfg, W, imgs, ids, path, T1, T2, precision="fp32"):
    """An episodic call of T1 steps, then a continuing call (no reset) of T2
    steps on the same handle, and the same two calls on one oracle; returns
    ([gpu1, gpu2], [ref1, ref2]) with each call's records and the weights and
    thresholds after it."""
    from paper_1909_02549_amd.snn import Net, unpack_bits
    B = len(ids)
    net = Net(cfg, max_batch=B, path=path, precision=precision)
    net.snn_set_weights(W)
    d_imgs, d_ids = to_dev(torch, imgs), to_dev(torch, ids.astype(np.int64))
    orc = oracle_mod.OracleNet(cfg, W.astype(np.float64), precision=precision)
    rec = ("in", "exc", "inh", "v_exc", "counts")
    gs, rs = [], []
    for T, reset in ((T1, True), (T2, False)):
        out = net.snn_run(d_imgs, d_ids, T, reset=reset, record=rec)
        torch.cuda.synchronize()
        g = {"in": unpack_bits(out["in"].cpu().numpy(), cfg["n_in"]).transpose(1, 0, 2),
             "exc": unpack_bits(out["exc"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2),
             "inh": unpack_bits(out["inh"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2),
             "v_exc": out["v_exc"].cpu().numpy().transpose(1, 0, 2),
             "counts": out["counts"].cpu().numpy().astype(np.int64),
             "W": net.snn_get_weights(), "theta": net.snn_get_theta(), "path": net.snn_last_path()}
        r = orc.run(imgs, ids, T, reset=reset, record=rec)
        r["W"], r["theta"] = orc.W.copy(), orc.theta.copy()
        gs.append(g)
        rs.append(r)
    net.close()
    return gs, rs


def call_sequence(torch, oracle_mod, cfg, W, max_batch, path, ops, precision="fp32"):
    """Calls on one handle and, in step, on one oracle: ("run", imgs, ids, T,
    reset) or ("rebatch", keep, batch).  Returns ([gpu], [ref]) with each
    run's records and the weights and thresholds after it."""
    from paper_1909_02549_amd.snn import Net, unpack_bits
    net = Net(cfg, max_batch=max_batch, path=path, precision=precision)
    net.snn_set_weights(W)
    orc = oracle_mod.OracleNet(cfg, W.astype(np.float64), precision=precision)
    rec = ("in", "exc", "inh", "v_exc", "counts")
    gs, rs = [], []
    for op in ops:
        if op[0] == "rebatch":
            net.snn_rebatch(op[1], op[2])
            orc.rebatch(op[1], op[2])
            continue
        _, imgs, ids, T, reset = op
        out = net.snn_run(to_dev(torch, imgs), to_dev(torch, ids.astype(np.int64)), T, reset=reset, record=rec)
        torch.cuda.synchronize()
        g = {"in": unpack_bits(out["in"].cpu().numpy(), cfg["n_in"]).transpose(1, 0, 2),
             "exc": unpack_bits(out["exc"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2),
             "inh": unpack_bits(out["inh"].cpu().numpy(), cfg["n_exc"]).transpose(1, 0, 2),
             "v_exc": out["v_exc"].cpu().numpy().transpose(1, 0, 2),
             "counts": out["counts"].cpu().numpy().astype(np.int64),
             "W": net.snn_get_weights(), "theta": net.snn_get_theta(), "path": net.snn_last_path()}
        r = orc.run(imgs, ids, T, reset=reset, record=rec)
        r["W"], r["theta"] = orc.W.copy(), orc.theta.copy()
        gs.append(g)
        rs.append(r)
    net.close()
    return gs, rs


@pytest.mark.parametrize("path", PATHS + ["auto"])
def test_rebatch_parity(torch_cuda, oracle_mod, path):
    """Continuing across re-formed batches (snn_rebatch): 8 samples for 30
    steps; samples 5, 2 and 7 kept as slots 0-2 with three new samples, 30
    steps; then all six kept in a new order with six more (12 slots, above
    the capacity the handle had allocated), 20 steps.  Kept samples continue
    their input streams at their own local steps, new ones start at step 0.
    Every call meets the parity bars against the oracle doing the same."""
    cfg = dc_config(100)
    W = uniform_weights(784, 100, 0.0, 0.3, 11)
    imgs8, ids8 = stroke_images(8, 31, 0.19), sample_ids(8, 300)
    new3, nid3 = stroke_images(3, 32, 0.19), sample_ids(3, 400)
    imgs6 = np.concatenate([imgs8[[5, 2, 7]], new3])
    ids6 = np.concatenate([ids8[[5, 2, 7]], nid3])
    order = [4, 0, 5, 1, 3, 2]
    new6, nid6 = stroke_images(6, 33, 0.19), sample_ids(6, 500)
    imgs12 = np.concatenate([imgs6[order], new6])
    ids12 = np.concatenate([ids6[order], nid6])
    ops = [("run", imgs8, ids8, 30, True), ("rebatch", [5, 2, 7], 6), ("run", imgs6, ids6, 30, False),
           ("rebatch", order, 12), ("run", imgs12, ids12, 20, False)]
    gs, rs = call_sequence(torch_cuda, oracle_mod, cfg, W, 12, path, ops)
    for g, r in zip(gs, rs):
        assert g["path"] == path or path == "auto"
        check_parity(g, r)
    assert rs[1]["exc"].sum() > 20 and rs[2]["exc"].sum() > 20


@pytest.mark.parametrize("path", PATHS)
def test_rebatch_keeps_samples_independent(torch_cuda, path):
    """Learning off, so samples do not interact: after snn_rebatch each kept
    sample's spikes and voltages continue exactly as in the original batch,
    bit for bit, and a new sample's equal its own episodic run."""
    from paper_1909_02549_amd.snn import Net, unpack_bits
    cfg = dc_config(100, learn=False)
    W = uniform_weights(784, 100, 0.0, 0.3, 12)
    imgs, ids = stroke_images(6, 34, 0.19), sample_ids(6, 600)
    new, nid = stroke_images(1, 35, 0.19), sample_ids(1, 700)
    rec = ("exc", "v_exc")

    def run(net, im, i, T, reset):
        out = net.snn_run(to_dev(torch_cuda, im), to_dev(torch_cuda, i.astype(np.int64)), T, reset=reset,
                          record=rec)
        torch_cuda.cuda.synchronize()
        return (unpack_bits(out["exc"].cpu().numpy(), 100).transpose(1, 0, 2),
                out["v_exc"].cpu().numpy().transpose(1, 0, 2))
    a = Net(cfg, max_batch=8, path=path)
    a.snn_set_weights(W)
    run(a, imgs, ids, 25, True)
    ea, va = run(a, imgs, ids, 25, False)
    b = Net(cfg, max_batch=8, path=path)
    b.snn_set_weights(W)
    run(b, imgs, ids, 25, True)
    b.snn_rebatch([4, 1], 3)
    eb, vb = run(b, np.concatenate([imgs[[4, 1]], new]), np.concatenate([ids[[4, 1]], nid]), 25, False)
    c = Net(cfg, max_batch=8, path=path)
    c.snn_set_weights(W)
    ec, vc = run(c, new, nid, 25, True)
    assert np.array_equal(eb[0], ea[4]) and np.array_equal(eb[1], ea[1]) and np.array_equal(eb[2], ec[0])
    assert np.array_equal(vb[0], va[4]) and np.array_equal(vb[1], va[1]) and np.array_equal(vb[2], vc[0])
    assert ea[[1, 4]].sum() > 0
    for n in (a, b, c):
        n.close()


def test_rebatch_errors(torch_cuda):
    from paper_1909_02549_amd.snn import Net, SnnError
    cfg = dc_config(100)
    net = Net(cfg, max_batch=8)
    net.snn_set_weights(uniform_weights(784, 100, 0.0, 0.3, 13))
    with pytest.raises(SnnError):
        net.snn_rebatch([0], 4)                  # no samples yet
    net.snn_rebatch([], 4)                       # a fresh batch of 4
    imgs, ids = stroke_images(4, 36, 0.19), sample_ids(4, 800)
    net.snn_run(to_dev(torch_cuda, imgs), to_dev(torch_cuda, ids.astype(np.int64)), 5, reset=False)
    for keep, B in (([4], 4), ([1, 1], 4), ([0, 1, 2], 2), ([0], 0)):
        with pytest.raises(SnnError) as e:
            net.snn_rebatch(keep, B)
        assert e.value.status == -1
    with pytest.raises(SnnError) as e:
        net.snn_rebatch([0], 9)
    assert e.value.status == -2
    net.snn_rebatch([3, 0], 2)                   # still usable after the refusals
    net.snn_run(to_dev(torch_cuda, imgs[[3, 0]]), to_dev(torch_cuda, ids[[3, 0]].astype(np.int64)), 5, reset=False)
    net.snn_sync()
    net.close()


@pytest.mark.parametrize("path", PATHS)
def test_continuing_run_parity(torch_cuda, oracle_mod, path):
    """Continuing simulation (Episodic vs. continuing simulation section): a
    40-step episode, then 10 more steps without a reset, every-step
    normalisation.  The second call starts from the first call's voltages,
    refractory counts, traces and previous spikes, and its encoder continues
    at local step 40; both calls meet every parity bar."""
    cfg = dc_config(100)
    imgs = stroke_images(8, 14, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 15)
    gs, rs = continuing_pair(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(8, 130), path, 40, 10)
    assert gs[1]["path"] == path
    assert rs[1]["exc"].sum() > 5
    for g, r in zip(gs, rs):
        check_parity(g, r)
    assert first_divergence(gs[0], rs[0]) == 40, "first call diverged: continuation not tested"


@pytest.mark.parametrize("path", ["fused", "persistent"])
def test_per_run_normalisation_across_chunks(torch_cuda, oracle_mod, path):
    """A run longer than one encoder chunk (512 steps, two persistent
    launches): the columns are normalised after the run's last step only, not
    at the end of the first chunk."""
    cfg = dc_config(100, norm_per_run=1)
    imgs = stroke_images(4, 6, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 8)
    T = 520
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(4, 40), T, path=path)
    assert g["path"] == path
    assert ref["exc"].sum() > 50
    t_div = check_parity(g, ref)
    assert t_div > 512, f"rasters diverged at step {t_div}, before the chunk boundary"
    np.testing.assert_allclose(g["W"].astype(np.float64).sum(axis=0), 78.4, rtol=1e-5)


@pytest.mark.parametrize("path", PATHS)
def test_run_errors_leave_the_handle_usable(torch_cuda, oracle_mod, path):
    """Invalid calls return an error without touching the state: a run on the
    same handle afterwards still matches the oracle from the initial state."""
    from paper_1909_02549_amd.snn import SnnError
    torch = torch_cuda
    cfg = dc_config(100)
    imgs = stroke_images(4, 2, 0.19)
    ids = sample_ids(4, 50)
    W = uniform_weights(784, 100, 0.0, 0.3, 2)
    d_imgs, d_ids = to_dev(torch, imgs), to_dev(torch, ids.astype(np.int64))

    def invalid_calls(net):
        with pytest.raises(SnnError, match="EINVAL"):
            net.snn_run(d_imgs, d_ids, 0)
        with pytest.raises(SnnError, match="ENOMEM"):  # more samples than max_batch
            net.snn_run(to_dev(torch, stroke_images(5, 2, 0.19)), to_dev(torch, sample_ids(5).astype(np.int64)), 10)
        assert net.lib.snn_run(net.h, d_imgs.data_ptr(), None, 4, 10, 1, None) == -1  # no sample ids
        assert net.lib.snn_run(net.h, None, d_ids.data_ptr(), 4, 10, 1, None) == -1  # no images, no uniform rate
        assert net.lib.snn_run(net.h, d_imgs.data_ptr(), d_ids.data_ptr(), 0, 10, 1, None) == -1
        assert net.lib.snn_run_spikes(net.h, None, 4, 10, 1, None) == -1

    g, ref = run_both(torch, oracle_mod, cfg, W, imgs, ids, 40, path=path, before=invalid_calls)
    assert ref["exc"].sum() > 20
    assert check_parity(g, ref) == 40
    assert np.array_equal(g["counts"], ref["counts"].astype(np.int64))


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("level", [0, 255])
def test_blank_and_saturated_images(torch_cuda, oracle_mod, path, level):
    """Degenerate inputs with learning on: blank images give no input or
    output spike, so the weights change only by the per-step normalisation;
    saturated images drive every input at the highest rate (B = 3, ragged
    batch word)."""
    cfg = dc_config(100)
    imgs = np.full((3, 784), level, np.uint8)
    W = uniform_weights(784, 100, 0.0, 0.3, 3)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(3, 60), 30, path=path)
    if level == 0:
        assert ref["in"].sum() == 0 and ref["exc"].sum() == 0
    else:
        assert ref["in"].mean() > 0.03
    assert check_parity(g, ref) == 30
    assert np.array_equal(g["counts"], ref["counts"].astype(np.int64))


@pytest.mark.parametrize("path", PATHS)
def test_ragged_batch_and_inputs(torch_cuda, oracle_mod, path):
    """B = 70 (two 64-sample tiles, three 32-sample words), n_in = 50
    (ragged input word), n_exc = 37 (ragged column block)."""
    cfg = dc_config(37, n_in=50)
    rng = np.random.default_rng(0)
    imgs = (rng.random((70, 50)) < 0.5) * rng.integers(1, 256, (70, 50))
    imgs = imgs.astype(np.uint8)
    W = uniform_weights(50, 37, 0.0, 1.5, 2)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(70, 5), 40, path=path)
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS)
def test_no_learning_scaling_net(torch_cuda, oracle_mod, path):
    """Uniform 20 Hz inputs -> LIF layer without inhibition or learning."""
    cfg = inputs.scaling_config(n_in=200, n_out=150)
    W = inputs.normal_weights(200, 150, 0.5, 0.2, 0)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, sample_ids(16), 120, path=path,
                      record=("in", "exc", "v_exc", "counts"))
    assert ref["exc"].sum() > 100
    check_parity(g, ref, learn=False)


@pytest.mark.parametrize("path", PATHS)
def test_forced_stdp_pairs(torch_cuda, oracle_mod, path):
    """Forced input rasters through snn_run_spikes: pre/post pairs at several
    offsets in different samples, compared with the oracle."""
    cfg = dc_config(1, n_in=2, reduce="sum", norm=0.0, w_max=100.0, exc=dict(adaptive=0))
    cfg["n_inh"] = 0
    T = 40
    deltas = [-7, -3, -1, 0, 1, 2, 5, 12]
    forced = np.zeros((len(deltas), T, 2), np.uint8)
    for b, d in enumerate(deltas):
        t_pre = 10 if d >= 0 else 10 - d
        forced[b, t_pre, 0] = 1
        forced[b, t_pre + d, 1] = 1
    W = np.array([[0.5], [20.0]], np.float32)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, sample_ids(len(deltas)), T, path=path,
                      forced=forced, record=("in", "exc", "v_exc"))
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS)
def test_long_run_crosses_encoder_chunks(torch_cuda, oracle_mod, path):
    """T = 300 > 256 steps per encoder chunk: the chunk boundary (next-step
    inputs for the presynaptic traces) is seamless."""
    cfg = dc_config(40)
    imgs = stroke_images(3, 21, 0.25)
    W = uniform_weights(784, 40, 0.0, 0.3, 4)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(3, 77), 300, path=path)
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS)
def test_batch_equals_separate_runs_bit_exact(torch_cuda, path):
    """Learning off: a batch of 8 gives each sample exactly the spikes and
    voltages it gets when run alone (every sample's arithmetic is its own;
    the encoder is keyed by sample id, not by batch slot)."""
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net
    cfg = dc_config(100, learn=False)
    imgs = stroke_images(8, 31, 0.19)
    ids = sample_ids(8, 900)
    W = inputs.frozen_weights(784, 100, 78.4, 6)
    T = 60
    net = Net(cfg, max_batch=8, path=path)
    net.snn_set_weights(W)
    full = net.snn_run(to_dev(torch, imgs), to_dev(torch, ids.astype(np.int64)), T, record=("exc", "v_exc"))
    torch.cuda.synchronize()
    fe, fv = full["exc"].cpu().numpy(), full["v_exc"].cpu().numpy()
    assert net.snn_last_path() == path
    assert fe.any()
    for b in range(8):
        one = net.snn_run(to_dev(torch, imgs[b:b + 1]), to_dev(torch, ids[b:b + 1].astype(np.int64)), T,
                          record=("exc", "v_exc"))
        torch.cuda.synchronize()
        assert np.array_equal(one["exc"].cpu().numpy()[:, 0], fe[:, b]), f"sample {b}: spikes differ"
        assert np.array_equal(one["v_exc"].cpu().numpy()[:, 0], fv[:, b]), f"sample {b}: voltages differ"
    net.close()


@pytest.mark.parametrize("path", PATHS)
def test_additive_traces_parity(torch_cuda, oracle_mod, path):
    """Additive traces (x <- lam x + 1 on a spike, the flag of the trace
    form): a learning run of the 784 -> 100/100 network, B = 8, on every
    path.  Pre traces exceed 1 where inputs fire in consecutive steps."""
    cfg = dc_config(100, trace_additive=1)
    imgs = stroke_images(8, 17, 0.19)
    W = uniform_weights(784, 100, 0.0, 0.3, 16)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(8, 160), 80, path=path)
    assert g["path"] == path
    assert ref["exc"].sum() > 50
    # the additive form changes the result: the nearest-spike run differs
    orc = oracle_mod.OracleNet(dc_config(100), W.astype(np.float64))
    orc.run(imgs, sample_ids(8, 160), 80, record=())
    assert np.abs(orc.W - ref["W"]).max() > 1e-4
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS)
def test_additive_forced_spike_trains(torch_cuda, oracle_mod, path):
    """Additive traces from forced trains of several pre and post spikes per
    sample (the closed forms the oracle is pinned to), through
    snn_run_spikes: input 0 is the plastic synapse, input 1 (weight 20)
    drives the neuron."""
    cfg = dc_config(1, n_in=2, reduce="sum", norm=0.0, w_max=100.0, exc=dict(adaptive=0), trace_additive=1)
    cfg["n_inh"] = 0
    T = 40
    trains = [([4, 9], [15]), ([22], [4, 13]), ([6, 11], [11]), ([3, 4, 5, 6], [7, 20, 30]),
              ([10, 20, 30], [12, 25]), ([1], [1])]
    forced = np.zeros((len(trains), T, 2), np.uint8)
    for b, (pre, post) in enumerate(trains):
        forced[b, pre, 0] = 1
        forced[b, post, 1] = 1
    W = np.array([[0.5], [20.0]], np.float32)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, sample_ids(len(trains)), T, path=path,
                      forced=forced, record=("in", "exc", "v_exc"))
    assert ref["exc"].sum() == sum(len(p) for _, p in trains)
    check_parity(g, ref)
