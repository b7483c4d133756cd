"""GPU tests of the chunk kernel for networks whose tasks are independent.

A network without learning and without an inhibitory layer (the batch-scaling
network of the scaling experiment) couples no two neurons: each (sample,
column) evolves from the sample's own input spikes through frozen weights.
The persistent path then runs every step of an encoder chunk in one launch
with no grid barrier, one thread per (sample, 8 columns) task and any number
of workgroups, so it also serves batches too large for the cooperative
kernel.  Its per-step arithmetic is the fused kernel's, so the two agree bit
for bit; against the oracle it meets the usual parity bars.

Shapes: ragged layers (150 columns: the last 8-column group holds 6), column
blocks of 8, 13 and 32 columns, batches that leave the last workgroup of
each column block partly empty, runs that cross an encoder chunk (512
steps), continuing runs, the reduced operand forms, serving, and each
number of columns per lane (small batches spread a task over several
lanes).
"""
import numpy as np
import pytest

from paper_1909_02549_amd import inputs
from paper_1909_02549_amd.inputs import sample_ids
from test_parity_gpu import check_parity, run_both, to_dev, torch_cuda  # noqa: F401
from test_serve_gpu import wait_all

pytestmark = pytest.mark.gpu

REC = ("in", "exc", "v_exc", "counts")


def scaling_net(n_in=200, n_out=150):
    cfg = inputs.scaling_config(n_in=n_in, n_out=n_out)
    W = inputs.normal_weights(n_in, n_out, 0.5, 0.2, 0)
    return cfg, W


def run_path(torch, cfg, W, ids, T, path, precision="fp32", record=REC, calls=None):
    """Outputs of one run (or of consecutive calls of the given lengths
    without a reset) on `path`, as host arrays, and the path that ran."""
    from paper_1909_02549_amd.snn import Net
    net = Net(cfg, max_batch=len(ids), path=path, precision=precision)
    net.snn_set_weights(W)
    outs = []
    for k, t in enumerate(calls or [T]):
        out = net.snn_run(None, to_dev(torch, ids.astype(np.int64)), t, record=record, reset=(k == 0))
        torch.cuda.synchronize()
        outs.append({key: v.cpu().numpy() for key, v in out.items()})
    used = net.snn_last_path()
    net.close()
    if calls:
        return {key: np.concatenate([o[key] for o in outs]) if key != "counts" else sum(o[key] for o in outs)
                for key in outs[0]}, used
    return outs[0], used


@pytest.mark.parametrize("jb", [8, 13, 32])
def test_matches_oracle(torch_cuda, oracle_mod, monkeypatch, jb):
    monkeypatch.setenv("SNN_JB", str(jb))
    cfg, W = scaling_net()
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, sample_ids(37, 11), 150, path="persistent",
                      record=REC)
    assert g["path"] == "persistent"
    assert ref["exc"].sum() > 100
    check_parity(g, ref, learn=False)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("B", [1, 300])
def test_bit_exact_against_fused(torch_cuda, precision, B):
    """Same gather order and neuron update as the fused kernel: every
    recorded raster, voltage and count is identical."""
    cfg, W = scaling_net()
    ids = sample_ids(B, 70)
    gp, used_p = run_path(torch_cuda, cfg, W, ids, 120, "persistent", precision)
    gf, used_f = run_path(torch_cuda, cfg, W, ids, 120, "fused", precision)
    assert (used_p, used_f) == ("persistent", "fused")
    assert gp["exc"].any()
    for key in REC:
        assert np.array_equal(gp[key], gf[key]), key


def test_run_across_encoder_chunks(torch_cuda, oracle_mod):
    """600 steps: two chunk launches, the second starting from the state the
    first stored."""
    cfg, W = scaling_net(120, 40)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, sample_ids(6, 90), 600, path="persistent", record=REC)
    assert g["path"] == "persistent"
    assert ref["exc"][:, 512:].sum() > 10
    check_parity(g, ref, learn=False)


def test_continuing_runs_equal_one_run(torch_cuda):
    """Calls of 70, 1 and 49 steps without a reset equal one 120-step run."""
    cfg, W = scaling_net()
    ids = sample_ids(50, 120)
    one, _ = run_path(torch_cuda, cfg, W, ids, 120, "persistent")
    parts, used = run_path(torch_cuda, cfg, W, ids, 120, "persistent", calls=[70, 1, 49])
    assert used == "persistent"
    for key in REC:
        assert np.array_equal(one[key], parts[key]), key


def test_large_batch_runs_persistent(torch_cuda):
    """B = 3000 x 1000 columns: past what the cooperative kernel holds, the
    chunk kernel still runs it; sampled rows equal the fused path's."""
    cfg, W = scaling_net(300, 1000)
    ids = sample_ids(3000, 5)
    rec = ("exc", "counts")
    gp, used = run_path(torch_cuda, cfg, W, ids, 40, "persistent", record=rec)
    gf, _ = run_path(torch_cuda, cfg, W, ids, 40, "fused", record=rec)
    assert used == "persistent"
    assert gp["counts"].sum() > 1000
    for key in rec:
        assert np.array_equal(gp[key], gf[key]), key


def test_serving_alone_equals_mix(torch_cuda, oracle_mod):
    """A frozen image-driven network without inhibitory layer served through
    the chunk kernel: each request's counts are the same alone and in the
    mix, and agree with the oracle."""
    from paper_1909_02549_amd.snn import Net, Server
    cfg = inputs.dc_config(48, learn=False, n_inh=0, w_ei=0.0, w_ie=0.0)
    W = inputs.frozen_weights(784, 48, 78.4, 9)
    net = Net(cfg, max_batch=1, path="persistent")
    net.snn_set_weights(W)
    imgs = inputs.stroke_images(8, 35, 0.19)
    Ts = [20, 45, 70, 20, 33, 64, 17, 90]
    ids = list(range(700, 708))
    srv1 = Server(net, max_slots=1, chunk_steps=16)
    alone = []
    for k in range(8):
        rid = srv1.snn_serve_submit(imgs[k], ids[k], Ts[k])
        alone.append(wait_all(srv1, [rid])[rid][0])
    srv1.snn_serve_destroy()
    srv = Server(net, max_slots=5, chunk_steps=16)
    rids = [srv.snn_serve_submit(imgs[k], ids[k], Ts[k]) for k in range(8)]
    res = wait_all(srv, rids)
    st = srv.snn_serve_stats()
    srv.snn_serve_destroy()
    net.close()
    assert st["completed"] == 8 and st["peak_active"] > 1
    for k, r in enumerate(rids):
        assert np.array_equal(res[r][0], alone[k]), f"request {k} differs alone vs in the mix"
    assert sum(a.sum() for a in alone) > 0
    for k in range(8):
        ref = oracle_mod.OracleNet(cfg, W.astype(np.float64)).run(imgs[k:k + 1], np.array([ids[k]], np.uint64),
                                                                  Ts[k], record=("counts",))
        assert (ref["counts"][0] == alone[k]).mean() >= 0.99


@pytest.mark.parametrize("path", ["persistent", "fused"])
def test_forced_input_spikes(torch_cuda, oracle_mod, path):
    """Caller-given input spikes (snn_run_spikes) on a network without
    learning: the encoder copies the words and builds the lists from them
    (inputs 0 .. 69, so the last 16-input group of the lanes is ragged and
    one 32-input word is half empty)."""
    cfg = inputs.scaling_config(n_in=70, n_out=40)
    W = inputs.normal_weights(70, 40, 0.8, 0.3, 4)
    rng = np.random.default_rng(12)
    B, T = 21, 90
    forced = (rng.random((B, T, 70)) < 0.06).astype(np.uint8)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, sample_ids(B, 40), T, path=path, forced=forced,
                      record=REC)
    assert g["path"] == path
    assert ref["exc"].sum() > 20
    check_parity(g, ref, learn=False)


@pytest.mark.parametrize("cols", [1, 2, 4, 8])
@pytest.mark.parametrize("jb", [8, 13])
def test_columns_per_lane_bit_exact(torch_cuda, oracle_mod, monkeypatch, cols, jb):
    """Small batches spread each 8-column task over 8 / cols lanes (the
    library picks the width from the grid size; SNN_INDEP_COLS fixes it).
    Every width gives the fused kernel's outputs bit for bit, in every operand
    form, and meets the oracle's bars."""
    monkeypatch.setenv("SNN_JB", str(jb))
    monkeypatch.setenv("SNN_INDEP_COLS", str(cols))
    cfg, W = scaling_net()
    ids = sample_ids(37, 130)
    for precision in ("fp32", "bf16", "fp8"):
        gp, used_p = run_path(torch_cuda, cfg, W, ids, 70, "persistent", precision)
        gf, used_f = run_path(torch_cuda, cfg, W, ids, 70, "fused", precision)
        assert (used_p, used_f) == ("persistent", "fused")
        for key in REC:
            assert np.array_equal(gp[key], gf[key]), (precision, key)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, ids, 70, path="persistent", record=REC)
    assert ref["exc"].sum() > 50
    check_parity(g, ref, learn=False)


@pytest.mark.parametrize("cols", [1, 2, 4, 8])
def test_tiny_network(torch_cuda, oracle_mod, monkeypatch, cols):
    """10 inputs (one 32-input word, mostly padding) -> 3 neurons (one
    4-column plane, partly padding), B = 5: every width against the oracle
    and bit for bit against the fused kernel."""
    monkeypatch.setenv("SNN_INDEP_COLS", str(cols))
    cfg = inputs.scaling_config(n_in=10, n_out=3, rate_hz=150.0)
    W = inputs.normal_weights(10, 3, 4.0, 1.0, 8)
    ids = sample_ids(5, 300)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, None, ids, 80, path="persistent", record=REC)
    assert g["path"] == "persistent"
    assert ref["exc"].sum() > 10
    check_parity(g, ref, learn=False)
    gf, _ = run_path(torch_cuda, cfg, W, ids, 80, "fused")
    gp, _ = run_path(torch_cuda, cfg, W, ids, 80, "persistent")
    for key in REC:
        assert np.array_equal(gp[key], gf[key]), key


def test_very_large_batch(torch_cuda, oracle_mod):
    """B = 20 000 on the 1000 -> 1000 scaling network (twice the largest
    batch of the scaling sweep; the grid has 125 x 313 workgroups): sampled
    samples against the oracle, every row against the fused kernel."""
    wl = inputs.workload("scale")
    cfg = wl["cfg"]
    W = inputs.normal_weights(1000, 1000, wl["wmean"], wl["wstd"], 0)
    B, T = 20000, 24
    ids = sample_ids(B, 9)
    rec = ("exc", "counts")
    gp, used = run_path(torch_cuda, cfg, W, ids, T, "persistent", record=rec)
    gf, _ = run_path(torch_cuda, cfg, W, ids, T, "fused", record=rec)
    assert used == "persistent"
    for key in rec:
        assert np.array_equal(gp[key], gf[key]), key
    sel = np.array([0, 1, 9999, 19998, 19999])
    ref = oracle_mod.OracleNet(cfg, W.astype(np.float64)).run(None, ids[sel], T, record=("counts",))
    assert ref["counts"].sum() > 0
    assert (gp["counts"][sel] == ref["counts"]).mean() >= 0.999
