"""GPU: episodic runs replayed from captured HIP graphs give exactly the
results of launching every kernel.

Two handles with the same weights run the same sequence of episodic trials,
one with graphs on and one without; after every trial (with unrelated eager
GPU work and synchronisations between the replays) the counts, rasters,
voltages, weights and thresholds must be identical bit for bit.
"""
import numpy as np
import pytest

from paper_1909_02549_amd import inputs
from paper_1909_02549_amd.inputs import dc_config, sample_ids, stroke_images, uniform_weights
from test_parity_gpu import torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


def trial_outputs(torch, net, imgs_d, ids_d, T):
    out = net.snn_run(imgs_d, ids_d, T, reset=True, record=("exc", "inh", "v_exc", "counts"))
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["W"] = net.snn_get_weights()
    res["theta"] = net.snn_get_theta()
    res["path"] = net.snn_last_path()
    return res


@pytest.mark.parametrize("path", ["plain", "mfma", "fused", "persistent"])
def test_graph_replays_equal_launches(torch_cuda, path):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net
    cfg = dc_config(64)
    B, T = 8, 50
    imgs = stroke_images(B, 80, 0.19)
    W = uniform_weights(784, 64, 0.0, 0.3, 21)
    imgs_d = torch.from_numpy(imgs).cuda()
    ids_d = torch.from_numpy(sample_ids(B, 31).astype(np.int64)).cuda()
    g_net = Net(cfg, max_batch=B, path=path)
    e_net = Net(cfg, max_batch=B, path=path)
    g_net.snn_set_weights(W)
    e_net.snn_set_weights(W)
    g_net.snn_set_graphs(True)
    junk = torch.randn(1 << 20, device="cuda")
    for trial in range(4):
        a = trial_outputs(torch, g_net, imgs_d, ids_d, T)
        b = trial_outputs(torch, e_net, imgs_d, ids_d, T)
        assert a["path"] == b["path"] == path
        for k in ("exc", "inh", "v_exc", "counts", "W", "theta"):
            assert np.array_equal(a[k], b[k]), f"trial {trial}: {k} differs"
        # unrelated eager work between replays
        junk = (junk * 1.0001).sin_()
        torch.cuda.synchronize()
    assert a["counts"].sum() > 0
    g_net.close()
    e_net.close()


@pytest.mark.parametrize("path,T", [("plain", 40), ("fused", 40), ("persistent", 40), ("persistent", 530)])
def test_graph_with_changing_batch_and_frozen_weights(torch_cuda, path, T):
    """No learning: replays of the same trial repeat exactly; a different
    batch size captures a new graph and still equals the launched kernels.
    Without an inhibitory layer the persistent path runs the barrier-free
    chunk kernel (530 steps: two encoder chunks inside one graph)."""
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net
    cfg = inputs.scaling_config(n_in=300, n_out=200)
    W = inputs.normal_weights(300, 200, 0.5, 0.2, 3)
    g_net = Net(cfg, max_batch=64, path=path)
    e_net = Net(cfg, max_batch=64, path=path)
    g_net.snn_set_weights(W)
    e_net.snn_set_weights(W)
    g_net.snn_set_graphs(True)
    first = None
    for B in (64, 16, 64, 16):
        ids_d = torch.from_numpy(sample_ids(B, 5).astype(np.int64)).cuda()
        a = trial_outputs(torch, g_net, None, ids_d, T)
        b = trial_outputs(torch, e_net, None, ids_d, T)
        assert g_net.snn_last_path() == e_net.snn_last_path() == path
        for k in ("exc", "v_exc", "counts"):
            assert np.array_equal(a[k], b[k]), f"B={B}: {k} differs"
        if B == 64:
            if first is None:
                first = a
            else:
                assert np.array_equal(first["counts"], a["counts"])
    g_net.close()
    e_net.close()


def test_persistent_graph_full_size_trial(torch_cuda):
    """The benchmark's workload (784 -> 6400/6400, B = 256, T = 350, STDP) on
    the persistent path replayed from a captured graph: three trials in a
    row, each bit-identical (spike counts, weights, thresholds) to the same
    trial launched directly, with the device error flag clear."""
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net
    wl = inputs.workload("dc6400")
    cfg, B, T = wl["cfg"], wl["B"], wl["T"]
    imgs_d = torch.from_numpy(stroke_images(B, 1234, wl["density"])).cuda()
    ids_d = torch.from_numpy(sample_ids(B).astype(np.int64)).cuda()
    W = uniform_weights(784, cfg["n_exc"], wl["wlo"], wl["whi"], 0)
    g_net = Net(cfg, max_batch=B, path="persistent")
    e_net = Net(cfg, max_batch=B, path="persistent")
    g_net.snn_set_weights(W)
    e_net.snn_set_weights(W)
    g_net.snn_set_graphs(True)
    for trial in range(3):
        outs = []
        for net in (g_net, e_net):
            out = net.snn_run(imgs_d, ids_d, T, reset=True, record=("counts",))
            net.snn_sync()
            outs.append((out["counts"].cpu().numpy(), net.snn_get_weights(), net.snn_get_theta(),
                         net.snn_last_path()))
        (ca, wa, ta, pa), (cb, wb, tb, pb) = outs
        assert pa == pb == "persistent"
        assert np.array_equal(ca, cb) and np.array_equal(wa, wb) and np.array_equal(ta, tb), f"trial {trial}"
        assert ca.sum() > 0
    g_net.close()
    e_net.close()
