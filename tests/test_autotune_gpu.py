"""GPU tests of the autotuner (SNN_PATH_AUTO): its choice of execution path
and column block width, and the re-layout of a handle whose width changes.

The weights and thresholds a handle holds must survive the re-layout
exactly, and the tuned handle must meet every parity bar against the oracle
(learning on and off)."""
import os

import numpy as np
import pytest

from paper_1909_02549_amd.inputs import dc_config, sample_ids, stroke_images, uniform_weights
from test_parity_gpu import check_parity, run_both, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_exc", [100, 400])
def test_tuned_handle_keeps_parameters(torch_cuda, n_exc):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net
    cfg = dc_config(n_exc, learn=False)
    W = uniform_weights(784, n_exc, 0.0, 0.3, 40)
    th = np.random.default_rng(0).uniform(0.0, 2.0, n_exc)
    net = Net(cfg, max_batch=32, path="auto")
    net.snn_set_weights(W)
    net.snn_set_theta(th)
    imgs = torch.from_numpy(stroke_images(32, 41, 0.19)).cuda()
    ids = torch.from_numpy(sample_ids(32, 7).astype(np.int64)).cuda()
    out = net.snn_run(imgs, ids, 60, record=("counts",))
    torch.cuda.synchronize()
    assert net.snn_last_path() in ("persistent", "fused", "mfma", "plain")
    assert np.array_equal(net.snn_get_weights(), W)
    assert np.array_equal(net.snn_get_theta(), th)
    assert out["counts"].sum().item() > 0
    net.close()


@pytest.mark.parametrize("learn", [True, False])
def test_tuned_handle_matches_oracle(torch_cuda, oracle_mod, learn):
    """784 -> 400/400, B = 64: the autotuner times (path, width) pairs on
    scratch copies, the handle re-lays out for the winner, and the run meets
    the parity bars."""
    cfg = dc_config(400, learn=learn)
    imgs = stroke_images(64, 42, 0.19)
    W = uniform_weights(784, 400, 0.0, 0.3, 43)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(64, 900), 60, path="auto")
    assert ref["exc"].sum() > 100
    check_parity(g, ref, learn=learn)
