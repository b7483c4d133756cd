"""GPU parity at the column-block widths of large layers.

The library gives each workgroup a block of 8 to 32 post-synaptic columns
(one block per compute unit for large layers: 25 columns for 784 -> 6400).
Blocks wider than 8 columns span several 8-column groups, and the per-step
kernels then split each weight row over two threads and test the spike masks
of the groups separately.  SNN_JB sets the block width of a small layer, so
that these code paths are checked against the oracle at sizes it finishes in
seconds: 13 columns (two groups, the second ragged), 20 (three groups) and 25
(four groups, the 784 -> 6400 layout).

The short runs cover the first synchronous burst of excitatory spikes (many
samples firing in one block in the same step, so the potentiation terms take
several passes over the list of spiking samples) and must not diverge, so the
learned weights are compared; the longer runs check rasters, voltages and, if
nothing diverged, weights.
"""
import numpy as np
import pytest

from paper_1909_02549_amd.inputs import dc_config, sample_ids, stroke_images, uniform_weights
from test_parity_gpu import check_parity, run_both, torch_cuda  # noqa: F401

pytestmark = pytest.mark.gpu

PATHS = ["plain", "mfma", "fused", "persistent"]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("jb", [13, 20, 25])
def test_wide_block_burst_weights(torch_cuda, oracle_mod, monkeypatch, jb, path):
    monkeypatch.setenv("SNN_JB", str(jb))
    cfg = dc_config(300)
    T = 14
    imgs = stroke_images(64, 77, 0.19)
    W = uniform_weights(784, 300, 0.0, 0.3, 41)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(64, 500), T, path=path)
    assert g["path"] == path
    fired = ref["exc"].reshape(64, T, -1, jb).any(axis=3) if 300 % jb == 0 else None
    if fired is not None:
        assert fired.sum(axis=0).max() > 8, "no block with more than 8 spiking samples in one step"
    assert ref["exc"].sum() > 100
    t_div = check_parity(g, ref)
    assert t_div == T, f"rasters diverged at step {t_div}: weights not compared"


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("reduce", ["mean", "sum", "max"])
def test_wide_block_reductions(torch_cuda, oracle_mod, monkeypatch, reduce, path):
    monkeypatch.setenv("SNN_JB", "25")
    cfg = dc_config(300, reduce=reduce)
    imgs = stroke_images(16, 78, 0.19)
    W = uniform_weights(784, 300, 0.0, 0.3, 42)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(16, 600), 60, path=path)
    assert g["path"] == path
    check_parity(g, ref)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_wide_block_reduced_forms(torch_cuda, oracle_mod, monkeypatch, precision, path):
    """Against the oracle in the same operand form."""
    monkeypatch.setenv("SNN_JB", "25")
    cfg = dc_config(300)
    T = 14
    imgs = stroke_images(32, 79, 0.19)
    W = uniform_weights(784, 300, 0.0, 0.3, 43)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(32, 700), T, path=path,
                      precision=precision)
    assert g["path"] == path
    t_div = check_parity(g, ref)
    assert t_div == T, f"rasters diverged at step {t_div}: weights not compared"
    assert np.isfinite(g["W"]).all()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("variant", ["max_signed", "soft_max", "norm_per_run"])
def test_wide_block_reduction_variants(torch_cuda, oracle_mod, monkeypatch, variant, path):
    """The signed-max and soft-max reductions and per-run normalisation at the
    25-column block of the 784 -> 6400 layout, through the first burst."""
    monkeypatch.setenv("SNN_JB", "25")
    cfg = (dc_config(300, reduce=variant, reduce_tau=0.1) if variant != "norm_per_run"
           else dc_config(300, norm_per_run=1))
    T = 14
    imgs = stroke_images(32, 80, 0.19)
    W = uniform_weights(784, 300, 0.0, 0.3, 44)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(32, 800), T, path=path)
    assert g["path"] == path
    assert ref["exc"].sum() > 100
    t_div = check_parity(g, ref)
    assert t_div == T, f"rasters diverged at step {t_div}: weights not compared"


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("reduce", ["max_signed", "soft_max"])
def test_wide_block_reduced_forms_variant_reductions(torch_cuda, oracle_mod, monkeypatch, reduce, precision, path):
    """The signed and soft maxima in the reduced operand forms, against the
    oracle in the same form, through the first burst."""
    monkeypatch.setenv("SNN_JB", "25")
    cfg = dc_config(300, reduce=reduce, reduce_tau=0.1)
    T = 14
    imgs = stroke_images(32, 81, 0.19)
    W = uniform_weights(784, 300, 0.0, 0.3, 45)
    g, ref = run_both(torch_cuda, oracle_mod, cfg, W, imgs, sample_ids(32, 900), T, path=path,
                      precision=precision)
    assert g["path"] == path
    assert ref["exc"].sum() > 100
    t_div = check_parity(g, ref)
    assert t_div == T, f"rasters diverged at step {t_div}: weights not compared"
