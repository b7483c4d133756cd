"""CPU tests of the benchmark's host-side arithmetic: workload sizes,
algorithmic bytes and flops (against hand-computed figures), the roofline
fractions, and the single-GPU guard."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import bench as b
    return b


def test_dims_expected_input_spikes(bench):
    from paper_1909_02549_amd import inputs
    # uniform 20 Hz at dt = 1 ms: p = 0.02 per input and step
    d = bench.dims(inputs.scaling_config(n_in=1000, n_out=1000), 64)
    assert d["s_in"] == pytest.approx(64 * 1000 * 0.02)
    assert d["n_in_pad"] == 1024 and d["in_words"] == 32 and d["bwords"] == 2
    # images: a 255 pixel fires with p = 0.128, a 51 pixel with 0.0256
    img = np.zeros((2, 784), np.uint8)
    img[0, :3] = 255
    img[1, 0] = 51
    d = bench.dims(inputs.dc_config(100), 2, img)
    assert d["s_in"] == pytest.approx(3 * 0.128 + 0.0256)
    assert d["n_in_pad"] == 800


def test_persistent_bytes_hand_value(bench):
    """784 -> 6400/6400 learning, B = 256, one 350-step launch:
    weights 784 * 6400 * 4 = 20 070 400 B read and written;
    state 256 * 6400 * (4 + 2 + 4 + 4) = 22 937 600 B read and written;
    per step x_pre 256 * 800 * 4 = 819 200 B read and written and input spikes
    256 * 25 * 4 + 800 * 8 * 4 = 51 200 B:
    2 * 20 070 400 + 2 * 22 937 600 + 350 * (2 * 819 200 + 51 200) = 677 376 000."""
    from paper_1909_02549_amd import inputs
    d = bench.dims(inputs.dc_config(6400), 256)
    assert bench.algorithmic_bytes("persistent", d, 350) == 677_376_000
    assert bench.algorithmic_bytes("no_such_kernel", d) is None


def test_step_model_hand_values(bench):
    """One learning step of 784 (800) -> 6400 at B = 256:
    bytes 2 * 800 * 6400 * 4 + 2 * 256 * 6400 * 14 + 2 * 256 * 800 * 4
          = 40 960 000 + 45 875 200 + 1 638 400 = 88 473 600;
    flops 6 * 256 * 800 * 6400 = 7 864 320 000."""
    from paper_1909_02549_amd import inputs
    d = bench.dims(inputs.dc_config(6400), 256)
    assert bench.step_bytes(d) == 88_473_600
    assert bench.step_flops(d) == 7_864_320_000


def test_roofline_fractions_and_bound(bench):
    from paper_1909_02549_amd import inputs
    d = bench.dims(inputs.dc_config(6400), 256)
    per = bench.algorithmic_bytes("fused_step", d)
    # 10 launches in 1 ms: 100 us each
    r = bench.kernel_roofline("fused_step", d, "fp32", 10, 1.0, 1.0)
    assert r["bytes_per_launch"] == per
    assert r["alu"]["frac"] == pytest.approx(bench.alu_ops("fused_step", d) / 100e-6 / 1e12 / 157.3)
    hbm = per / 100e-6 / 1e9 / 8000.0
    assert r["alu"]["hbm_frac"] == pytest.approx(hbm)
    # the kernel's own models, then the whole-step HBM figure as the bound
    assert r["kernel_model"]["frac"] == pytest.approx(max(hbm, r["alu"]["frac"]))
    assert r["bound"] == "hbm" and r["frac"] == pytest.approx(88_473_600 / 100e-6 / 1e9 / 8000.0)
    # persistent: one launch of 350 steps in 10 ms, graded on the step's
    # 88.5 MB times 350 against the HBM peak; the dense-equivalent flops
    # against the BF16 matrix-core peak are context
    q = bench.kernel_roofline("persistent", d, "fp32", 1, 10.0, 350.0)
    assert q["bound"] == "hbm" and q["peak"] == 8000.0 and q["unit"] == "GB/s"
    assert q["algorithmic_bytes_per_launch"] == 350 * 88_473_600
    assert q["frac"] == pytest.approx(350 * 88_473_600 / 10e-3 / 1e9 / 8000.0)
    assert q["step_model"]["mfma_frac"] == pytest.approx(350 * 7_864_320_000 / 10e-3 / 1e12 / 2500.0)
    m = bench.kernel_roofline("mfma_front", d, "fp32", 1, 0.01, 1.0)
    tf = 2.0 * 256 * 784 * 6400 / 10e-6 / 1e12
    assert m["mfma"]["achieved"] == pytest.approx(tf)
    assert m["mfma"]["frac"] == pytest.approx(3 * tf / 2500.0)


def test_conversion_flops_hand_value(bench):
    """784-256-128-10, B = 1024, T = 10:
    2 * 1024 * (784 * 256 + 10 * (256 * 128 + 128 * 10)) = 1 108 344 832."""
    assert bench.conversion_flops((784, 256, 128, 10), 1024, 10) == 1_108_344_832
    # issued: 3 planes, n_out padded to 32: 6 * 1024 * (784 * 256 + 10 * (256 * 128 + 128 * 32))
    assert bench.conversion_issued_flops((784, 256, 128, 10), 1024, 10) == 6.0 * 1024 * (
        784 * 256 + 10 * (256 * 128 + 128 * 32))


def test_single_gpu_guard():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_sweep_selection_flags():
    """--sweep-paths must name entries of the scaling sweep; a bad entry is
    refused before anything runs (no GPU needed)."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--sweep", "scale", "--sweep-paths",
                        "persistent,bogus"], capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "--sweep-paths entries must be among" in r.stderr


def test_scale_sweep_entries(bench):
    assert "persistent" in bench.SCALE_PATHS and "fused+graph" in bench.SCALE_PATHS
    for e in bench.SCALE_PATHS:
        path, _, g = e.partition("+")
        assert path in ("plain", "mfma", "fused", "persistent") and g in ("", "graph")
