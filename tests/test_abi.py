"""CPU tests of the C-ABI library: it loads without a GPU, exports every
symbol include/snn.h declares, and rejects invalid configurations before
touching the device.  No compute call is made here."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "snn.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(snn_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1909_02549_amd import snn
    if not os.path.exists(snn.LIB_PATH):
        pytest.skip("libsnn.so not built")
    return snn.load_library()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 20
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_1909_02549_amd import snn
    assert sorted(snn.EXPORTED) == declared_symbols()


def test_abi_version(lib):
    assert lib.snn_abi_version() == 2


def _cfg(**over):
    from paper_1909_02549_amd import inputs, snn
    cfg = inputs.dc_config(100)
    c = snn.make_config(cfg, max_batch=4)
    for k, v in over.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("field,value", [("abi_version", 7), ("n_in", 0), ("n_exc", 0), ("n_inh", 5),
                                         ("reduce", 9), ("precision", 5), ("path", 8), ("max_batch", 0),
                                         ("dt_ms", 0.0), ("w_min", 2.0)])
def test_invalid_config_rejected_without_gpu(lib, field, value):
    c = _cfg(**{field: value})
    h = C.c_void_p()
    st = lib.snn_create(C.byref(c), None, C.byref(h))
    assert st == -1 and not h.value
    assert lib.snn_last_error().decode()


@pytest.mark.parametrize("tau,additive", [(1e-3, 0), (float("inf"), 0), (float("nan"), 0), (-1.0, 0),
                                          (0.1, 1)])
def test_soft_max_temperature_bound_rejected(lib, tau, additive):
    """The soft maximum needs a finite temperature of at least x_max / 64
    (x_max = 1 for nearest-spike traces, 1 / (1 - exp(-dt / tau_trace)),
    about 20.5, for additive ones at 20 ms)."""
    c = _cfg(reduce=4, reduce_tau=tau, trace_additive=additive)
    h = C.c_void_p()
    assert lib.snn_create(C.byref(c), None, C.byref(h)) == -1 and not h.value
    assert "reduce_tau" in lib.snn_last_error().decode()


def test_refractory_bound_rejected(lib):
    c = _cfg()
    c.exc.refrac_steps = 200
    h = C.c_void_p()
    assert lib.snn_create(C.byref(c), None, C.byref(h)) == -1


def test_null_handle_calls(lib):
    assert lib.snn_run(None, None, None, 1, 1, 0, None) == -1
    assert lib.snn_sync(None) == -1
    assert lib.snn_stdp_reduce(None, 0) == -1
    assert lib.snn_stdp_reduce_soft(None, 1.0) == -1
    assert lib.snn_serve_poll(None, 1, None, None) == -1


def test_state_bytes_grow_with_batch(lib):
    c = _cfg()
    b1 = lib.snn_state_bytes(C.byref(c), 1)
    b64 = lib.snn_state_bytes(C.byref(c), 64)
    assert 0 < b1 < b64


def test_bit_packing_roundtrip():
    from paper_1909_02549_amd.snn import pack_bits, unpack_bits
    rng = np.random.default_rng(0)
    for n in (1, 31, 32, 33, 784, 1000):
        x = (rng.random((3, 5, n)) < 0.3).astype(np.uint8)
        w = pack_bits(x)
        assert w.shape == (3, 5, (n + 31) // 32)
        assert np.array_equal(unpack_bits(w, n), x)
    assert pack_bits(np.array([1, 0, 0, 0, 0, 1] + [0] * 26, np.uint8))[0] == (1 | 1 << 5)


@pytest.mark.parametrize("field,value", [("abi_version", 7), ("n_in", 0), ("n_h1", 0), ("n_h1", 257),
                                         ("n_h2", 129), ("n_out", 33), ("n_out", 0), ("max_batch", 0),
                                         ("theta_h1", 0.0), ("theta_h2", -1.0)])
def test_invalid_ifnet_config_rejected_without_gpu(lib, field, value):
    from paper_1909_02549_amd import snn
    c = snn.make_ifnet_config((784, 256, 128, 10), (1.0, 1.0), 16)
    setattr(c, field, value)
    h = C.c_void_p()
    assert lib.snn_ifnet_create(C.byref(c), None, C.byref(h)) == -1 and not h.value
    assert lib.snn_last_error().decode()


def test_ifnet_null_handle_calls(lib):
    assert lib.snn_ifnet_run(None, None, 1, 1, None) == -1
    assert lib.snn_ifnet_sync(None) == -1
    assert lib.snn_ifnet_set_layer(None, 1, None, 0, None, 0) == -1


def test_product_package_never_uses_the_oracle():
    """The HIP path has no CPU fallback: no module of the package imports the
    oracle (test infrastructure), and the oracle does not import the package's
    binding."""
    pkg = os.path.join(ROOT, "paper_1909_02549_amd")
    for name in os.listdir(pkg):
        if name.endswith(".py"):
            src = open(os.path.join(pkg, name)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), name
    for name in ("oracle.py", "ifnet.py"):
        src = open(os.path.join(ROOT, "oracle", name)).read()
        assert "paper_1909_02549_amd.snn" not in src and "libsnn" not in src, name


def test_handles_raise_without_gpu_or_library(monkeypatch):
    torch = pytest.importorskip("torch")
    from paper_1909_02549_amd import inputs, snn
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            snn.Net(inputs.dc_config(100), max_batch=4)
        with pytest.raises(RuntimeError, match="no CPU fallback"):
            snn.IFNet((784, 256, 128, 10))
    monkeypatch.setattr(snn, "_lib", None)
    monkeypatch.setattr(snn, "LIB_PATH", os.path.join(ROOT, "no_such_libsnn.so"))
    with pytest.raises(RuntimeError, match="not built"):
        snn.load_library()


def test_resource_report_parser():
    from paper_1909_02549_amd import build
    text = ("a.hip:3:1: remark: Function Name: k_a [-Rpass-analysis=kernel-resource-usage]\n"
            "    3 | {\n      | ^\n"
            "a.hip:3:1: remark:     VGPRs: 121 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:3:1: remark:     ScratchSize [bytes/lane]: 448 [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:9:1: remark: Function Name: k_b [-Rpass-analysis=kernel-resource-usage]\n"
            "a.hip:9:1: remark:     Occupancy [waves/SIMD]: 5 [-Rpass-analysis=kernel-resource-usage]\n")
    assert build.parse_resources(text) == {"k_a": {"vgpr": 121, "scratch": 448}, "k_b": {"occupancy": 5}}


def test_no_kernel_spills_to_scratch():
    """Every kernel keeps its state in registers and LDS: a kernel that
    starts spilling to scratch memory runs several times slower (the FP32
    fused step at 448 bytes per lane took three times as long per step)."""
    from paper_1909_02549_amd import build, snn
    if not os.path.exists(build.RESOURCES) or not os.path.exists(snn.LIB_PATH):
        pytest.skip("library not built")
    res = json.load(open(build.RESOURCES))
    assert os.path.getmtime(build.RESOURCES) >= os.path.getmtime(snn.LIB_PATH) - 5
    assert any("k_fused_step" in k for k in res) and any("k_persist" in k for k in res)
    spilling = {k: r["scratch"] for k, r in res.items() if r.get("scratch", 0)}
    assert not spilling, spilling
