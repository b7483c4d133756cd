"""ctypes front end of the FP64 CPU oracle (``snn_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It does not
import the HIP binding and the HIP binding does not import it.

``OracleNet`` mirrors the minibatched simulation of the paper's
Implementation section: per-sample state duplicated B times (voltages,
refractory counters, traces, previous spikes), one shared copy of the weights
and adaptive thresholds, an episodic reset between trials (Episodic vs.
continuing simulation) and re-initialisation when the batch size changes
(Dynamic minibatch size).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")


class _Lif(C.Structure):
    _fields_ = [("v_rest", C.c_double), ("v_reset", C.c_double), ("v_thresh", C.c_double),
                ("tau_ms", C.c_double), ("refrac_steps", C.c_int32), ("adaptive", C.c_int32),
                ("theta_plus", C.c_double), ("tau_theta_ms", C.c_double)]


class _Config(C.Structure):
    _fields_ = [("n_in", C.c_int32), ("n_exc", C.c_int32), ("n_inh", C.c_int32),
                ("uniform_rate", C.c_int32), ("learn", C.c_int32),
                ("trace_additive", C.c_int32), ("reduce", C.c_int32), ("precision", C.c_int32),
                ("dt_ms", C.c_double), ("max_rate_hz", C.c_double),
                ("exc", _Lif), ("inh", _Lif), ("w_ei", C.c_double), ("w_ie", C.c_double),
                ("nu_pre", C.c_double), ("nu_post", C.c_double), ("tau_pre_ms", C.c_double),
                ("tau_post_ms", C.c_double), ("w_min", C.c_double), ("w_max", C.c_double),
                ("norm", C.c_double), ("seed", C.c_uint64), ("norm_per_run", C.c_int32),
                ("reduce_tau", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64)] * 3
        _lib.orc_philox4x64_10.restype = None
        _lib.orc_uniform32.argtypes = [C.c_uint64] * 4
        _lib.orc_uniform32.restype = C.c_uint32
        _lib.orc_threshold.argtypes = [C.POINTER(_Config), C.c_int]
        _lib.orc_threshold.restype = C.c_uint32
        _lib.orc_run.restype = C.c_int
        _lib.orc_quantize.argtypes = [C.c_double, C.c_int]
        _lib.orc_quantize.restype = C.c_double
        _lib.orc_set_threads.argtypes = [C.c_int]
        _lib.orc_set_threads.restype = None
        _lib.orc_threads.argtypes = []
        _lib.orc_threads.restype = C.c_int
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ctype))


PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2}


def make_config(cfg: dict, precision=0) -> _Config:
    c = _Config()
    for k in ("n_in", "n_exc", "n_inh", "uniform_rate", "learn", "trace_additive", "reduce"):
        setattr(c, k, int(cfg[k]))
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for k in ("dt_ms", "max_rate_hz", "w_ei", "w_ie", "nu_pre", "nu_post", "tau_pre_ms",
              "tau_post_ms", "w_min", "w_max", "norm"):
        setattr(c, k, float(cfg[k]))
    c.seed = int(cfg["seed"])
    c.norm_per_run = int(cfg.get("norm_per_run", 0))
    c.reduce_tau = float(cfg.get("reduce_tau", 1.0))
    for layer in ("exc", "inh"):
        L = getattr(c, layer)
        p = cfg[layer]
        for k in ("v_rest", "v_reset", "v_thresh", "tau_ms", "theta_plus", "tau_theta_ms"):
            setattr(L, k, float(p[k]))
        L.refrac_steps = int(p["refrac_steps"])
        L.adaptive = int(p["adaptive"])
    return c


def philox4x64_10(counter, key) -> np.ndarray:
    """One Philox4x64-10 block: 4 uint64 outputs for a 4-word counter and a
    2-word key."""
    ctr = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(ctr, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def uniform32(seed: int, sample_id: int, t: int, i: int) -> int:
    return int(lib().orc_uniform32(seed, sample_id, t, i))


def quantize(x, precision) -> np.ndarray:
    """Operand rounding of the reduced-precision forms (``orc_quantize``):
    0 none, 1 bfloat16, 2 OCP FP8 E4M3, each from the value's FP32 form,
    round to nearest even."""
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    f = lib().orc_quantize
    return np.array([f(float(v), p) for v in np.ravel(x)]).reshape(np.shape(x))


def threshold_table(cfg: dict) -> np.ndarray:
    c = make_config(cfg)
    return np.array([lib().orc_threshold(C.byref(c), p) for p in range(256)], dtype=np.uint64)


class OracleNet:
    """FP64 reference network.  ``W`` is (n_in, n_exc) float64, shared;
    ``theta`` is (n_exc,) float64, shared.  ``precision`` ("fp32", "bf16",
    "fp8") rounds the weight and trace operands of the two contractions (see
    ``quantize``); "fp32" leaves them in FP64."""

    def __init__(self, cfg: dict, W: np.ndarray, theta: np.ndarray | None = None, precision="fp32"):
        self.cfg = dict(cfg)
        self.c = make_config(cfg, precision)
        n_in, n_exc = cfg["n_in"], cfg["n_exc"]
        assert W.shape == (n_in, n_exc)
        self.W = np.ascontiguousarray(W, dtype=np.float64).copy()
        self.theta = np.zeros(n_exc) if theta is None else np.ascontiguousarray(theta, np.float64).copy()
        self.B = 0
        self.tl = np.zeros(0, np.int64)

    # -- state ---------------------------------------------------------------
    def reset(self, B: int):
        """Episodic reset: every per-sample variable back to its initial value.
        Shared parameters (W, theta) are kept."""
        cfg = self.cfg
        n_in, n_exc, n_inh = cfg["n_in"], cfg["n_exc"], cfg["n_inh"]
        ni = max(n_inh, 1)
        self.B = B
        self.tl = np.zeros(B, np.int64)  # per-sample local step
        self.v_exc = np.full((B, n_exc), float(cfg["exc"]["v_rest"]))
        self.v_inh = np.full((B, ni), float(cfg["inh"]["v_rest"]))
        self.r_exc = np.zeros((B, n_exc), np.int32)
        self.r_inh = np.zeros((B, ni), np.int32)
        self.x_pre = np.zeros((B, n_in))
        self.x_post = np.zeros((B, n_exc))
        self.s_exc = np.zeros((B, n_exc), np.uint8)
        self.s_inh = np.zeros((B, ni), np.uint8)

    # -- run -----------------------------------------------------------------
    def run(self, images, ids, T: int, reset: bool = True, forced_in=None,
            record=("exc", "inh", "in", "v_exc", "counts")) -> dict:
        """Simulate T steps for the batch.  ``images`` (B, n_in) uint8 or None
        (uniform rate / forced inputs); ``ids`` (B,) uint64; ``forced_in``
        optional (B, T, n_in) 0/1 raster replacing the Poisson encoder."""
        cfg = self.cfg
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        B = int(ids.shape[0])
        if reset or B != self.B:
            self.reset(B)
        n_in, n_exc, n_inh = cfg["n_in"], cfg["n_exc"], cfg["n_inh"]
        if images is not None:
            images = np.ascontiguousarray(images, dtype=np.uint8)
            assert images.shape == (B, n_in)
        elif not cfg["uniform_rate"] and forced_in is None:
            raise ValueError("images required")
        if forced_in is not None:
            forced_in = np.ascontiguousarray(forced_in, dtype=np.uint8)
            assert forced_in.shape == (B, T, n_in)
        out = {}

        def rec(name, shape, dtype):
            if name in record:
                out[name] = np.zeros(shape, dtype)
                return out[name]
            return None

        r_in = rec("in", (B, T, n_in), np.uint8)
        r_exc = rec("exc", (B, T, n_exc), np.uint8)
        r_inh = rec("inh", (B, T, max(n_inh, 1)), np.uint8)
        r_ve = rec("v_exc", (B, T, n_exc), np.float64)
        r_vi = rec("v_inh", (B, T, max(n_inh, 1)), np.float64)
        cnt = rec("counts", (B, n_exc), np.uint32)
        r_th = rec("theta", (T, n_exc), np.float64)
        rc = lib().orc_run(
            C.byref(self.c), C.c_int(B), C.c_int(T), _ptr(self.tl, C.c_int64),
            _ptr(images, C.c_uint8), _ptr(ids, C.c_uint64), _ptr(forced_in, C.c_uint8),
            _ptr(self.W, C.c_double), _ptr(self.theta, C.c_double),
            _ptr(self.v_exc, C.c_double), _ptr(self.v_inh, C.c_double),
            _ptr(self.r_exc, C.c_int32), _ptr(self.r_inh, C.c_int32),
            _ptr(self.x_pre, C.c_double), _ptr(self.x_post, C.c_double),
            _ptr(self.s_exc, C.c_uint8), _ptr(self.s_inh, C.c_uint8),
            _ptr(r_in, C.c_uint8), _ptr(r_exc, C.c_uint8), _ptr(r_inh, C.c_uint8),
            _ptr(r_ve, C.c_double), _ptr(r_vi, C.c_double), _ptr(cnt, C.c_uint32),
            _ptr(r_th, C.c_double))
        if rc != 0:
            raise RuntimeError(f"orc_run failed: {rc}")
        self.tl += T
        return out

    def rebatch(self, keep, B: int):
        """Re-form the batch without a reset (an extension of the Dynamic
        minibatch size section, whose re-initialisation on a size change
        this avoids for the samples kept): new sample k < len(keep) takes
        every per-sample variable of old sample keep[k], its local step
        included; samples len(keep) .. B-1 start from the initial state at
        local step 0.  Shared parameters are untouched."""
        keep = np.asarray(keep, dtype=np.int64)
        assert keep.ndim == 1 and len(keep) <= B and len(set(keep.tolist())) == len(keep)
        assert (keep >= 0).all() and (keep < self.B).all()
        old = {k: getattr(self, k) for k in ("v_exc", "v_inh", "r_exc", "r_inh", "x_pre", "x_post",
                                             "s_exc", "s_inh", "tl")}
        self.reset(B)
        n = len(keep)
        for k, a in old.items():
            getattr(self, k)[:n] = a[keep]
