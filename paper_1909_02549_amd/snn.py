"""Python binding of the C ABI in ``include/snn.h`` (argument marshalling only).

Every step of the simulation runs in the HIP kernels of ``libsnn.so``; this
module converts dictionaries and torch tensors into the plain structs and
device pointers the library takes.  torch provides device memory and the
stream.  There is no CPU fallback: without the built library, or without a
GPU, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsnn.so")

SNN_ABI_VERSION = 2
SNN_RUN_RESET = 1
PATHS = {"plain": 0, "fused": 1, "persistent": 2, "auto": 3, "mfma": 4}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2}
REDUCES = {"sum": 0, "mean": 1, "max": 2, "max_signed": 3, "soft_max": 4}
STATUS = {0: "SNN_OK", -1: "SNN_EINVAL", -2: "SNN_ENOMEM", -3: "SNN_EDEVICE", -4: "SNN_EAGAIN",
          -5: "SNN_ENOTFOUND", -6: "SNN_ESTATE"}

EXPORTED = ["snn_abi_version", "snn_last_error", "snn_create", "snn_destroy", "snn_set_stream",
            "snn_set_weights", "snn_get_weights", "snn_set_theta", "snn_get_theta", "snn_stdp_reduce", "snn_stdp_reduce_soft",
            "snn_set_path", "snn_rebatch", "snn_last_path", "snn_set_graphs", "snn_run", "snn_run_spikes", "snn_sync", "snn_state_bytes",
            "snn_profile_enable", "snn_profile_get",
            "snn_serve_create", "snn_serve_submit", "snn_serve_poll", "snn_serve_stats",
            "snn_serve_destroy", "snn_ifnet_create", "snn_ifnet_destroy", "snn_ifnet_set_layer", "snn_ifnet_run",
            "snn_ifnet_run_noalloc", "snn_ifnet_sync"]


class SnnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class snn_lif(C.Structure):
    _fields_ = [("v_rest", C.c_double), ("v_reset", C.c_double), ("v_thresh", C.c_double),
                ("tau_ms", C.c_double), ("refrac_steps", C.c_int32), ("adaptive", C.c_int32),
                ("theta_plus", C.c_double), ("tau_theta_ms", C.c_double)]


class snn_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("n_in", C.c_uint32), ("n_exc", C.c_uint32),
                ("n_inh", C.c_uint32), ("uniform_rate", C.c_int32), ("learn", C.c_int32),
                ("trace_additive", C.c_int32), ("reduce", C.c_int32), ("precision", C.c_int32),
                ("path", C.c_int32), ("dt_ms", C.c_double), ("max_rate_hz", C.c_double),
                ("exc", snn_lif), ("inh", snn_lif), ("w_ei", C.c_double), ("w_ie", C.c_double),
                ("nu_pre", C.c_double), ("nu_post", C.c_double), ("tau_pre_ms", C.c_double),
                ("tau_post_ms", C.c_double), ("w_min", C.c_double), ("w_max", C.c_double),
                ("norm", C.c_double), ("seed", C.c_uint64), ("max_batch", C.c_uint32),
                ("norm_per_run", C.c_uint32), ("hbm_budget_bytes", C.c_uint64), ("reduce_tau", C.c_double)]


class snn_outputs(C.Structure):
    _fields_ = [("counts", C.c_void_p), ("raster_in", C.c_void_p), ("raster_exc", C.c_void_p),
                ("raster_inh", C.c_void_p), ("v_exc", C.c_void_p), ("v_inh", C.c_void_p)]


class snn_ifnet_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("n_in", C.c_uint32), ("n_h1", C.c_uint32), ("n_h2", C.c_uint32),
                ("n_out", C.c_uint32), ("max_batch", C.c_uint32), ("theta_h1", C.c_double),
                ("theta_h2", C.c_double)]


class snn_ifnet_outputs(C.Structure):
    _fields_ = [("out_sum", C.c_void_p), ("pred", C.c_void_p), ("counts_h1", C.c_void_p),
                ("counts_h2", C.c_void_p), ("raster_h1", C.c_void_p), ("raster_h2", C.c_void_p),
                ("v_h1", C.c_void_p), ("v_h2", C.c_void_p)]


_lib = None


def load_library():
    """Load ``libsnn.so`` after torch, so that both share one HIP runtime."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the process's HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    P, VP, U32, U64, I32, SZ = C.POINTER, C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32, C.c_size_t
    sig = {
        "snn_abi_version": ([], U32),
        "snn_last_error": ([], C.c_char_p),
        "snn_create": ([P(snn_config), VP, P(VP)], I32),
        "snn_destroy": ([VP], None),
        "snn_set_stream": ([VP, VP], I32),
        "snn_set_weights": ([VP, VP, SZ], I32),
        "snn_get_weights": ([VP, VP, SZ], I32),
        "snn_set_theta": ([VP, VP, SZ], I32),
        "snn_get_theta": ([VP, VP, SZ], I32),
        "snn_stdp_reduce": ([VP, I32], I32),
        "snn_stdp_reduce_soft": ([VP, C.c_double], I32),
        "snn_set_path": ([VP, I32, I32], I32),
        "snn_rebatch": ([VP, VP, U32, U32], I32),
        "snn_last_path": ([VP, P(I32)], I32),
        "snn_set_graphs": ([VP, I32], I32),
        "snn_run": ([VP, VP, VP, U32, U32, U32, P(snn_outputs)], I32),
        "snn_run_spikes": ([VP, VP, U32, U32, U32, P(snn_outputs)], I32),
        "snn_sync": ([VP], I32),
        "snn_state_bytes": ([P(snn_config), U32], SZ),
        "snn_profile_enable": ([VP, I32], I32),
        "snn_profile_get": ([VP, U32, C.c_char_p, SZ, P(U64), P(C.c_double)], I32),
        "snn_serve_create": ([VP, U32, U64, U32, P(VP)], I32),
        "snn_serve_submit": ([VP, VP, U64, U32, P(U64)], I32),
        "snn_serve_poll": ([VP, U64, VP, P(C.c_double)], I32),
        "snn_serve_stats": ([VP, P(U64), P(U64), P(U32), P(C.c_double)], I32),
        "snn_serve_destroy": ([VP], I32),
        "snn_ifnet_create": ([P(snn_ifnet_config), VP, P(VP)], I32),
        "snn_ifnet_destroy": ([VP], None),
        "snn_ifnet_set_layer": ([VP, U32, VP, SZ, VP, SZ], I32),
        "snn_ifnet_run": ([VP, VP, U32, U32, P(snn_ifnet_outputs)], I32),
        "snn_ifnet_run_noalloc": ([VP, VP, U32, U32, P(snn_ifnet_outputs)], I32),
        "snn_ifnet_sync": ([VP], I32),
    }
    for name, (args, res) in sig.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if lib.snn_abi_version() != SNN_ABI_VERSION:
        raise RuntimeError("libsnn.so ABI version mismatch")
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().snn_last_error()
        raise SnnError(status, msg.decode() if msg else "")


def make_config(cfg: dict, max_batch: int, path="plain", precision="fp32", hbm_budget: int = 0) -> snn_config:
    c = snn_config()
    c.abi_version = SNN_ABI_VERSION
    for k in ("n_in", "n_exc", "n_inh", "uniform_rate", "learn", "trace_additive", "reduce"):
        setattr(c, k, int(cfg[k]))
    for k in ("dt_ms", "max_rate_hz", "w_ei", "w_ie", "nu_pre", "nu_post", "tau_pre_ms",
              "tau_post_ms", "w_min", "w_max", "norm"):
        setattr(c, k, float(cfg[k]))
    for layer in ("exc", "inh"):
        L = getattr(c, layer)
        p = cfg[layer]
        for k in ("v_rest", "v_reset", "v_thresh", "tau_ms", "theta_plus", "tau_theta_ms"):
            setattr(L, k, float(p[k]))
        L.refrac_steps = int(p["refrac_steps"])
        L.adaptive = int(p["adaptive"])
    c.seed = int(cfg["seed"])
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.path = PATHS[path] if isinstance(path, str) else int(path)
    c.max_batch = int(max_batch)
    c.norm_per_run = int(cfg.get("norm_per_run", 0))
    c.hbm_budget_bytes = int(hbm_budget)
    c.reduce_tau = float(cfg.get("reduce_tau", 1.0))
    return c


def snn_state_bytes(cfg: dict, batch: int) -> int:
    c = make_config(cfg, max(batch, 1))
    return int(load_library().snn_state_bytes(C.byref(c), int(batch)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Net:
    """One network handle (``snn_create`` ... ``snn_destroy``)."""

    def __init__(self, cfg: dict, max_batch: int, path="plain", precision="fp32", hbm_budget: int = 0,
                 stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP path has no CPU fallback")
        self.lib = load_library()
        self.cfg = dict(cfg)
        self.c = make_config(cfg, max_batch, path, precision, hbm_budget)
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        h = C.c_void_p()
        _check(self.lib.snn_create(C.byref(self.c), C.c_void_p(s.cuda_stream), C.byref(h)))
        self.h = h
        self.n_in, self.n_exc = int(cfg["n_in"]), int(cfg["n_exc"])

    def close(self):
        if getattr(self, "h", None):
            self.lib.snn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters -----------------------------------------------------------
    def snn_set_weights(self, W: np.ndarray):
        w = np.ascontiguousarray(W, dtype=np.float32)
        assert w.shape == (self.n_in, self.n_exc)
        _check(self.lib.snn_set_weights(self.h, w.ctypes.data, w.size))

    def snn_get_weights(self) -> np.ndarray:
        w = np.zeros((self.n_in, self.n_exc), np.float32)
        _check(self.lib.snn_get_weights(self.h, w.ctypes.data, w.size))
        return w

    def snn_set_theta(self, th: np.ndarray):
        t = np.ascontiguousarray(th, dtype=np.float64)
        _check(self.lib.snn_set_theta(self.h, t.ctypes.data, t.size))

    def snn_get_theta(self) -> np.ndarray:
        t = np.zeros(self.n_exc, np.float64)
        _check(self.lib.snn_get_theta(self.h, t.ctypes.data, t.size))
        return t

    def snn_stdp_reduce(self, mode):
        _check(self.lib.snn_stdp_reduce(self.h, REDUCES[mode] if isinstance(mode, str) else int(mode)))

    def snn_stdp_reduce_soft(self, tau: float):
        _check(self.lib.snn_stdp_reduce_soft(self.h, float(tau)))

    def snn_set_path(self, path="plain", precision="fp32"):
        _check(self.lib.snn_set_path(self.h, PATHS[path] if isinstance(path, str) else int(path),
                                     PRECISIONS[precision] if isinstance(precision, str) else int(precision)))

    def snn_rebatch(self, keep, batch: int):
        """Re-form the batch without a reset: new slot k < len(keep) takes
        the state of current slot keep[k]; the other slots start fresh."""
        k = np.ascontiguousarray(np.asarray(keep, dtype=np.uint32))
        _check(self.lib.snn_rebatch(self.h, k.ctypes.data if k.size else None, int(k.size), int(batch)))

    def snn_set_graphs(self, on: bool = True):
        _check(self.lib.snn_set_graphs(self.h, 1 if on else 0))

    def snn_last_path(self) -> str:
        v = C.c_int32()
        _check(self.lib.snn_last_path(self.h, C.byref(v)))
        return {v_: k for k, v_ in PATHS.items()}.get(v.value, str(v.value))

    def snn_sync(self):
        _check(self.lib.snn_sync(self.h))

    def snn_profile_enable(self, on: bool = True):
        _check(self.lib.snn_profile_enable(self.h, 1 if on else 0))

    def snn_profile_get(self) -> dict:
        """{kernel name: (launches, total_ms)} accumulated since profiling on."""
        res, idx = {}, 0
        name = C.create_string_buffer(64)
        while True:
            n, ms = C.c_uint64(), C.c_double()
            st = self.lib.snn_profile_get(self.h, idx, name, 64, C.byref(n), C.byref(ms))
            if st == -5:
                break
            _check(st)
            res[name.value.decode()] = (int(n.value), float(ms.value))
            idx += 1
        return res

    # -- running --------------------------------------------------------------
    def _outputs(self, B, T, record):
        import torch
        dev = torch.device("cuda")
        ni_w = (self.n_in + 31) // 32
        ne_w = (self.n_exc + 31) // 32
        out = {}
        if "counts" in record:
            out["counts"] = torch.empty((B, self.n_exc), dtype=torch.int32, device=dev)
        if "in" in record:
            out["in"] = torch.empty((T, B, ni_w), dtype=torch.int32, device=dev)
        if "exc" in record:
            out["exc"] = torch.empty((T, B, ne_w), dtype=torch.int32, device=dev)
        if "inh" in record:
            out["inh"] = torch.empty((T, B, ne_w), dtype=torch.int32, device=dev)
        if "v_exc" in record:
            out["v_exc"] = torch.empty((T, B, self.n_exc), dtype=torch.float32, device=dev)
        if "v_inh" in record:
            out["v_inh"] = torch.empty((T, B, self.n_exc), dtype=torch.float32, device=dev)
        o = snn_outputs(_ptr(out.get("counts")), _ptr(out.get("in")), _ptr(out.get("exc")),
                        _ptr(out.get("inh")), _ptr(out.get("v_exc")), _ptr(out.get("v_inh")))
        return out, o

    def outputs(self, B: int, T: int, record=("counts",)) -> dict:
        """Device output tensors for a run of B samples and T steps, to be
        passed to snn_run(..., out=) (allocated once, reused by many runs)."""
        return self._outputs(B, T, record)[0]

    def snn_run(self, images, ids, T: int, reset: bool = True, record=("counts",), out=None):
        """images: cuda uint8 (B, n_in) or None (uniform rate); ids: cuda
        int64 (B,).  Returns the requested device outputs (asynchronous);
        with ``out`` (from ``outputs``) the run writes into those tensors."""
        B = int(ids.shape[0])
        assert ids.is_cuda and ids.dtype.itemsize == 8 and ids.is_contiguous()
        if images is not None:
            assert images.is_cuda and images.shape == (B, self.n_in) and images.is_contiguous()
        if out is None:
            out, o = self._outputs(B, T, record)
        else:
            o = snn_outputs(_ptr(out.get("counts")), _ptr(out.get("in")), _ptr(out.get("exc")),
                            _ptr(out.get("inh")), _ptr(out.get("v_exc")), _ptr(out.get("v_inh")))
        _check(self.lib.snn_run(self.h, _ptr(images), _ptr(ids), B, int(T),
                                SNN_RUN_RESET if reset else 0, C.byref(o)))
        return out

    def snn_run_spikes(self, in_bits, T: int, reset: bool = True, record=("counts",)):
        """in_bits: cuda int32 (T, B, ceil(n_in/32)) packed input spikes."""
        B = int(in_bits.shape[1])
        assert in_bits.is_cuda and in_bits.is_contiguous() and in_bits.shape[0] == T
        out, o = self._outputs(B, T, record)
        _check(self.lib.snn_run_spikes(self.h, _ptr(in_bits), B, int(T),
                                       SNN_RUN_RESET if reset else 0, C.byref(o)))
        return out


class Server:
    """Continuous-batching server over a frozen Net (snn_serve_* calls)."""

    def __init__(self, net: Net, max_slots: int, hbm_budget: int = 0, chunk_steps: int = 25):
        self.lib = net.lib
        self.net = net
        self.n_exc = net.n_exc
        h = C.c_void_p()
        _check(self.lib.snn_serve_create(net.h, int(max_slots), int(hbm_budget), int(chunk_steps), C.byref(h)))
        self.h = h

    def snn_serve_submit(self, image: np.ndarray, sample_id: int, T: int) -> int:
        img = np.ascontiguousarray(image, dtype=np.uint8)
        rid = C.c_uint64()
        _check(self.lib.snn_serve_submit(self.h, img.ctypes.data, int(sample_id), int(T), C.byref(rid)))
        return int(rid.value)

    def snn_serve_poll(self, req_id: int):
        """(counts, latency_s) when finished, None while queued or running."""
        counts = np.zeros(self.n_exc, np.uint32)
        lat = C.c_double()
        st = self.lib.snn_serve_poll(self.h, int(req_id), counts.ctypes.data, C.byref(lat))
        if st == -4:
            return None
        _check(st)
        return counts, float(lat.value)

    def snn_serve_stats(self) -> dict:
        c, s, pk, bs = C.c_uint64(), C.c_uint64(), C.c_uint32(), C.c_double()
        _check(self.lib.snn_serve_stats(self.h, C.byref(c), C.byref(s), C.byref(pk), C.byref(bs)))
        return {"completed": c.value, "slot_steps": s.value, "peak_active": pk.value, "busy_s": bs.value}

    def snn_serve_destroy(self):
        if getattr(self, "h", None):
            h, self.h = self.h, None
            _check(self.lib.snn_serve_destroy(h))

    def __del__(self):
        try:
            self.snn_serve_destroy()
        except Exception:
            pass


def make_ifnet_config(sizes, thresholds=(1.0, 1.0), max_batch: int = 1024) -> snn_ifnet_config:
    c = snn_ifnet_config()
    c.abi_version = SNN_ABI_VERSION
    c.n_in, c.n_h1, c.n_h2, c.n_out = (int(x) for x in sizes)
    c.max_batch = int(max_batch)
    c.theta_h1, c.theta_h2 = (float(x) for x in thresholds)
    return c


class IFNet:
    """Converted feed-forward IF network handle (``snn_ifnet_*`` calls)."""

    def __init__(self, sizes, thresholds=(1.0, 1.0), max_batch: int = 1024, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the HIP path has no CPU fallback")
        self.lib = load_library()
        self.sizes = tuple(int(x) for x in sizes)
        self.c = make_ifnet_config(self.sizes, thresholds, max_batch)
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        h = C.c_void_p()
        _check(self.lib.snn_ifnet_create(C.byref(self.c), C.c_void_p(s.cuda_stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.snn_ifnet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def snn_ifnet_set_layer(self, layer: int, W: np.ndarray, b: np.ndarray):
        w = np.ascontiguousarray(W, dtype=np.float32)
        bb = np.ascontiguousarray(b, dtype=np.float32)
        assert w.shape == (self.sizes[layer - 1], self.sizes[layer]) and bb.shape == (self.sizes[layer],)
        _check(self.lib.snn_ifnet_set_layer(self.h, int(layer), w.ctypes.data, w.size, bb.ctypes.data, bb.size))

    def set_layers(self, layers):
        for l, (W, b) in enumerate(layers, start=1):
            self.snn_ifnet_set_layer(l, W, b)

    def snn_ifnet_run(self, images, T: int, record=("out_sum", "pred"), noalloc: bool = False):
        """images: cuda uint8 (B, n_in).  Returns the requested device outputs
        (asynchronous): out_sum, pred, counts_h1/h2, raster_h1/h2, v_h1/h2.
        ``noalloc`` calls snn_ifnet_run_noalloc (scratch in the library's
        fixed device array instead of the handle's buffers)."""
        import torch
        B = int(images.shape[0])
        assert images.is_cuda and images.dtype == torch.uint8 and images.is_contiguous()
        assert images.shape == (B, self.sizes[0])
        dev = images.device
        n1, n2, no = self.sizes[1], self.sizes[2], self.sizes[3]
        shapes = {"out_sum": ((B, no), torch.float32), "pred": ((B,), torch.int32),
                  "counts_h1": ((B, n1), torch.int32), "counts_h2": ((B, n2), torch.int32),
                  "raster_h1": ((T, B, (n1 + 31) // 32), torch.int32),
                  "raster_h2": ((T, B, (n2 + 31) // 32), torch.int32),
                  "v_h1": ((T, B, n1), torch.float32), "v_h2": ((T, B, n2), torch.float32)}
        out = {k: torch.empty(shapes[k][0], dtype=shapes[k][1], device=dev) for k in record}
        o = snn_ifnet_outputs(*(_ptr(out.get(k)) for k in ("out_sum", "pred", "counts_h1", "counts_h2",
                                                           "raster_h1", "raster_h2", "v_h1", "v_h2")))
        fn = self.lib.snn_ifnet_run_noalloc if noalloc else self.lib.snn_ifnet_run
        _check(fn(self.h, _ptr(images), B, int(T), C.byref(o)))
        return out

    def snn_ifnet_sync(self):
        _check(self.lib.snn_ifnet_sync(self.h))


def unpack_bits(words, n: int) -> np.ndarray:
    """(..., n_words) int32/uint32 bit rasters -> (..., n) uint8 0/1."""
    w = np.ascontiguousarray(np.asarray(words)).astype(np.uint32)
    bytes_ = w.view(np.uint8).reshape(w.shape[:-1] + (w.shape[-1] * 4,))
    bits = np.unpackbits(bytes_, axis=-1, bitorder="little")
    return bits[..., :n]


def pack_bits(x: np.ndarray) -> np.ndarray:
    """(..., n) 0/1 -> (..., ceil(n/32)) uint32 packed, bit k of word k // 32."""
    x = np.asarray(x, dtype=np.uint8)
    n = x.shape[-1]
    nw = (n + 31) // 32
    pad = np.zeros(x.shape[:-1] + (nw * 32,), np.uint8)
    pad[..., :n] = x
    by = np.packbits(pad, axis=-1, bitorder="little")
    return np.ascontiguousarray(by).view(np.uint32)
