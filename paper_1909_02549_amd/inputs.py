"""Seeded synthetic inputs and workload presets.

This module is shared by the oracle-side tests and the HIP path.  It holds no
arithmetic of the simulated method: only random inputs (stroke images, initial
weights, sample ids, serving arrival times) and the parameter values of the
workloads, so that both sides receive byte-identical inputs.

The paper trains on MNIST digits (Unsupervised Learning section) and uses
random Poisson rates and random Gaussian weights for its scaling experiment
(Scaling a Two Layer Network section).  Neither dataset is available here; the
images below are synthetic pen strokes of the same 28x28 uint8 shape and a
comparable fraction of nonzero pixels.  No dataset item is reproduced.
"""

from __future__ import annotations

import numpy as np

IMG_SIDE = 28
N_PIXELS = IMG_SIDE * IMG_SIDE  # 784


# ---------------------------------------------------------------------------
# synthetic stroke images
# ---------------------------------------------------------------------------

def _gauss_kernel(sigma: float) -> np.ndarray:
    r = int(np.ceil(3 * sigma))
    x = np.arange(-r, r + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sigma) ** 2)
    return k / k.sum()


def _blur(img: np.ndarray, sigma: float) -> np.ndarray:
    k = _gauss_kernel(sigma)
    out = np.apply_along_axis(lambda r: np.convolve(r, k, mode="same"), 1, img)
    out = np.apply_along_axis(lambda c: np.convolve(c, k, mode="same"), 0, out)
    return out


def stroke_image(seed: int, index: int, density: float | tuple = 0.19) -> np.ndarray:
    """One 28x28 uint8 image of 1-4 blurred quadratic Bezier pen strokes.

    ``density`` is the target fraction of nonzero pixels (a float), or a
    ``(lo, hi)`` range from which it is drawn uniformly per image.  The image
    depends only on ``(seed, index)``, never on the batch it is placed in.
    """
    rng = np.random.default_rng([int(seed), int(index)])
    if isinstance(density, tuple):
        dens = float(rng.uniform(density[0], density[1]))
    else:
        dens = float(density)
    yy, xx = np.mgrid[0:IMG_SIDE, 0:IMG_SIDE].astype(np.float64)
    canvas = np.zeros((IMG_SIDE, IMG_SIDE))
    n_strokes = int(rng.integers(1, 5))
    for _ in range(n_strokes):
        p = rng.uniform(4.0, 24.0, size=(3, 2))
        width = rng.uniform(1.5, 2.5)
        s = np.linspace(0.0, 1.0, 64)[:, None]
        pts = (1 - s) ** 2 * p[0] + 2 * (1 - s) * s * p[1] + s ** 2 * p[2]
        d2 = (yy[None] - pts[:, 0, None, None]) ** 2 + (xx[None] - pts[:, 1, None, None]) ** 2
        d = np.sqrt(d2.min(axis=0))
        canvas = np.maximum(canvas, np.clip(1.0 - (d - 0.5 * width), 0.0, 1.0))
    canvas = _blur(canvas, 1.0)
    flat = canvas.ravel()
    keep = max(1, int(round(dens * N_PIXELS)))
    order = np.argsort(-flat, kind="stable")
    out = np.zeros(N_PIXELS, dtype=np.float64)
    top = flat[order[:keep]]
    peak = top[0] if top[0] > 0 else 1.0
    out[order[:keep]] = np.maximum(1.0, np.round(255.0 * top / peak))
    return out.astype(np.uint8)


def stroke_images(n: int, seed: int, density: float | tuple = 0.19, start: int = 0) -> np.ndarray:
    """``n`` stroke images, shape (n, 784) uint8; image k uses ``(seed, start + k)``."""
    return np.stack([stroke_image(seed, start + k, density) for k in range(n)])


# ---------------------------------------------------------------------------
# initial weights and ids
# ---------------------------------------------------------------------------

def uniform_weights(n_in: int, n_out: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Row-major (n_in, n_out) float32 weights drawn from U(lo, hi)."""
    rng = np.random.default_rng([int(seed), 0x5741])
    return rng.uniform(lo, hi, size=(n_in, n_out)).astype(np.float32)


def normal_weights(n_in: int, n_out: int, mean: float, std: float, seed: int) -> np.ndarray:
    """Row-major (n_in, n_out) float32 weights drawn from N(mean, std^2)."""
    rng = np.random.default_rng([int(seed), 0x4E57])
    return rng.normal(mean, std, size=(n_in, n_out)).astype(np.float32)


def frozen_weights(n_in: int, n_out: int, col_sum: float, seed: int, alpha: float = 3.0) -> np.ndarray:
    """Row-major (n_in, n_out) float32 weights of a frozen (inference) network
    whose columns sum to ``col_sum``: each column is ``col_sum`` times a draw
    from a symmetric Dirichlet distribution of concentration ``alpha``.  Its
    entries have mean col_sum / n_in and coefficient of variation about
    1 / sqrt(alpha) (0.58 at alpha = 3, that of U(0, 0.3) weights)."""
    rng = np.random.default_rng([int(seed), 0x465A])
    cols = rng.dirichlet(np.full(n_in, float(alpha)), size=n_out)
    return (col_sum * cols.T).astype(np.float32)


def conversion_mlp(sizes=(784, 256, 128, 10), seed: int = 0, calib_images: np.ndarray | None = None,
                   percentile: float = 99.9) -> list:
    """Stand-in for the trained MLP of the conversion experiment (ANN to SNN
    conversion section), prepared for IF neurons with threshold 1.

    No trained network exists here, so the weights are random: He-normal
    N(0, 2 / fan_in) and biases N(0, 0.01^2), float64 draws.  They are then
    rescaled layer by layer as the conversion method prescribes (data-based
    normalisation, Rueckauer et al. 2017): lambda_l is the given percentile
    of layer l's ReLU activations on calibration images (pixels / 255), and
    W_l, b_l become W_l * lambda_{l-1} / lambda_l and b_l / lambda_l
    (lambda_0 = 1; the output layer keeps lambda_L = 1).  Returns
    [(W_l float32 (n_{l-1}, n_l), b_l float32 (n_l,)), ...].
    """
    rng = np.random.default_rng([int(seed), 0x434E])
    raw = []
    for n0, n1 in zip(sizes[:-1], sizes[1:]):
        raw.append((rng.normal(0.0, np.sqrt(2.0 / n0), size=(n0, n1)), rng.normal(0.0, 0.01, size=n1)))
    if calib_images is None:
        calib_images = stroke_images(256, 0xCA1B, 0.19)
    a = np.asarray(calib_images, np.float64) / 255.0
    lam_prev, out = 1.0, []
    for l, (W, b) in enumerate(raw):
        z = a @ W + b
        if l == len(raw) - 1:
            lam = 1.0
        else:
            a = np.maximum(z, 0.0)
            pos = a[a > 0]
            lam = float(np.percentile(pos, percentile)) if pos.size else 1.0
        out.append(((W * (lam_prev / lam)).astype(np.float32), (b / lam).astype(np.float32)))
        lam_prev = lam
    return out


def sample_ids(n: int, base: int = 0) -> np.ndarray:
    """Per-sample ids; the Poisson encoder is keyed by id, not batch slot."""
    return (np.arange(n, dtype=np.uint64) + np.uint64(base)).astype(np.uint64)


def poisson_arrivals(n: int, rate_hz: float, seed: int = 1) -> np.ndarray:
    """Arrival times (s) of a Poisson process with ``rate_hz`` requests/s."""
    rng = np.random.default_rng([int(seed), 0x5356])
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n))


def request_durations(n: int, choices=(100, 250, 500), seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng([int(seed), 0x4455])
    return rng.choice(np.asarray(choices, dtype=np.uint32), size=n)


# ---------------------------------------------------------------------------
# workload presets (parameter values only)
# ---------------------------------------------------------------------------

# Diehl & Cook style excitatory (adaptive threshold) and inhibitory LIF layers.
DC_EXC = dict(v_rest=-65.0, v_reset=-60.0, v_thresh=-52.0, tau_ms=100.0, refrac_steps=5,
              adaptive=1, theta_plus=0.05, tau_theta_ms=1e7)
DC_INH = dict(v_rest=-60.0, v_reset=-45.0, v_thresh=-40.0, tau_ms=10.0, refrac_steps=2,
              adaptive=0, theta_plus=0.0, tau_theta_ms=1e7)
# Plain LIF layer of the batch-scaling workload (no reset / refractory stated:
# reset to rest and 5 refractory steps are the documented readings).
SCALING_LIF = dict(v_rest=-65.0, v_reset=-65.0, v_thresh=-52.0, tau_ms=100.0, refrac_steps=5,
                   adaptive=0, theta_plus=0.0, tau_theta_ms=1e7)

REDUCE = {"sum": 0, "mean": 1, "max": 2, "max_signed": 3, "soft_max": 4}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2}


def dc_config(n_exc: int, learn: bool = True, reduce: str = "mean", seed: int = 0,
              n_in: int = N_PIXELS, **over) -> dict:
    """Diehl & Cook style network: Poisson inputs -> adaptive-LIF exc layer
    with a one-to-one exc->inh layer and all-but-self inh->exc inhibition."""
    cfg = dict(
        n_in=n_in, n_exc=n_exc, n_inh=n_exc,
        dt_ms=1.0, max_rate_hz=128.0, uniform_rate=0, learn=int(bool(learn)),
        exc=dict(DC_EXC), inh=dict(DC_INH), w_ei=22.5, w_ie=-120.0,
        nu_pre=1e-4, nu_post=1e-2, tau_pre_ms=20.0, tau_post_ms=20.0,
        w_min=0.0, w_max=1.0, norm=78.4, trace_additive=0,
        reduce=REDUCE[reduce] if isinstance(reduce, str) else int(reduce), seed=seed,
    )
    for k, v in over.items():
        if k in ("exc", "inh"):
            cfg[k] = dict(cfg[k], **v)
        else:
            cfg[k] = v
    return cfg


def scaling_config(n_in: int = 1000, n_out: int = 1000, rate_hz: float = 20.0, seed: int = 0) -> dict:
    """Two-layer batch-scaling network: uniform-rate Poisson inputs -> LIF
    layer, dense weights, no inhibition and no learning."""
    return dict(
        n_in=n_in, n_exc=n_out, n_inh=0, dt_ms=1.0, max_rate_hz=rate_hz, uniform_rate=1,
        learn=0, exc=dict(SCALING_LIF), inh=dict(DC_INH), w_ei=0.0, w_ie=0.0,
        nu_pre=0.0, nu_post=0.0, tau_pre_ms=20.0, tau_post_ms=20.0, w_min=0.0, w_max=1.0,
        norm=0.0, trace_additive=0, reduce=REDUCE["mean"], seed=seed,
    )


def workload(name: str) -> dict:
    """Named workloads (shapes, densities and seeds) used by tests and bench.

    dc100   784->100/100, B=4, T=100, learning, mean reduction (parity case)
    scale   1000 uniform-20Hz inputs -> 1000 LIF, no learning, T=1000
    dc400   784->400/400, T=250, learning, reduction sum/mean/max
    dc6400  784->6400/6400, B=256, T=350, learning, 10-30 % nonzero images
    shard8  784->800/800, otherwise as dc6400: the per-GPU column share of
            dc6400 split over 8 GPUs (its own inhibition only: the count
            exchange between shards is not part of it)
    serve   frozen 784->1600/1600 inference, T in {100,250,500}
    conv    converted IF network 784-256-128-10, B=1024, T=10, 10000 images
    """
    if name == "dc100":
        return dict(cfg=dc_config(100), B=4, T=100, density=0.19, wlo=0.0, whi=0.3)
    if name == "scale":
        return dict(cfg=scaling_config(), B=64, T=1000, density=None, wmean=0.05, wstd=0.02)
    if name == "dc400":
        return dict(cfg=dc_config(400), B=64, T=250, density=0.19, wlo=0.0, whi=0.3)
    if name == "dc6400":
        return dict(cfg=dc_config(6400), B=256, T=350, density=(0.10, 0.30), wlo=0.0, whi=0.3)
    if name == "shard8":
        return dict(cfg=dc_config(800), B=256, T=350, density=(0.10, 0.30), wlo=0.0, whi=0.3)
    if name == "serve":
        return dict(cfg=dc_config(1600, learn=False), B=4096, T=None, density=0.19, wlo=0.0, whi=0.3)
    if name == "conv":
        return dict(sizes=(784, 256, 128, 10), thresholds=(1.0, 1.0), B=1024, T=10, n_images=10000,
                    density=0.19, seed=0)
    raise KeyError(name)
