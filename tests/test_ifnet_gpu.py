"""GPU parity of the converted IF network (ANN to SNN conversion section)
against the FP64 oracle, through the C ABI (snn_ifnet_*).

Bars (FP32 path against FP64):
- spike rasters of both hidden layers agree in >= 99.9 % of (sample, step,
  neuron) entries, and at a sample's first differing step every differing
  entry of the first layer that differs is an oracle near-tie (voltage before
  the reset within 1e-3 of the threshold);
- voltages agree within 1e-3 + 4e-6 |v| (threshold units) before a
  sample's first differing step: a neuron driven above threshold keeps the
  excess, so its voltage grows with the run (about 10^3 after 300 steps,
  where FP32 spacing is 6e-5 and hundreds of rounded additions accumulate
  past 1e-3); the relative term is the one of the learning network's
  voltage bar;
- samples that never differ: spike counts equal, summed output input within
  the FP32 summation bound gamma_m * sum |terms| (m = the number of terms
  added per output: 3 planes x 16-deep chunks x steps, plus the partial sums
  and the bias term), and the predicted class equal unless the oracle's two
  largest sums are closer than twice that bound.
"""
import numpy as np
import pytest

from oracle.ifnet import OracleIFNet
from paper_1909_02549_amd import inputs

pytestmark = pytest.mark.gpu

RASTER_AGREE = 0.999
V_TOL = 1e-3
V_RTOL = 4e-6
TIE_TOL = 1e-3
U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gamma(m):
    return m * U / (1 - m * U)


def run_gpu(torch, layers, thresholds, imgs, T, max_batch=None):
    from paper_1909_02549_amd.snn import IFNet, unpack_bits
    sizes = (layers[0][0].shape[0],) + tuple(W.shape[1] for W, _ in layers)
    net = IFNet(sizes, thresholds, max_batch=max_batch or len(imgs))
    net.set_layers(layers)
    out = net.snn_ifnet_run(torch.from_numpy(imgs).cuda(), T,
                            record=("out_sum", "pred", "counts_h1", "counts_h2", "raster_h1", "raster_h2",
                                    "v_h1", "v_h2"))
    net.snn_ifnet_sync()
    g = {"out": out["out_sum"].cpu().numpy(), "pred": out["pred"].cpu().numpy(),
         "c1": out["counts_h1"].cpu().numpy(), "c2": out["counts_h2"].cpu().numpy(),
         "s1": unpack_bits(out["raster_h1"].cpu().numpy(), sizes[1]).transpose(1, 0, 2),
         "s2": unpack_bits(out["raster_h2"].cpu().numpy(), sizes[2]).transpose(1, 0, 2),
         "v1": out["v_h1"].cpu().numpy().transpose(1, 0, 2), "v2": out["v_h2"].cpu().numpy().transpose(1, 0, 2)}
    net.close()
    return g


def check(g, ref, layers, thresholds, T, min_clean=0.95, spikes=True):
    B = ref["out"].shape[0]
    for k in ("s1", "s2"):
        agree = (g[k] == ref[k]).mean()
        assert agree >= RASTER_AGREE, f"{k} raster agreement {agree}"
    if spikes:  # the case exercises both spiking layers
        assert ref["s1"].sum() > 0 and ref["s2"].sum() > 0
    d1 = (g["s1"] != ref["s1"]).any(axis=2)
    d2 = (g["s2"] != ref["s2"]).any(axis=2)
    diff = d1 | d2
    t_div = np.where(diff.any(axis=1), diff.argmax(axis=1), T)
    for b in np.nonzero(t_div < T)[0]:
        t = t_div[b]
        key, ukey, th = ("s1", "u1", thresholds[0]) if d1[b, t] else ("s2", "u2", thresholds[1])
        units = np.nonzero(g[key][b, t] != ref[key][b, t])[0]
        margin = np.abs(ref[ukey][b, t, units] - th).max()
        assert margin < TIE_TOL, f"sample {b} step {t}: {key} differs away from a near-tie ({margin})"
    for key in ("v1", "v2"):
        for b in range(B):
            t = t_div[b]
            if t:
                vr = ref[key][b, :t]
                dv = np.abs(g[key][b, :t] - vr)
                assert (dv <= V_TOL + V_RTOL * np.abs(vr)).all(), f"sample {b}: {key} error {dv.max()} before step {t}"
    clean = t_div == T
    assert clean.mean() >= min_clean, f"only {clean.mean():.3f} of the samples never differ"
    assert np.array_equal(g["c1"][clean], ref["c1"][clean])
    assert np.array_equal(g["c2"][clean], ref["c2"][clean])
    W3, b3 = (x.astype(np.float64) for x in layers[2])
    k3 = (W3.shape[0] + 15) // 16
    bound = gamma(3 * 16 * k3 * T + 6) * (ref["c2"] @ np.abs(W3) + T * np.abs(b3)) + 1e-30
    err = np.abs(g["out"] - ref["out"])
    assert (err[clean] <= bound[clean]).all(), f"readout error {(err / bound)[clean].max()} x the bound"
    top2 = np.sort(ref["out"], axis=1)[:, -2:] if ref["out"].shape[1] > 1 else None
    for b in np.nonzero(clean)[0]:
        if top2 is None or top2[b, 1] - top2[b, 0] > 2 * bound[b].max():
            assert g["pred"][b] == ref["pred"][b], f"sample {b}: class {g['pred'][b]} vs {ref['pred'][b]}"
    return clean


def oracle_run(layers, thresholds, imgs, T):
    return OracleIFNet([(W.astype(np.float64), b.astype(np.float64)) for W, b in layers], thresholds).run(
        imgs, T, record=("s1", "s2", "v1", "v2", "u1", "u2", "c1", "c2"))


@pytest.fixture(scope="module")
def conv():
    wl = inputs.workload("conv")
    return wl, inputs.conversion_mlp(wl["sizes"], wl["seed"])


def test_conversion_full_batch(torch_cuda, conv):
    """784-256-128-10 at B = 1024, T = 10: the configuration of the
    conversion timing, every sample checked."""
    wl, layers = conv
    imgs = inputs.stroke_images(wl["B"], 21, wl["density"])
    g = run_gpu(torch_cuda, layers, wl["thresholds"], imgs, wl["T"])
    ref = oracle_run(layers, wl["thresholds"], imgs, wl["T"])
    check(g, ref, layers, wl["thresholds"], wl["T"])


@pytest.mark.parametrize("B,T", [(1, 1), (37, 25), (33, 3)])
def test_conversion_ragged_batches(torch_cuda, conv, B, T):
    wl, layers = conv
    imgs = inputs.stroke_images(B, 22, wl["density"])
    g = run_gpu(torch_cuda, layers, wl["thresholds"], imgs, T, max_batch=64)
    ref = oracle_run(layers, wl["thresholds"], imgs, T)
    check(g, ref, layers, wl["thresholds"], T, min_clean=0.9 if B > 1 else 1.0, spikes=B * T > 1)


def test_odd_layer_sizes_and_thresholds(torch_cuda):
    """100 inputs (no 8-pixel loads), 40 and 24 hidden neurons (ragged tiles
    and chunks), 3 outputs, thresholds 0.75 and 1.5."""
    sizes, th = (100, 40, 24, 3), (0.75, 1.5)
    layers = inputs.conversion_mlp(sizes, 5, calib_images=inputs.stroke_images(128, 9, 0.19)[:, :100])
    imgs = np.ascontiguousarray(inputs.stroke_images(70, 23, 0.3)[:, 300:400])
    T = 12
    g = run_gpu(torch_cuda, layers, th, imgs, T)
    ref = oracle_run(layers, th, imgs, T)
    check(g, ref, layers, th, T, min_clean=0.9)


def test_largest_layer_sizes(torch_cuda):
    """The largest supported layers: 256 and 128 hidden neurons, 32 outputs,
    with 1000 inputs."""
    sizes = (1000, 256, 128, 32)
    calib = np.random.default_rng(3).integers(0, 256, size=(128, 1000)).astype(np.uint8)
    layers = inputs.conversion_mlp(sizes, 6, calib_images=calib)
    imgs = np.random.default_rng(4).integers(0, 256, size=(64, 1000)).astype(np.uint8)
    T = 8
    g = run_gpu(torch_cuda, layers, (1.0, 1.0), imgs, T)
    ref = oracle_run(layers, (1.0, 1.0), imgs, T)
    check(g, ref, layers, (1.0, 1.0), T, min_clean=0.9)


def test_sample_results_do_not_depend_on_the_batch(torch_cuda, conv):
    """A sample's outputs are bit-identical alone, in a small batch and in a
    large one (its rows of every tile are computed independently)."""
    torch = torch_cuda
    from paper_1909_02549_amd.snn import IFNet
    wl, layers = conv
    imgs = inputs.stroke_images(300, 24, wl["density"])
    net = IFNet(wl["sizes"], wl["thresholds"], max_batch=300)
    net.set_layers(layers)
    rec = ("out_sum", "pred", "raster_h1", "raster_h2")
    full = net.snn_ifnet_run(torch.from_numpy(imgs).cuda(), 10, record=rec)
    part = net.snn_ifnet_run(torch.from_numpy(np.ascontiguousarray(imgs[100:140])).cuda(), 10, record=rec)
    one = net.snn_ifnet_run(torch.from_numpy(np.ascontiguousarray(imgs[123:124])).cuda(), 10, record=rec)
    again = net.snn_ifnet_run(torch.from_numpy(imgs).cuda(), 10, record=rec)
    net.snn_ifnet_sync()
    for k in rec:
        f = full[k].cpu().numpy()
        bd = 1 if k.startswith("raster") else 0
        sl = [slice(None)] * f.ndim
        sl[bd] = slice(100, 140)
        assert np.array_equal(f[tuple(sl)], part[k].cpu().numpy()), k
        sl[bd] = slice(123, 124)
        assert np.array_equal(f[tuple(sl)], one[k].cpu().numpy()), k
        assert np.array_equal(f, again[k].cpu().numpy()), k
    net.close()


def test_run_errors(torch_cuda, conv):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import IFNet, SnnError
    wl, layers = conv
    net = IFNet(wl["sizes"], wl["thresholds"], max_batch=8)
    imgs = torch.zeros((8, 784), dtype=torch.uint8, device="cuda")
    with pytest.raises(SnnError, match="EINVAL"):  # layers not set
        net.snn_ifnet_run(imgs, 5)
    W1, b1 = layers[0]
    assert net.lib.snn_ifnet_set_layer(net.h, 1, W1.ctypes.data, W1.size, b1.ctypes.data, 3) == -1
    assert net.lib.snn_ifnet_set_layer(net.h, 4, W1.ctypes.data, W1.size, b1.ctypes.data, b1.size) == -1
    assert net.lib.snn_ifnet_set_layer(net.h, 2, W1.ctypes.data, W1.size, b1.ctypes.data, b1.size) == -1
    net.set_layers(layers)
    big = torch.zeros((9, 784), dtype=torch.uint8, device="cuda")
    with pytest.raises(SnnError, match="ENOMEM"):
        net.snn_ifnet_run(big, 5)
    with pytest.raises(SnnError, match="EINVAL"):
        net.snn_ifnet_run(imgs, 0)
    assert net.lib.snn_ifnet_run(net.h, None, 8, 5, None) == -1
    out = net.snn_ifnet_run(imgs, 3)
    net.snn_ifnet_sync()
    # blank images: the first layer sees only its biases, every sample alike
    o = out["out_sum"].cpu().numpy()
    assert o.shape == (8, 10) and (o == o[0]).all()
    net.close()
    assert net.lib.snn_ifnet_sync(None) == -1
    assert net.lib.snn_ifnet_set_layer(None, 1, None, 0, None, 0) == -1


def test_long_run(torch_cuda, conv):
    """T = 300 (long accumulations; 16-bit packed spike counters).  Over this
    many steps an FP32 near-tie flip becomes likely in some samples, so the
    bar is the raster agreement, the near-tie rule at each sample's first
    differing step, and exact counts and readout where nothing differed."""
    wl, layers = conv
    imgs = inputs.stroke_images(40, 25, wl["density"])
    T = 300
    g = run_gpu(torch_cuda, layers, wl["thresholds"], imgs, T)
    ref = oracle_run(layers, wl["thresholds"], imgs, T)
    check(g, ref, layers, wl["thresholds"], T, min_clean=0.0)
    assert g["c1"].max() > 255 or g["c2"].max() > 255 or ref["c1"].max() <= 255
