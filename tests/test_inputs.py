"""CPU tests of the seeded synthetic inputs (shared by oracle and HIP runs)."""
import numpy as np

from paper_1909_02549_amd import inputs


def test_stroke_images_shape_density_determinism():
    a = inputs.stroke_images(8, 5, 0.19)
    b = inputs.stroke_images(8, 5, 0.19)
    assert a.shape == (8, 784) and a.dtype == np.uint8
    assert np.array_equal(a, b)
    assert np.allclose((a > 0).mean(axis=1), 0.19, atol=0.002)
    assert a.max() == 255
    c = inputs.stroke_images(8, 5, (0.1, 0.3))
    d = (c > 0).mean(axis=1)
    assert d.min() >= 0.099 and d.max() <= 0.301


def test_image_depends_only_on_seed_and_index():
    a = inputs.stroke_images(4, 9, 0.2, start=10)
    b = np.stack([inputs.stroke_image(9, 10 + k, 0.2) for k in range(4)])
    assert np.array_equal(a, b)


def test_weights_and_arrivals():
    w = inputs.uniform_weights(784, 10, 0.0, 0.3, 0)
    assert w.dtype == np.float32 and 0 <= w.min() and w.max() < 0.3
    f = inputs.frozen_weights(784, 50, 78.4, 0)
    assert f.dtype == np.float32 and f.min() > 0 and np.array_equal(f, inputs.frozen_weights(784, 50, 78.4, 0))
    assert np.allclose(f.astype(np.float64).sum(0), 78.4, rtol=1e-5)
    assert abs(f.mean() - 0.1) < 2e-3 and abs(f.std() / f.mean() - 1 / np.sqrt(3.0)) < 0.02
    t = inputs.poisson_arrivals(20000, 5000.0)
    assert abs(np.diff(t).mean() - 1 / 5000.0) < 1e-5
    T = inputs.request_durations(3000)
    assert set(np.unique(T)) == {100, 250, 500}


def test_conversion_mlp_is_seeded_and_shaped():
    """The converted network's weights depend only on the seed (and the
    calibration images); shapes and dtypes follow the layer sizes."""
    from paper_1909_02549_amd.inputs import conversion_mlp, stroke_images
    calib = stroke_images(32, 5, 0.19)
    a = conversion_mlp((784, 64, 32, 10), 3, calib_images=calib)
    b = conversion_mlp((784, 64, 32, 10), 3, calib_images=calib)
    c = conversion_mlp((784, 64, 32, 10), 4, calib_images=calib)
    assert [w.shape for w, _ in a] == [(784, 64), (64, 32), (32, 10)]
    assert [bb.shape for _, bb in a] == [(64,), (32,), (10,)]
    assert all(w.dtype == np.float32 and bb.dtype == np.float32 for w, bb in a)
    assert all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) for x, y in zip(a, b))
    assert not np.array_equal(a[0][0], c[0][0])
