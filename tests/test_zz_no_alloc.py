"""GPU test of snn_ifnet_run_noalloc, the converted network's run with its
scratch in the library's fixed device array (for callers that cannot
allocate): through the C ABI, its outputs equal snn_ifnet_run's bit for bit
on two calls in a row, the second with a smaller batch (so the array holds
the first call's larger contents when the second starts), and a batch beyond
the array's capacity is refused before anything runs."""
import numpy as np
import pytest

from paper_1909_02549_amd import inputs

pytestmark = pytest.mark.gpu

KEYS = ("out_sum", "pred", "counts_h1", "counts_h2", "raster_h1", "raster_h2", "v_h1", "v_h2")


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_noalloc_equals_run_on_two_calls(torch_cuda):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import IFNet
    wl = inputs.workload("conv")
    sizes, T = wl["sizes"], 12
    layers = inputs.conversion_mlp(sizes, wl["seed"])
    imgs = torch.from_numpy(inputs.stroke_images(1100, 77, wl["density"])).cuda()
    net = IFNet(sizes, wl["thresholds"], max_batch=1100)
    net.set_layers(layers)
    for B in (1100, 45):
        x = imgs[:B].contiguous()
        ref = net.snn_ifnet_run(x, T, record=KEYS)
        got = net.snn_ifnet_run(x, T, record=KEYS, noalloc=True)
        torch.cuda.synchronize()
        for k in KEYS:
            a, b = ref[k].cpu().numpy(), got[k].cpu().numpy()
            assert np.array_equal(a, b), f"B={B}: {k} differs between snn_ifnet_run and the no-allocation run"
        assert ref["counts_h1"].sum().item() > 0
    net.close()


def test_noalloc_refuses_batches_beyond_its_array(torch_cuda):
    torch = torch_cuda
    from paper_1909_02549_amd.snn import IFNet, SnnError
    wl = inputs.workload("conv")
    sizes = wl["sizes"]
    net = IFNet(sizes, wl["thresholds"], max_batch=8)
    net.set_layers(inputs.conversion_mlp(sizes, wl["seed"]))
    # 256 h1 and 128 h2 neurons take (256 + 128) * 4 bytes per sample of the
    # 6 MiB array: 4096 samples fit, 4097 do not
    x = torch.zeros((4097, sizes[0]), dtype=torch.uint8, device="cuda")
    with pytest.raises(SnnError) as e:
        net.snn_ifnet_run(x, 10, record=("pred",), noalloc=True)
    assert e.value.status == -2
    out = net.snn_ifnet_run(x[:4096].contiguous(), 10, record=("pred",), noalloc=True)
    torch.cuda.synchronize()
    assert out["pred"].shape[0] == 4096
    net.close()
