"""GPU tests of the continuous-batching server (snn_serve_*).

A request's spike counts must not depend on which other requests share the
device batch: each request run alone and the same request in a mix of
concurrent requests of different durations give identical counts, and both
agree with the FP64 oracle run of that single sample.
"""
import time

import numpy as np
import pytest

from paper_1909_02549_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def frozen_net(n_exc=64, path="auto"):
    from paper_1909_02549_amd.snn import Net
    cfg = inputs.dc_config(n_exc, learn=False)
    W = inputs.frozen_weights(784, n_exc, 78.4, 7)
    net = Net(cfg, max_batch=1, path=path)
    net.snn_set_weights(W)
    return cfg, W, net


def wait_all(srv, rids, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(rids):
        for r in rids:
            if r in out:
                continue
            res = srv.snn_serve_poll(r)
            if res is not None:
                out[r] = res
        assert time.time() - t0 < timeout, "serving did not finish"
        time.sleep(0.001)
    return out


@pytest.mark.parametrize("path", ["auto", "plain", "fused", "persistent", "mfma"])
def test_alone_equals_mix_and_oracle(torch_cuda, oracle_mod, path):
    """Ten requests of mixed lengths through six slots: chunks run in full
    with per-slot count limits, finished slots' places are taken by moving
    the highest active slots down, new requests join above them.  Every
    request's counts equal its run alone, bit for bit, on every path."""
    from paper_1909_02549_amd.snn import Server
    cfg, W, net = frozen_net(path=path)
    imgs = inputs.stroke_images(10, 33, 0.19)
    Ts = [20, 50, 80, 20, 50, 80, 35, 64, 17, 90]
    ids = list(range(500, 510))
    alone = []
    srv1 = Server(net, max_slots=1, chunk_steps=16)
    for k in range(10):
        rid = srv1.snn_serve_submit(imgs[k], ids[k], Ts[k])
        alone.append(wait_all(srv1, [rid])[rid][0])
    srv1.snn_serve_destroy()
    srv = Server(net, max_slots=6, chunk_steps=16)
    rids = [srv.snn_serve_submit(imgs[k], ids[k], Ts[k]) for k in range(10)]
    res = wait_all(srv, rids)
    st = srv.snn_serve_stats()
    srv.snn_serve_destroy()
    assert st["completed"] == 10 and st["peak_active"] > 1
    for k, r in enumerate(rids):
        assert np.array_equal(res[r][0], alone[k]), f"request {k} differs alone vs in the mix"
    agree = []
    for k in range(10):
        orc = oracle_mod.OracleNet(cfg, W.astype(np.float64))
        ref = orc.run(imgs[k:k + 1], np.array([ids[k]], np.uint64), Ts[k], record=("counts",))
        agree.append((ref["counts"][0] == alone[k]).mean())
    assert min(agree) >= 0.99, agree
    assert sum(a.sum() for a in alone) > 0


def test_budget_queues_instead_of_dropping(torch_cuda):
    from paper_1909_02549_amd.snn import Server, snn_state_bytes
    cfg, W, net = frozen_net()
    budget = snn_state_bytes(cfg, 2) + 1
    srv = Server(net, max_slots=64, hbm_budget=budget, chunk_steps=10)
    imgs = inputs.stroke_images(6, 3, 0.19)
    rids = [srv.snn_serve_submit(imgs[k], 900 + k, 30) for k in range(6)]
    res = wait_all(srv, rids)
    st = srv.snn_serve_stats()
    srv.snn_serve_destroy()
    assert len(res) == 6 and st["completed"] == 6
    assert 1 <= st["peak_active"] <= 2


def test_error_paths(torch_cuda):
    from paper_1909_02549_amd.snn import Net, Server, SnnError
    cfg, W, net = frozen_net()
    srv = Server(net, max_slots=4, hbm_budget=1, chunk_steps=10)
    with pytest.raises(SnnError) as e:
        srv.snn_serve_submit(np.zeros(784, np.uint8), 1, 10)
    assert e.value.status == -2
    srv.snn_serve_destroy()
    srv = Server(net, max_slots=4, chunk_steps=10)
    with pytest.raises(SnnError) as e:
        srv.snn_serve_poll(12345)
    assert e.value.status == -5
    rid = srv.snn_serve_submit(np.zeros(784, np.uint8), 1, 5)
    wait_all(srv, [rid])
    with pytest.raises(SnnError) as e:
        srv.snn_serve_poll(rid)
    assert e.value.status == -5
    with pytest.raises(SnnError):
        srv.snn_serve_submit(np.zeros(784, np.uint8), 1, 0)
    srv.snn_serve_destroy()
    learn_net = Net(inputs.dc_config(16), max_batch=2)
    with pytest.raises(SnnError) as e:
        Server(learn_net, max_slots=2)
    assert e.value.status == -1


def test_server_takes_the_frozen_handles_precision(torch_cuda, oracle_mod):
    """A server built from a handle switched to BF16 with snn_set_path serves
    in BF16: each request equals the BF16 run of its sample on the handle
    itself, bit for bit, and the BF16-rounding oracle's counts.  Request 3 is
    one whose BF16 and FP32 counts differ (oracle), so an FP32 server fails."""
    torch = torch_cuda
    from paper_1909_02549_amd.snn import Net, Server
    cfg = inputs.dc_config(64, learn=False)
    W = inputs.frozen_weights(784, 64, 78.4, 9)
    net = Net(cfg, max_batch=1, path="fused", precision="fp32")
    net.snn_set_weights(W)
    net.snn_set_path("fused", "bf16")
    imgs = inputs.stroke_images(4, 44, 0.19)
    T = 60
    srv = Server(net, max_slots=4, chunk_steps=20)
    rids = [srv.snn_serve_submit(imgs[k], 40 + k, T) for k in range(4)]
    res = wait_all(srv, rids)
    srv.snn_serve_destroy()
    for k, r in enumerate(rids):
        out = net.snn_run(torch.from_numpy(imgs[k:k + 1]).cuda(), torch.tensor([40 + k], dtype=torch.int64).cuda(),
                          T, record=("counts",))
        torch.cuda.synchronize()
        alone = out["counts"].cpu().numpy()[0].astype(np.uint32)
        assert np.array_equal(res[r][0], alone), f"request {k}: served counts differ from the BF16 run"
        ref = oracle_mod.OracleNet(cfg, W.astype(np.float64), precision="bf16").run(
            imgs[k:k + 1], np.array([40 + k], np.uint64), T, record=("counts",))
        assert np.array_equal(ref["counts"][0], alone), f"request {k}: counts differ from the BF16 oracle"
    ref32 = oracle_mod.OracleNet(cfg, W.astype(np.float64), precision="fp32").run(
        imgs[3:4], np.array([43], np.uint64), T, record=("counts",))
    assert not np.array_equal(ref32["counts"][0], res[rids[3]][0])
    net.close()
