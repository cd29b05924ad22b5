"""The learned-split network's device kernels against the oracle (oracle/mlp.py): forward pass,
loss, back-propagated gradient (per-tensor relative error <= 1e-4 against FP64), one Adam step,
training descent and determinism."""
import numpy as np
import pytest

from oracle import mlp as omlp

torch = pytest.importorskip("torch")
cr = pytest.importorskip("paper_1409_4441_amd")
from paper_1409_4441_amd import learn  # noqa: E402

pytestmark = pytest.mark.gpu

TENSORS = [("W1", 0, 192), ("b1", 192, 256), ("W2", 256, 4352), ("b2", 4352, 4416), ("W3", 4416, 4544),
           ("b3", 4544, 4546)]


def _data(seed, n):
    g = np.random.default_rng(seed)
    x = g.uniform(-1, 1, (n, 3))
    t = np.stack([np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2], np.cos(x[:, 1]) - 0.5 * x[:, 0]], axis=1)
    return x.astype(np.float32), t.astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


@pytest.mark.parametrize("n", [1, 37, 300, 2000])
def test_forward_and_loss_match_oracle(cuda_device, n):
    p = learn.init_params(11)
    x, t = _data(n, n)
    net = learn.Network(max_batch=2048)
    net.set_params(p)
    y = net.forward(_dev(x)).cpu().numpy()
    yo, _, _ = omlp.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.max(np.abs(y - yo)) <= 2e-5 * max(1.0, np.max(np.abs(yo)))
    loss, _ = net.gradient(_dev(x), _dev(t))
    lo = omlp.loss(p.astype(np.float64), x, t)
    assert float(loss.cpu()[0]) == pytest.approx(lo, rel=1e-5)
    assert np.array_equal(net.get_params(), p)
    net.close()


@pytest.mark.parametrize("n,seed", [(64, 1), (2000, 2)])
def test_gradient_matches_fp64_backprop(cuda_device, n, seed):
    p = (np.random.default_rng(seed).normal(0, 0.4, omlp.N_PARAMS)).astype(np.float32)
    x, t = _data(seed + 10, n)
    net = learn.Network(max_batch=n)
    net.set_params(p)
    _, g = net.gradient(_dev(x), _dev(t))
    g = g.cpu().numpy().astype(np.float64)
    go = omlp.gradient(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    for name, a, b in TENSORS:
        err = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        assert err <= 1e-4, (name, err)
    net.close()


def test_adam_steps_match_oracle(cuda_device):
    p = learn.init_params(5)
    x, t = _data(6, 128)
    net = learn.Network(max_batch=128)
    net.set_params(p)
    hist = net.train(_dev(x), _dev(t), steps=5, lr=1e-3).cpu().numpy()
    po, ho = omlp.adam(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), steps=5, lr=1e-3)
    q = net.get_params().astype(np.float64)
    assert np.allclose(hist, ho, rtol=1e-5)
    # Adam moves each parameter by about lr per step whatever the gradient's size, so a parameter
    # whose gradient nearly cancels can move differently in FP32; compare the whole update
    du, duo = q - p.astype(np.float64), po - p.astype(np.float64)
    assert np.linalg.norm(du - duo) <= 1e-3 * np.linalg.norm(duo)
    net.close()


def test_training_descends_and_is_deterministic(cuda_device):
    x, t = _data(7, 1000)
    runs = []
    for _ in range(2):
        net = learn.Network(max_batch=1000)
        net.set_params(learn.init_params(3))
        hist = net.train(_dev(x), _dev(t), steps=400, lr=3e-3).cpu().numpy()
        runs.append((hist, net.get_params()))
        net.close()
    assert runs[0][0][-1] < 0.1 * runs[0][0][0]
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    # continuing a run carries the Adam step count: 200 + 200 steps equal 400 steps
    net = learn.Network(max_batch=1000)
    net.set_params(learn.init_params(3))
    net.train(_dev(x), _dev(t), steps=200, lr=3e-3)
    net.train(_dev(x), _dev(t), steps=200, lr=3e-3)
    assert np.array_equal(net.get_params(), runs[0][1])
    net.close()


def test_bad_arguments(cuda_device):
    net = learn.Network(max_batch=16)
    with pytest.raises(cr.ConvRealError):
        net.set_params(np.full(learn.N_PARAMS, np.nan, dtype=np.float32))
    x = torch.zeros((17, 3), device="cuda:0")
    with pytest.raises(cr.ConvRealError):
        net.forward(x)                       # batch above max_batch
    with pytest.raises(cr.ConvRealError):
        net.forward(torch.zeros((4, 3), device="cuda:0", dtype=torch.float64))
    with pytest.raises(cr.ConvRealError):
        net.train(torch.zeros((4, 3), device="cuda:0"), torch.zeros((4, 2), device="cuda:0"), steps=1, lr=-1.0)
    net.close()
    with pytest.raises(cr.ConvRealError):
        learn.Network(max_batch=0)
