"""GPU checks of the contact-surrogate MLP kernels (BF16 matrix-core
products, FP32 accumulation) against the FP64 reference in oracle/mlp.py,
which uses the same BF16-rounded operands. Differences come from FP32
accumulation order and from activations that sit on a BF16 rounding
boundary, so the bounds are a few 1e-3 of the output / gradient scale."""
import numpy as np
import pytest

from oracle import mlp as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mlp(params=None, seed=0):
    from paper_2207_03530_amd import binding as B
    return B.Mlp(None if params is None else M.pack(params), seed=seed)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to("cuda:0")


def _rel(a, b):
    return np.abs(np.asarray(a, np.float64) - b).max() / max(np.abs(b).max(), 1e-12)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4097])
def test_forward_matches_reference(n):
    p = M.init_params(1)
    x = np.random.default_rng(n).standard_normal((n, 12)).astype(np.float32)
    net = _mlp(p)
    Y = torch.zeros(n, 2, device="cuda:0")
    net.forward(_dev(x), Y)
    torch.cuda.synchronize()
    y_ref, _, _ = M.forward(p, x)
    err = _rel(Y.cpu().numpy(), y_ref)
    print(f"forward n={n}: rel err {err:.3g}")
    assert err <= 5e-3


def test_backward_matches_reference():
    n = 777
    rng = np.random.default_rng(5)
    p = M.init_params(2)
    x = rng.standard_normal((n, 12)).astype(np.float32)
    dy = (rng.standard_normal((n, 2)) / n).astype(np.float32)
    net = _mlp(p)
    grad = torch.zeros(M.pack(p).size, device="cuda:0")
    dX = torch.zeros(n, 12, device="cuda:0")
    net.backward(_dev(x), _dev(dy), grad, dX)
    torch.cuda.synchronize()
    g = M.backward(p, x, dy.astype(np.float64))
    gg = M.unpack(grad.cpu().numpy())
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        err = _rel(gg[k], g[k])
        print(f"grad {k}: rel err {err:.3g}")
        assert err <= 1e-2, k
    assert _rel(dX.cpu().numpy(), g["x"]) <= 1e-2


def test_training_reduces_loss_and_is_deterministic():
    """Adam on a smooth regression target: the loss falls by 10x in 300
    steps, and two runs from the same seed give identical parameters."""
    rng = np.random.default_rng(0)
    n = 4096
    x = rng.uniform(-1, 1, (n, 12)).astype(np.float32)
    t = np.stack([np.sin(2 * x[:, 0]) * x[:, 1], np.tanh(x[:, 2] - x[:, 3] ** 2)], 1).astype(np.float32)
    X, Tt = _dev(x), _dev(t)
    runs = []
    for _ in range(2):
        net = _mlp(seed=7)
        loss = torch.zeros(1, device="cuda:0")
        hist = []
        for step in range(300):
            net.train_step(X, Tt, 3e-3, loss)
            if step in (0, 299):
                torch.cuda.synchronize()
                hist.append(float(loss.item()))
        runs.append((net.params(), hist))
        net.close()
    print(f"training loss {runs[0][1][0]:.4g} -> {runs[0][1][1]:.4g}")
    assert runs[0][1][1] < 0.1 * runs[0][1][0]
    assert np.array_equal(runs[0][0], runs[1][0])
