"""Pins of the FP64 reference MLP used to check the GPU surrogate kernels:
its gradients against central differences (exact arithmetic), and its BF16
rounding against the format's definition."""
import numpy as np

from oracle import mlp as M


def test_bf16_rounding_definition():
    # exactly representable values survive, halfway cases go to even
    vals = np.array([1.0, -2.5, 0.0, 2.0 ** 127, 1.0 + 2.0 ** -7], np.float32)
    np.testing.assert_array_equal(M.bf16_round(vals), vals.astype(np.float64))
    one_ulp = 2.0 ** -7
    assert M.bf16_round(np.float32(1.0 + one_ulp / 2)) == 1.0            # tie -> even (1.0)
    assert M.bf16_round(np.float32(1.0 + 3 * one_ulp / 2)) == 1.0 + 2 * one_ulp  # tie -> even
    assert M.bf16_round(np.float32(1.0 + one_ulp * 0.75)) == 1.0 + one_ulp
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    r = M.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 + 1e-45)
    assert np.all((r.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_mlp_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    p = {k: v.astype(np.float64) for k, v in M.init_params(3).items()}
    x = rng.standard_normal((7, 12))
    t = rng.standard_normal((7, 2))
    _, g = M.loss_and_grads(p, x, t, rounded=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, min(5, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = M.loss_and_grads(p, x, t, rounded=False)
            flat[idx] = old - h
            lm, _ = M.loss_and_grads(p, x, t, rounded=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name].reshape(-1)[idx]) <= 1e-7 + 1e-6 * abs(fd), name
    for idx in range(12):
        xp = x.copy()
        xp[2, idx] += h
        lp, _ = M.loss_and_grads(p, xp, t, rounded=False)
        xp[2, idx] -= 2 * h
        lm, _ = M.loss_and_grads(p, xp, t, rounded=False)
        assert abs((lp - lm) / (2 * h) - g["x"][2, idx]) <= 1e-7
