"""The allocation-free rollout adjoint (vmas_rollout_backward_noalloc)
against vmas_rollout_backward, through the C boundary: the same kernels on
the same inputs, so the gradients must agree bit for bit, on two calls in a
row (the second on a smaller input, which finds the previous call's data in
the shared static scratch), and a workspace beyond the scratch is refused
before any device work."""
import numpy as np
import pytest

from paper_2207_03530_amd import binding as B
from paper_2207_03530_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to("cuda:0")


def _grads(b, w, T, k, noalloc):
    rng = np.random.default_rng(T * 100 + k)
    acts = _dev(w.actions(T))
    gT = _dev(rng.standard_normal((6, w.n_entities)))
    gs = torch.full((6 * w.n_entities,), 7.0, device="cuda:0")
    ga = torch.full((T * 2 * w.n_agents_total,), 7.0, device="cuda:0")
    b.rollout_backward(_dev(w.state0), acts, gT, k, gs, ga, noalloc=noalloc)
    torch.cuda.synchronize()
    return gs, ga


def test_noalloc_adjoint_equals_allocating_adjoint():
    cases = [(W.mixed(96, seed=31), 24, 5), (W.mixed(20, n_spheres=6, n_boxes=2, n_lines=3,
                                                   seed=32), 7, 3)]
    for w, T, k in cases:  # the second call is the smaller one
        b = B.Batch(w, 0)
        ref_s, ref_a = _grads(b, w, T, k, noalloc=False)
        got_s, got_a = _grads(b, w, T, k, noalloc=True)
        assert torch.equal(got_s, ref_s), (w.name, T, k)
        assert torch.equal(got_a, ref_a), (w.name, T, k)
        assert torch.isfinite(got_s).all() and got_s.abs().max() > 0
        b.close()


def test_noalloc_adjoint_refuses_workspace_beyond_scratch():
    w = W.spread(30000)
    b = B.Batch(w, 0)
    T = 400
    acts = torch.zeros((T, w.n_agents_total, 2), device="cuda:0")
    g = torch.zeros(6 * w.n_entities, device="cuda:0")
    with pytest.raises(B.VmasError) as ex:
        b.rollout_backward(g, acts, g, 200, noalloc=True)
    assert ex.value.status == 1 and "scratch" in str(ex.value)
    b.close()
