"""The size-bucketed plan of uneven sphere batches: every bucket of
environment sizes (1-4, 5-8, 9-16, 17-32, 33-64, 65-) runs its own plan --
the ordered quad plan over the bucket's environments where they fit it,
else a size-sorted entity-lane plan -- and the buckets' launches run at the
same time on side streams (or as independent nodes of the rollout graph).
Checked bit for bit against the single-plan lane schedule, before and after
the autotuner's per-bucket choice, eagerly and replayed from the graph; the
autotuner's choice is cached across handles of the same environment-shape
histogram."""
import numpy as np
import pytest

from paper_2207_03530_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32)).to("cuda:0")


def _names(b):
    return [b.schedule_name(q) for q in range(b.n_schedules)]


def _bucketed(b):
    names = _names(b)
    q = [i for i, n in enumerate(names) if n.startswith("bucketed")]
    assert len(q) == 1, names
    return q[0]


def _lane(b):
    """The first valid single-plan entity-lane schedule (the reference)."""
    return next(i for i, n in enumerate(_names(b)) if n.startswith("entity-lane"))


def _run(b, w, q, T, traj=False, mask=False, graph=False, drawn=False):
    b.set_schedule(q)
    s = _dev(w.state0)
    tr = torch.zeros((T + 1) * 6 * w.n_entities, device="cuda:0") if traj else None
    mk = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0") if mask else None
    if drawn:
        b.rollout(s, None, T=T, seed=3, traj=tr, final_mask=mk, graph=graph)
    else:
        b.rollout(s, _dev(w.actions(T)), traj=tr, final_mask=mk, graph=graph)
    torch.cuda.synchronize()
    return s, tr, mk


@pytest.mark.parametrize("drawn", [False, True])
def test_bucketed_plan_bitwise_equals_lane_plan(drawn):
    from paper_2207_03530_amd import binding as B
    w = W.uneven(700, lo=1, hi=70, radius=0.08, seed=7)
    b = B.Batch(w, 0)
    qb = _bucketed(b)
    name0 = b.schedule_name(qb)
    assert "quad-ordered" in name0, name0  # the smallest bucket takes the quad plan
    ref = _run(b, w, _lane(b), 30, traj=True, mask=True, drawn=drawn)
    out = _run(b, w, qb, 30, traj=True, mask=True, drawn=drawn)
    for r, o, what in zip(ref, out, ("state", "trajectory", "final mask")):
        assert torch.equal(r, o), (name0, what)
    assert int(ref[2].sum()) > 0
    # after the per-bucket choice of the autotuner, still the same bits
    q = b.autotune(_dev(w.state0), 10)
    print(f"default {name0}; tuned {b.schedule_name(qb)}; chosen {b.schedule_name(q)}")
    out = _run(b, w, qb, 30, traj=True, mask=True, drawn=drawn)
    for r, o, what in zip(ref, out, ("state", "trajectory", "final mask")):
        assert torch.equal(r, o), (b.schedule_name(qb), what)


def test_bucketed_plan_graph_replay_and_steps():
    """The bucketed plan replayed from its rollout graph (one node per
    bucket) with eager work in between, and single steps with masks and
    forces, against the lane plan."""
    from paper_2207_03530_amd import binding as B
    w = W.uneven(400, lo=2, hi=40, radius=0.1, seed=8)
    b = B.Batch(w, 0)
    qb = _bucketed(b)
    ref, _, _ = _run(b, w, _lane(b), 20, drawn=True)
    for rep in range(3):
        junk = torch.randn(1000, device="cuda:0").sum()
        s, _, _ = _run(b, w, qb, 20, graph=True, drawn=True)
        assert torch.equal(s, ref), rep
        del junk
    acts = _dev(w.actions(1)[0])
    outs = []
    for q in (_lane(b), qb):
        b.set_schedule(q)
        s = _dev(w.state0)
        m = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
        f = torch.zeros(3 * w.n_entities, device="cuda:0")
        b.step(s, acts, m, f)
        torch.cuda.synchronize()
        outs.append((s, m, f))
    for r, o in zip(*outs):
        assert torch.equal(r, o)


def test_autotune_choice_cached_across_handles():
    """A second batch with the same environment-shape histogram (other
    positions) takes the first one's choice from the cache, without timing."""
    from paper_2207_03530_amd import binding as B
    w1 = W.uneven(500, lo=2, hi=30, seed=9)
    w2 = W.uneven(500, lo=2, hi=30, seed=9)
    w2.state0 = (w1.state0 + np.float32(0.01)).astype(np.float32)
    b1 = B.Batch(w1, 0)
    q1 = b1.autotune(_dev(w1.state0), 12)
    assert b1.info().tune_cached == 0
    b2 = B.Batch(w2, 0)
    q2 = b2.autotune(_dev(w2.state0), 12)
    assert b2.info().tune_cached == 1
    assert q2 == q1 and b2.schedule_name(q2) == b1.schedule_name(q1)
    # a different rollout length bucket is tuned anew
    b2.autotune(_dev(w2.state0), 200)
    assert b2.info().tune_cached == 0
