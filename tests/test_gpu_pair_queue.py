"""The pair-queue schedule (every pair with a box or a segment evaluated once,
from per-class queues in LDS, results summed per entity in the plain order)
against the entity-lane schedule of the same block size, bit for bit: final
state, trajectory, final contact mask and one step's forces, with given and
in-kernel actions, joints, a minimum distance, static boxes and segments
(pairs owned by the lane of the moving side), queues that overflow (the
pairs beyond a full queue are evaluated by both of their lanes), and more
broad-phase pairs per lane than the registers hold."""
import dataclasses

import numpy as np
import pytest

from paper_2207_03530_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda:0", dtype)


def _bits(t):
    return t.view(torch.int32) if t.dtype == torch.float32 else t


def _worlds():
    base = W.mixed(60, seed=11)
    static = W.mixed(50, seed=12)
    fl = static.flags.copy()
    n = 28
    fl[17::n] = W.COLLIDABLE   # box 1 of every environment does not move or turn
    fl[20::n] = W.COLLIDABLE   # segment 0 likewise
    static = dataclasses.replace(static, flags=fl, min_dist=0.005)
    # segments of length 2 in a 2 x 2 square: nearly all of the 378
    # segment pairs of an environment are candidates, beyond the queue's 256
    dense = W.mixed(6, n_spheres=2, n_boxes=2, n_lines=28, line_len=2.0, joints=False, seed=13)
    # 4 sphere movers among 28 static segments: 118 pairs per environment
    # and 16 environments per 64 lanes, about 30 pairs per lane (more than a
    # lane keeps in registers: the broad phase reads its pairs from LDS)
    walls = W.mixed(48, n_spheres=4, n_boxes=0, n_lines=28, joints=False, seed=14)
    fl = walls.flags.copy()
    fl[(np.arange(walls.n_entities) % 32) >= 4] = W.COLLIDABLE
    walls = dataclasses.replace(walls, flags=fl)
    return {"mixed": base, "static": static, "dense": dense, "walls": walls}


def _plans(b):
    names = {b.schedule_name(q): q for q in range(b.n_schedules)}
    pairs = []
    for nm, q in names.items():
        if nm.startswith("pair-queue/"):
            # an evenly spread plan against the entity-lane plan of its block
            ref = "entity-lane/" + nm[len("pair-queue/"):].removesuffix("/even")
            assert ref in names, (nm, sorted(names))
            pairs.append((nm, q, names[ref]))
    assert pairs, sorted(names)
    return pairs


def _run(b, w, q, T, drawn):
    b.set_schedule(q)
    s = _dev(w.state0)
    traj = torch.zeros((T + 1) * 6 * w.n_entities, device="cuda:0")
    mk = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
    if drawn:
        b.rollout(s, None, T=T, seed=5, traj=traj, final_mask=mk)
    else:
        b.rollout(s, _dev(w.actions(T)), traj=traj, final_mask=mk)
    s1 = _dev(w.state0)
    m1 = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
    f1 = torch.zeros(3 * w.n_entities, device="cuda:0")
    b.step(s1, _dev(w.actions(1)[0]), m1, f1)
    torch.cuda.synchronize()
    return s, traj, mk, s1, m1, f1


@pytest.mark.parametrize("name", ["mixed", "static", "dense", "walls"])
@pytest.mark.parametrize("drawn", [False, True])
def test_pair_queue_bitwise_equals_entity_lane(name, drawn):
    from paper_2207_03530_amd import binding as B
    w = _worlds()[name]
    b = B.Batch(w, 0)
    T = 12 if name == "dense" else 40
    for nm, q_pq, q_ref in _plans(b):
        print(f"{name}: {w.n_envs} envs, {w.n_entities} entities, {nm}, drawn={drawn}", flush=True)
        ref = _run(b, w, q_ref, T, drawn)
        out = _run(b, w, q_pq, T, drawn)
        for r, o, what in zip(ref, out, ("state", "traj", "final mask", "step state", "step mask",
                                         "step forces")):
            assert torch.equal(_bits(r), _bits(o)), (nm, what)
        assert int(ref[4].sum()) > 0  # contacts in the first step


def test_dense_world_overflows_the_queue():
    """The dense world really has more segment-pair candidates per
    environment than the queue holds (so the both-lanes path runs): pairs
    whose centres lie within the sum of the bounding radii (1 + 1) always
    pass the broad phase."""
    w = _worlds()["dense"]
    n = 32
    x = w.state0[0].reshape(-1, n)
    y = w.state0[1].reshape(-1, n)
    seg = np.arange(4, n)  # 2 spheres, 2 boxes, then the segments
    iu = np.triu_indices(len(seg), 1)
    dist = np.hypot(x[:, seg[iu[0]]] - x[:, seg[iu[1]]], y[:, seg[iu[0]]] - y[:, seg[iu[1]]])
    per_env = (dist <= 2.0).sum(axis=1)
    assert per_env.min() > 256, per_env


def test_pair_queue_graph_replay():
    from paper_2207_03530_amd import binding as B
    w = _worlds()["mixed"]
    b = B.Batch(w, 0)
    nm, q_pq, q_ref = _plans(b)[-1]
    acts = _dev(w.actions(20))
    b.set_schedule(q_ref)
    ref = _dev(w.state0)
    b.rollout(ref, acts)
    b.set_schedule(q_pq)
    for _ in range(3):
        s = _dev(w.state0)
        b.rollout(s, acts, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(s, ref), nm


def test_pair_queue_offered_only_where_it_fits():
    from paper_2207_03530_amd import binding as B
    for w, ok in ((W.spread(40, seed=1), False),                       # spheres only
                  (W.mixed(10, n_spheres=20, n_lines=12, seed=1), False),  # 36 entities
                  (W.mixed(10, seed=1), True)):
        b = B.Batch(w, 0)
        names = [b.schedule_name(q) for q in range(b.n_schedules)]
        assert any(n.startswith("pair-queue/") for n in names) == ok, (w.name, names)
