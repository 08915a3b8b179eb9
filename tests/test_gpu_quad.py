"""The quad schedules (the movers of an environment on one aligned lane
quad, partner centres by DPP, static partners in registers, no LDS; the
ordered variant for environments whose movers come first) against the
entity-lane schedule, bit for bit: final state, trajectory, final contact
mask and forces, with given and in-kernel actions, idle lanes, zero to four
static entities, a static entity that does not collide, a minimum distance,
a speed limit, and gravity."""
import dataclasses

import numpy as np
import pytest

from paper_2207_03530_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

QUAD = "quad/256"
QUADS = ["quad/256", "quad-ordered/64"]


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda:0", dtype)


def _worlds():
    dense = W.spread(500, 4, 2, radius=0.15, seed=1)
    idle = W.spread(300, 3, 4, radius=0.2, seed=2)
    ragged = W.uneven(400, lo=1, hi=4, radius=0.2, seed=3)
    odd = W.spread(257, 2, 3, radius=0.2, seed=4)
    fl = odd.flags.copy()
    fl[2::5] = 0  # the first landmark of every environment takes no part
    odd = dataclasses.replace(odd, flags=fl, min_dist=0.01,
                              max_speed=np.full(odd.n_entities, 0.5, np.float32))
    # spinning spheres (omega != 0, angles that turn) of unequal masses, and
    # environments whose last movers are not agents (no action)
    spin = W.spread(300, 4, 2, radius=0.15, seed=5)
    st = spin.state0.copy()
    rng = np.random.default_rng(5)
    st[5] = rng.uniform(-2, 2, spin.n_entities).astype(np.float32)
    st[4] = rng.uniform(-3, 3, spin.n_entities).astype(np.float32)
    spin = dataclasses.replace(spin, state0=st,
                               mass=rng.uniform(0.5, 2.0, spin.n_entities).astype(np.float32))
    mute = W.spread(300, 4, 2, radius=0.15, seed=6)
    mute = dataclasses.replace(mute, n_agents=np.full(300, 2, np.int32))
    # gravity on the movers (the quad kernels then read the full entity
    # record for m g), with explicit moments of inertia
    grav = W.spread(300, 4, 2, radius=0.15, seed=7)
    grav = dataclasses.replace(grav, gravity=(0.3, -0.5),
                               inertia=np.full(grav.n_entities, 0.02, np.float32))
    return {"dense": dense, "idle": idle, "ragged": ragged, "odd": odd, "spin": spin,
            "mute": mute, "grav": grav}


def _schedules(b, quad=QUAD):
    names = {b.schedule_name(q): q for q in range(b.n_schedules)}
    assert quad in names, names
    return names[quad], 0


def _run(b, w, q, T, drawn):
    b.set_schedule(q)
    s = _dev(w.state0)
    traj = torch.zeros((T + 1) * 6 * w.n_entities, device="cuda:0")
    mk = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
    if drawn:
        b.rollout(s, None, T=T, seed=7, traj=traj, final_mask=mk)
    else:
        b.rollout(s, _dev(w.actions(T)), traj=traj, final_mask=mk)
    s1 = _dev(w.state0)
    m1 = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
    f1 = torch.zeros(3 * w.n_entities, device="cuda:0")
    b.step(s1, _dev(w.actions(1)[0]), m1, f1)
    torch.cuda.synchronize()
    return s, traj, mk, s1, m1, f1


@pytest.mark.parametrize("quad", QUADS)
@pytest.mark.parametrize("name", ["dense", "idle", "ragged", "odd", "spin", "mute", "grav"])
@pytest.mark.parametrize("drawn", [False, True])
def test_quad_schedule_bitwise_equals_lane_schedule(name, drawn, quad):
    from paper_2207_03530_amd import binding as B
    w = _worlds()[name]
    b = B.Batch(w, 0)
    q_quad, q_lane = _schedules(b, quad)
    print(f"{name}: {w.n_envs} envs, {w.n_entities} entities, drawn={drawn}", flush=True)
    ref = _run(b, w, q_lane, 40, drawn)
    out = _run(b, w, q_quad, 40, drawn)
    for r, o, what in zip(ref, out, ("state", "traj", "final mask", "step state", "step mask",
                                     "step forces")):
        assert torch.equal(r, o), what
    assert int(ref[2].sum()) > 0  # contacts happened


@pytest.mark.parametrize("quad", QUADS)
def test_quad_schedule_graph_replay(quad):
    from paper_2207_03530_amd import binding as B
    w = _worlds()["dense"]
    b = B.Batch(w, 0)
    q_quad, q_lane = _schedules(b, quad)
    acts = _dev(w.actions(24))
    b.set_schedule(q_lane)
    ref = _dev(w.state0)
    b.rollout(ref, acts)
    b.set_schedule(q_quad)
    for _ in range(3):
        s = _dev(w.state0)
        b.rollout(s, acts, graph=True)
        torch.cuda.synchronize()
        assert torch.equal(s, ref)


def test_quad_schedule_offered_only_where_it_fits():
    from paper_2207_03530_amd import binding as B
    for w, ok in ((W.uneven(40, lo=5, hi=5, seed=1), False),   # 5 movers
                  (W.spread(40, 2, 5, seed=1), False),         # 5 static collidables
                  (W.mixed(8, seed=1), False),                 # not spheres only
                  (W.spread(40, 4, 4, seed=1), True)):
        b = B.Batch(w, 0)
        names = [b.schedule_name(q) for q in range(b.n_schedules)]
        assert (QUAD in names) == ok, (w.name, names)
        assert ("quad-ordered/64" in names) == ok, (w.name, names)
    # movers not first: the quad schedule fits, the ordered one does not
    w = W.spread(40, 4, 2, seed=1)
    fl = w.flags.copy()
    fl[0::6] = W.COLLIDABLE
    fl[4::6] = W.MOVABLE | W.ROTATABLE | W.COLLIDABLE
    w = dataclasses.replace(w, flags=fl)
    b = B.Batch(w, 0)
    names = [b.schedule_name(q) for q in range(b.n_schedules)]
    assert QUAD in names and "quad-ordered/64" not in names, names
