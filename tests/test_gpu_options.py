"""GPU parity of the options of the problem statement (Sec. 3) that the
benchmark configurations leave at their defaults: gravity, an extra
minimum distance, explicit moments of inertia, jointed pairs that collide,
an immovable but rotatable segment (the anchored line of the paper's Wheel
scenario, Sec. 4), non-sphere environments with more movers than a 256-lane
workgroup holds, and the non-finite debug check of the boundary.

Every option is compared with the FP64 oracle: one step from t = 0 (both
error metrics of tests/parity.py, masks up to band cases) and teacher
forcing along a GPU trajectory (the oracle steps from the GPU's state at
every step)."""
import dataclasses

import numpy as np
import pytest

from oracle import oracle as O
from paper_2207_03530_amd import workloads as W
from tests import parity as PU

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests.gpu_common import (_batch, _dev, _gpu_run, _gpu_step, _mask_check,  # noqa: E402
                              _one_step_check, _teacher_forced_check)


def _check_world(w, name, T=30, min_plain=0.85):
    """One step from t = 0 (forces and torques too), then teacher forcing
    along a T-step GPU trajectory."""
    b = _batch(w)
    acts = w.actions(T)
    ow = O.OracleWorld(w)
    g, gm, gf = _gpu_step(b, w.state0, acts[0], forces=True)
    o, om, of = ow.step(w.state0, acts[0], want_forces=True)
    band = _mask_check(w, ow, w.state0, gm, om, name)
    skip = np.zeros(w.n_envs, bool)
    skip[PU.pair_env(w.env_offset)[band]] = True
    _one_step_check(w, ow, w.state0, acts[0], g, o, name, skip=skip)
    # forces and torques of the entities that can move or rotate (the others
    # report 0), on the environments that are not ill-conditioned
    ent_env = np.repeat(np.arange(w.n_envs), np.diff(w.env_offset))
    ill = skip | PU.ill_conditioned_step(ow, w.state0, acts[0])
    ok = ~ill[ent_env] & ((w.flags & (W.MOVABLE | W.ROTATABLE)) != 0)
    fscale = np.abs(of[:, ok]).max(1, keepdims=True) + 1e-6
    ferr = (np.abs(gf - of)[:, ok] / fscale).max(1)
    print(f"{name}: force/torque err {ferr} on {(~ill).sum()}/{w.n_envs} envs")
    assert ferr.max() <= 1e-5
    assert om.sum() > 0, f"{name}: the world has no contact at t = 0"
    _, gtraj, gmasks = _gpu_run(b, w.state0, acts)
    _teacher_forced_check(w, ow, gtraj, gmasks, acts, f"{name}, teacher-forced",
                          min_plain=min_plain)
    return b, gtraj


def test_gravity_with_immovable_entities():
    """g = (0.3, -0.7): m g on movable entities only (an immovable but
    rotatable box and an immovable segment feel no gravity)."""
    w = W.mixed(64, seed=7)
    w.gravity = (0.3, -0.7)
    fl = w.flags.copy()
    local = np.tile(np.arange(28), 64)
    fl[local == 17] = W.ROTATABLE | W.COLLIDABLE   # box 1: anchored, free to turn
    fl[local == 27] = W.COLLIDABLE                  # last segment: static
    w.flags = fl
    _, gtraj = _check_world(w, "gravity")
    st = w.state0
    assert np.all(gtraj[-1][0:4, local == 17] == st[0:4, local == 17])
    assert np.all(gtraj[-1][:, local == 27] == st[:, local == 27])


@pytest.mark.parametrize("kind", ["mixed", "spread"])
def test_min_dist(kind):
    """An extra minimum distance of 0.02 in every pair's d_min (the kernels'
    nonzero-d_min variants, sphere and generic)."""
    if kind == "mixed":
        w = dataclasses.replace(W.mixed(64, seed=8), min_dist=0.02)
    else:
        w = dataclasses.replace(W.spread(256, seed=8), min_dist=0.02)
    _check_world(w, f"min_dist {kind}")


def test_explicit_inertia():
    """Moments of inertia given per entity (a quarter of them <= 0, which
    selects the textbook default)."""
    w = W.mixed(64, seed=9)
    rng = np.random.default_rng(9)
    I = rng.uniform(0.002, 0.05, w.n_entities).astype(np.float32)
    I[rng.random(w.n_entities) < 0.25] = 0.0
    w.inertia = I
    _check_world(w, "explicit inertia")


def test_joint_collide():
    """Jointed pairs that collide (joint_collide = 1 for every other joint),
    with jointed agents placed inside their box so the contact is active."""
    w = W.mixed(64, seed=10)
    J = w.n_joints
    w.joint_collide = (np.arange(J) % 2 == 0).astype(np.uint8)
    st = w.state0.copy()
    for q in range(J):
        a, c = w.joint_a[q], w.joint_b[q]
        st[0, a] = st[0, c] + 0.01 * (1 if q % 2 == 0 else -1)
        st[1, a] = st[1, c]
    w.state0 = st
    w.joint_rest = np.full(J, 0.12, np.float32)
    b, _ = _check_world(w, "joint_collide")
    ow = O.OracleWorld(w)
    _, om, _ = ow.step(w.state0, w.actions(1)[0])
    n = 28
    # slot of the pair (agent, box 0) in each environment's mask
    for q in range(0, J, 2):
        e = w.joint_a[q] // n
        la, lc = w.joint_a[q] % n, w.joint_b[q] % n
        slot = e * (n * (n - 1) // 2) + la * n - la * (la + 1) // 2 + (lc - la - 1)
        assert om[slot] == 1


def test_joint_anchor_off_sphere_centre():
    """Joints anchored off the centre of a sphere agent (the sphere's
    orientation then enters the joint geometry, and the joint's torque turns
    it): agents 0 and 1 tied at local (0.02, 0.01) to box 0, agents 2 and 3
    tied to each other at (-0.02, 0) and (0, 0.025); rest lengths from the
    initial state."""
    w = W.mixed(64, seed=16)
    n = 28
    base = np.arange(64, dtype=np.int32) * n
    ja = np.concatenate([w.joint_a, base + 2]).astype(np.int32)
    jb = np.concatenate([w.joint_b, base + 3]).astype(np.int32)
    aa = np.concatenate([np.tile([[0.02, 0.01]], (w.n_joints, 1)),
                         np.tile([[-0.02, 0.0]], (64, 1))]).astype(np.float32)
    ab = np.concatenate([w.anchor_b, np.tile([[0.0, 0.025]], (64, 1))]).astype(np.float32)
    w.joint_a, w.joint_b, w.anchor_a, w.anchor_b = ja, jb, aa, ab
    w.joint_rest = np.full(len(ja), -1.0, np.float32)
    st = w.state0.copy()
    st[4, (np.arange(w.n_entities) % n) < 4] = 0.3  # sphere agents start turned
    w.state0 = st
    _, gtraj = _check_world(w, "anchors off sphere centres")
    agents = np.nonzero((np.arange(w.n_entities) % n) < 4)[0]
    assert np.abs(gtraj[-1][5, agents]).max() > 1e-3  # the joints turn the spheres


def test_entity_with_four_joints():
    """Box 0 of every environment tied to agents 0 .. 3 (four joints on one
    entity, evaluated in joint order: the first two kept in registers, the
    others read each step), rest lengths from the initial state, agents
    started off their rest positions by their actions."""
    w = W.mixed(64, seed=17)
    n = 28
    base = np.arange(64, dtype=np.int32) * n
    ja = np.stack([base + k for k in range(4)], 1).reshape(-1).astype(np.int32)
    jb = np.repeat(base + 16, 4).astype(np.int32)
    J = len(ja)
    w.joint_a, w.joint_b = ja, jb
    w.anchor_a = np.zeros((J, 2), np.float32)
    w.anchor_b = np.tile(np.array([[0.0, 0.15], [0.0, -0.15], [0.05, 0.0], [-0.05, 0.1]],
                                  np.float32), (64, 1))
    w.joint_rest = np.full(J, -1.0, np.float32)
    # four springs of stiffness 100 on one box are stiff enough that even the
    # oracle's own definition evaluated in FP32 meets the plain 1e-5 on only
    # 0.76 of the teacher-forced environment-steps; at stiffness 25 it meets
    # it on 0.88 (every step is still held to the conditioning allowance)
    w = dataclasses.replace(w, joint_stiffness=25.0)
    _, gtraj = _check_world(w, "four joints on one entity", min_plain=0.8)
    boxes = base + 16
    assert np.abs(gtraj[-1][5, boxes]).max() > 1e-3  # the joints turn the boxes


def test_joint_rest_from_state_is_exactly_at_rest():
    """A joint whose rest length is taken from the initial state exerts no
    force in that state: with no actions, no contacts and no gravity one
    step leaves every velocity exactly zero."""
    w = W.mixed(32, seed=17, half_width=2.0, separated=True)
    b = _batch(w)
    g, _, f = _gpu_step(b, w.state0, np.zeros((w.n_agents_total, 2), np.float32), forces=True)
    assert np.all(g[2:4] == 0) and np.all(g[5] == 0) and np.all(f == 0)


def test_immovable_rotatable_segment():
    """The anchored line of the Wheel scenario (Sec. 4): a segment that can
    turn but not move, pushed off-centre by four sphere agents; its centre
    and linear velocity never change, its angle does."""
    E = 128
    n = 5
    N = E * n
    rng = np.random.default_rng(12)
    shape = np.tile(np.array([W.SPHERE] * 4 + [W.LINE], np.uint8), E)
    dims = np.tile(np.array([[0.05, 0]] * 4 + [[0.8, 0]], np.float32), (E, 1))
    flags = np.tile(np.array([7, 7, 7, 7, W.ROTATABLE | W.COLLIDABLE], np.uint8), E)
    st = np.zeros((6, N), np.float32)
    for e in range(E):
        o = e * n
        st[4, o + 4] = rng.uniform(-np.pi, np.pi)
        c, s = np.cos(st[4, o + 4]), np.sin(st[4, o + 4])
        for a in range(4):
            u = rng.uniform(-0.38, 0.38)  # along the segment, off centre
            v = rng.choice([-1, 1]) * rng.uniform(0.02, 0.06)
            st[0, o + a] = c * u - s * v
            st[1, o + a] = s * u + c * v
    w = W.World(env_offset=(np.arange(E + 1) * n).astype(np.int32),
                n_agents=np.full(E, 4, np.int32), shape=shape, dims=dims,
                mass=np.ones(N, np.float32), flags=flags, state0=st, seed=12)
    _, gtraj = _check_world(w, "anchored segment", T=40)
    seg = np.arange(E) * n + 4
    assert np.all(gtraj[:, 0:4, seg] == st[None, 0:4, seg])
    assert np.abs(gtraj[-1][4, seg] - st[4, seg]).max() > 1e-3  # it turned


def _large_mixed_world(seed=13):
    """Two environments of 300 entities (200 spheres, 40 boxes, 60 segments)
    in [-3, 3]^2: more movers than a 256-lane workgroup. A non-colliding
    joint ties local entities 0 and 1; local entity 255 sits on entity 0, so
    their contact must be active (local index 255 is never excluded by a
    joint)."""
    E, n = 2, 300
    N = E * n
    rng = np.random.default_rng(seed)
    local = np.tile(np.arange(n), E)
    shape = np.where(local < 200, W.SPHERE, np.where(local < 240, W.BOX, W.LINE)).astype(np.uint8)
    # local 255 is a box; make it a sphere so the overlap with sphere 0 is a plain pair
    shape[local == 255] = W.SPHERE
    dims = np.zeros((N, 2), np.float32)
    dims[shape == W.SPHERE, 0] = 0.05
    dims[shape == W.BOX] = (0.15, 0.3)
    dims[shape == W.LINE, 0] = 0.5
    st = np.zeros((6, N), np.float32)
    st[0:2] = rng.uniform(-3, 3, (2, N)).astype(np.float32)
    st[4] = np.where(shape == W.SPHERE, 0, rng.uniform(-np.pi, np.pi, N)).astype(np.float32)
    for e in range(E):
        st[0:2, e * n + 255] = st[0:2, e * n] + np.float32(0.03)
    ja = np.array([e * n for e in range(E)], np.int32)
    jb = ja + 1
    w = W.World(env_offset=(np.arange(E + 1) * n).astype(np.int32),
                n_agents=np.full(E, 100, np.int32), shape=shape, dims=dims,
                mass=np.ones(N, np.float32), flags=np.full(N, 7, np.uint8), state0=st,
                joint_a=ja, joint_b=jb, anchor_a=np.zeros((E, 2), np.float32),
                anchor_b=np.zeros((E, 2), np.float32), joint_rest=np.full(E, -1.0, np.float32),
                seed=seed)
    return w


def test_large_mixed_environments():
    """Non-sphere environments of 300 movers (1024-lane workgroups of the
    generic kernel), joint exclusion next to local index 255."""
    w = _large_mixed_world()
    b, _ = _check_world(w, "large mixed (300 movers)", T=20)
    print(f"plan {b.schedule_name(0)}")
    ow = O.OracleWorld(w)
    _, om, _ = ow.step(w.state0, w.actions(1)[0])
    n = 300
    la, lc = 0, 255
    slot = la * n - la * (la + 1) // 2 + (lc - la - 1)
    assert om[slot] == 1


def test_large_mixed_adjoint_dot_test():
    """The adjoint on 300-entity environments (adjoint workgroups above 64
    lanes) and on the options world with gravity and explicit inertia: the
    dot test <J^T w, v> = <w, J v> against the oracle's forward-mode JVP."""
    from tests.test_gpu_adjoint import _dot_test
    _dot_test(_large_mixed_world(), 1, 1, "large mixed step", tol=1e-4, min_frac=0.5)
    w = W.mixed(64, seed=14)
    w.gravity = (0.3, -0.7)
    w.inertia = np.random.default_rng(14).uniform(0.002, 0.05, w.n_entities).astype(np.float32)
    w.min_dist = 0.01
    _dot_test(w, 6, 2, "options T=6", tol=1e-3, min_frac=0.5)


def test_nonfinite_debug_flag():
    """VMAS_DEBUG_NONFINITE: a NaN fed into one environment's state (plain
    data) is found by the check after the rollout; the next call returns
    VMAS_ERR_NONFINITE (and enqueues nothing), the call after it proceeds,
    the marks name exactly that environment, and the other environments'
    results are bitwise those of a batch without the NaN."""
    from paper_2207_03530_amd import binding as B
    w = W.mixed(32, seed=15)
    T = 10
    acts = _dev(w.actions(T))
    b = B.Batch(w, 0, debug_nonfinite=True)
    st = w.state0.copy()
    bad_env = 5
    st[2, w.env_offset[bad_env] + 3] = np.nan
    s = _dev(st)
    b.rollout(s, acts)
    s_before = s.clone()
    with pytest.raises(B.VmasError) as ex:
        b.rollout(s, acts)
    assert ex.value.status == 5 and "1 environment" in str(ex.value)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(s, nan=7.0), torch.nan_to_num(s_before, nan=7.0))
    marks, cnt = b.nonfinite_envs()
    assert cnt == 1 and marks[bad_env] == 1 and marks.sum() == 1
    b.rollout(s, acts)  # reported once: this call proceeds
    torch.cuda.synchronize()
    marks, cnt = b.nonfinite_envs(clear=True)
    assert cnt == 1
    marks, cnt = b.nonfinite_envs()
    assert cnt == 0 and marks.sum() == 0
    # the other environments are untouched by the NaN
    ref = B.Batch(w, 0)
    r = _dev(w.state0)
    ref.rollout(r, acts)
    torch.cuda.synchronize()
    seg = np.repeat(np.arange(w.n_envs), np.diff(w.env_offset))
    good = torch.as_tensor(np.tile(seg != bad_env, 6).reshape(6, -1), device="cuda:0")
    sv = s_before.view(6, -1)
    rv = r.view(6, -1)
    assert torch.equal(sv[good], rv[good])
    # a finite batch never reports
    s2 = _dev(w.state0)
    b.rollout(s2, acts)
    b.step(s2, acts[0].contiguous())
    torch.cuda.synchronize()
    assert b.nonfinite_envs()[1] == 0
