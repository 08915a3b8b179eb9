"""Seeded synthetic workloads for the batched 2D physics step.

This module only *draws* inputs: entity layouts, initial states and action
sequences shaped like the paper's scenarios. It holds none of the physics
(no forces, no geometry, no integration, no inertia or rest-length
defaults) and is the one module shared by the HIP path's tests and the CPU
oracle's tests.

Random numbers come from a counter-based SplitMix64 (Steele, Lea, Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014):

    key(seed, stream)   = mix64(seed + (stream + 1) * GOLDEN)
    draw(seed, stream, i) = mix64(key + (i + 1) * GOLDEN)      (mod 2^64)

i.e. draw(., ., i) is output i of a SplitMix64 generator started at ``key``.
A draw becomes a uniform u = (draw >> 40) * 2^-24 and a = 2u - 1, exact in
FP32, so both sides consume identical values. Streams: 1 positions,
2 actions, 3 orientations, 4 per-environment agent counts, 5 candidate
positions of the separated layout (rejection sampling).

Action element (t, agent, comp) of a batch with A agents in total is draw
index (t * A + agent) * 2 + comp; the GPU rollout can regenerate the same
numbers in-kernel from the same definition.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)

STREAM_POS, STREAM_ACT, STREAM_THETA, STREAM_COUNT, STREAM_SEP = 1, 2, 3, 4, 5

SPHERE, BOX, LINE = 0, 1, 2
MOVABLE, ROTATABLE, COLLIDABLE = 1, 2, 4


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = np.uint64(seed) + np.uint64(stream + 1) * GOLDEN
    return mix64(np.array([k], dtype=np.uint64))[0]


def draw_u64(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    key = stream_key(seed, stream)
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + (idx + np.uint64(1)) * GOLDEN)


def draw_sym(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Uniform in [-1, 1) on the 2^-23 grid, exactly representable in FP32."""
    k = (draw_u64(seed, stream, idx) >> np.uint64(40)).astype(np.int64)
    return ((k - (1 << 23)).astype(np.float64) / float(1 << 23)).astype(np.float32)


def draw_int(seed: int, stream: int, idx: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """Integers uniform in [lo, hi] by multiply-shift of 24 random bits."""
    k = (draw_u64(seed, stream, idx) >> np.uint64(40)).astype(np.int64)
    return lo + ((k * (hi - lo + 1)) >> 24)


@dataclasses.dataclass
class World:
    """Entity layout of a batch plus world parameters and an initial state.

    Arrays follow the C boundary: entity e of environment b is global index
    env_offset[b] + e, the agents of b are its first n_agents[b] entities,
    state is float32 [6, N] (x, y, vx, vy, theta, omega).
    """

    env_offset: np.ndarray      # int32 [E + 1]
    n_agents: np.ndarray        # int32 [E]
    shape: np.ndarray           # uint8 [N]
    dims: np.ndarray            # float32 [N, 2]
    mass: np.ndarray            # float32 [N]
    flags: np.ndarray           # uint8 [N]
    state0: np.ndarray          # float32 [6, N]
    inertia: Optional[np.ndarray] = None    # float32 [N] or None (textbook)
    max_speed: Optional[np.ndarray] = None  # float32 [N] or None
    joint_a: Optional[np.ndarray] = None    # int32 [J]
    joint_b: Optional[np.ndarray] = None
    anchor_a: Optional[np.ndarray] = None   # float32 [J, 2]
    anchor_b: Optional[np.ndarray] = None
    joint_rest: Optional[np.ndarray] = None  # float32 [J]; < 0: from state0
    joint_collide: Optional[np.ndarray] = None
    dt: float = 0.1
    drag: float = 0.25
    gravity: tuple = (0.0, 0.0)
    contact_force: float = 100.0
    contact_margin: float = 1e-3
    min_dist: float = 0.0
    joint_stiffness: float = 100.0
    seed: int = 0
    name: str = ""

    @property
    def n_envs(self) -> int:
        return int(self.env_offset.shape[0] - 1)

    @property
    def n_entities(self) -> int:
        return int(self.env_offset[-1])

    @property
    def n_agents_total(self) -> int:
        return int(self.n_agents.sum())

    @property
    def n_joints(self) -> int:
        return 0 if self.joint_a is None else int(self.joint_a.shape[0])

    def agent_ids(self) -> np.ndarray:
        """Global entity id of every agent, in action-row order."""
        ids = [np.arange(self.env_offset[b], self.env_offset[b] + self.n_agents[b])
               for b in range(self.n_envs)]
        return np.concatenate(ids).astype(np.int64) if ids else np.zeros(0, np.int64)

    def actions(self, T: int, t0: int = 0) -> np.ndarray:
        """float32 [T, A, 2] actions uniform in [-1, 1)^2 for steps t0 .. t0+T-1."""
        A = self.n_agents_total
        t = np.arange(t0, t0 + T, dtype=np.uint64)[:, None, None]
        a = np.arange(A, dtype=np.uint64)[None, :, None]
        c = np.arange(2, dtype=np.uint64)[None, None, :]
        idx = (t * np.uint64(A) + a) * np.uint64(2) + c
        return draw_sym(self.seed, STREAM_ACT, idx)

    def pair_slots(self) -> int:
        n = np.diff(self.env_offset).astype(np.int64)
        return int((n * (n - 1) // 2).sum())


def _positions(seed: int, N: int) -> np.ndarray:
    idx = np.arange(2 * N, dtype=np.uint64)
    return draw_sym(seed, STREAM_POS, idx).reshape(N, 2)


def _orientations(seed: int, N: int) -> np.ndarray:
    u = draw_sym(seed, STREAM_THETA, np.arange(N, dtype=np.uint64))
    return (u * np.float32(np.pi)).astype(np.float32)


def _state(pos: np.ndarray, theta: Optional[np.ndarray]) -> np.ndarray:
    N = pos.shape[0]
    s = np.zeros((6, N), np.float32)
    s[0] = pos[:, 0]
    s[1] = pos[:, 1]
    if theta is not None:
        s[4] = theta
    return s


def spread(n_envs: int, n_agents: int = 4, n_landmarks: int = 2, radius: float = 0.05,
           seed: int = 0) -> World:
    """Sphere agents plus immovable sphere landmarks per environment (the
    shape of the MPE 'simple_spread' task used for the paper's scalability
    comparison; 4 agents + 2 landmarks, r = 0.05, m = 1 by default).
    Positions uniform in [-1, 1]^2, velocities and angles zero."""
    n = n_agents + n_landmarks
    N = n_envs * n
    env_offset = (np.arange(n_envs + 1) * n).astype(np.int32)
    local = np.tile(np.arange(n), n_envs)
    is_agent = local < n_agents
    shape = np.full(N, SPHERE, np.uint8)
    dims = np.zeros((N, 2), np.float32)
    dims[:, 0] = radius
    flags = np.where(is_agent, MOVABLE | ROTATABLE | COLLIDABLE, COLLIDABLE).astype(np.uint8)
    return World(env_offset=env_offset, n_agents=np.full(n_envs, n_agents, np.int32),
                 shape=shape, dims=dims, mass=np.ones(N, np.float32), flags=flags,
                 state0=_state(_positions(seed, N), None), seed=seed,
                 name=f"spread{n_envs}x({n_agents}a+{n_landmarks}l)")


def _separated_positions(seed: int, n_envs: int, reach: np.ndarray, half_width: float,
                         gap: float, tries: int = 256) -> np.ndarray:
    """[n_envs * n, 2] positions, uniform in [-half_width, half_width]^2 and
    rejection-sampled per environment: entity i takes the first of its
    candidates (stream 5, candidate k of entity i of environment b is draw
    pair ((b * n + i) * tries + k)) whose circle of radius reach[i] keeps
    `gap` from the circles of entities 0 .. i-1 already placed. `reach` is
    a radius that covers the entity's whole shape, so no two shapes touch."""
    n = reach.shape[0]
    pos = np.zeros((n_envs, n, 2), np.float32)
    for i in range(n):
        placed = np.zeros(n_envs, bool)
        for k0 in range(0, tries, 16):
            ks = np.arange(k0, k0 + 16, dtype=np.uint64)
            base = ((np.arange(n_envs, dtype=np.uint64)[:, None] * np.uint64(n) + np.uint64(i))
                    * np.uint64(tries) + ks[None, :]) * np.uint64(2)
            cx = draw_sym(seed, STREAM_SEP, base) * np.float32(half_width)
            cy = draw_sym(seed, STREAM_SEP, base + np.uint64(1)) * np.float32(half_width)
            ok = np.ones(cx.shape, bool)
            for j in range(i):
                dd = np.hypot(cx.astype(np.float64) - pos[:, j, 0:1], cy.astype(np.float64) - pos[:, j, 1:2])
                ok &= dd > reach[i] + reach[j] + gap
            first = np.argmax(ok, 1)
            take = ~placed & ok[np.arange(n_envs), first]
            pos[take, i, 0] = cx[take, first[take]]
            pos[take, i, 1] = cy[take, first[take]]
            placed |= take
            if placed.all():
                break
        if not placed.all():
            raise ValueError(f"entity {i}: no separated position in {tries} tries")
    return pos.reshape(-1, 2)


def mixed(n_envs: int, n_spheres: int = 16, n_boxes: int = 4, n_lines: int = 8,
          radius: float = 0.03, box=(0.1, 0.3), line_len: float = 0.5, joints: bool = True,
          seed: int = 0, half_width: float = 1.0, separated: bool = False) -> World:
    """Mixed shapes and joints: sphere agents, boxes and line segments, all
    movable and rotatable, random poses in [-1, 1]^2 with angles uniform in
    [-pi, pi); two joints per environment tie agents 0 and 1 (at their
    centres) to box 0 at its local (0, +ly/2) and (0, -ly/2).

    separated=True: positions uniform in [-half_width, half_width]^2 but
    rejection-sampled so that no two shapes are within 0.02 of each other at
    t = 0 (by circles covering each shape: sphere radius, half the box
    diagonal, half the segment); the joints' rest lengths are the anchor
    distances of that layout."""
    n = n_spheres + n_boxes + n_lines
    N = n_envs * n
    env_offset = (np.arange(n_envs + 1) * n).astype(np.int32)
    local = np.tile(np.arange(n), n_envs)
    shape = np.where(local < n_spheres, SPHERE,
                     np.where(local < n_spheres + n_boxes, BOX, LINE)).astype(np.uint8)
    dims = np.zeros((N, 2), np.float32)
    dims[shape == SPHERE, 0] = radius
    dims[shape == BOX, 0] = box[0]
    dims[shape == BOX, 1] = box[1]
    dims[shape == LINE, 0] = line_len
    flags = np.full(N, MOVABLE | ROTATABLE | COLLIDABLE, np.uint8)
    theta = _orientations(seed, N)
    theta[shape == SPHERE] = 0.0
    if separated:
        kinds = shape[:n]
        reach = np.where(kinds == SPHERE, radius,
                         np.where(kinds == BOX, 0.5 * np.hypot(box[0], box[1]), 0.5 * line_len))
        pos = _separated_positions(seed, n_envs, reach.astype(np.float64), half_width, 0.02)
    else:
        pos = _positions(seed, N) * np.float32(half_width)
    w = World(env_offset=env_offset, n_agents=np.full(n_envs, n_spheres, np.int32),
              shape=shape, dims=dims, mass=np.ones(N, np.float32), flags=flags,
              state0=_state(pos, theta), seed=seed,
              name=f"mixed{n_envs}x({n_spheres}s+{n_boxes}b+{n_lines}l)"
                   + ("-separated" if separated else ""))
    if joints and n_boxes > 0 and n_spheres >= 2:
        base = np.arange(n_envs, dtype=np.int32) * n
        box0 = base + n_spheres
        w.joint_a = np.stack([base, base + 1], 1).reshape(-1).astype(np.int32)
        w.joint_b = np.stack([box0, box0], 1).reshape(-1).astype(np.int32)
        J = w.joint_a.shape[0]
        w.anchor_a = np.zeros((J, 2), np.float32)
        w.anchor_b = np.zeros((J, 2), np.float32)
        w.anchor_b[0::2, 1] = box[1] / 2
        w.anchor_b[1::2, 1] = -box[1] / 2
        w.joint_rest = np.full(J, -1.0, np.float32)
    return w


def uneven(n_envs: int, lo: int = 2, hi: int = 64, radius: float = 0.05, seed: int = 0) -> World:
    """Environments of sphere agents only, agent counts uniform in {lo..hi};
    same position and action distributions as :func:`spread`."""
    counts = draw_int(seed, STREAM_COUNT, np.arange(n_envs, dtype=np.uint64), lo, hi)
    counts = counts.astype(np.int32)
    env_offset = np.zeros(n_envs + 1, np.int32)
    env_offset[1:] = np.cumsum(counts)
    N = int(env_offset[-1])
    shape = np.full(N, SPHERE, np.uint8)
    dims = np.zeros((N, 2), np.float32)
    dims[:, 0] = radius
    flags = np.full(N, MOVABLE | ROTATABLE | COLLIDABLE, np.uint8)
    return World(env_offset=env_offset, n_agents=counts.copy(), shape=shape, dims=dims,
                 mass=np.ones(N, np.float32), flags=flags,
                 state0=_state(_positions(seed, N), None), seed=seed,
                 name=f"uneven{n_envs}x({lo}..{hi})")


def subset(w: World, envs: np.ndarray) -> World:
    """The same environments, re-indexed: a batch made of envs[k] of w, in order
    (joints follow their environment)."""
    envs = np.asarray(envs, np.int64)
    sizes = np.diff(w.env_offset)[envs]
    off = np.zeros(len(envs) + 1, np.int32)
    off[1:] = np.cumsum(sizes)
    ids = np.concatenate([np.arange(w.env_offset[b], w.env_offset[b + 1]) for b in envs])
    remap = -np.ones(w.n_entities, np.int64)
    remap[ids] = np.arange(len(ids))
    out = dataclasses.replace(
        w, env_offset=off, n_agents=w.n_agents[envs].copy(), shape=w.shape[ids].copy(),
        dims=w.dims[ids].copy(), mass=w.mass[ids].copy(), flags=w.flags[ids].copy(),
        state0=w.state0[:, ids].copy(),
        inertia=None if w.inertia is None else w.inertia[ids].copy(),
        max_speed=None if w.max_speed is None else w.max_speed[ids].copy())
    if w.n_joints:
        keep = remap[w.joint_a] >= 0
        out.joint_a = remap[w.joint_a[keep]].astype(np.int32)
        out.joint_b = remap[w.joint_b[keep]].astype(np.int32)
        out.anchor_a = w.anchor_a[keep].copy()
        out.anchor_b = w.anchor_b[keep].copy()
        out.joint_rest = w.joint_rest[keep].copy()
        out.joint_collide = None if w.joint_collide is None else w.joint_collide[keep].copy()
    return out
