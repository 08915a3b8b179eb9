"""Helpers shared by the GPU parity tests: error metrics, conditioning checks
and the fork-aware comparison of free-running trajectories.

Relative error (the reading of "1e-5 relative after one step, 1e-3 after
100" used throughout): normwise per field group {position, velocity,
angle, angular velocity}. For environment e and group G the per-environment
error is

    err[e, G] = ||g_e,G - o_e,G||_inf / max(||o_e,G||_inf, 1e-6)

(numerator and denominator over the entities of e: env_rel_err_local). The
tests assert it together with the batch-scaled variant env_err, whose
denominator is the group's magnitude over the whole batch.

Conditioning: the state checks (conditioned_check) add to the relative
tolerance K times rho, the largest distance from the exact (FP64) result
of five other results that are equally correct at FP32 precision: the exact
results from two FP32-rounding-size (1e-7 relative) perturbations of the
input poses, and the oracle's own definition evaluated in FP32 from the
input and from both perturbed inputs (perturbed_steps,
perturbed_trajectories). On a well-conditioned environment that allowance is
far below the tolerance; it matters where no FP32 computation can meet the
relative tolerance (a quantity that is exactly zero in the exact result but
rounding-sized in FP32, where the per-environment denominator is its 1e-6
floor, or a stiff contact that amplifies rounding). No environment is
excluded; the tests bound K for all environments and, tighter, for all but
a small tail, and print how many needed the allowance at all.

Forks: the contact decision of Eq. (2) is a threshold, so two correct
trajectories may take different decisions once rounding has moved them
apart. Each step's masks are compared; the first step where they differ is
a valid fork only if every differing pair sat within the measured
trajectory deviation of d_min. After a valid fork the environment's
trajectories are no longer comparable and it leaves the final comparison
(counted).
"""
import numpy as np

GROUPS = {"pos": (0, 1), "vel": (2, 3), "theta": (4,), "omega": (5,)}


def group_scale(ora: np.ndarray) -> np.ndarray:
    ora = np.asarray(ora, np.float64)
    return np.array([max(np.abs(ora[list(r)]).max() if ora.size else 0.0, 1e-6)
                     for r in GROUPS.values()])


def env_err(gpu, ora, env_offset, scale=None) -> np.ndarray:
    """[E, 4]: per-environment max abs error of each group over the group's
    batch-wide magnitude (see module docstring)."""
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    scale = group_scale(ora) if scale is None else scale
    E = len(env_offset) - 1
    seg = np.repeat(np.arange(E), np.diff(env_offset))
    out = np.zeros((E, len(GROUPS)))
    for k, rows in enumerate(GROUPS.values()):
        diff = np.abs(gpu[list(rows)] - ora[list(rows)]).max(0)
        dmax = np.zeros(E)
        np.maximum.at(dmax, seg, diff)
        out[:, k] = dmax / scale[k]
    return out


def env_rel_err_local(gpu, ora, env_offset) -> np.ndarray:
    """[E, 4] with per-environment denominators (reported only)."""
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    E = len(env_offset) - 1
    seg = np.repeat(np.arange(E), np.diff(env_offset))
    out = np.zeros((E, len(GROUPS)))
    for k, rows in enumerate(GROUPS.values()):
        diff = np.abs(gpu[list(rows)] - ora[list(rows)]).max(0)
        mag = np.abs(ora[list(rows)]).max(0)
        dmax, mmax = np.zeros(E), np.zeros(E)
        np.maximum.at(dmax, seg, diff)
        np.maximum.at(mmax, seg, mag)
        out[:, k] = dmax / np.maximum(mmax, 1e-6)
    return out


def pair_env(env_offset: np.ndarray) -> np.ndarray:
    """Environment of every pair slot."""
    n = np.diff(env_offset).astype(np.int64)
    return np.repeat(np.arange(len(n)), n * (n - 1) // 2)


def pair_members(env_offset: np.ndarray):
    """(i, j) global entity ids of every pair slot, lexicographic per env."""
    I, J = [], []
    for b in range(len(env_offset) - 1):
        o, n = env_offset[b], env_offset[b + 1] - env_offset[b]
        a, c = np.triu_indices(n, 1)
        I.append(o + a)
        J.append(o + c)
    if not I:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(I), np.concatenate(J)


def pair_shapes(shape: np.ndarray, env_offset: np.ndarray):
    i, j = pair_members(env_offset)
    return shape[i], shape[j]


def ulp32(x) -> np.ndarray:
    """Spacing of FP32 numbers at |x| (in FP64)."""
    return np.spacing(np.abs(np.asarray(x, np.float64)).astype(np.float32)).astype(np.float64)


def in_band(ow, state, ulps=8):
    """Per pair slot: whether the exact distance lies within `ulps` FP32 ulps
    of d_min (see mask_compare); also returns (d64, d_min)."""
    from oracle import oracle as O
    w = ow.w
    st = np.asarray(state, np.float64)
    d, dm = O.pair_distances(ow, st)
    i, j = pair_members(w.env_offset)
    sph = (w.shape[i] == 0) & (w.shape[j] == 0)
    s = np.maximum(np.abs(d), dm)
    coord = np.max(np.abs(np.stack([st[0, i], st[1, i], st[0, j], st[1, j],
                                    w.dims[i, 0], w.dims[i, 1], w.dims[j, 0], w.dims[j, 1]])), 0)
    s = np.where(sph, s, np.maximum(s, coord))
    with np.errstate(invalid="ignore"):
        band = np.abs(d - dm) <= ulps * ulp32(s)
    return band, d, dm


def mask_compare(ow, state, gmask, omask, ulps=8):
    """Contact masks of one step from the same input state, compared the way
    Eq. (2)'s threshold allows.

    The oracle decides |x_ij| <= d_min in FP64 on its own signed distance;
    the GPU decides in FP32. A disagreement is admissible only for a pair
    whose exact distance lies within `ulps` FP32 ulps of the threshold:
    |d64 - d_min| <= ulps * ulp32(s). For two spheres s = max(|d|, d_min)
    (the decision is a difference of centres, squared and summed, whose
    rounding is relative to d). For a pair with a box or a segment the FP32
    distance is built from vertex coordinates, so s also covers the largest
    coordinate and size of the two entities. Any other disagreement raises.
    Returns the slots of the admissible ("band") disagreements."""
    gmask = np.asarray(gmask)
    omask = np.asarray(omask)
    diff = gmask != omask
    if not np.any(diff):
        return np.zeros(0, np.int64)
    band, d, dm = in_band(ow, state, ulps)
    bad = diff & ~band
    assert not np.any(bad), (
        f"contact mask differs outside the FP32 band at slots {np.nonzero(bad)[0][:10]}: "
        f"d - d_min = {(d - dm)[bad][:10]}, gpu {gmask[bad][:10]}, oracle {omask[bad][:10]}")
    return np.nonzero(diff)[0]


def nearest_to_threshold(ow, state):
    """Smallest |d64 - d_min| over the eligible pairs (how close the input
    comes to the band), for reporting."""
    from oracle import oracle as O
    d, dm = O.pair_distances(ow, np.asarray(state, np.float64))
    g = np.abs(d - dm)
    g = g[np.isfinite(g)]
    return float(g.min()) if g.size else float("inf")


def _perturb(state, rel, seed, shape=None):
    """Poses moved by +-rel (positions, in world units, and the angles of
    boxes and lines, in radians): the size of FP32 rounding of O(1)
    coordinates. A sphere's angle plays no part in its geometry."""
    rng = np.random.default_rng(seed)
    s = np.asarray(state, np.float64).copy()
    for r in (0, 1, 4):
        d = rel * rng.choice([-1.0, 1.0], size=s[r].shape)
        if r == 4 and shape is not None:
            d = np.where(shape == 0, 0.0, d)
        s[r] += d
    return s


def both_errs(gpu, ora, env_offset, scale=None) -> np.ndarray:
    """[E]: the larger of the batch-scaled and the per-environment error."""
    return np.maximum(env_err(gpu, ora, env_offset, scale).max(1),
                      env_rel_err_local(gpu, ora, env_offset).max(1))


def conditioned_check(gpu, ora, perts, env_offset, tol, K=4.0):
    """The per-environment comparison the parity tests assert (S23 reading
    with a conditioning allowance). For environment e and field group G,

        |g - o|_e,G <= tol * max(|o|_e,G, 1e-6) + K * rho_e,G

    (inf-norms over the entities of e), where rho_e,G is the largest
    |o' - o|_e,G over the results `perts` (perturbed_steps): how far the
    exact result moves when the input poses move by FP32 rounding size, and
    how far the same definition evaluated in FP32 lands from it.
    The first term is the relative tolerance with the per-environment
    denominator; the second admits what no FP32 computation can avoid on an
    ill-conditioned environment (a contact decision or a quantity that is
    exactly zero in the exact result but rounding-sized in FP32), so no
    environment is excluded. Returns (ok [E] bool, plain [E]: the plain
    relative error max_G |g - o|_e,G / max(|o|_e,G, 1e-6), allow [E]: whether
    the allowance was needed). With K=None, ok holds the multiple of rho each
    environment needs instead (0 where the plain tolerance holds)."""
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    E = len(env_offset) - 1
    seg = np.repeat(np.arange(E), np.diff(env_offset))
    need = np.zeros(E)
    plain = np.zeros(E)
    for rows in GROUPS.values():
        r = list(rows)
        num, mag, rho = np.zeros(E), np.zeros(E), np.zeros(E)
        np.maximum.at(num, seg, np.abs(gpu[r] - ora[r]).max(0))
        np.maximum.at(mag, seg, np.abs(ora[r]).max(0))
        for p in perts:
            np.maximum.at(rho, seg, np.abs(np.asarray(p, np.float64)[r] - ora[r]).max(0))
        den = np.maximum(mag, 1e-6)
        with np.errstate(invalid="ignore", divide="ignore"):
            over = np.maximum(num - tol * den, 0.0)
            need = np.maximum(need, np.where(over > 0, over / rho, 0.0))
        plain = np.maximum(plain, num / den)
    if K is None:
        return need, plain, plain > tol
    return need <= K, plain, plain > tol


def conditioned_detail(gpu, ora, perts, env_offset, e):
    """Per group of environment e: (|g - o|, |o|, rho) for failure messages."""
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    sl = slice(int(env_offset[e]), int(env_offset[e + 1]))
    out = {}
    for name, rows in GROUPS.items():
        r = list(rows)
        rho = max([np.abs(np.asarray(p, np.float64)[r, sl] - ora[r, sl]).max() for p in perts]
                  or [0.0])
        out[name] = (float(np.abs(gpu[r, sl] - ora[r, sl]).max()),
                     float(np.abs(ora[r, sl]).max()), float(rho))
    return out


def perturbed_steps(ow, state, act, rel=1e-7, seeds=(7, 8)):
    """The results that size the allowance of conditioned_check: the exact
    one-step results from FP32-rounding-size perturbations of the input
    poses, and the oracle's own definition evaluated in FP32 from the input
    and from the perturbed inputs (which carries the rounding of
    intermediate values: vertex coordinates, contact arms, spring
    stretches)."""
    pert = [_perturb(state, rel, sd, ow.w.shape) for sd in seeds]
    out = [ow.step(p, act, want_mask=False)[0] for p in pert]
    # FP32 evaluations from the input and from the perturbed inputs: several
    # realisations of FP32 rounding (one alone can be luckily small)
    out += [ow.rollout_fp32(p, np.asarray(act)[None])[0] for p in [state] + pert]
    return out


def perturbed_trajectories(ow, state0, actions, rel=1e-7, seeds=(7, 8)):
    """[T+1, 6, N] trajectories that size the allowance of a free run: exact
    ones from perturbed initial poses, and the oracle's definition evaluated
    in FP32."""
    pert = [_perturb(state0, rel, sd, ow.w.shape) for sd in seeds]
    out = [ow.rollout(p, actions, traj=True, want_mask=False)[2] for p in pert]
    out += [ow.rollout_fp32(p, actions, traj=True)[1] for p in [state0] + pert]
    return out


def ill_conditioned_step(ow, state, act, tol=1e-5, rel=1e-7, seeds=(7, 8)) -> np.ndarray:
    """Environments whose exact (FP64) one-step result moves by more than the
    tolerance itself (batch-scaled metric) when the input poses move by FP32
    rounding (`rel`): there even an exact computation on FP32 inputs cannot
    promise `tol`. (Used by the auxiliary force and adjoint checks; the
    state checks use conditioned_check.)"""
    ref, _, _ = ow.step(state, act, want_mask=False)
    scale = group_scale(ref)
    out = np.zeros(ow.w.n_envs, bool)
    for sd in seeds:
        pert, _, _ = ow.step(_perturb(state, rel, sd, ow.w.shape), act, want_mask=False)
        out |= env_err(pert, ref, ow.w.env_offset, scale).max(1) > tol
    return out


def ill_conditioned_rollout(ow, state0, actions, tol=1e-3, rel=1e-7, seeds=(7, 8)) -> np.ndarray:
    ref, _, _ = ow.rollout(state0, actions, want_mask=False)
    scale = group_scale(ref)
    out = np.zeros(ow.w.n_envs, bool)
    for sd in seeds:
        pert, _, _ = ow.rollout(_perturb(state0, rel, sd, ow.w.shape), actions, want_mask=False)
        out |= env_err(pert, ref, ow.w.env_offset, scale).max(1) > tol
    return out


def horizon(ow, state0, actions, tol=1e-3, rel=1e-7, seeds=(7, 8)) -> np.ndarray:
    """Per environment, the first step at which the exact (FP64) trajectory
    moves by more than tol/10 (batch-scaled metric) under an FP32-sized
    perturbation of the initial poses (T if never): beyond it the trajectory
    is chaotic at FP32 precision and two correct implementations need not
    agree."""
    T = actions.shape[0]
    _, _, ref = ow.rollout(state0, actions, traj=True, want_mask=False)
    E = ow.w.n_envs
    h = np.full(E, T)
    # group magnitudes over the whole run (a group that is exactly zero at one
    # step, e.g. every angular velocity before the first torque, is not
    # unpredictable because a perturbation makes it rounding-sized)
    scale = group_scale(np.concatenate(list(ref), axis=1))
    for sd in seeds:
        _, _, pt = ow.rollout(_perturb(state0, rel, sd, ow.w.shape), actions, traj=True,
                              want_mask=False)
        for t in range(1, T + 1):
            moved = env_err(pt[t], ref[t], ow.w.env_offset, scale).max(1) > tol / 10
            h = np.where(moved & (h > t - 1), np.minimum(h, t - 1), h)
    return h


def fork_compare(ow, gpu_traj, gpu_masks, state0, actions):
    """Step the oracle along the same inputs and compare per-step masks.

    gpu_traj: [T+1, 6, N] GPU states, gpu_masks: [T, P] GPU masks.
    Returns (ora_traj [T+1,6,N], fork_step [E] (T = no fork), invalid list)
    where `invalid` lists (step, slot) mask differences that were NOT within
    the trajectory deviation of the threshold (real failures)."""
    from oracle import oracle as O
    w = ow.w
    T = actions.shape[0]
    E = w.n_envs
    penv = pair_env(w.env_offset)
    pi, pj = pair_members(w.env_offset)
    seg = np.repeat(np.arange(E), np.diff(w.env_offset))
    ora = np.zeros((T + 1,) + np.shape(state0), np.float64)
    ora[0] = state0
    fork = np.full(E, T)
    invalid = []
    for t in range(T):
        o, om, _ = ow.step(ora[t], actions[t])
        ora[t + 1] = o
        diff = (gpu_masks[t] != om) & (fork[penv] == T)
        if np.any(diff):
            slots = np.nonzero(diff)[0]
            d, dm = O.pair_distances(ow, ora[t])
            dev = np.zeros(E)
            delta = np.maximum(np.abs(gpu_traj[t, 0:2] - ora[t, 0:2]).max(0),
                               0.5 * np.abs(gpu_traj[t, 4] - ora[t, 4]))
            np.maximum.at(dev, seg, delta)
            for q in slots:
                band = 4.0 * dev[penv[q]] + 2e-6 * max(1.0, abs(dm[q]))
                if not (abs(d[q] - dm[q]) <= band):
                    invalid.append((t, int(q), float(d[q] - dm[q]), float(band)))
            fork[np.unique(penv[slots])] = t
    return ora, fork, invalid
