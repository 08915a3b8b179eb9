"""Helpers shared by the GPU parity tests: error metrics and oracle runs.

State parity is normwise per environment per field group {position,
velocity, angle, angular velocity}: ||g - o||_inf / max(||o||_inf, 1e-6),
with the infinity norm over the entities of the environment.
"""
import numpy as np

GROUPS = {"pos": (0, 1), "vel": (2, 3), "theta": (4,), "omega": (5,)}


def env_rel_err(gpu: np.ndarray, ora: np.ndarray, env_offset: np.ndarray) -> np.ndarray:
    """[E, 4] relative error of each field group of each environment."""
    gpu = np.asarray(gpu, np.float64)
    ora = np.asarray(ora, np.float64)
    E = len(env_offset) - 1
    out = np.zeros((E, len(GROUPS)))
    seg = np.repeat(np.arange(E), np.diff(env_offset))
    for k, rows in enumerate(GROUPS.values()):
        diff = np.abs(gpu[list(rows)] - ora[list(rows)]).max(0)
        mag = np.abs(ora[list(rows)]).max(0)
        dmax = np.zeros(E)
        mmax = np.zeros(E)
        np.maximum.at(dmax, seg, diff)
        np.maximum.at(mmax, seg, mag)
        out[:, k] = dmax / np.maximum(mmax, 1e-6)
    return out


def pair_env(env_offset: np.ndarray) -> np.ndarray:
    """Environment of every pair slot."""
    n = np.diff(env_offset).astype(np.int64)
    return np.repeat(np.arange(len(n)), n * (n - 1) // 2)


def pair_shapes(shape: np.ndarray, env_offset: np.ndarray):
    """(shape_lo, shape_hi) of every pair slot, lexicographic within envs."""
    lo, hi = [], []
    for b in range(len(env_offset) - 1):
        o, n = env_offset[b], env_offset[b + 1] - env_offset[b]
        a, c = np.triu_indices(n, 1)
        lo.append(shape[o + a])
        hi.append(shape[o + c])
    if not lo:
        return np.zeros(0, np.uint8), np.zeros(0, np.uint8)
    return np.concatenate(lo), np.concatenate(hi)


def ill_conditioned(ow, state0: np.ndarray, actions: np.ndarray, rel: float = 1e-7,
                    thresh: float = 1e-4, seed: int = 7) -> np.ndarray:
    """Environments whose FP64 trajectory moves by more than `thresh` (same
    metric) when the initial positions are perturbed by `rel` relative."""
    ref, _, _ = ow.rollout(state0, actions, want_mask=False)
    rng = np.random.default_rng(seed)
    s = np.asarray(state0, np.float64).copy()
    s[0:2] *= 1.0 + rel * rng.choice([-1.0, 1.0], size=s[0:2].shape)
    pert, _, _ = ow.rollout(s, actions, want_mask=False)
    return env_rel_err(pert, ref, ow.w.env_offset).max(1) > thresh


def near_threshold_envs(ow, traj: np.ndarray, band: float) -> np.ndarray:
    """Environments where some eligible pair came within `band` of its
    contact threshold d_min at some step of an oracle trajectory: there the
    discontinuous force of Eq. (2) makes the outcome depend on rounding."""
    from oracle import oracle as O
    penv = pair_env(ow.w.env_offset)
    flag = np.zeros(ow.w.n_envs, bool)
    for t in range(traj.shape[0] - 1):
        d, dm = O.pair_distances(ow, traj[t])
        close = np.abs(d - dm) <= band
        close &= ~np.isnan(d)
        flag[penv[close]] = True
    return flag
