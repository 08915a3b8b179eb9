"""Helpers of the GPU parity tests: device copies, step loops through the C
boundary, and the checks of one step and of free-running trajectories
against the FP64 oracle (metrics in tests/parity.py)."""
import numpy as np
import pytest

from tests import parity as PU

torch = pytest.importorskip("torch")


def _batch(w):
    from paper_2207_03530_amd import binding as B
    return B.Batch(w, 0)


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda:0", dtype)


def _gpu_step(b, state, act, masks=True, forces=False):
    st = _dev(state)
    mk = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0") if masks else None
    fo = torch.zeros(3 * b.N, dtype=torch.float32, device="cuda:0") if forces else None
    b.step(st, _dev(act), mk, fo)
    torch.cuda.synchronize()
    out = [st.cpu().numpy().reshape(6, -1)]
    out.append(mk.cpu().numpy() if masks else None)
    out.append(fo.cpu().numpy().reshape(3, -1) if forces else None)
    return out


def _gpu_run(b, state0, acts, ids=None, slots=None):
    """Step loop on the GPU: states [T+1, 6, n] and masks [T, p] (restricted
    to entity ids / pair slots when given)."""
    T = acts.shape[0]
    s = _dev(state0)
    a = _dev(acts)
    mk = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
    ids_t = None if ids is None else torch.as_tensor(ids, device="cuda:0")
    sl_t = None if slots is None else torch.as_tensor(slots, device="cuda:0")
    trs, mks = [], []
    pick = (lambda x: x.view(6, -1)) if ids_t is None else (lambda x: x.view(6, -1)[:, ids_t])
    trs.append(pick(s).cpu().numpy())
    for t in range(T):
        b.step(s, a[t], mk)
        trs.append(pick(s).cpu().numpy())
        mks.append((mk if sl_t is None else mk[sl_t]).cpu().numpy())
    return s, np.stack(trs), np.stack(mks)


def _mask_check(w, ow, state, gmask, omask, name=""):
    """Masks equal except for band cases (tests/parity.py mask_compare);
    returns the band slots."""
    band = PU.mask_compare(ow, state, gmask, omask)
    print(f"{name} mask: contacts {int(np.sum(omask))}, band cases {len(band)}, nearest "
          f"|d - d_min| {PU.nearest_to_threshold(ow, state):.3g}")
    return band


def _one_step_check(w, ow, st, act, g, o, name, skip=None, min_plain=0.5):
    """One step from the same FP32 input, every environment asserted with
    tests/parity.py conditioned_check at 1e-5 (per-environment denominator
    plus the allowance of the exact result's own FP32-size sensitivity); the
    batch-scaled metric is printed. `skip`: environments with a band case
    (their contact decision legitimately differs), counted. At least
    `min_plain` of the environments must meet the plain 1e-5 without the
    allowance."""
    perts = PU.perturbed_steps(ow, st, act)
    ok, plain, allow = PU.conditioned_check(g, o, perts, w.env_offset, 1e-5)
    if skip is not None:
        ok = ok | skip
        allow = allow & ~skip
    err = PU.env_err(g, o, w.env_offset)
    bad = np.nonzero(~ok)[0]
    frac_plain = 1.0 - allow.mean()
    print(f"{name}: per-env err median {np.median(plain):.3g}, plain 1e-5 met by "
          f"{frac_plain:.3f} of envs, allowance used by {allow.sum()}/{w.n_envs}, band skips "
          f"{0 if skip is None else int(skip.sum())}, batch-scaled max {err.max():.3g}")
    assert bad.size == 0, (f"{name}: envs {bad[:8]} fail even with the allowance (plain "
                           f"{plain[bad[:8]]}); env {bad[0]} (|g-o|, |o|, rho) per group: "
                           f"{PU.conditioned_detail(g, o, perts, w.env_offset, bad[0])}")
    assert frac_plain >= min_plain, f"{name}: plain 1e-5 only on {frac_plain:.3f} of envs"
    return err


def _free_run_check(w, ow, gtraj, gmasks, acts, name, tol=1e-3, min_full=0.75, min_steps=None):
    """Free-running comparison of a T-step GPU trajectory with the oracle's.
    Each environment is compared at every step up to its cutoff with
    conditioned_check at `tol` (the allowance sized by the exact trajectory's
    own deviation under an FP32-size perturbation of the initial poses and by
    FP32 evaluations of the oracle's definition; K = 4 on at least 99.9 % of
    the compared environment-steps, K = 32 on all). The
    cutoff is the first valid mask fork (tests/parity.py fork_compare: a
    contact decision that differs only where the pair sat within the
    trajectories' deviation of d_min; after it the two runs are different
    but equally valid trajectories) or the FP64 predictability horizon
    (tests/parity.py horizon), whichever comes first. At least `min_full` of
    the environments must be compared for `min_steps` steps (default T).
    Printed for comparison: how many environments the exact trajectory
    itself forks on under that perturbation, and the fraction meeting the
    plain tolerance at every compared step."""
    ora, fork, invalid = PU.fork_compare(ow, gtraj, gmasks, w.state0, acts)
    assert not invalid, f"{name}: mask forks outside the deviation band: {invalid[:5]}"
    T = acts.shape[0]
    perts = PU.perturbed_trajectories(ow, w.state0, acts)
    hor = PU.horizon(ow, w.state0, acts, tol=tol)
    cut = np.minimum(fork, hor)
    plain_all = np.ones(w.n_envs, bool)
    worst = 0.0
    needs = []
    for t in range(1, T + 1):
        live = cut >= t
        if not live.any():
            break
        pt = [p[t] for p in perts]
        need, plain, allow = PU.conditioned_check(gtraj[t], ora[t], pt, w.env_offset, tol, K=None)
        bad = np.nonzero(live & (need > 32))[0]
        assert bad.size == 0, (f"{name}: step {t}: envs {bad[:8]} plain err {plain[bad[:8]]}; env "
                               f"{bad[0]} (|g-o|, |o|, rho) per group: "
                               f"{PU.conditioned_detail(gtraj[t], ora[t], pt, w.env_offset, bad[0])}")
        needs.append(need[live])
        plain_all &= ~(live & allow)
        worst = max(worst, plain[live].max())
    needs = np.concatenate(needs) if needs else np.zeros(1)
    assert (needs > 4).mean() <= 1e-3, f"{name}: allowance K > 4 on {(needs > 4).mean():.4f}"
    # forks of the exact trajectory against its own perturbed copy (intrinsic)
    penv = PU.pair_env(w.env_offset)
    self_fork = np.zeros(w.n_envs, bool)
    for p in perts:
        for t in range(T):
            _, m1, _ = ow.step(ora[t], acts[t])
            _, m2, _ = ow.step(p[t], acts[t])
            self_fork[np.unique(penv[m1 != m2])] = True
    need = T if min_steps is None else min_steps
    full = (cut >= need).mean()
    print(f"{name}: forks {(fork < T).sum()} (exact run vs its perturbed copy: "
          f"{self_fork.sum()}), FP64 horizon < T {(hor < T).sum()}, median cutoff "
          f"{np.median(cut):.0f}/{T}, compared for {need} steps {full:.2f}, plain {tol:g} at every "
          f"compared step {plain_all.mean():.2f}, max plain err {worst:.3g}, allowance K > 4 on "
          f"{(needs > 4).mean():.5f} of env-steps, largest K {needs.max():.3g}")
    assert full >= min_full
    return ora


def _teacher_forced_check(w, ow, gtraj, gmasks, acts, name, tol=1e-5, min_plain=0.85):
    """Teacher forcing along a GPU trajectory: at every step t the oracle
    steps from the GPU's own FP32 state gtraj[t] with the same actions; its
    result must match gtraj[t + 1] by conditioned_check at `tol` (allowance
    K = 4 times the FP32 rounding realisations' spread on at least 99.9 % of
    environment-steps, K = 32 on all: the ratio of two rounding errors has a
    long tail) and its contact mask gmasks[t] up to band cases
    (environment-steps with a band case are counted and skipped). At least
    `min_plain` of the environment-steps must meet the plain tolerance."""
    T = acts.shape[0]
    penv = PU.pair_env(w.env_offset)
    worst = 0.0
    nband = 0
    contacts = 0
    allowed = 0
    needs = []
    for t in range(T):
        st = gtraj[t]
        o, om, _ = ow.step(st, acts[t])
        band = PU.mask_compare(ow, st, gmasks[t], om)
        nband += len(band)
        contacts += int(om.sum())
        skip = np.zeros(w.n_envs, bool)
        skip[penv[band]] = True
        perts = PU.perturbed_steps(ow, st, acts[t])
        need, plain, allow = PU.conditioned_check(gtraj[t + 1], o, perts, w.env_offset, tol, K=None)
        need = np.where(skip, 0.0, need)
        bad = np.nonzero(need > 32)[0]
        assert bad.size == 0, (f"{name}: step {t}: envs {bad[:8]} plain err {plain[bad[:8]]}; env "
                               f"{bad[0]} (|g-o|, |o|, rho) per group: "
                               f"{PU.conditioned_detail(gtraj[t + 1], o, perts, w.env_offset, bad[0])}")
        needs.append(need)
        allowed += int((allow & ~skip).sum())
        worst = max(worst, plain[~skip].max() if (~skip).any() else 0.0)
    needs = np.concatenate(needs)
    frac = 1.0 - allowed / (T * w.n_envs)
    over4 = (needs > 4).mean()
    print(f"{name}: {T} teacher-forced steps x {w.n_envs} envs, contacts {contacts}, band cases "
          f"{nband}, plain {tol:g} met by {frac:.4f} of env-steps, allowance K > 1 on "
          f"{(needs > 1).mean():.4f}, K > 4 on {over4:.5f}, largest K {needs.max():.3g}, max plain "
          f"err {worst:.3g}")
    assert frac >= min_plain, f"{name}: plain {tol:g} met by {frac:.4f} of env-steps < {min_plain}"
    assert over4 <= 1e-3
    return worst
