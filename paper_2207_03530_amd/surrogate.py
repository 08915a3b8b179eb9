"""Training and evaluation driver of the learned contact surrogate.

Orchestration only: the dataset comes from the exact HIP step
(vmas_rollout trajectories and vmas_pair_features), the network is
trained by the HIP MLP kernels (vmas_mlp_train_step), and evaluation runs
vmas_step_surrogate next to the exact vmas_step. Host code selects which
pair slots become samples, shapes the training set and shuffles minibatch
order. The shaping evaluates Eq. (2) and its inverse on the targets (torch,
on the device): targets of contacts deeper than twice the fallback depth
are scaled to the force at that depth, and contacts within 2 k of onset are
repeated. This prepares training data only; the surrogate step itself,
including its fallback rule, runs in the HIP kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding as B
from . import workloads as W

BAND = 0.01          # candidate reach beyond touching bounding circles
FALLBACK = 0.5       # exact step when the predicted penetration exceeds 0.5 r
FEAT_L, FORCE_L = 0.1, 0.02   # feature length scale and target force scale c * FORCE_L


def _half_size(dims_over_l, code):
    """Length that the fallback rule compares penetration with: sphere r,
    box half its shorter side, line half its length (features -> metres)."""
    import torch
    d0, d1 = dims_over_l[:, 0] * FEAT_L, dims_over_l[:, 1] * FEAT_L
    return torch.where(code == 0, d0, torch.where(code == 0.5, 0.5 * torch.minimum(d0, d1), 0.5 * d0))


def penetration_of(y, c: float, k: float):
    """Penetration implied by a target / output through the inverse of Eq. (2)."""
    import torch
    mag = torch.linalg.norm(y, dim=1).double() * c * FORCE_L
    return (k * torch.log(torch.expm1(mag / (c * k)))).float()


def make_dataset(world, T: int, stride: int, max_samples: int, seed: int = 0, device: int = 0):
    """Candidate pair samples (features [n, 12], targets [n, 2]) from an
    exact rollout of `world`, taken every `stride` steps."""
    import torch
    dev = torch.device("cuda", device)
    b = B.Batch(world, device)
    N, P = world.n_entities, world.pair_slots()
    traj = torch.zeros((T + 1) * 6 * N, device=dev)
    st = torch.as_tensor(world.state0).to(dev).contiguous()
    b.rollout(st, torch.as_tensor(world.actions(T)).to(dev).contiguous(), traj=traj)
    feats, targs = [], []
    flags = torch.zeros(P, dtype=torch.uint8, device=dev)
    fbuf = torch.zeros(P, 12, device=dev)
    rng = np.random.default_rng(seed)
    total = 0
    for t in range(0, T + 1, stride):
        s_t = traj.view(T + 1, -1)[t].contiguous()
        b.pair_features(s_t, fbuf, flags, band=BAND)
        cand = np.nonzero(flags.cpu().numpy() & 1)[0]
        if cand.size == 0:
            continue
        slots = torch.as_tensor(cand.astype(np.int64), device=dev)
        f = torch.zeros(cand.size, 12, device=dev)
        y = torch.zeros(cand.size, 2, device=dev)
        fl = torch.zeros(cand.size, dtype=torch.uint8, device=dev)
        b.pair_features(s_t, f, fl, targets=y, slots=slots, band=BAND)
        # contacts deeper than twice the fallback threshold are taught as
        # exactly that deep: their prediction only has to trigger the exact
        # fallback, so the network need not fit the unbounded force there
        rr = torch.minimum(_half_size(f[:, 6:8], f[:, 10]), _half_size(f[:, 8:10], f[:, 11]))
        c, k = world.contact_force, world.contact_margin
        pen = penetration_of(y, c, k)
        cap = 2.0 * FALLBACK * rr
        deep = ((fl & 2) != 0) & (pen > cap)
        if bool(deep.any()):
            m_cap = c * k * torch.nn.functional.softplus(cap[deep].double() / k) / (c * FORCE_L)
            m = torch.linalg.norm(y[deep], dim=1).double()
            y[deep] = y[deep] * (m_cap / m).float().unsqueeze(1)
        # contacts within 2 k of onset, where Eq. (2) jumps and bends, are
        # taught four times as often
        pen = penetration_of(y, c, k)
        near = ((fl & 2) != 0) & (pen <= 2.0 * k)
        if bool(near.any()):
            f = torch.cat([f] + [f[near]] * 3)
            y = torch.cat([y] + [y[near]] * 3)
        feats.append(f)
        targs.append(y)
        total += f.shape[0]
        if total >= max_samples:
            break
    b.close()
    X = torch.cat(feats)[:max_samples].contiguous()
    Y = torch.cat(targs)[:max_samples].contiguous()
    perm = torch.as_tensor(rng.permutation(X.shape[0]), device=dev)
    return X[perm].contiguous(), Y[perm].contiguous()


def train(mlp: "B.Mlp", X, Y, epochs: int, batch: int = 8192, lr: float = 2e-3,
          lr_final: float = 1e-4, seed: int = 0, log=None):
    """Adam over minibatches reshuffled every epoch (seeded), learning rate
    decayed geometrically from lr to lr_final; returns the per-epoch mean loss."""
    import torch
    n = X.shape[0]
    nb = n // batch
    loss = torch.zeros(1, device=X.device)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    hist = []
    steps = epochs * nb
    k = 0
    for ep in range(epochs):
        order = torch.randperm(n, device=X.device, generator=gen)
        acc = torch.zeros(1, device=X.device)
        for q in range(nb):
            idx = order[q * batch:(q + 1) * batch]
            rate = lr * (lr_final / lr) ** (k / max(1, steps - 1))
            mlp.train_step(X[idx], Y[idx], rate, loss)
            acc += loss
            k += 1
        hist.append(float(acc.item()) / max(1, nb))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4g}")
    return hist


def training_set(parts, seed: int = 0):
    """Concatenates (X, Y) datasets and shuffles the rows with a seeded
    generator."""
    import torch
    X = torch.cat([p[0] for p in parts])
    Y = torch.cat([p[1] for p in parts])
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    perm = torch.randperm(X.shape[0], device=X.device, generator=gen)
    return X[perm].contiguous(), Y[perm].contiguous()


def contact_force_error(world, mlp: "B.Mlp", steps: int = 5, device: int = 0,
                        fallback: float = FALLBACK):
    """Normwise relative error ||F_sur - F||_2 / ||F||_2 of the contact forces
    (total force minus action and gravity) of the surrogate step against the
    exact step, from the same states along an exact trajectory; also the
    number of fallback pair sides per step."""
    import torch
    dev = torch.device("cuda", device)
    b = B.Batch(world, device)
    N = world.n_entities
    acts = torch.as_tensor(world.actions(steps)).to(dev).contiguous()
    st = torch.as_tensor(world.state0).to(dev).contiguous()
    errs, fbs = [], []
    agents = torch.as_tensor(world.agent_ids(), device=dev)
    for t in range(steps):
        fe = torch.zeros(3 * N, device=dev)
        fs = torch.zeros(3 * N, device=dev)
        nfb = torch.zeros(1, dtype=torch.int32, device=dev)
        s_exact = st.clone()
        b.step(s_exact, acts[t], None, fe)
        s_sur = st.clone()
        b.step_surrogate(mlp, s_sur, acts[t], BAND, fallback, fs, nfb)
        torch.cuda.synchronize()
        Fe = fe.view(3, N)[0:2].clone()
        Fs = fs.view(3, N)[0:2].clone()
        Fe[:, agents] -= acts[t].T
        Fs[:, agents] -= acts[t].T
        errs.append(float(torch.linalg.norm(Fs - Fe) / torch.linalg.norm(Fe)))
        fbs.append(int(nfb.item()))
        st = s_exact
    b.close()
    return errs, fbs


def time_steps(world, mlp: "B.Mlp", reps: int = 20, device: int = 0, fallback: float = FALLBACK):
    """Mean milliseconds of one exact step and of one surrogate step."""
    import torch
    dev = torch.device("cuda", device)
    b = B.Batch(world, device)
    act = torch.as_tensor(world.actions(1)[0]).to(dev).contiguous()
    st = torch.as_tensor(world.state0).to(dev).contiguous()
    out = {}
    for name, fn in (("exact", lambda s: b.step(s, act)),
                     ("surrogate", lambda s: b.step_surrogate(mlp, s, act, BAND, fallback))):
        s = st.clone()
        for _ in range(3):
            fn(s)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(s)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    b.close()
    return out


def inference_world(n_envs: int = 65536, seed: int = 11):
    """16 sphere agents (r = 0.03) per environment, positions uniform in [-1, 1]^2."""
    return W.uneven(n_envs, lo=16, hi=16, radius=0.03, seed=seed)
