"""Benchmark of the batched 2D physics step on one MI355X.

A bench step is one 100-step rollout (every row of the hot path, every
physics step: staging, per-entity geometry, actions, pair loop with the
narrow phase and Eq. 2 contact forces, joints, Eq. 1/Eq. 3 integration) of
the 30,000-environment workload: 4 sphere agents (r = 0.05, m = 1) and 2
immovable sphere landmarks per environment, positions uniform in [-1, 1]^2,
actions uniform in [-1, 1)^2 per agent per step, dt 0.1, drag 0.25. Inputs
(state and all 100 steps of actions) are resident in HBM before the timed
region; the state carries over from step to step.

Prints one JSON line (rank 0): throughput in agent-steps/s, the roofline
of the dominant kernel measured with HIP events on the launch stream, and
the FP64 CPU oracle timed on the host cores on the same workload.

--workload mixed4096 measures the mixed-shape workload instead: 4,096
environments of 16 sphere agents (r = 0.03), 4 boxes (0.1 x 0.3) and 8
segments (length 0.5), all movable and rotatable, two joints each, one
200-step rollout per bench step; its roofline is the FP32 vector peak.

--workload uneven16384: 16,384 environments of 2..64 sphere agents
(r = 0.05, uniform counts), one 500-step rollout per bench step replayed
from the rollout graph with the actions drawn in the kernel; FP32 vector
roofline by the model count (5 FLOP per pair test, 16 per agent update).

--workload adjoint16384: the same batch, one 50-step rollout adjoint per
bench step (checkpoints every 10 steps: the forward replays and the reverse
steps), actions from HBM, the gradient of sum |x_T|^2 seeded as 2 x_T.

--workload surrogate65536: the learned contact surrogate. The network is
trained on the GPU (its own kernels) on pair samples of exact rollouts, then
the surrogate step and the exact step run from the same states of an exact
trajectory of 65,536 environments x 16 sphere agents (r = 0.03) at three
fallback fractions; the line reports the surrogate's speed relative to the
exact step at the largest fraction whose contact-force error stays within
1e-2 at every step, the network kernel's BF16 matrix-core roofline, and the
same comparison on the mixed 4,096-environment batch (box pairs through
the network, segment pairs exact).
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# sources of the rollout kernels (the traffic summaries name their hash)
KERNEL_SRC = [os.path.join(ROOT, "paper_2207_03530_amd", "csrc", f)
              for f in ("vmas_kernels.hip", "vmas_geom.h", "vmas_internal.h")]
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes of one environment-step / one entity of the spread
# workload (see the roofline section of the design notes):
#   actions 4 agents x 2 x 4 B per step;
#   per rollout: state read 6 x 4 B per entity, state written 6 x 4 B per
#   agent, static parameters (radius, inverse mass, flags) 12 B per entity.
ACTION_BYTES_PER_AGENT_STEP = 8
STATE_READ_PER_ENTITY = 24
STATE_WRITE_PER_ACTIVE = 24
STATIC_PER_ENTITY = 12


# Model FLOP count of one environment-step of the mixed workload (FMA = 2,
# transcendental = 1; every pair tested once): sphere-sphere 120 x 5,
# sphere-segment 128 x 15, sphere-box 64 x 20, segment-segment 28 x 75,
# segment-box 32 x 150, box-box 6 x 200 (11,900), integration 28 x 16 and
# box/segment geometry 12 x 20.
MIXED_FLOP_PER_ENV_STEP = 12600
# Model FLOP count of the uneven sphere workload: 5 per pair test, 16 per
# agent update (a model count for sphere batches).
UNEVEN_FLOP_PER_PAIR = 5
UNEVEN_FLOP_PER_AGENT = 16


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n_envs, agents, landmarks, T):
    N = n_envs * (agents + landmarks)
    A = n_envs * agents
    return (T * A * ACTION_BYTES_PER_AGENT_STEP + N * STATE_READ_PER_ENTITY
            + A * STATE_WRITE_PER_ACTIVE + N * STATIC_PER_ENTITY)


def kernel_of(schedule: str, spheres_only: bool = True) -> str:
    """Device function that runs a rollout under the given schedule."""
    if not spheres_only:
        return "k_rollout"
    if schedule.startswith("quad-ordered"):
        return "k_rollout_quad_ord"
    return "k_rollout_quad" if schedule.startswith("quad") else "k_rollout_sph"


def traffic_per_launch(kernel: str, tag: str = "spread30k", schedule: str = None):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary of `kernel` on workload `tag`, if it was taken on the current
    kernel source and (when given) under the same launch plan; else None."""
    try:
        d = json.load(open(os.path.join(PROFILES, f"{kernel}_{tag}_traffic.json")))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_sha():
        return None
    if schedule is not None and d.get("schedule") != schedule:
        return None
    return d.get("hbm_bytes_per_launch")


CALIBRATION_BYTES = 256 * 1024 * 1024  # the --pmc-calibration copy, read and written


def _counter_dispatches(csv_path):
    """Per dispatch of a rocprofv3 counter collection: kernel name, grid size
    and the sum over instances of every counter."""
    import csv
    out = {}
    for r in csv.DictReader(open(csv_path)):
        d = out.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"],
                                                   "grid": int(r["Grid_Size"]), "c": {}})
        d["c"][r["Counter_Name"]] = d["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def write_traffic_summary(kernel, tag, fetch_csv, write_csv, schedule, workload):
    """profiles/<kernel>_<tag>_traffic.json from the FETCH_SIZE and WRITE_SIZE
    passes of a --pmc-calibration bench run: the kernel's mean per dispatch,
    scaled by what the same counter reads for the 256 MiB copy."""
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        ds = _counter_dispatches(path).values()
        kv = [d["c"][counter] for d in ds
              if f"::{kernel}<" in d["name"] or f"::{kernel}(" in d["name"]]
        copies = [d for d in ds if "copyBuffer" in d["name"]]
        big = max(d["grid"] for d in copies)
        cv = sorted(d["c"][counter] for d in copies if d["grid"] == big)
        if not kv or not cv:
            sys.exit(f"no {kernel} or calibration copy dispatches in {path}")
        per[counter] = (float(np.mean(kv)), cv[len(cv) // 2], len(kv))
    fetch_kib, fetch_copy, n = per["FETCH_SIZE"]
    write_kib, write_copy, _ = per["WRITE_SIZE"]
    fs, ws = CALIBRATION_BYTES / (fetch_copy * 1024), CALIBRATION_BYTES / (write_copy * 1024)
    d = {"kernel": kernel, "schedule": schedule, "workload": workload,
         "kernel_source_sha": kernel_sha(), "dispatches": n,
         "fetch_kib_per_dispatch_raw": fetch_kib, "write_kib_per_dispatch_raw": write_kib,
         "copy_fetch_kib_raw": fetch_copy, "copy_write_kib_raw": write_copy,
         "fetch_scale_from_copy": fs, "write_scale_from_copy": ws,
         "fetch_bytes_per_launch": fetch_kib * 1024 * fs,
         "write_bytes_per_launch": write_kib * 1024 * ws}
    d["hbm_bytes_per_launch"] = d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
    path = os.path.join(PROFILES, f"{kernel}_{tag}_traffic.json")
    with open(path, "w") as f:
        json.dump(d, f, indent=1)
    print(json.dumps(d))


def cpu_baseline(w, acts, T):
    """The FP64 oracle, unchanged, on the same workload, environments split
    over the host cores (one thread per core, contiguous ranges)."""
    from oracle import oracle as O
    threads = min(16, len(os.sched_getaffinity(0)))
    ow = O.OracleWorld(w)
    times = []
    t_start = time.perf_counter()
    while len(times) < 3 or time.perf_counter() - t_start < 10.0:
        t = time.perf_counter()
        O.rollout_threaded(ow, w.state0, acts, threads)
        times.append(time.perf_counter() - t)
    sec = float(np.median(times))
    # the same oracle on one core (at least one full run, then until about 10 s)
    times1 = []
    t_start = time.perf_counter()
    while not times1 or time.perf_counter() - t_start < 10.0:
        t = time.perf_counter()
        O.rollout_threaded(ow, w.state0, acts, 1)
        times1.append(time.perf_counter() - t)
    sec1 = float(np.median(times1))
    return {"value": w.n_agents_total * T / sec, "unit": "agent-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the full workload ({w.n_envs} envs x {T} steps, FP64) repeated {len(times)} "
                      f"times (about 10 s), median {sec:.3f} s per run, {threads} threads on "
                      f"disjoint environment ranges",
            "single_core": {"value": w.n_agents_total * T / sec1, "cores": 1,
                            "sample": f"the same workload on one thread, {len(times1)} run(s), "
                                      f"median {sec1:.3f} s"}}


MLP_FLOP_PER_ROW = 2 * (12 * 128 + 128 * 128 + 128 * 2)  # the three products of one row
BF16_PEAK_TFLOPS = 2500.0


def surrogate_bench(args):
    """The surrogate workload (see the module docstring): one JSON line."""
    import torch
    from paper_2207_03530_amd import binding as B, surrogate as S, workloads as W
    t = time.perf_counter()
    X, Y = S.training_set([
        S.make_dataset(W.mixed(16384, seed=21), T=600, stride=1, max_samples=6_000_000),
        S.make_dataset(W.uneven(65536, lo=16, hi=16, radius=0.03, seed=22), T=300, stride=1,
                       max_samples=4_000_000)])
    t_data = time.perf_counter() - t
    net = B.Mlp(seed=0)
    t = time.perf_counter()
    hist = S.train(net, X, Y, epochs=300, batch=8192, lr=3e-3, lr_final=1e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t
    print(f"surrogate: {X.shape[0]} samples in {t_data:.1f} s, trained in {t_train:.1f} s, "
          f"loss {hist[0]:.4g} -> {hist[-1]:.4g}", file=sys.stderr, flush=True)
    reps = max(5, args.steps)
    results = {}
    for name, w in (("spheres65536x16", S.inference_world(65536)), ("mixed4096", W.mixed(4096))):
        rows = []
        for frac in (0.5, 0.25, 0.1):
            errs, fbs = S.contact_force_error(w, net, steps=5, fallback=frac)
            times = S.time_steps(w, net, reps=reps, fallback=frac)
            rows.append({"fallback_frac": frac, "max_rel_force_err": float(np.max(errs)),
                         "rel_force_err_per_step": [round(float(e), 5) for e in errs],
                         "exact_ms": times["exact"], "surrogate_ms": times["surrogate"],
                         "speed_vs_exact": times["exact"] / times["surrogate"]})
            print(f"{name} fallback {frac}: err {np.round(errs, 4)}, exact {times['exact']:.4f} ms, "
                  f"surrogate {times['surrogate']:.4f} ms", file=sys.stderr, flush=True)
        results[name] = rows
    # the network kernel alone on as many rows as the sphere batch has candidates
    w = S.inference_world(65536)
    b = B.Batch(w, 0)
    st = torch.as_tensor(w.state0).cuda().contiguous()
    fl = torch.zeros(b.P, dtype=torch.uint8, device="cuda:0")
    fb = torch.zeros(b.P, 12, device="cuda:0")
    b.pair_features(st, fb, fl, band=S.BAND)
    n_cand = int((fl & 1).sum())
    b.close()
    n_rows = max(n_cand, 1 << 20)
    Xr = X[:n_rows].contiguous() if X.shape[0] >= n_rows else X.repeat(n_rows // X.shape[0] + 1, 1)[:n_rows].contiguous()
    Yr = torch.zeros(n_rows, 2, device="cuda:0")
    for _ in range(3):
        net.forward(Xr, Yr)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        net.forward(Xr, Yr)
    e1.record()
    torch.cuda.synchronize()
    mlp_ms = e0.elapsed_time(e1) / reps
    achieved = MLP_FLOP_PER_ROW * n_rows / (mlp_ms * 1e-3) / 1e12
    sph = results["spheres65536x16"]
    within = [r for r in sph if r["max_rel_force_err"] <= 1e-2]
    best = within[0] if within else None
    out = {
        "metric": "surrogate step speed relative to the exact step at <= 1e-2 relative "
                  "contact-force error (65,536 envs x 16 sphere agents)",
        "value": best["speed_vs_exact"] if best else None,
        "unit": "x exact step",
        "n_gpus": 1, "steps": reps, "warmup": 3,
        "ms_per_step": best["surrogate_ms"] if best else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 (network) / f32 (step)", "data": "synthetic",
        "config": {"workload": "surrogate65536: 12-128-128-2 MLP trained on the GPU on exact "
                               "pair samples, surrogate step vs exact step from the same states",
                   "n_envs": 65536, "agents_per_env": 16, "fallback_frac":
                       best["fallback_frac"] if best else None,
                   "training_samples": int(X.shape[0]), "training_s": round(t_train, 1)},
        "surrogate": results,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_mlp_infer", "kernel_ms": mlp_ms, "rows": n_rows,
                     "algorithmic_flop_per_row": MLP_FLOP_PER_ROW,
                     "candidate_rows_per_step": n_cand},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", choices=("spread30000", "mixed4096", "uneven16384", "adjoint16384",
                                           "surrogate65536"), default="spread30000")
    ap.add_argument("--envs", type=int, default=None,
                    help="environments (default 30000 spread, 4096 mixed)")
    ap.add_argument("--T", type=int, default=None, help="rollout length (default 100 spread, 200 mixed)")
    ap.add_argument("--graph", action="store_true", help="replay a captured hipGraph")
    ap.add_argument("--schedule", default=None,
                    help="run this launch plan (vmas_schedule_name) instead of autotuning")
    ap.add_argument("--drawn-actions", action="store_true",
                    help="draw the actions in the kernel instead of reading them from HBM")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="also run a plain copy of known size (traffic counter calibration)")
    ap.add_argument("--traffic-summary", nargs=6,
                    metavar=("KERNEL", "TAG", "FETCH_CSV", "WRITE_CSV", "SCHEDULE", "WORKLOAD"),
                    help="write the traffic summary of KERNEL from two rocprofv3 counter "
                         "collections (FETCH_SIZE, WRITE_SIZE) of a --pmc-calibration run")
    args = ap.parse_args()
    if args.traffic_summary:
        return write_traffic_summary(*args.traffic_summary)
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1); "
              "environments are independent and shard by environment range",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_03530_amd import binding, workloads as W

    if args.workload == "surrogate65536":
        return surrogate_bench(args)
    mixed = args.workload == "mixed4096"
    uneven = args.workload in ("uneven16384", "adjoint16384")
    adjoint = args.workload == "adjoint16384"
    if uneven:
        T = args.T or (50 if adjoint else 500)
        w = W.uneven(args.envs or 16384, lo=2, hi=64, seed=0)
        if not adjoint:
            args.graph = True
            args.drawn_actions = True
    else:
        T = args.T or (200 if mixed else 100)
        w = W.mixed(args.envs or 4096) if mixed else W.spread(args.envs or 30000)
    acts_np = w.actions(T)
    dev = torch.device("cuda", 0)
    batch = binding.vmas_create_batch(w, 0)
    state = torch.as_tensor(w.state0).to(dev).contiguous()
    acts = torch.as_tensor(acts_np).to(dev).contiguous()
    if args.schedule:
        names = [batch.schedule_name(q) for q in range(batch.n_schedules)]
        if args.schedule not in names:
            sys.exit(f"unknown schedule {args.schedule!r}; valid: {[n for n in names if n]}")
        plan = names.index(args.schedule)
        batch.set_schedule(plan)
    else:
        plan = batch.autotune(state, T, None if args.drawn_actions else acts)
    stream = torch.cuda.current_stream(dev)

    if args.pmc_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)  # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(10):
            dst.copy_(src)
        c1.record(stream)
        torch.cuda.synchronize()
        sec = c0.elapsed_time(c1) * 1e-3 / 10
        print(f"calibration copy: {src.numel() * 4} bytes read and written per launch, "
              f"{2 * src.numel() * 4 / sec / 1e9:.0f} GB/s (read + write)",
              file=sys.stderr, flush=True)

    # one step = one T-step rollout of the whole batch (for adjoint16384 one
    # rollout adjoint); arguments marshalled once
    if adjoint:
        s0 = state.clone()
        gT = torch.zeros_like(state)
        gs = torch.zeros_like(state)
        ga = torch.zeros_like(acts)

        def one_step():
            batch.rollout_backward(s0, acts, gT, 10, gs, ga)
    elif args.drawn_actions:
        one_step = batch.prepare_rollout(state, None, T=T, seed=w.seed, graph=args.graph)
    else:
        one_step = batch.prepare_rollout(state, acts, graph=args.graph)

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    # HIP events on the launch stream bracket the whole timed region: the
    # kernel's average launch duration is their interval over the K launches,
    # which run back to back (the host enqueues faster than the GPU drains)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        one_step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = e0.elapsed_time(e1) / args.steps
    ms_per_step = wall * 1e3 / args.steps
    agent_steps = w.n_agents_total * T
    value = agent_steps / (ms_per_step * 1e-3)

    kernel = kernel_of(batch.schedule_name(plan), not mixed)
    if adjoint:
        kernel = "k_step_backward"
    tag = "mixed4096" if mixed else ("uneven16384" if uneven else "spread30k")
    default_size = w.n_envs == (4096 if mixed else 30000) and T == (200 if mixed else 100)
    traffic = (traffic_per_launch(kernel, tag, batch.schedule_name(plan))
               if not (args.drawn_actions or args.graph) and default_size else None)
    if uneven:
        n = np.diff(w.env_offset).astype(np.int64)
        pairs = int((n * (n - 1) // 2).sum())
        # model count per step: 5 FLOP per pair test, 16 per agent update;
        # the adjoint counts its forward replays (one per step) and its
        # reverse step at twice the forward work (value and three tangents
        # on the contacting pairs only, the reverse of the update)
        flop_step = UNEVEN_FLOP_PER_PAIR * pairs + UNEVEN_FLOP_PER_AGENT * w.n_agents_total
        flop = flop_step * T * (3 if adjoint else 1)
        achieved = flop / (kernel_ms * 1e-3) / 1e12
        roofline = {
            "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": None,
            "kernel": kernel, "kernel_ms": kernel_ms, "algorithmic_flop_per_launch": flop,
            "algorithmic_flop_per_env_step": flop / (w.n_envs * T),
        }
        if adjoint:
            workload = (f"adjoint{w.n_envs}: {w.n_envs} envs x 2..64 sphere agents, backward of "
                        f"sum |x_T|^2 through a {T}-step rollout, checkpoints every 10 steps")
            metric = f"agent-steps/s of the {T}-step rollout adjoint at {w.n_envs} uneven envs"
        else:
            workload = (f"uneven{w.n_envs}: {w.n_envs} envs x 2..64 sphere agents, one {T}-step "
                        f"rollout per step replayed from the rollout graph, actions drawn in-kernel")
            metric = f"agent-steps/s at {w.n_envs} uneven envs (2..64 agents)"
        shape = {"n_envs": w.n_envs, "agents_per_env": "2..64 (uniform)",
                 "pair_slots": pairs}
    elif mixed:
        flop = MIXED_FLOP_PER_ENV_STEP * w.n_envs * T
        achieved = flop / (kernel_ms * 1e-3) / 1e12
        roofline = {
            "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
            "kernel": kernel, "kernel_ms": kernel_ms,
            "algorithmic_flop_per_launch": flop,
            "algorithmic_flop_per_env_step": MIXED_FLOP_PER_ENV_STEP,
        }
        workload = (f"mixed{w.n_envs}: {w.n_envs} envs x (16 sphere agents + 4 boxes + 8 segments, "
                    f"2 joints), one {T}-step rollout per step, actions "
                    + ("drawn in-kernel" if args.drawn_actions else "read from HBM"))
        metric = f"agent-steps/s at {w.n_envs} envs x (16 spheres + 4 boxes + 8 segments)"
        shape = {"n_envs": w.n_envs, "agents_per_env": 16, "boxes_per_env": 4,
                 "segments_per_env": 8, "joints_per_env": 2}
    else:
        nbytes = algorithmic_bytes(w.n_envs, 4, 2, T)
        if args.drawn_actions:
            nbytes -= T * w.n_agents_total * ACTION_BYTES_PER_AGENT_STEP
        achieved = nbytes / (kernel_ms * 1e-3) / 1e9
        roofline = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": kernel, "kernel_ms": kernel_ms,
            "algorithmic_bytes_per_launch": nbytes,
            "algorithmic_bytes_per_env_step": nbytes / (w.n_envs * T),
        }
        workload = (f"spread{w.n_envs}: {w.n_envs} envs x (4 sphere agents + 2 sphere "
                    f"landmarks), one {T}-step rollout per step, actions "
                    + ("drawn in-kernel" if args.drawn_actions else "read from HBM"))
        metric = "agent-steps/s at 30k envs x 4 agents"
        shape = {"n_envs": w.n_envs, "agents_per_env": 4, "landmarks_per_env": 2}
    out = {
        "metric": metric,
        "value": value,
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload, **shape, "rollout_T": T,
            "dt": w.dt, "drag": w.drag, "schedule": batch.schedule_name(plan),
            "graph": bool(args.graph),
        },
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, acts_np, T)
    print(json.dumps(out), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
