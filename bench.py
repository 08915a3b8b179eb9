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
    return "k_rollout_quad" if schedule.startswith("quad") else "k_rollout_sph"


def traffic_per_launch(kernel: str, tag: str = "spread30k"):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary of `kernel` on workload `tag`, if it was taken on the current
    kernel source; else None."""
    try:
        d = json.load(open(os.path.join(PROFILES, f"{kernel}_{tag}_traffic.json")))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_sha():
        return None
    return d.get("hbm_bytes_per_launch")


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", choices=("spread30000", "mixed4096"), default="spread30000")
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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build runs a single MI355X (--gpus 1); "
              "environments are independent, see the sharding notes in DESIGN.md",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2207_03530_amd import binding, workloads as W

    mixed = args.workload == "mixed4096"
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

    # one step = one T-step rollout of the whole batch; arguments marshalled once
    if args.drawn_actions:
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
    tag = "mixed4096" if mixed else "spread30k"
    default_size = w.n_envs == (4096 if mixed else 30000) and T == (200 if mixed else 100)
    traffic = (traffic_per_launch(kernel, tag)
               if not (args.drawn_actions or args.graph) and default_size else None)
    if mixed:
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
