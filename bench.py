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
KERNEL_SRC = os.path.join(ROOT, "paper_2207_03530_amd", "csrc", "vmas_kernels.hip")
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


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def algorithmic_bytes(n_envs, agents, landmarks, T):
    N = n_envs * (agents + landmarks)
    A = n_envs * agents
    return (T * A * ACTION_BYTES_PER_AGENT_STEP + N * STATE_READ_PER_ENTITY
            + A * STATE_WRITE_PER_ACTIVE + N * STATIC_PER_ENTITY)


def kernel_of(schedule: str) -> str:
    """Device function that runs a rollout under the given schedule."""
    return "k_rollout_quad" if schedule.startswith("quad") else "k_rollout_sph"


def traffic_per_launch(kernel: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary of `kernel`, if it was taken on the current kernel source; else None."""
    try:
        d = json.load(open(os.path.join(PROFILES, f"{kernel}_spread30k_traffic.json")))
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
    return {"value": w.n_agents_total * T / sec, "unit": "agent-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the full workload ({w.n_envs} envs x {T} steps, FP64) repeated {len(times)} "
                      f"times (about 10 s), median {sec:.3f} s per run, {threads} threads on "
                      f"disjoint environment ranges"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--envs", type=int, default=30000)
    ap.add_argument("--T", type=int, default=100)
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

    T = args.T
    w = W.spread(args.envs)
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
        print(f"calibration copy: {src.numel() * 4} bytes read and written per launch",
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

    nbytes = algorithmic_bytes(w.n_envs, 4, 2, T)
    if args.drawn_actions:
        nbytes -= T * w.n_agents_total * ACTION_BYTES_PER_AGENT_STEP
    achieved = nbytes / (kernel_ms * 1e-3) / 1e9
    kernel = kernel_of(batch.schedule_name(plan))
    traffic = traffic_per_launch(kernel) if not (args.drawn_actions or args.graph) else None
    out = {
        "metric": "agent-steps/s at 30k envs x 4 agents",
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
            "workload": f"spread{w.n_envs}: {w.n_envs} envs x (4 sphere agents + 2 sphere "
                        f"landmarks), one {T}-step rollout per step, actions "
                        + ("drawn in-kernel" if args.drawn_actions else "read from HBM"),
            "n_envs": w.n_envs, "agents_per_env": 4, "landmarks_per_env": 2, "rollout_T": T,
            "dt": w.dt, "drag": w.drag, "schedule": batch.schedule_name(plan),
            "graph": bool(args.graph),
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": kernel, "kernel_ms": kernel_ms,
            "algorithmic_bytes_per_launch": nbytes,
            "algorithmic_bytes_per_env_step": nbytes / (w.n_envs * T),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, acts_np, T)
    print(json.dumps(out), flush=True)
    batch.close()


if __name__ == "__main__":
    main()
