#!/usr/bin/env python3
"""Benchmark of the batched differentiable rope simulation on one MI355X.

Workload (the configuration the headline metric is quoted on): 1024 ropes of
64 nodes, 100 steps, dt = 0.005, stiffness ~ U[300, 800], three random
spheres + ground, gripper controls ~ N(0, 0.05^2).  One timed step is the
whole hot path over that batch:

  1. forward rollout (full trajectory stored)          cord_rollout
  2. adjoint of a terminal cotangent -> s0_bar, u_bar   cord_rollout_backward
  3. dense A_t (384 x 384) and B_t (384 x 3), all t     cord_linearize

value = particle-steps (sum n T) per second of that whole pass.  Inputs are
resident in HBM before timing starts.  Per-kernel durations come from HIP
events recorded on the stream the kernels run on (torch's current stream).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3        # MI355X FP32 vector, published
HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published

# Algorithmic FP32 operations per particle, counted from the kernel source
# ("Algorithmic work"): per conjugate-gradient iteration,
# per Newton iteration (gradient + Hessian data + preconditioner + line
# search), per interior-point iteration (residuals, right-hand side, step
# rule) and per solved step (predictor, contacts, output).
FLOPS_PER_PARTICLE = {
    "rope": {"pcg": 135.0, "newton": 350.0, "ipm": 400.0, "step": 150.0},
    "cloth": {"pcg": 300.0, "newton": 900.0, "ipm": 500.0, "step": 150.0},
}


def workload(B=1024, n=64, T=100):
    import workloads as W
    return W.config_c2(B=B, n=n, T=T)


# ---------------------------------------------------------------- CPU baseline
def _oracle_job(args):
    import numpy as np
    import workloads as W
    from oracle.derivatives import rollout_backward, rollout_linearize
    from oracle.step import rollout
    idx, B, n, T, with_lin = args
    inst = W.config_c2(B=B, n=n, T=T)[idx]
    t0 = time.perf_counter()
    traj, _ = rollout(inst)
    sb = W.random_cotangent(inst.n_s, 5000 + idx)
    rollout_backward(inst, traj, sT_bar=sb)
    if with_lin:
        rollout_linearize(inst, traj)
    return time.perf_counter() - t0, inst.n * inst.T


def cpu_baseline(workers: int, per_worker: int, T: int, with_lin: bool):
    """The FP64 oracle on a bounded sample of the same workload: `workers`
    processes, each running `per_worker` instances (forward, adjoint and
    dense linearization, as in the GPU step) over the first T steps."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(i, 1024, 64, T, with_lin) for i in range(workers * per_worker)]
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_job, jobs))
    wall = time.perf_counter() - t0
    ps = sum(r[1] for r in res)
    return {"value": ps / wall, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(jobs)} of the 1024 ropes (64 nodes), first {T} steps, forward + adjoint"
                      f"{' + dense A/B' if with_lin else ''}, {workers} processes, {wall:.1f} s wall"}


# ---------------------------------------------------------------- GPU
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-linearize", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-workers", type=int, default=8)
    ap.add_argument("--cpu-per-worker", type=int, default=1)
    ap.add_argument("--cpu-T", type=int, default=25)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); instances are independent "
              "and would shard by instance across GPUs, which this build does not launch.", file=sys.stderr)
        sys.exit(2)

    with_lin = not args.no_linearize
    cpu = None
    if not args.no_cpu:
        # before any GPU initialisation: the pool is started from a clean process
        cpu = cpu_baseline(args.cpu_workers, args.cpu_per_worker, args.cpu_T, with_lin)
        print("cpu baseline:", json.dumps(cpu), file=sys.stderr, flush=True)

    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim

    insts = workload()
    B, n, T = len(insts), insts[0].n, insts[0].T
    sim = Sim(insts)
    dev = sim.device
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    sT = sim.pack_states([W.random_cotangent(i.n_s, 7000 + j) for j, i in enumerate(insts)])
    traj = torch.empty(sim.info.traj_floats, dtype=torch.float32, device=dev)
    A = torch.empty(sim.info.A_floats, dtype=torch.float32, device=dev) if with_lin else None
    Bm = torch.empty(sim.info.B_floats, dtype=torch.float32, device=dev) if with_lin else None
    status = torch.zeros(B, dtype=torch.int32, device=dev)
    print(f"workload: {B} ropes x {n} nodes x {T} steps; A {sim.info.A_floats * 4 / 1e9:.1f} GB", file=sys.stderr, flush=True)

    ev = {k: [] for k in ("rollout", "backward", "linearize")}

    def one_step(record):
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record:
            marks[0].record()
        sim.rollout(s0, u, out=traj, status=status)
        if record:
            marks[1].record()
        sim.backward(u, traj, sT_bar=sT)
        if record:
            marks[2].record()
        if with_lin:
            sim.linearize(traj, u, A=A, Bm=Bm)
        if record:
            marks[3].record()
            ev["rollout"].append((marks[0], marks[1]))
            ev["backward"].append((marks[1], marks[2]))
            if with_lin:
                ev["linearize"].append((marks[2], marks[3]))

    for _ in range(args.warmup):
        one_step(False)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    kern_ms = {k: (float(np.mean([a.elapsed_time(b) for a, b in v])) if v else 0.0) for k, v in ev.items()}
    st = status.cpu().numpy()

    # iteration counters of one extra (untimed) pass -> algorithmic FLOPs
    cr = torch.zeros(4 * B, dtype=torch.int32, device=dev)
    cb = torch.zeros(4 * B, dtype=torch.int32, device=dev)
    sim.rollout(s0, u, out=traj, counters=cr)
    sim.backward(u, traj, sT_bar=sT, counters=cb)
    torch.cuda.synchronize()
    fp = FLOPS_PER_PARTICLE["rope"]

    def flops(c):
        c = c.cpu().numpy().reshape(B, 4).astype(np.float64)
        per = c[:, 1] * fp["pcg"] + c[:, 0] * fp["newton"] + c[:, 2] * fp["ipm"] + c[:, 3] * fp["step"]
        return float(np.sum(per * n))

    f_roll, f_bwd = flops(cr), flops(cb)
    particle_steps = B * n * T
    value = particle_steps / (ms / 1e3)
    lin_bytes = 4.0 * (sim.info.A_floats + sim.info.B_floats)
    kernels = {
        "rollout": {"bound": "alu", "achieved": f_roll / (kern_ms["rollout"] / 1e3) / 1e12,
                    "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s"},
        "backward": {"bound": "alu", "achieved": f_bwd / (kern_ms["backward"] / 1e3) / 1e12,
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s"},
    }
    if with_lin:
        kernels["linearize"] = {"bound": "hbm", "achieved": lin_bytes / (kern_ms["linearize"] / 1e3) / 1e9,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    dom = max(kernels, key=lambda k: kern_ms[k])
    roof = dict(kernels[dom])
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["kernel"] = dom
    out = {
        "metric": "particle-steps/s fwd+bwd (rope/cloth batch); MPC plan p50/p99 ms vs plain",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "rope-64 x 1024, T=100, dt=0.005, 3 spheres + ground: forward + adjoint"
                               + (" + dense A_t/B_t" if with_lin else ""),
                   "batch": B, "nodes": n, "horizon": T},
        "kernel_ms": kern_ms,
        "kernel_roofline": {k: dict(v, frac=v["achieved"] / v["peak"]) for k, v in kernels.items()},
        "status_nonzero": int((st != 0).sum()),
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
