#!/usr/bin/env python3
"""Benchmark of the batched differentiable rope simulation on one MI355X.

Workload (the configuration the headline metric is quoted on): 1024 ropes of
64 nodes, 100 steps, dt = 0.005, stiffness ~ U[300, 800], three random
spheres + ground, gripper controls ~ N(0, 0.05^2).  One timed step is the
whole hot path over that batch:

  1. forward rollout (full trajectory stored)          cord_rollout
  2. adjoint of a terminal cotangent -> s0_bar, u_bar   cord_rollout_backward
  3. dense A_t (384 x 384) and B_t (384 x 3), all t     cord_linearize

Steps 2 and 3 read only the rollout's output; by default they run one after
the other on one stream (--overlap runs them concurrently on two streams).
value = particle-steps (sum n T) per second of that whole pass.  Inputs are
resident in HBM before timing starts.  Per-kernel durations come from HIP
events recorded on the stream each kernel runs on.

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

# Algorithmic FP32 operations per particle, counted from the kernel source:
# per conjugate-gradient iteration,
# per Newton iteration (gradient + Hessian data + preconditioner + line
# search), per interior-point iteration (residuals, right-hand side, step
# rule) and per solved step (predictor, contacts, output).  Ropes with one
# particle per lane apply and build the pair-block preconditioner: 18 more
# per iteration, about 250 more per build (Newton and interior point).
FLOPS_PER_PARTICLE = {
    "rope": {"pcg": 153.0, "newton": 600.0, "ipm": 650.0, "step": 150.0},
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


def _one_thread():
    # one BLAS / OpenMP thread per worker process, so that `cores` is the
    # number of threads the baseline used (set before numpy is imported);
    # the oracle and its libraries are imported before the clock starts
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    import numpy  # noqa: F401
    import scipy.sparse.linalg  # noqa: F401
    import oracle.derivatives  # noqa: F401
    import workloads  # noqa: F401


def _ready(_):
    return os.getpid()


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_cores():
    """Host cores this process may use, at most 16 (the machine's CPU share for one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(workers: int, sample: int, T: int, with_lin: bool):
    """The FP64 oracle on a bounded sample of the same workload: `sample`
    seeded instances of the rope batch (forward, adjoint and dense
    linearization, as in the GPU step, over the first T steps) spread over
    `workers` single-threaded processes, timed once the processes are up;
    then one instance alone (the single-thread figure)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(i, 1024, 64, T, with_lin) for i in range(sample)]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"),
                                initializer=_one_thread) as ex:
        list(ex.map(_ready, range(4 * workers)))          # every worker started and imported
        t0 = time.perf_counter()
        res = list(ex.map(_oracle_job, jobs))
        wall = time.perf_counter() - t0
        t1 = time.perf_counter()
        one = ex.submit(_oracle_job, jobs[0]).result()
        wall1 = time.perf_counter() - t1
    ps = sum(r[1] for r in res)
    what = f"forward + adjoint{' + dense A/B' if with_lin else ''} over {T} of 100 steps"
    return {"value": ps / wall, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(jobs)} of the 1024 ropes (64 nodes), {what}, {workers} single-threaded processes, "
                      f"{wall:.1f} s wall after start-up",
            "cpu_model": _cpu_model(),
            "single_thread": {"value": one[1] / wall1, "unit": "particle-steps/s",
                              "sample": f"rope 0 alone, {what}, {wall1:.1f} s"}}


# ---------------------------------------------------------------- other workloads
def _time(fn, warmup, steps):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def bench_c3(args):
    """256 cloths 32x32, T = 60: forward with checkpoints every 10 steps,
    checkpointed adjoint, and 6 JVP tangents per step (the B_t columns)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim, _lib as L
    insts = W.config_c3()
    sim = Sim(insts)
    if not args.no_aux:
        sim.use_aux(True)      # the full rollout keeps its step internals for the JVPs
    B, n, T = len(insts), insts[0].n, insts[0].T
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    sT = sim.pack_states([W.random_cotangent(i.n_s, 8000 + j) for j, i in enumerate(insts)])
    k = 6
    du = np.zeros((B, T, k, 6), np.float32)
    du[:, :, np.arange(6), np.arange(6)] = 1.0
    dut = torch.from_numpy(du.ravel()).to(sim.device)
    ck = torch.empty(sim.ckpt_floats(10), dtype=torch.float32, device=sim.device)
    full = torch.empty(sim.info.traj_floats, dtype=torch.float32, device=sim.device)
    ms = {}

    def step():
        e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        e[0].record()
        sim.rollout(s0, u, store=L.STORE_CKPT, ckpt_every=10, out=ck)
        e[1].record()
        sim.backward(u, ck, sT_bar=sT, store=L.STORE_CKPT, ckpt_every=10)
        e[2].record()
        sim.rollout(s0, u, out=full)
        e[3].record()
        sim.linearize(full, u, dense=False, want_B=False, jvp_k=k, jvp_du=dut)
        e[4].record()
        step.ev.append(e)
    step.ev = []
    tms = _time(step, args.warmup, args.steps)
    ev = step.ev[args.warmup:]
    names = ["rollout_ckpt", "backward_ckpt", "rollout_full", "jvp6"]
    for j, nm in enumerate(names):
        ms[nm] = float(np.mean([x[j].elapsed_time(x[j + 1]) for x in ev]))
    ps = B * n * T
    return {"workload": "cloth-32x32 x 256, T=60: forward (ckpt 10) + checkpointed adjoint + 6 JVP tangents/step",
            "steps": args.steps, "ms_per_step": tms, "particle_steps_per_s": ps / (tms / 1e3), "kernel_ms": ms,
            "fwd_bwd_particle_steps_per_s": ps / ((ms["rollout_ckpt"] + ms["backward_ckpt"]) / 1e3)}


def bench_c4(args):
    """4096 mixed ropes (16..256 nodes) and cloths (8x8..48x48), T 30..120,
    forward + adjoint, as one hipGraph of persistent per-class launches,
    persistent, grouped, and one launch per instance (the plain launch)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim, _lib as L
    insts = W.config_c4()
    sim = Sim(insts)
    if not args.no_aux:
        sim.use_aux(True)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    sT = sim.pack_states([W.random_cotangent(i.n_s, 9000 + j) for j, i in enumerate(insts)])
    traj = torch.empty(sim.info.traj_floats, dtype=torch.float32, device=sim.device)
    ps = sum(i.n * i.T for i in insts)
    out = {"workload": "C4 mixed: 4096 instances (ropes 16..256, cloths 8x8..48x48), T 30..120, forward + adjoint",
           "particle_steps": ps}
    if args.autotune:
        out["tuned"] = sim.autotune(s0, u, sample=64)
    out["classes"] = sim.classes()
    for name, mode in (("graph", L.LAUNCH_GRAPH), ("persistent", L.LAUNCH_PERSISTENT),
                       ("grouped", L.LAUNCH_GROUPED), ("per_instance", L.LAUNCH_PER_INSTANCE)):
        sim.set_launch(mode)

        def step():
            sim.rollout(s0, u, out=traj)
            sim.backward(u, traj, sT_bar=sT)
        if mode == L.LAUNCH_PER_INSTANCE:
            # one launch per instance, one instance after another: timed on
            # every 8th instance and scaled by particle-steps
            sub = insts[::8]
            ss = Sim(sub)
            ss.set_launch(mode)
            s0s = ss.pack_states([i.s0 for i in sub])
            us = ss.pack_controls([i.u for i in sub])
            sTs = ss.pack_states([W.random_cotangent(i.n_s, 9000 + 8 * j) for j, i in enumerate(sub)])
            trs = torch.empty(ss.info.traj_floats, dtype=torch.float32, device=ss.device)

            def sub_step():
                ss.rollout(s0s, us, out=trs)
                ss.backward(us, trs, sT_bar=sTs)
            pss = sum(i.n * i.T for i in sub)
            tsub = _time(sub_step, 0, 1)
            out[name] = {"ms_per_step": tsub * ps / pss, "particle_steps_per_s": pss / (tsub / 1e3),
                         "sample": f"every 8th instance ({len(sub)}), {tsub:.0f} ms, scaled by particle-steps"}
            print(name, out[name], file=sys.stderr, flush=True)
            continue
        tms = _time(step, 1, max(1, args.steps // 2))
        out[name] = {"ms_per_step": tms, "particle_steps_per_s": ps / (tms / 1e3)}
        print(name, out[name], file=sys.stderr, flush=True)
    out["graph_vs_per_instance"] = out["per_instance"]["ms_per_step"] / out["graph"]["ms_per_step"]
    return out


def sls_tri_flops(N, n, ra_list):
    """Algorithmic FLOPs of the assembly products C = A B with A block-lower
    (row blocks of ra, column blocks of n) and B block-lower (n x n blocks):
    output block (i, j), j <= i, sums i - j + 1 products of ra x n by n x n,
    so 2 ra n^2 sum_i (i+1)(i+2)/2 per product."""
    s = sum((i + 1) * (i + 2) // 2 for i in range(N + 1))
    return float(sum(2.0 * ra * n * n * s for ra in ra_list))


def bench_sls(args):
    """Output-feedback SLS stage 3 on the A_t of 64 ropes of 13 nodes
    (n_s = 78, the paper's output-feedback rope has 13 nodes) over N = 40
    steps, C = I, E = r_CP I, F = rho I: the Kalman recursion serially and as
    the associative scan (batch 64 and batch 1), the observer responses, the
    state-feedback stand-in, the block-triangular assembly and the tubes."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim
    from paper_2606_14188_amd.sls import SCAN, SERIAL, SLS
    B, nodes, N = 64, 13, 40
    insts = W.small_rope_batch(B, nodes, N, seed=1019)
    sim = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    traj = sim.rollout(s0, u)
    A, Bm, _ = sim.linearize(traj, u)
    ns, m = insts[0].n_s, insts[0].n_u
    A = A.reshape(B, N, ns, ns)
    Bm = Bm.reshape(B, N, ns, m)
    del sim, traj
    eye = torch.eye(ns, device=A.device)
    r_cp, rho = 1e-3, 2e-3
    E = (r_cp * eye).expand(B, N, ns, ns).contiguous()
    F = (rho * eye).expand(B, N, ns, ns).contiguous()
    Xi = (rho * eye).expand(B, ns, ns).contiguous()
    K = torch.from_numpy(W.sls_system(B, N, ns, m, seed=1020)["K"]).to(A.device)
    h = SLS(B, N, ns, m)
    h1 = SLS(1, N, ns, m)
    reps = max(3, args.steps)
    out = {"workload": f"SLS stage 3 on rope-{nodes} A_t (n_s={ns}, n_u={m}) x {B}, N={N}, C=I",
           "B": B, "N": N, "n": ns, "m": m}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            res = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), res

    ms = {}
    ms["kalman_serial_b64"], _ = timed(lambda: h.kalman(A, E, F, Xi, mode=SERIAL))
    ms["kalman_scan_b64"], (Pi, Lg, st) = timed(lambda: h.kalman(A, E, F, Xi, mode=SCAN))
    A1, E1, F1, X1 = A[:1].contiguous(), E[:1].contiguous(), F[:1].contiguous(), Xi[:1].contiguous()
    ms["kalman_serial_b1"], _ = timed(lambda: h1.kalman(A1, E1, F1, X1, mode=SERIAL))
    ms["kalman_scan_b1"], _ = timed(lambda: h1.kalman(A1, E1, F1, X1, mode=SCAN))
    ms["observer"], (Phx, Phy) = timed(lambda: h.observer(A, Lg))
    ms["state_feedback"], (Pbx, Pbu) = timed(lambda: h.state_feedback(A, Bm, K))
    ms["assemble"], (xw, uw, xe, ue) = timed(lambda: h.assemble(A, Pbx, Pbu, Phx, Phy))
    ms["tubes"], (tx, tu) = timed(lambda: h.tubes(xw, xe, E, F, uw, ue))
    out["ms"] = ms
    out["status_nonzero"] = int((st.cpu().numpy() != 0).sum())
    out["tau_x_final_max"] = float(tx[:, -1].max())
    f = B * sls_tri_flops(N, ns, [ns, ns, m, m])
    achieved = f / (ms["assemble"] / 1e3) / 1e12
    out["assemble_roofline"] = {"bound": "mfma", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                                "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS, "flops": f}
    return out


def bench_next(args):
    """The widened rows: friction (the C2 batch of 1024 ropes x 64 nodes x
    100 steps, forward + adjoint, frictionless and with mu = 0.5 on every
    contact; dense A_t/B_t of 64 of them with friction, by the row-by-row
    kernel), analytical policy gradients (one training iteration of the
    lift task: 64 environments x 20 steps, forward and backward through
    the simulator and the policy), and the conformal radius (scores of
    10 000 calibration transitions and the order statistic)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim, cp_radius
    from paper_2606_14188_amd.apg import MLPPolicy, lift_loss, policy_rollout, sim_step
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    reps = max(3, args.steps)
    # friction at the C2 size
    base = workload()
    B, n, T = len(base), base[0].n, base[0].T
    fr = {}
    for label, insts in (("frictionless", base), ("mu_0.5", [i.replace(mu=0.5) for i in base])):
        sim = Sim(insts)
        s0 = sim.pack_states([i.s0 for i in insts])
        u = sim.pack_controls([i.u for i in insts])
        traj = torch.empty(sim.info.traj_floats, dtype=torch.float32, device=sim.device)
        sT = sim.pack_states([W.random_cotangent(i.n_s, 7000 + j) for j, i in enumerate(insts)])
        st = torch.zeros(B, dtype=torch.int32, device=sim.device)
        ms_f = timed(lambda: sim.rollout(s0, u, out=traj, status=st), reps)
        ms_b = timed(lambda: sim.backward(u, traj, sT_bar=sT), reps)
        fr[label] = {"rollout_ms": ms_f, "backward_ms": ms_b,
                     "particle_steps_per_s": B * n * T / ((ms_f + ms_b) / 1e3),
                     "status_nonzero": int((st.cpu().numpy() != 0).sum())}
        del sim, traj
        torch.cuda.empty_cache()
    sub = [i.replace(mu=0.5) for i in base[:64]]
    sim = Sim(sub)
    s0 = sim.pack_states([i.s0 for i in sub])
    u = sim.pack_controls([i.u for i in sub])
    traj = sim.rollout(s0, u)
    A = torch.empty(sim.info.A_floats, dtype=torch.float32, device=sim.device)
    Bm = torch.empty(sim.info.B_floats, dtype=torch.float32, device=sim.device)
    fr["mu_0.5_linearize_64_ms"] = timed(lambda: sim.linearize(traj, u, A=A, Bm=Bm), reps)
    del sim, traj, A, Bm
    torch.cuda.empty_cache()
    out["friction"] = {"workload": f"rope-{n} x {B}, T={T}: forward + adjoint; A_t/B_t of 64 with friction", **fr}
    # analytical policy gradients
    torch.manual_seed(5)
    envs = W.lift_rope_envs(64, n=12, seed=1011)
    sim = Sim(envs)
    policy = MLPPolicy(u_max=0.5).to(sim.device)
    s0 = sim.pack_states([i.s0 for i in envs]).reshape(len(envs), -1)
    step = sim_step(sim)
    Tl = 20

    def it():
        policy.zero_grad()
        sT, us = policy_rollout(step, policy, s0, 12, Tl)
        lift_loss(sT, us, 12, 0.02).backward()

    ms_it = timed(it, reps)
    out["apg"] = {"workload": "lift task: 64 environments x 20 steps, rope-12 with penalty grippers, "
                              "hard forward / smoothed gradient", "ms_per_iteration": ms_it,
                  "env_steps_per_s": 64 * Tl / (ms_it / 1e3)}
    del sim
    # conformal radius
    cal = W.calibration_set(10000, seed=1030)
    insts = [c[0] for c in cal]
    sim = Sim(insts)
    s0 = sim.pack_states([i.s0 for i in insts])
    u = sim.pack_controls([i.u for i in insts])
    s_next = sim.pack_states([np.concatenate([c[1].ravel(), np.zeros(3 * c[0].n)]) for c in cal])
    ms_s = timed(lambda: sim.cp_scores(s0, u, s_next), reps)
    sc = sim.cp_scores(s0, u, s_next)
    ms_r = timed(lambda: cp_radius(sc, 0.05, 40), reps)
    out["conformal"] = {"workload": "10000 calibration transitions of an 11-node rope", "scores_ms": ms_s,
                        "radius_ms": ms_r, "radius_m": float(cp_radius(sc, 0.05, 40)[0])}
    return out


HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE = os.path.join(HERE, "profiles", "rollout_backward_linearize__rope64x1024_T100.md")
LIN_SOURCES = ["cord_lin_direct.h", "cord_solver.h", "cord_lin_rope.hip"]


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None if there is none for it or the
    kernel's sources have changed since the counters were taken."""
    import hashlib
    import re
    if kernel != "linearize" or not os.path.exists(PROFILE):
        return None
    m = re.search(r"traffic: kernel=linearize bytes_per_launch=(\d+) sources_sha1=([0-9a-f]{40})",
                  open(PROFILE).read())
    if not m:
        return None
    h = hashlib.sha1()
    for f in LIN_SOURCES:
        with open(os.path.join(HERE, "paper_2606_14188_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m.group(1)) if h.hexdigest() == m.group(2) else None


def copy_calibration():
    """Plain device copy of 256 MiB, three times: the reference dispatch that
    scales the FETCH_SIZE / WRITE_SIZE counters of a profile to bytes."""
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy calibration", "bytes_per_copy": n * 4, "copies": 3}), flush=True)


def bench_probe(args):
    """Context probe at batch 1: one step of a 20-node rope and of a 10x10
    cloth, forward alone and the dense step Jacobian (A_t, B_t), each the
    median of repeated launches.  The paper's simulator-speed table quotes
    the same shapes on unstated hardware; it is context, not a target."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim
    rope = W.config_c1().replace(T=1)
    rope = rope.replace(u=rope.u[:1])
    cloth = W.small_cloth_batch(1, 10, 10, 1, seed=1006)[0]
    out = {"workload": "batch-1 probe: one step of a 20-node rope and of a 10x10 cloth (forward; dense A_t/B_t)",
           "paper_context_ms": {"rope": {"forward": 1.095, "jacobian": 5.198},
                                "cloth": {"forward": 15.08, "jacobian": 10.06},
                                "note": "paper's table, hardware not stated; forward may be a rollout"}}
    for name, inst in (("rope", rope), ("cloth", cloth)):
        sim = Sim([inst])
        s0 = sim.pack_states([inst.s0])
        u = sim.pack_controls([inst.u])
        traj = sim.rollout(s0, u)
        A, Bm, _ = sim.linearize(traj, u)
        times = {"forward": [], "jacobian": []}
        for _ in range(max(20, args.steps)):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            sim.rollout(s0, u, out=traj)
            e[1].record()
            sim.linearize(traj, u, A=A, Bm=Bm)
            e[2].record()
            torch.cuda.synchronize()
            times["forward"].append(e[0].elapsed_time(e[1]))
            times["jacobian"].append(e[1].elapsed_time(e[2]))
        out[name] = {k: float(np.median(v)) for k, v in times.items()}
        out[name]["n"] = inst.n
    print(json.dumps(out), flush=True)


def _serve_once(trace, slots, discard=0.0):
    """Replay a request trace against one server; latencies are measured from
    each request's scheduled arrival (so a slow submit counts against the
    server) to the moment its result is ready.  Requests that arrive in the
    first `discard` seconds are served but left out of the latency figures."""
    import threading
    import numpy as np
    from paper_2606_14188_amd.serve import Server
    srv = Server(hbm_budget=64 << 30, max_slots=slots, queue_cap=1 << 20)
    tickets, late = [], []

    def submitter():
        t0 = time.perf_counter()
        for (ta, inst, gn, goal) in trace:
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            late.append(max(0.0, time.perf_counter() - t0 - ta))
            tickets.append(srv.submit(inst, goal_node=gn, goal=goal, n_cand=128, iters=10, step=0.05,
                                      sigma=0.05, seed=len(tickets), want_AB=(inst.kind == "rope"), u_warm=inst.u))
    t_start = time.perf_counter()
    th = threading.Thread(target=submitter)
    th.start()
    th.join()
    lat, fails = [], 0
    for (ta, *_), t, lt in zip(trace, tickets, late):
        r = srv.wait(t, 600000)
        if ta >= discard:
            lat.append(lt + r.latency)
        fails += int(r.status != 0 or r.sim_status != 0)
        srv.release(t)
    wall = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    lat = np.array(lat) * 1e3
    return {"slots": slots, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "measured_requests": int(len(lat)),
            "throughput_req_s": len(trace) / wall, "wall_s": wall, "drain_s": wall - trace[-1][0],
            "peak_queue": st["peak_queue"], "failed_or_flagged": fails}


def bench_c5(args, quiet=False):
    """Served planning stream: each request plans 128 candidates x T=30 x 10
    gradient steps on a rope (48..128 nodes, plus A_t/B_t along the winner)
    or a cloth (16x16..32x32).  Continuous batching (8 slots) against one
    request at a time on the same inputs:
      capacity  a burst of requests all arriving at once, drained by each
                server: requests per second each sustains; the offered
                200 req/s divided by it is the utilisation rho;
      stable    Poisson arrivals at 80 % of the batched capacity for
                `serve_seconds` (first 2 s discarded): p50 / p99 latency of
                both servers (one at a time is unstable at that rate if its
                capacity is lower, and then says so)."""
    import workloads as W
    out = {"workload": "planning stream: 128 candidates x T=30 x 10 gradient steps, "
                       "ropes 48..128 (+A_t/B_t) / cloths 16x16..32x32"}
    burst = [(0.0, inst, gn, goal) for (_, inst, gn, goal) in W.serve_trace(200.0, 0.4, seed=1015)]
    cap = {}
    for name, slots in (("batched", args.slots), ("plain", 1)):
        r = _serve_once(burst, slots)
        cap[name] = r["throughput_req_s"]
        if not quiet:
            print("capacity", name, r, file=sys.stderr, flush=True)
    out["capacity"] = {"requests": len(burst), "batched_req_s": cap["batched"], "plain_req_s": cap["plain"],
                       "rho_at_200_req_s": {"batched": 200.0 / cap["batched"], "plain": 200.0 / cap["plain"]},
                       "offered_load_note": "rho > 1: the 200 req/s stream exceeds what one GPU serves; "
                                            "its queue grows without bound"}
    rate = 0.8 * cap["batched"]
    trace = W.serve_trace(rate, args.serve_seconds)
    res = {"offered_req_s": rate, "duration_s": args.serve_seconds, "requests": len(trace), "discarded_s": 2.0}
    for name, slots in (("batched", args.slots), ("plain", 1)):
        res[name] = _serve_once(trace, slots, discard=2.0)
        res[name]["keeps_up"] = bool(res[name]["drain_s"] < 2.0)
        if not quiet:
            print("stable", name, res[name], file=sys.stderr, flush=True)
    out["stable"] = res
    return out


# ---------------------------------------------------------------- GPU
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-linearize", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (default: host cores, at most 16)")
    ap.add_argument("--cpu-sample", type=int, default=32, help="oracle instances of the rope batch")
    ap.add_argument("--cpu-T", type=int, default=100)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "probe", "copy", "sls", "next"])
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=22.0,
                    help="length of the Poisson trace of the serving leg (the first 2 s are discarded)")
    ap.add_argument("--slots", type=int, default=8, help="device slots of the batched planning server")
    ap.add_argument("--no-aux", action="store_true",
                    help="re-solve every step in the adjoint and linearize instead of keeping the step internals")
    ap.add_argument("--grasp", default="dirichlet", choices=["dirichlet", "penalty"],
                    help="grasp of the rope batch (penalty: holonomic penalty with smoothed activation)")
    ap.add_argument("--no-serve", action="store_true", help="skip the planning-stream leg")
    ap.add_argument("--no-extras", action="store_true", help="skip the cloth (C3), mixed-batch (C4), SLS and widened-row legs")
    ap.add_argument("--overlap", action="store_true",
                    help="run the adjoint and the linearization concurrently on two streams, both after "
                         "the rollout (default: one after the other on one stream, so that each kernel's "
                         "duration, and the roofline fraction, is its own)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); instances are independent "
              "and would shard by instance across GPUs, which this build does not launch.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        print(json.dumps(bench_c3(args)), flush=True)
        return
    if args.workload == "c4":
        print(json.dumps(bench_c4(args)), flush=True)
        return
    if args.workload == "copy":
        return copy_calibration()
    if args.workload == "probe":
        return bench_probe(args)
    if args.workload == "c5":
        print(json.dumps(bench_c5(args)), flush=True)
        return
    if args.workload == "sls":
        print(json.dumps(bench_sls(args)), flush=True)
        return
    if args.workload == "next":
        print(json.dumps(bench_next(args)), flush=True)
        return

    with_lin = not args.no_linearize
    cpu = None
    if not args.no_cpu:
        # before any GPU initialisation: the pool is started from a clean process
        cpu = cpu_baseline(args.cpu_workers or cpu_cores(), args.cpu_sample, args.cpu_T, with_lin)
        print("cpu baseline:", json.dumps(cpu), file=sys.stderr, flush=True)

    import numpy as np
    import torch
    import workloads as W
    from paper_2606_14188_amd import Sim

    insts = workload()
    if args.grasp == "penalty":
        import workloads as W
        insts = [W.penalty_grasp(inst, seed=i) for i, inst in enumerate(insts)]
    B, n, T = len(insts), insts[0].n, insts[0].T
    sim = Sim(insts)
    if not args.no_aux:
        sim.use_aux(True)      # the adjoint and linearize reuse the rollout's step internals
    overlap = with_lin and args.overlap
    # The adjoint and the linearization both read only the rollout's output.
    # With --overlap they run concurrently: the linearization through a
    # second simulator over the same instances (a simulator serves one stream
    # at a time) that shares the step internals, on a second stream of
    # default priority.
    sim_lin = Sim(insts) if overlap else sim
    if overlap and not args.no_aux:
        sim_lin.use_aux(True, buffer=sim.aux)
    lin_stream = torch.cuda.Stream() if overlap else None
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
        # marks: rollout start/end, backward end (main stream); linearize
        # start/end (on the stream it runs on)
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if record else None
        main = torch.cuda.current_stream()
        if record:
            marks[0].record()
        sim.rollout(s0, u, out=traj, status=status)
        if record:
            marks[1].record()
        if overlap:
            lin_stream.wait_stream(main)          # trajectory and step internals written
            with torch.cuda.stream(lin_stream):
                if record:
                    marks[3].record()
                sim_lin.linearize(traj, u, A=A, Bm=Bm)
                if record:
                    marks[4].record()
        sim.backward(u, traj, sT_bar=sT)
        if record:
            marks[2].record()
        if with_lin and not overlap:
            sim.linearize(traj, u, A=A, Bm=Bm)
            if record:
                marks[4].record()
            marks_lin0 = marks[2] if record else None
        else:
            marks_lin0 = marks[3] if record else None
        if overlap:
            main.wait_stream(lin_stream)          # the next rollout overwrites both
        if record:
            ev["rollout"].append((marks[0], marks[1]))
            ev["backward"].append((marks[1], marks[2]))
            if with_lin:
                ev["linearize"].append((marks_lin0, marks[4]))

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
    roof["traffic"] = profiled_traffic(dom) if args.grasp == "dirichlet" else None
    roof["kernel"] = dom
    serve, extras = None, None
    if with_lin:
        del A, Bm
    del sim, sim_lin
    torch.cuda.empty_cache()
    # the other workloads: reported beside the headline figure (a failure
    # there is recorded instead of losing the line)
    if not args.no_extras:
        extras = {}
        for name, fn in (("c3", bench_c3), ("c4", bench_c4), ("sls", bench_sls), ("next", bench_next)):
            try:
                extras[name] = fn(args)
            except Exception as e:      # noqa: BLE001
                extras[name] = {"error": repr(e)}
            torch.cuda.empty_cache()
    if not args.no_serve:
        try:
            serve = bench_c5(args)
        except Exception as e:          # noqa: BLE001
            serve = {"error": repr(e)}
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
                               + (" + dense A_t/B_t" if with_lin else "")
                               + (", penalty grasp" if args.grasp == "penalty" else ""),
                   "batch": B, "nodes": n, "horizon": T,
                   "schedule": ("rollout, then adjoint and linearization concurrently on two streams" if overlap
                                else "rollout, adjoint, linearization on one stream")},
        "kernel_ms": kern_ms,
        "kernel_roofline": {k: dict(v, frac=v["achieved"] / v["peak"]) for k, v in kernels.items()},
        "status_nonzero": int((st != 0).sum()),
        "roofline": roof,
        "cpu_baseline": cpu,
        "serve": serve,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
