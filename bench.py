"""Benchmark of the fused SSP-RK3 stage path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rot2d_256_p2]

A step is one SSP-RK3 step (three fused stage launches, each evaluating the
whole stabilised DG operator: traces, volume and face quadrature with the LLF
flux, HWENO reconstruction, sensor, dissipation, mass inverse and the RK
combination) over the whole mesh of the workload.  K steps run as one dg_run
call (HIP graph replay) with the state already resident in HBM; the timed
region is bracketed by device synchronisation.

Printed: one JSON line with the metric (FP64 DOF-updates per second per RK
stage), the roofline of the stage kernel (algorithmic HBM bytes per launch over
its average duration, from HIP events on the stream the kernels run on), and
the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 DOF-updates/s per RK stage + %HBM roofline; batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0


def workload(name):
    from paper_2309_12019_amd import inputs
    table = {
        "rot2d_256_p2": lambda: inputs.rot2d(256, 2, seed=0, steps=200),
        "rot2d_256_p3": lambda: inputs.rot2d(256, 3, seed=0, steps=200),
        "burgers2d_1024_p2": lambda: inputs.burgers2d(1024, 2, seed=0),
        "adv1d_64_p2": lambda: inputs.adv1d(64, 2, steps=100),
        "rot2d_2048_p2": lambda: inputs.rot2d(2048, 2, seed=0, steps=50),
    }
    return table[name]()


def stage_bytes_per_dof():
    """Algorithmic HBM bytes per DOF per stage: stage 1 reads U^n and writes
    U^(1) (16 B); stages 2 and 3 also read U^n (24 B); mean 64/3 B."""
    return (16.0 + 24.0 + 24.0) / 3.0


def time_gpu(w, steps, warmup):
    import torch
    from paper_2309_12019_amd import dgweno
    g = dgweno.DG.from_workload(w)
    U0 = g.initial_state(w)
    dt = w.dt()
    U = U0.clone()
    if warmup:
        g.run(U, dt, warmup)
    torch.cuda.synchronize()
    U = U0.clone()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(st)
    g.run(U, dt, steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    bad = g.count_nonfinite(U)
    if bad:
        raise RuntimeError(f"{bad} non-finite values after the timed run")
    return dict(wall=wall, event_ms=ev_ms, ndof=w.ndof, steps=steps, tile=g.tile())


def cpu_baseline(w, budget_s=15.0):
    """The CPU oracle, as it stands, on the same workload: whole SSP-RK3 steps
    over the full mesh, as many as fit the time budget (at least one)."""
    import torch
    import numpy as np
    import oracle
    f = w.fields()
    O = oracle.Oracle(oracle.Problem(**{k: f[k] for k in oracle.Problem.__dataclass_fields__ if k in f}))
    U = O.project(torch.from_numpy(np.ascontiguousarray(w.eval_ic(O.proj_nodes().numpy()))))
    dt = w.dt()
    t0 = time.perf_counter()
    U = O.step(U, dt)
    one = time.perf_counter() - t0
    n = max(1, min(50, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    for _ in range(n):
        U = O.step(U, dt)
    t = time.perf_counter() - t0
    return {"value": 3.0 * w.ndof * n / t, "unit": "DOF-updates/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n} SSP-RK3 steps of {w.name} ({w.ndof} DOFs) after one warm-up step, "
                      f"PyTorch CPU fp64, {t:.1f} s"}


def bench_batch(steps=100, seed=0, count=512):
    """512 independent problems (1D advection / Burgers, 2D rotation, degrees
    1..4, seeded sizes) for `steps` SSP-RK3 steps each with its own dt: the
    batched graph-captured path against the same kernels launched one problem
    and one stage at a time (no graph), from the same initial state."""
    import torch
    from paper_2309_12019_amd import dgweno, inputs
    ws = inputs.batch_mix(seed, count, steps)
    B = dgweno.Batch.from_workloads(ws)
    arena = B.empty()
    for w, v in zip(ws, B.views(arena)):
        g = dgweno.DG.from_workload(w)
        pts = torch.from_numpy(g.proj_nodes()).to(g.device)
        g.project_ic(w.eval_ic(pts).reshape(-1).contiguous(), v)
        g.close()
    torch.cuda.synchronize()
    U0 = arena.clone()
    dts = [w.dt() for w in ws]
    report = B.tune(U0, dts, reps=3)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    B.run(arena, dts, steps)          # records the graph (untimed)
    torch.cuda.synchronize()
    arena.copy_(U0)
    torch.cuda.synchronize()
    ev[0].record(st)
    B.run(arena, dts, steps)
    ev[1].record(st)
    torch.cuda.synchronize()
    seq = U0.clone()
    torch.cuda.synchronize()
    ev[2].record(st)
    B.run_sequential(seq, dts, steps)
    ev[3].record(st)
    torch.cuda.synchronize()
    tb = ev[0].elapsed_time(ev[1]) / 1e3
    ts = ev[2].elapsed_time(ev[3]) / 1e3
    ndof = sum(w.ndof for w in ws)
    upd = 3.0 * steps * ndof
    return {"workload": f"{count} problems: 1D advection/Burgers 64-4096 cells, 2D rotation 32^2-512^2, "
                        f"p 1..4, seed {seed}, {steps} SSP-RK3 steps each",
            "problems": count, "dofs": ndof, "classes": B.num_classes(),
            "value": upd / tb, "unit": "DOF-updates/s",
            "one_launch_per_problem_value": upd / ts,
            "speedup_vs_one_launch_per_problem": ts / tb,
            "batched_s": tb, "one_launch_per_problem_s": ts,
            "max_abs_diff_vs_one_launch_per_problem": float((arena - seq).abs().max()),
            "tuned_schedule": [B.schedule(c) for c in range(B.num_classes())]}


def traffic_for(wname):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary,
    if one exists for this workload (else None)."""
    path = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        return d.get(wname, {}).get("bytes_per_launch")
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="rot2d_256_p2")
    ap.add_argument("--extra", default="rot2d_256_p3,burgers2d_1024_p2",
                    help="comma-separated workloads reported alongside (no cpu baseline)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU domain decomposition is a design note, not a code path.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    w = workload(args.workload)
    r = time_gpu(w, args.steps, args.warmup)
    sec = r["event_ms"] / 1e3
    launches = 3 * args.steps
    dof_rate = 3.0 * w.ndof * args.steps / sec
    bpd = stage_bytes_per_dof()
    bytes_per_launch = bpd * w.ndof
    avg_launch = sec / launches
    achieved = bytes_per_launch / avg_launch / 1e9
    traffic = traffic_for(args.workload)
    line = {
        "metric": METRIC,
        "value": dof_rate,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["event_ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "dim": w.dim, "cells": w.ncells, "p": w.p, "dofs": w.ndof,
                   "flux": "linear advection" if w.flux == 0 else "Burgers",
                   "mode": ["DG", "LO", "WENO"][w.mode], "ssp_rk3_steps": args.steps,
                   "dt": w.dt(), "tile": list(r["tile"])},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"stage_kernel<{w.dim},{w.p},{w.flux},{w.mode}>",
                     "bytes_per_dof": bpd, "avg_launch_us": avg_launch * 1e6},
        "wall_s": r["wall"],
    }
    extra = {}
    for name in [s for s in args.extra.split(",") if s]:
        we = workload(name)
        k = min(we.steps, 100)
        re_ = time_gpu(we, k, 5)
        s_ = re_["event_ms"] / 1e3
        extra[name] = {"value": 3.0 * we.ndof * k / s_, "steps": k, "dofs": we.ndof,
                       "avg_launch_us": s_ / (3 * k) * 1e6,
                       "hbm_frac": bpd * we.ndof / (s_ / (3 * k)) / 1e9 / HBM_PEAK_GBS}
    if extra:
        line["extra"] = extra
    if not args.no_batch:
        line["batched"] = bench_batch(args.batch_steps)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
