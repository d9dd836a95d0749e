"""Benchmark of the dissipative-WENO RKDG hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload burgers2d_1024_p2]

A step is one SSP-RK3 step over the whole mesh of the workload: the three
stages each evaluate the whole stabilised DG operator (traces, volume and face
quadrature with the LLF flux, HWENO reconstruction, sensor, dissipation, mass
inverse) and the RK combination.  K steps run as one dg_run call (HIP graph
replay) with the state already resident in HBM; the timed region is bracketed
by device synchronisation.  The default workload is 1024^2 P2 periodic 2D
Burgers with seeded Fourier data, time step CFL h / ((2p+1) lambda_max(U^0))
from the library's dg_stable_dt; dg_run takes the per-stage kernel there
(three launches per step).

Printed: one JSON line with the metric (FP64 DOF-updates per second per RK
stage), the HBM roofline of the per-stage kernel (algorithmic bytes per
launch over its average duration from HIP events on the stream the kernels
run on, against 8 TB/s), the same kernel's FP64 rate, the CPU oracle timed
on a bounded sample of the same workload (one thread and all threads),
further workloads, the batched extension and the adjoint extension.
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


def _order(w, k):
    w.rk_order = k
    return w


def workload(name):
    from paper_2309_12019_amd import inputs
    table = {
        "rot2d_256_p2": lambda: inputs.rot2d(256, 2, seed=0, steps=200),
        "rot2d_256_p3": lambda: inputs.rot2d(256, 3, seed=0, steps=200),
        "burgers2d_1024_p2": lambda: inputs.burgers2d(1024, 2, seed=0),
        "adv1d_64_p2": lambda: inputs.adv1d(64, 2, steps=100),
        "rot2d_2048_p2": lambda: inputs.rot2d(2048, 2, seed=0, steps=50),
        # the rotation at a bandwidth-bound size (per-stage kernel, 9.4 M DOFs)
        "rot2d_1024_p2": lambda: inputs.rot2d(1024, 2, seed=0, steps=100),
        # degree 3 on the per-stage kernel (16 M DOFs)
        "rot2d_1024_p3": lambda: inputs.rot2d(1024, 3, seed=0, steps=50),
        # the sensor of Zhao et al. (Sec. 5.6) in place of eq. (sensor)
        "rot2d_256_p2_zhao": lambda: inputs.rot2d(256, 2, seed=0, steps=200, mode=inputs.MODE_ZHAO),
        # the KPP problem of Sec. 5.5 at the paper's size (128^2, P2, lambda_e = 2, t = 1)
        "kpp2d_128_p2": lambda: inputs.kpp2d(128, 2),
        # DRAM-resident (302 MB per state array, beyond the 256 MB last-level
        # cache); initial data evaluated on the device
        "burgers2d_2048_p2": lambda: inputs.burgers2d(2048, 2, seed=0),
        # the five-stage fourth-order SSP method that Sec. 5.1 pairs with p = 3
        "rot2d_256_p3_rk4": lambda: _order(inputs.rot2d(256, 3, seed=0, steps=200), 4),
        "burgers2d_1024_p2_rk4": lambda: _order(inputs.burgers2d(1024, 2, seed=0), 4),
        # the four-quadrant problem of Sec. 5.4 at the paper's size (exact
        # exterior state at every stage time; steps launched without a graph)
        "burgers2d_riemann_128_p2": lambda: inputs.burgers2d_riemann(128, 2),
        # the 1D Euler equations of Sec. 5.6: Sod's tube at the paper's size,
        # and on 2^20 cells (28 MB per state) for the per-stage kernel's bandwidth
        "sod1d_128_p2": lambda: inputs.sod1d(128, 2),
        "sod1d_1m_p2": lambda: inputs.sod1d(1 << 20, 2, steps=100),
    }
    return table[name]()


# FP64 flops per cell and stage that the per-stage kernel executes
# (rocprofv3 SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_F64 per wave, one lane per
# cell, FMA counted twice; profiles/stage_kernel_hbm_counters.md): the
# per-unit figure of the arithmetic roofline.  Keyed by (dim, p, flux, mode).
FLOPS_PER_CELL_STAGE = {(2, 2, 0, 2): 990.0, (2, 3, 0, 2): 2118.0, (2, 2, 1, 2): 1026.0, (1, 2, 3, 2): 832.0}
FP64_PEAK_TFLOPS = 78.6


def stage_bytes_per_dof(rk_order=3):
    """Algorithmic HBM bytes per DOF per stage launch: the first stage reads
    U^n and writes U^(1) (16 B); every later launch also reads the state it
    combines with (24 B).  Three-stage method: mean 64/3 B; two-stage: 20 B;
    five-stage fourth-order (six launches): 136/6 B."""
    launches = LAUNCHES_PER_STEP[rk_order]
    return (16.0 + 24.0 * (launches - 1)) / launches


# RK stages and stage-kernel launches per step of each SSP method (the
# five-stage method evaluates the operator at U^(3) twice)
STAGES_PER_STEP = {2: 2, 3: 3, 4: 5}
LAUNCHES_PER_STEP = {2: 2, 3: 3, 4: 6}


def prepare(w, fused=None):
    """Handle, projected initial state (initial data evaluated on the device)
    and the workload's time step from lambda_max of that state (dg_stable_dt:
    CFL h / ((2p+1) lambda_max(U^0))); a workload with an end time then runs
    ceil(t_end / dt) steps.  Workloads with a stated speed bound instead
    (lambda_e fixed, the Euler system, inflow boundaries) keep it."""
    from paper_2309_12019_amd import dgweno
    g = dgweno.DG.from_workload(w)
    if fused is not None:
        g.set_fused(fused)
    U0 = g.initial_state(w, on_device=True)
    if w.flux in (0, 1) and w.bc_kind == 0 and w.lambda_override <= 0:
        w.with_dt(g.stable_dt(U0, w.cfl))
    return g, U0


def time_gpu(w, steps, warmup, fused=None, g=None, U0=None):
    """Time `steps` SSP steps (the workload's order) of dg_run; fused: None
    keeps the library's automatic choice of the fused step kernel, 0 / 1
    forces it off / on."""
    import torch
    if g is None:
        g, U0 = prepare(w, fused)
    elif fused is not None:
        g.set_fused(fused)
    dt = w.dt()
    # dg_run replays graphs cached per (state buffer, dt, chunk length): one
    # untimed call of the timed length on the timed buffer records them, so
    # the timed region holds no capture or instantiation
    U = U0.clone()
    g.run(U, dt, steps)
    U.copy_(U0)
    if warmup:
        g.run(U, dt, warmup)
    torch.cuda.synchronize()
    U.copy_(U0)
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
    return dict(wall=wall, event_ms=ev_ms, ndof=w.ndof, steps=steps, tile=g.tile(), fused=g.fused(), dt=dt,
                step_tile=g.step_tile())


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s=12.0):
    """The CPU oracle, as it stands, on the same workload: the plain C oracle
    (oracle/dgoracle.c, loops per cell, OpenMP over cells) from the oracle's
    projection of the initial data, whole SSP steps over the full mesh, as
    many as fit the time budget (at least one), with all host threads and
    with one."""
    import numpy as np
    import torch
    import oracle
    from oracle import coracle
    f = w.fields()
    prob = oracle.Problem(**{k: f[k] for k in oracle.Problem.__dataclass_fields__ if k in f})
    O = oracle.Oracle(prob)
    U = O.project(torch.from_numpy(np.ascontiguousarray(w.eval_ic(O.proj_nodes().numpy()))))
    del O
    C = coracle.COracle(prob)
    dt = w.dt()
    nmax = coracle.max_threads()
    legs = {}
    for threads in (nmax, 1):
        coracle.set_threads(threads)
        t0 = time.perf_counter()
        V = C.step(U, dt)
        one = time.perf_counter() - t0
        n = max(1, min(200, int(budget_s / max(one, 1e-3))))
        t0 = time.perf_counter()
        V = C.run(U, dt, n)
        t = time.perf_counter() - t0
        legs[threads] = {"value": w.ndof * 3.0 * n / t, "steps": n, "seconds": t}
    coracle.set_threads(nmax)
    big = legs[nmax]
    return {"value": big["value"], "unit": "DOF-updates/s", "cores": nmax, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{big['steps']} SSP-RK3 steps of {w.name} ({w.ndof} DOFs) after one warm-up step, "
                      f"C oracle, FP64, {nmax} OpenMP threads, {big['seconds']:.1f} s",
            "single_thread": {"value": legs[1]["value"], "cores": 1,
                              "sample": f"{legs[1]['steps']} steps, 1 thread, {legs[1]['seconds']:.1f} s"}}


def oracle_ops_per_cell(w):
    """FP64 operations per cell and stage of the oracle's own evaluation of
    the operator (oracle/opcounts.json, written by python -m oracle.opcount:
    dense products over all basis functions and nodes, so an upper bound on
    the method's arithmetic)."""
    path = os.path.join(ROOT, "oracle", "opcounts.json")
    try:
        d = json.load(open(path))["counts"]
        return d[f"{w.dim},{w.p},{w.flux},{w.mode}"]["ops_per_cell"]
    except (OSError, KeyError, ValueError):
        return None


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


def bench_adjoint(n=512, steps=400, ndir=32, seed=0, budget_bytes=1 << 30):
    """Gradient of J = int_W u(T)^2 dx, W = [0.25, 0.75]^2, with respect to all
    initial DOFs of 2D Burgers (n x n, P2, seeded Fourier data, `steps` steps)
    by the checkpointed discrete adjoint.  Cost (forward with checkpoints +
    backward) over the plain forward run for three memory budgets: binomial
    checkpointing within ~1 GB of snapshots (the headline), one snapshot per
    step, and every step's stage states kept (the upper-memory reference).
    Finite differences of the GPU forward map along `ndir` random unit
    directions: central differences Richardson-extrapolated over (delta,
    delta/2), delta = 1e-4 ||U^0||_inf (and 1e-5 for comparison); every
    direction's runs record their branches (dg_run_signature), and a
    direction whose records at U^0 +- delta d (or +- delta/2 d) differ has
    crossed a kink of the map, reported per kind (sensor, lambda_e, LLF)."""
    import numpy as np
    import torch
    from paper_2309_12019_amd import dgweno, inputs
    w = inputs.burgers2d(n, 2, seed=seed, steps=steps)
    g = dgweno.DG.from_workload(w)
    U0 = g.initial_state(w)
    dt = w.dt()
    dev = U0.device
    xc = (torch.arange(n, device=dev, dtype=torch.float64) + 0.5) / n
    win = (xc > 0.25) & (xc < 0.75)
    inside = (win[None, :] & win[:, None]).reshape(-1).to(torch.float64)
    mh = torch.tensor([4.0 / ((2 * a + 1) * (2 * b + 1)) for b in range(3) for a in range(3)],
                      dtype=torch.float64, device=dev) * (0.5 / n) ** 2

    st = torch.cuda.current_stream()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        out = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / 1e3

    # plain forward (graph-captured run), warmed
    U = U0.clone()
    g.run(U, dt, steps)             # records the graphs (untimed)
    U.copy_(U0)
    _, t_fwd = timed(lambda: g.run(U, dt, steps))
    state_bytes = w.ndof * 8
    res = {"workload": f"2D Burgers {n}x{n} P2 WENO, seeded Fourier data, {steps} SSP-RK3 steps, "
                       f"J = int over [0.25,0.75]^2 of u(T)^2", "dofs": w.ndof, "forward_s": t_fwd,
           "state_bytes": state_bytes}
    budget_snaps = max(1, budget_bytes // state_bytes - 2)   # + 2 working slots
    grad = None
    for key, ns, keep in (("budget_1GiB", budget_snaps, False), ("snapshot_every_step", steps, False),
                          ("every_stage_state_kept", steps, True)):
        ck = g.checkpoints(ns)
        stg = g.stage_checkpoints(steps) if keep else None
        for rep in range(2):  # the first pass warms the buffers, as the forward run above
            UT, t_f = timed(lambda: g.adjoint_forward(U0, dt, steps, ns, ck, stages=stg))
            lam = (2 * UT * mh[None, :] * inside[:, None]).contiguous()
            _, t_b = timed(lambda: g.adjoint_backward(dt, steps, ns, ck, lam, stages=stg))
        del ck, stg
        torch.cuda.empty_cache()
        rs = dgweno.revolve_stats(steps, ns)
        res[key] = {"snapshots": ns, "forward_with_checkpoints_s": t_f, "backward_s": t_b,
                    "cost_vs_forward": (t_f + t_b) / t_fwd, "recomputed_steps": rs["recomputed_steps"],
                    "checkpoint_bytes": (ns + 2 + (2 * steps if keep else 0)) * state_bytes}
        if grad is None:
            grad = lam.clone()
            JT = float(((UT * UT * mh[None, :]).sum(1) * inside).sum())
    res["cost_vs_forward"] = res["budget_1GiB"]["cost_vs_forward"]
    res["schedule"] = "budget_1GiB"
    res["upper_memory_reference"] = "every_stage_state_kept"

    # finite differences of the forward map, with branch records
    rng = np.random.default_rng(1)
    u0max = float(U0.abs().max())
    sig = [torch.empty((3, g.ncells), dtype=torch.int32, device=dev) for _ in range(4)]

    def runs(d, delta):
        """J(U(+s)) - J(U(-s)) for s = delta and delta/2, summed as (U+ - U-)(U+ + U-)
        (the two values of J agree to ~1e-9 of J, below the rounding of each sum),
        and the cells whose branch records differ between +s and -s, per kind."""
        out, crossed = [], np.zeros(3, dtype=np.int64)
        for k, s_ in enumerate((delta, 0.5 * delta)):
            Up = (U0 + s_ * d).contiguous()
            Um = (U0 - s_ * d).contiguous()
            g.run_signature(Up, dt, steps, sig[2 * k])
            g.run_signature(Um, dt, steps, sig[2 * k + 1])
            out.append(float((((Up - Um) * (Up + Um) * mh[None, :]).sum(1) * inside).sum()))
            crossed += (sig[2 * k] != sig[2 * k + 1]).sum(1).cpu().numpy()
        return out, crossed

    deltas = (("1e-4", 1e-4 * u0max), ("1e-5", 1e-5 * u0max))
    rows = {tag: [] for tag, _ in deltas}
    for j in range(ndir):
        d = torch.from_numpy(rng.standard_normal(U0.shape)).to(dev)
        d /= d.norm()
        ad = float((grad * d).sum())
        for tag, delta in deltas:
            (j1, j2), crossed = runs(d, delta)
            fd1, fd2 = j1 / (2 * delta), j2 / delta
            fd = (4 * fd2 - fd1) / 3
            rows[tag].append({"rel_err": abs(fd - ad) / abs(ad), "crossed": crossed.tolist()})
    for tag, delta in deltas:
        r = rows[tag]
        kink = [x for x in r if sum(x["crossed"]) > 0]
        clean = [x for x in r if sum(x["crossed"]) == 0]
        res[f"fd_delta_{tag}_u0max"] = {
            "delta": delta, "directions": ndir, "within_1e-6": int(sum(x["rel_err"] <= 1e-6 for x in r)),
            "kink_crossing": len(kink),
            "kink_crossing_by_kind": {k: int(sum(x["crossed"][i] > 0 for x in r))
                                      for i, k in enumerate(("sensor", "lambda_e", "llf"))},
            "without_kink": len(clean),
            "without_kink_within_1e-6": int(sum(x["rel_err"] <= 1e-6 for x in clean)),
            "failures_not_at_a_kink": int(sum(x["rel_err"] > 1e-6 for x in clean)),
            "max_rel_err": max(x["rel_err"] for x in r), "median_rel_err": float(np.median([x["rel_err"] for x in r])),
            "max_rel_err_without_kink": max((x["rel_err"] for x in clean), default=None),
            "median_cells_crossed": float(np.median([sum(x["crossed"]) for x in r]))}
    res["J"] = JT
    return res


STAGE_SOURCES = ("dg_kernels.hpp", "dg_tables.hpp", "dg_stage.hip", "dg_euler.hpp")


def stage_source_digest():
    """SHA-256 over the code (comments and blank space removed) of the sources
    the stage kernels are compiled from."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in STAGE_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_12019_amd", "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def traffic_for(wname):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary
    for this workload; None if there is none or if the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if d.get("kernel_source_sha256") != stage_source_digest():
            return None
        return d.get(wname, {}).get("bytes_per_launch")
    except Exception:
        return None


def measured_copy_gbs(mib=1024, reps=5):
    """Achieved bandwidth of the library's streaming copy (dg_stream_copy, 16
    bytes per lane) of `mib` MiB, beyond the last-level cache: read plus write
    bytes over the event time.  The practical ceiling the per-stage kernel's
    HBM fraction can also be read against (the roofline itself uses the
    published 8 TB/s)."""
    import torch
    from paper_2309_12019_amd import dgweno
    n = mib * 1024 * 1024 // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dgweno.stream_copy(src, dst)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        dgweno.stream_copy(src, dst)
    e1.record(st)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    ok = bool(torch.equal(dst, src))
    del src, dst
    torch.cuda.empty_cache()
    return {"gbs": 2.0 * n * 8 / sec / 1e9, "bytes_per_copy": n * 8, "copied_exactly": ok,
            "kind": f"dg_stream_copy of {mib} MiB (16 B per lane), read + write bytes"}


def copy_probe(mib):
    """A plain device-to-device copy of a known size, three times: the
    reference against which rocprofv3's FETCH_SIZE / WRITE_SIZE counters are
    scaled to bytes."""
    import torch
    n = mib * 1024 * 1024 // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    print(json.dumps({"copy_probe_bytes": n * 8, "copies": 3}), flush=True)


def stage_kernel_name(w, tile):
    """The per-stage kernel the library launches for this workload and tile
    (2D 8x8: KPP spreads each tile over several waves; the other fluxes take
    four-wave tiles up to three 8x8 tiles per compute unit)."""
    if w.flux == 3:
        return f"euler_stage_kernel<{w.p},{w.mode}>"
    if w.dim == 1:
        return f"stage_kernel<1,{w.p},{w.flux},{w.mode},{tile[0]},1>"
    tx, ty = tile
    if (tx, ty) == (8, 8):
        if w.flux == 2:
            return f"kpp_split_kernel<{w.p},{w.mode}> (8x8)"
        import torch
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        t8 = ((w.nx + 7) // 8) * ((w.ny + 7) // 8)
        if t8 <= 3 * cus:
            return f"roles_kernel<{w.p},{w.flux},{w.mode}> (8x8, four waves)"
    return f"stage_kernel<{w.dim},{w.p},{w.flux},{w.mode},{tx},{ty}>"


def stage_roofline(w, wname, sec, launches, copy_gbs=None, tile=(16, 16)):
    """HBM roofline of the per-stage kernel over `launches` launches taking
    `sec` in all: algorithmic bytes per launch (16 B per DOF for the first
    stage, 24 B for the others: 64/3 B on average for SSP-RK3) over the
    average launch duration, against 8 TB/s; with the kernel's executed FP64
    rate beside it (rocprofv3 SQ counters per cell) and the oracle's op count
    (an upper bound on the method's arithmetic)."""
    bpd = stage_bytes_per_dof(w.rk_order)
    avg = sec / launches
    ach = bpd * w.ndof / avg / 1e9
    key = (w.dim, w.p, w.flux, w.mode)
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(wname),
            "kernel": stage_kernel_name(w, tile),
            "bytes_per_dof": bpd, "bytes_per_launch": bpd * w.ndof, "avg_launch_us": avg * 1e6}
    if copy_gbs:
        roof["frac_of_measured_copy"] = ach / copy_gbs
    fx = FLOPS_PER_CELL_STAGE.get(key)
    if fx:
        tf = fx * w.ncells / avg / 1e12
        roof["executed_flops_per_cell"] = fx
        roof["executed_tflops"] = tf
        roof["executed_flop_frac"] = tf / FP64_PEAK_TFLOPS
    ops = oracle_ops_per_cell(w)
    if ops:
        roof["oracle_ops_per_cell"] = ops
        roof["oracle_ops_rate_tflops"] = ops * w.ncells / avg / 1e12
    return roof


def fused_roofline(w, wname, sec, steps, step_tile=None):
    """The fused step kernel (one launch per step: U^n in, U^(n+1) out, three
    stages of arithmetic): FP64 rate from the per-stage kernel's executed
    flops per cell (recomputed rings not counted) against the FP64 vector
    peak, and its HBM fraction."""
    key = (w.dim, w.p, w.flux, w.mode)
    avg = sec / steps
    flops = 3.0 * FLOPS_PER_CELL_STAGE[key] * w.ncells if key in FLOPS_PER_CELL_STAGE else None
    ach = flops / avg / 1e12 if flops else None
    return {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP64_PEAK_TFLOPS if ach else None,
            "traffic": traffic_for(wname + ":step"),
            "kernel": (f"euler_step_kernel<{w.p},{w.mode}>" if w.flux == 3 else
                       f"step_kernel<{w.dim},{w.p},{w.flux},{w.mode}" +
                       (f",{step_tile[0]},{step_tile[1]}>" if step_tile and w.dim == 2 else ">")) +
                      " (fused SSP-RK3 step)",
            "flops_per_launch": flops, "avg_launch_us": avg * 1e6,
            "hbm_bytes_per_launch": 16.0 * w.ndof,
            "hbm_frac": 16.0 * w.ndof / avg / 1e9 / HBM_PEAK_GBS}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="burgers2d_1024_p2")
    ap.add_argument("--extra", default="rot2d_256_p2,rot2d_256_p3,rot2d_1024_p2,burgers2d_2048_p2,"
                    "rot2d_256_p2_zhao,kpp2d_128_p2,rot2d_256_p3_rk4,burgers2d_1024_p2_rk4,"
                    "burgers2d_riemann_128_p2,sod1d_128_p2,sod1d_1m_p2",
                    help="comma-separated workloads reported alongside (no cpu baseline)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-n", type=int, default=512)
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--adjoint-dirs", type=int, default=32)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU domain decomposition is a design note, not a code path.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
        return

    copy = measured_copy_gbs()
    cgbs = copy["gbs"]
    w = workload(args.workload)
    g, U0 = prepare(w)
    r = time_gpu(w, args.steps, args.warmup, g=g, U0=U0)
    sec = r["event_ms"] / 1e3
    dof_rate = STAGES_PER_STEP[w.rk_order] * w.ndof * args.steps / sec
    if r["fused"]:
        roof = fused_roofline(w, args.workload, sec, args.steps, r["step_tile"])
    else:
        roof = stage_roofline(w, args.workload, sec, LAUNCHES_PER_STEP[w.rk_order] * args.steps, cgbs, r["tile"])
    del g, U0
    torch.cuda.empty_cache()
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
                   "flux": ["linear advection", "Burgers", "KPP", "Euler"][w.flux],
                   "mode": ["DG", "LO", "WENO", "Zhao"][w.mode], "ssp_order": w.rk_order,
                   "timed_steps": args.steps, "steps_to_end_time": w.steps,
                   "dt": r["dt"], "dt_rule": "CFL h / ((2p+1) lambda_max(U^0)), CFL 0.1 (dg_stable_dt)",
                   "tile": list(r["tile"]), "fused_step": r["fused"]},
        "roofline": roof,
        "wall_s": r["wall"],
        "measured_copy": copy,
    }
    extra = {}
    for name in [s for s in args.extra.split(",") if s]:
        we = workload(name)
        ge, Ue = prepare(we)
        k = min(we.steps, 100)
        re_ = time_gpu(we, k, 5, g=ge, U0=Ue)
        s_ = re_["event_ms"] / 1e3
        ko = we.rk_order
        launches = k if re_["fused"] else LAUNCHES_PER_STEP[ko] * k
        ex = {"value": STAGES_PER_STEP[ko] * we.ndof * k / s_, "steps": k, "dofs": we.ndof,
              "rk_order": ko, "fused_step": re_["fused"], "tile": list(re_["tile"]),
              "us_per_step": s_ / k * 1e6, "avg_launch_us": s_ / launches * 1e6}
        if re_["fused"]:
            ex["step_tile"] = list(re_["step_tile"])
            ex["roofline"] = fused_roofline(we, name, s_, k, re_["step_tile"])
            rs = time_gpu(we, k, 5, fused=0, g=ge, U0=Ue)
            ex["per_stage"] = stage_roofline(we, name, rs["event_ms"] / 1e3, LAUNCHES_PER_STEP[ko] * k, cgbs,
                                             rs["tile"])
            ex["per_stage"]["value"] = STAGES_PER_STEP[ko] * we.ndof * k / (rs["event_ms"] / 1e3)
        else:
            ex["roofline"] = stage_roofline(we, name, s_, launches, cgbs, re_["tile"])
        extra[name] = ex
        del ge, Ue
        torch.cuda.empty_cache()
    if extra:
        line["extra"] = extra
    if not args.no_batch:
        line["batched"] = bench_batch(args.batch_steps)
    if not args.no_adjoint:
        line["adjoint"] = bench_adjoint(args.adjoint_n, args.adjoint_steps, args.adjoint_dirs)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
