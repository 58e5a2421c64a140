"""Throughput of the RK3 MHD step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload strat512]
                    [--precision both|fp64|fp32_split] [--no-cpu-baseline]

One "step" is one full cmhd_rk3_step (three substages with all boundary work:
z ghosts, the Fourier potential-field ghosts, the fused stencil/RHS/RK kernel,
the nudged ghost rows) on the stratified 512 x 512 x 256 box, with the state
resident in HBM and dt fixed (computed once on the device before the timed
region).  As in the workload definition, the photospheric driver target is
re-seeded every 10 steps (device-resident targets, set with cmhd_set_driver).

Prints one JSON line: the FP64 throughput (zone-updates/s) as `value`, the
FP32-split form beside it, the HBM roofline of the fused kernel from HIP
events around its launches (with the rate of a plain device copy measured in
the same run, the counters' HBM traffic and VALU busy), 32^2 x 24 and 64^3 boxes
stepped eagerly and from a captured HIP graph, the same box on a non-uniform z grid (FP64), the
1024 x 1024 x 256 active-region box in the FP32-split form, the
granulation driver's cost per snapshot on the same photospheric plane (outside
the timed steps), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes per zone of the fused substage kernel (FP64 state,
# 8 fields): stage 1 reads f, writes f_next and dF; stage 2 reads f and dF,
# writes both; stage 3 reads f and dF, writes f_next
BYTES_PER_ZONE_STEP = 192 + 256 + 192
METRIC = ("zone-updates/s per RK3 step (FP64 vs FP32-split) + % HBM roofline, "
          "512²×256")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def copy_bandwidth(mib=2048, reps=10):
    """GB/s (bytes read + written) of a device-to-device copy of `mib` MiB,
    timed with HIP events on the current stream."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def measured_traffic():
    """HBM bytes per substage from the committed rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE scaled by the copy calibration), if they were taken on the
    kernel sources as they are now; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "substage_strat512_fp64_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        if not os.path.exists(os.path.join(ROOT, src)):
            return None
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec if h.hexdigest() == rec["sources_sha256"] else None


def run_gpu(w, precision, steps, warmup, drivers):
    import torch

    from paper_1908_08557_amd import cmhd
    g = w.grid
    zones = g["nx"] * g["ny"] * g["nz"]
    s = cmhd.solver_for(w, precision)
    st = s.new_state(w.state)
    dt = s.cfl_dt(st)
    t = 0.0
    for i in range(warmup):
        t, _ = s.rk3_step(st, t, dt)
    torch.cuda.synchronize()
    s.profile(True)
    s.profile_read("substage")
    s.profile_read("ghosts")
    torch.cuda.synchronize()
    # events at the thirds of the timed region (no synchronisation inside it)
    marks = sorted({0, steps // 3, (2 * steps) // 3, steps})
    evs = {m: torch.cuda.Event(enable_timing=True) for m in marks}
    t0 = time.perf_counter()
    for i in range(steps):
        if i in evs:
            evs[i].record()
        if i % 10 == 0:
            s.set_driver(drivers[(i // 10) % len(drivers)])
        t, _ = s.rk3_step(st, t, dt)
    evs[steps].record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    blocks = [evs[a].elapsed_time(evs[b]) / (b - a) for a, b in zip(marks[:-1], marks[1:])]
    kms, nl = s.profile_read("substage")
    gms, ng_ = s.profile_read("ghosts")
    s.profile(False)
    # the optional CFL selection of dt (outside the timed steps, which take dt
    # as given): one call = one read pass with x/y/z stencils of A, the
    # three maxima and their copy to the host
    t1 = time.perf_counter()
    for _ in range(5):
        s.cfl_dt(st)
    cfl_ms = 1e3 * (time.perf_counter() - t1) / 5
    finite = s.check_finite(st)
    s.close()
    del st
    torch.cuda.empty_cache()
    ms_step = 1e3 * elapsed / steps
    # one substage = the boundary work (ghost fill, Fourier filters, nudged
    # rows) + the fused substage kernel, which moves the method's algorithmic
    # bytes; the library's events bracket each on the stream of the step
    substage_ms = kms / max(nl, 1)
    ghosts_ms = gms / max(ng_, 1)
    kernel_ms_per_launch = substage_ms
    alg_bytes_launch = BYTES_PER_ZONE_STEP / 3.0 * zones
    achieved = alg_bytes_launch / (substage_ms * 1e-3) / 1e9
    return dict(value=zones / (elapsed / steps), ms_per_step=ms_step, dt=dt, finite=finite,
                ms_per_step_blocks=blocks, ms_per_step_median_block=float(np.median(blocks)),
                kernel_ms_per_launch=kernel_ms_per_launch, launches=nl,
                ghosts_ms=ghosts_ms, substage_ms=substage_ms, cfl_dt_ms=cfl_ms,
                achieved_GBs=achieved, frac=achieved / HBM_PEAK_GBS,
                step_GBs=BYTES_PER_ZONE_STEP * zones / (elapsed / steps) / 1e9)


def graph_bench(n=64, nz=64, nsteps=10, reps=5):
    """A small stratified box (each step is some 60 small launches) stepped
    eagerly and as replays of one captured HIP graph of nsteps steps (dt
    fixed, ramp off, so the steps are time-independent)."""
    import torch
    from paper_1908_08557_amd import cmhd
    from paper_1908_08557_amd import workloads as W
    w = W.stratified_box(n, n, nz, 50.0 * n / 64, 50.0 * nz / 64, 8, 2, 3, f"strat{n}", t_ramp=0.0)
    s = cmhd.solver_for(w)
    x = s.new_state(w.state)
    dt = s.cfl_dt(x)
    for _ in range(3):
        s.rk3_step(x, 0.0, dt)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(nsteps * reps):
        s.rk3_step(x, 0.0, dt)
    e1.record()
    torch.cuda.synchronize()
    eager = e0.elapsed_time(e1) / (nsteps * reps)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(nsteps):
            s.rk3_step(x, 0.0, dt)
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph = e0.elapsed_time(e1) / (nsteps * reps)
    finite = bool(torch.isfinite(x).all())
    del g
    s.close()
    return {"workload": f"{n}x{n}x{nz} stratified box, FP64, ramp off", "eager_ms_per_step": eager,
            "graph_ms_per_step": graph, "speedup": eager / graph,
            "steps_per_graph": nsteps, "finite": finite}


def driver_bench(w, dt, ms_per_step, reps=5):
    """The granulation driver on the workload's photospheric plane: host
    bookkeeping of the first fill and of a 10 s update, and the GPU snapshot
    (render + eq. 3 enhancement + eq. 4 rescaling), timed with HIP events on
    the stream the driver object launches on."""
    import torch
    from paper_1908_08557_amd import cmhd
    from paper_1908_08557_amd import workloads as W
    g = w.grid
    p = dict(nx=g["nx"], ny=g["ny"], Lx=g["Lx"], Ly=g["Ly"], r_gran=0.8, r_lane=1.04,
             r_excl=0.64, t_gran=0.3, v0=1.028, vmin_frac=0.78, life_var=0.10, amp_var=0.15,
             f_rot=5.0)
    n_pool = int(4 * g["Lx"] * g["Ly"]) + 1000
    u, xi = W.granulation_randoms(n_pool, 31)
    drv = cmhd.Granulation(p)
    t0 = time.perf_counter()
    b0 = drv.update(0.0, u, xi)
    fill_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    b1 = drv.update(0.01, u[b0:], xi[2 * b0:])     # 10 s later
    update_ms = (time.perf_counter() - t0) * 1e3
    n = len(drv.granules())
    out = torch.empty((2, g["ny"], g["nx"]), dtype=torch.float64, device="cuda")
    drv.velocity(0.01, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        drv.velocity(0.01, out)
    e1.record()
    torch.cuda.synchronize()
    vel_ms = e0.elapsed_time(e1) / reps
    finite = bool(torch.isfinite(out).all().item())
    drv.close()
    steps_per_snapshot = 0.01 / dt            # one snapshot every 10 s of model time
    return {"plane": f"{g['nx']}x{g['ny']} over {g['Lx']}x{g['Ly']} Mm", "granules": n,
            "births_first_fill": b0, "births_10s_update": b1,
            "fill_ms_host": fill_ms, "update_ms_host": update_ms, "snapshot_ms_gpu": vel_ms,
            "steps_per_snapshot": steps_per_snapshot,
            "share_of_step_time": (update_ms + vel_ms) / (steps_per_snapshot * ms_per_step),
            "finite": finite}


def split_error(w, nsteps, drivers):
    """Per-field error of the FP32-split form against plain FP64 after nsteps
    steps from the same state with the same dt, the driver target re-seeded
    every 10 steps as in the timed runs (both on the GPU): max |diff| over
    the interior and the u_x, u_y ghost rows, divided by the max norm of the
    physical field (A and u as vectors, ln rho, ln T) of the FP64 run, and by
    the component's own max norm, except A_z: of a potential-field state it is
    a cancellation residue, measured against |A| in both figures (its own
    scale, max |A_z| / max |A|, is returned beside them)."""
    import torch
    from paper_1908_08557_amd import cmhd
    outs = {}
    dt = None
    for prec in ("fp64", "fp32_split"):
        s = cmhd.solver_for(w, prec)
        st = s.new_state(w.state)
        if dt is None:
            dt = s.cfl_dt(st)
        t = 0.0
        for i in range(nsteps):
            if i % 10 == 0:
                s.set_driver(drivers[(i // 10) % len(drivers)])
            t, _ = s.rk3_step(st, t, dt)
        torch.cuda.synchronize()
        outs[prec] = st
        s.close()
    a, b = outs["fp64"], outs["fp32_split"]
    names = ("Ax", "Ay", "Az", "ux", "uy", "uz", "lnrho", "lnT")
    groups = [(0, 1, 2)] * 3 + [(3, 4, 5)] * 3 + [(6,), (7,)]

    def vals(x, f):
        v = x[f, 3:-3].reshape(-1)
        if f in (3, 4):
            v = torch.cat([x[f, :3].reshape(-1), v])
        return v

    err, own = {}, {}
    for f in range(8):
        diff = float((vals(b, f) - vals(a, f)).abs().max())
        field = max(float(vals(a, q).abs().max()) for q in groups[f])
        err[names[f]] = diff / field
        own[names[f]] = diff / (field if names[f] == "Az" else float(vals(a, f).abs().max()))
    az_scale = float(vals(a, 2).abs().max()) / max(float(vals(a, q).abs().max()) for q in range(3))
    del outs, a, b
    torch.cuda.empty_cache()
    return err, own, az_scale


ORACLE_JOBS = {
    # name: (description, steps)
    "C1": ("periodic 16^3, 10 RK3 steps (the small parity case, in full)", 10),
    "C2": ("stratified 64^3 over 50 Mm, full physics, 100 RK3 steps (in full)", 100),
    "strat512-sample": ("128x128x64 box with the 512x512x256 box's grid spacing and physics, "
                        "8 RK3 steps", 8),
}


def _oracle_job(name):
    """One oracle run in a child process (numpy float64, one thread)."""
    from oracle import mhd as O
    from paper_1908_08557_amd import workloads as W
    desc, nsteps = ORACLE_JOBS[name]
    if name == "C1":
        w = W.periodic_box(16)
    elif name == "C2":
        w = W.strat64()
    else:
        nx, nz = 128, 64
        dz = 50.0 / 255.0
        w = W.stratified_box(nx, nx, nz, 50.0 * nx / 512, dz * (nz - 1), 2, 2, 3,
                             "strat512-sample")
    g = w.grid
    F = O.from_compact(w.state)
    O.fill_ghosts(F, g, w.params, w.lnrho0_z)
    dt = O.cfl_dt(F, g, w.params)
    drv = dict(uh=w.uh_target, ah=w.ah_target) if g["zbc"] == "solar" else None
    t0 = time.perf_counter()
    O.run(F, 0.0, dt, nsteps, g, w.params, w.lnrho0_z, drv)
    el = time.perf_counter() - t0
    zones = g["nx"] * g["ny"] * g["nz"]
    return dict(workload=desc, steps=nsteps, seconds=el, value=zones * nsteps / el,
                unit="zone-updates/s")


def cpu_model():
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _spawn_pool(nworkers):
    """A pool of fresh child processes (spawned, so that no GPU state is
    inherited) whose numpy runs on one thread each."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    ex = ProcessPoolExecutor(max_workers=nworkers, mp_context=mp.get_context("spawn"))
    ex.submit(int, 0).result()   # start the workers now, with this environment
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v
    return ex


def start_cpu_baseline():
    """The oracle as it stands on the host cores, started in child processes
    (one thread each, in parallel with the GPU timing): the two small cases in
    full and a bounded sample of the 512^2 x 256 workload."""
    ex = _spawn_pool(len(ORACLE_JOBS))
    futs = {name: ex.submit(_oracle_job, name) for name in ORACLE_JOBS}
    return ex, futs


def all_cores_run(name, ncores):
    """ncores independent copies of one oracle run at once, one per core (the
    oracle is single-threaded numpy): the host's aggregate rate."""
    ex = _spawn_pool(ncores)
    for _ in ex.map(int, range(ncores)):   # every worker started before the clock
        pass
    t0 = time.perf_counter()
    res = list(ex.map(_oracle_job, [name] * ncores))
    el = time.perf_counter() - t0
    ex.shutdown()
    desc, nsteps = ORACLE_JOBS[name]
    zu = sum(r["value"] * r["seconds"] for r in res)   # zone-updates done in all
    return dict(workload=desc, copies=ncores, seconds=el, value=zu / el,
                unit="zone-updates/s")


def finish_cpu_baseline(ex, futs, all_cores=True):
    res = {name: f.result() for name, f in futs.items()}
    ex.shutdown()
    smp = res["strat512-sample"]
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    out = dict(value=smp["value"], unit="zone-updates/s", cores=1, kind="oracle",
               sample=f"{smp['workload']}, numpy float64 on one thread, "
                      f"{smp['seconds']:.1f} s",
               threads_per_run=1, nproc=os.cpu_count(), cores_available=ncores,
               cpu_model=cpu_model(), omp_num_threads_of_runs=1, one_thread=res)
    if all_cores:
        # after the GPU timing, so that the oracle copies do not slow the
        # process that launches the GPU work
        out["all_cores"] = {name: all_cores_run(name, ncores) for name in ORACLE_JOBS}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="strat512")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "fp32_split"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-driver", action="store_true", help="skip the granulation-driver timing")
    ap.add_argument("--no-stretched", action="store_true",
                    help="skip the same box on the non-uniform z grid")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the eager vs HIP-graph timing of the small boxes")
    ap.add_argument("--no-ar1024", action="store_true",
                    help="skip the 1024x1024x256 active-region box (FP32-split)")
    ap.add_argument("--ar1024-steps", type=int, default=200,
                    help="timed steps of the 1024x1024x256 box (its workload runs 200)")
    ap.add_argument("--split-error-steps", type=int, default=100,
                    help="steps of the FP32-split vs FP64 error run (0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this implementation runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is a design note, not part of the build)", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration_mib:
        # a plain copy of known size: FETCH_SIZE/WRITE_SIZE per dispatch of this
        # kernel give the scale of the HBM counters
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "copies": args.steps}))
        return
    from paper_1908_08557_amd import workloads as W

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: oracle runs started in child processes")
        cpu = start_cpu_baseline()
    log(f"[bench] building workload {args.workload}")
    w = W.WORKLOADS[args.workload]()
    g = w.grid
    drivers = [W.driver_reseed(w, 100 + k) for k in range(4)]
    drivers = [torch.as_tensor(d, device="cuda") for d in drivers]
    res = {}
    precs = ["fp64", "fp32_split"] if args.precision == "both" else [args.precision]
    for prec in precs:
        log(f"[bench] {prec}: {args.warmup} warmup + {args.steps} timed steps")
        res[prec] = run_gpu(w, prec, args.steps, args.warmup, drivers)
        log(f"[bench] {prec}: {res[prec]}")
    main_prec = "fp64" if "fp64" in res else precs[0]
    r = res[main_prec]
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "ms_per_step_blocks": r["ms_per_step_blocks"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32-rhs/f64-state",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: stratified coronal box {g['nx']}x{g['ny']}x{g['nz']}, "
                               "solar boundaries, fixed dt, driver re-seeded every 10 steps",
                   "nx": g["nx"], "ny": g["ny"], "nz": g["nz"], "dt": r["dt"],
                   "precision": main_prec},
        "roofline": {"bound": "hbm", "achieved": r["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r["frac"], "traffic": None,
                     "kernel": "k_substage (fused z window, stencils, RHS and RK update "
                               "of one substage)",
                     "kernel_ms_per_launch": r["substage_ms"],
                     "ghosts_ms": r["ghosts_ms"],
                     "alg_bytes_per_launch": BYTES_PER_ZONE_STEP / 3.0 * g["nx"] * g["ny"] * g["nz"],
                     # the whole step (three substages and their boundary
                     # work) against the same 640 B per zone
                     "step_GBs": r["step_GBs"], "step_frac": r["step_GBs"] / HBM_PEAK_GBS},
        # dt by the CFL condition (cmhd_rk3_step with dt <= 0 adds this per step)
        "cfl_dt_ms": r["cfl_dt_ms"],
    }
    if "fp32_split" in res and main_prec == "fp64":
        s = res["fp32_split"]
        out["fp32_split"] = {"value": s["value"], "ms_per_step": s["ms_per_step"],
                             "speedup_vs_fp64": s["value"] / r["value"],
                             "roofline_frac": s["frac"],
                             "step_frac": s["step_GBs"] / HBM_PEAK_GBS,
                             "substage_ms": s["substage_ms"],
                             "ghosts_ms": s["ghosts_ms"]}
        if args.split_error_steps > 0:
            log(f"[bench] fp32_split vs fp64 error after {args.split_error_steps} steps")
            e, eo, azs = split_error(w, args.split_error_steps, drivers)
            log(f"[bench] split error: {e} (own maxima {eo})")
            out["fp32_split"]["rel_err_vs_fp64"] = e
            out["fp32_split"]["rel_err_vs_fp64_own_max"] = eo
            out["fp32_split"]["Az_residue_scale"] = azs
            out["fp32_split"]["rel_err_steps"] = args.split_error_steps
    # the HBM rate a plain device copy reaches on this GPU (read + write), the
    # practical ceiling beside the published peak
    cbw = copy_bandwidth()
    out["roofline"]["copy_GBs"] = cbw
    out["roofline"]["frac_of_copy"] = r["achieved_GBs"] / cbw
    tr = measured_traffic() if (w.name == "strat512" and main_prec == "fp64") else None
    if tr is not None:
        out["roofline"]["traffic"] = tr["hbm_bytes_per_substage"]
        out["roofline"]["traffic_GBs"] = tr["hbm_bytes_per_substage"] / (r["substage_ms"] * 1e-3) / 1e9
        out["roofline"]["traffic_source"] = tr["profile"]
        out["roofline"]["valu_busy_pct"] = tr["valu_busy_pct"]
    out["finite"] = all(v["finite"] for v in res.values())
    if not args.no_stretched and w.name == "strat512":
        # the same box on the paper's kind of z grid (100 km -> 800 km), FP64
        log("[bench] strat512_stretched fp64")
        ws = W.strat512_stretched()
        rs = run_gpu(ws, "fp64", max(args.steps // 2, 1), args.warmup,
                     [torch.as_tensor(W.driver_reseed(ws, 100 + k), device="cuda")
                      for k in range(2)])
        log(f"[bench] strat512_stretched: {rs}")
        out["stretched_z"] = {"workload": "strat512_stretched: 512x512x256, z spacing 0.1 -> "
                                          "0.8 Mm (top 141 Mm)",
                              "value": rs["value"], "ms_per_step": rs["ms_per_step"],
                              "substage_ms": rs["substage_ms"], "roofline_frac": rs["frac"],
                              "step_frac": rs["step_GBs"] / HBM_PEAK_GBS,
                              "steps": max(args.steps // 2, 1), "finite": rs["finite"]}
    if not args.no_ar1024 and w.name == "strat512":
        # the active-region box of the same physics, 1024 x 1024 x 256 over
        # 64 Mm with 32 bipoles, in the FP32-split form
        log("[bench] ar1024 fp32_split")
        wa = W.ar1024()
        ra = run_gpu(wa, "fp32_split", args.ar1024_steps, args.warmup,
                     [torch.as_tensor(W.driver_reseed(wa, 100 + k), device="cuda")
                      for k in range(4)])
        log(f"[bench] ar1024: {ra}")
        out["ar1024"] = {"workload": "ar1024: 1024x1024x256 over 64 Mm, 32 bipoles, FP32-split, "
                                     "driver re-seeded every 10 steps",
                         "value": ra["value"], "ms_per_step": ra["ms_per_step"],
                         "substage_ms": ra["substage_ms"], "roofline_frac": ra["frac"],
                         "step_frac": ra["step_GBs"] / HBM_PEAK_GBS,
                         "steps": args.ar1024_steps, "finite": ra["finite"]}
        del wa
    if not args.no_graph:
        log("[bench] small boxes, eager vs HIP graph")
        out["graph"] = [graph_bench(32, 24), graph_bench(64, 64)]
        log(f"[bench] graph: {out['graph']}")
    if not args.no_driver and g["zbc"] == "solar":
        log("[bench] granulation driver")
        out["driver"] = driver_bench(w, r["dt"], r["ms_per_step"])
        log(f"[bench] driver: {out['driver']}")
    if cpu is not None:
        log("[bench] cpu baseline: waiting for the oracle runs")
        out["cpu_baseline"] = finish_cpu_baseline(*cpu)
        log(f"[bench] cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
