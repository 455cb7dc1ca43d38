#!/usr/bin/env python3
"""Benchmark of the short-characteristics RTS on one MI355X.

Workload (default): 288^3 grid, four opacity bins plus the grey band (5
band sweeps), 24 rays (S4, three per octant), periodic x/y with 3 boundary
iterations, FP32 sweep with compensated partial sums and FP64 final
reduction; seeded synthetic stratified atmosphere.  A step is one complete
rts_solve: chi preparation, every sweep of every band and ray, and the final
reduction, with inputs already resident in HBM.

Prints one JSON line.  `value` is nominal cell-ray-band updates per second
(N * rays * bands per step); the timed calls are replays of one captured
hipGraph of the whole call (--no-graph: eager calls).  `roofline` describes
the sweep kernel, timed with HIP events on its stream inside the timed region
(event-record nodes of the replayed graph), against the published FP32 vector
peak.  `adjoint` is the adjoint / forward time on the 128^3 adjoint workload
with the training-step split.  `cpu_baseline` times the FP64 oracle on the
whole workload on this host's cores (at most 16 threads; about 15 s) and,
single-threaded, on a bounded sample of it.  The schedule (rows per strip,
queue order) is picked by the library's autotuner before the warm-up unless
--rows is given.

Other modes: --adjoint (adjoint/forward time on the 128^3 adjoint workload),
--workload boxes6 (six uneven boxes in one batched, graph-replayed call).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector (published; needs packed FP32 instructions)
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector (published)
# The sweep is bound by vector ALU issue (counters: VALU busy, HBM well below
# its peak).  The kernels issue no packed FP32 instructions, so their FP32 ALU
# peak is 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP (FMA) x 2.4 GHz = 78.6 TFLOP/s.
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FLOPS_PER_UPDATE = 32          # algorithmic FP operations of one D-form update: three bilinear
                               # interpolations 3 x 7, dtau 2, exp 1, c 2, the update 4, the sum 2


def sweep_model(p, plan_sched_tasks, esz):
    """Executed updates and algorithmic bytes of one sweep launch."""
    N = p.ncells
    executed = 0
    nbytes = 0
    for laps, nrays in plan_sched_tasks:
        executed += N * nrays * laps
        nbytes += laps * N * 2 * esz + N * esz   # chi and S per lap, one partial write
    return executed, nbytes


def task_list(p):
    """(laps, rays) of every sweep task of problem p: rays grouped by dominant
    axis and direction, four per task (equal spacing: 6 tasks per band)."""
    tasks = []
    d = (p.dx, p.dy, p.dz)
    groups = {}
    for m in p.mu:
        s = [d[a] / abs(m[a]) if m[a] != 0 else math.inf for a in range(3)]
        ax = max(a for a in range(3) if s[a] == min(s))
        groups.setdefault((ax, m[ax] > 0), []).append(m)
    for (ax, _), rays in groups.items():
        for i in range(0, len(rays), 4):
            tasks.append((1 if ax == 2 else p.n_iter, len(rays[i:i + 4])))
    return tasks * p.nbands


def kernel_hash(prefix="rts_sweep"):
    """Hash of a kernel's device sources (the files named prefix*, the device helpers and
    the shared structures; rts_sweep: the forward sweep, rts_reverse: the adjoint's reverse
    sweep): its counter summaries hold while it is unchanged."""
    d = os.path.join(ROOT, "paper_2107_08145_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.startswith(prefix) or f in ("rts_device.hpp", "rts_internal.h"):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, rows):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source and holds this strip height;
    else None."""
    f = os.path.join(ROOT, "profiles", f"rts_sweep_{workload}_pmc.json")
    if not os.path.exists(f):
        return None
    try:
        d = json.load(open(f))
    except ValueError:
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("by_rows", {}).get(str(rows), {}).get("hbm_bytes_per_launch")


COPY_BYTES = 1 << 30


def calibrate_copy():
    """A plain device copy of COPY_BYTES bytes: reads and writes exactly that many."""
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES}))


def _db_files(d):
    import glob
    return sorted(glob.glob(os.path.join(d, "**", "*.db"), recursive=True))


def _pmc_rows(d, counter):
    """(kernel name, value) of every dispatch in the rocprofv3 databases under d."""
    import sqlite3
    rows = []
    for f in _db_files(d):
        c = sqlite3.connect(f)
        q = ("select k.name, p.counter_value from pmc_events p join kernels k "
             "on p.dispatch_id = k.dispatch_id where p.counter_name = ?")
        rows += [(n, float(v)) for n, v in c.execute(q, (counter,)).fetchall()]
    return rows


def trace_summary(d, by_workgroup=False):
    """Per-kernel calls and mean duration from a rocprofv3 --kernel-trace database
    (per kernel and workgroup size with by_workgroup)."""
    import sqlite3
    out = []
    for f in _db_files(d):
        c = sqlite3.connect(f)
        if by_workgroup:
            q = ("select name || ' [workgroup ' || workgroup_x || ']', count(*), avg(duration), "
                 "sum(duration) from kernels group by name, workgroup_x "
                 "order by sum(duration) desc")
        else:
            q = ("select name, count(*), avg(duration), sum(duration) from kernels "
                 "group by name order by sum(duration) desc")
        out += [(n, k, a / 1e3, s / 1e6) for n, k, a, s in c.execute(q).fetchall()]
    return out


def counter_summary(dirs, key):
    """Per kernel whose name contains `key`: dispatches and the mean per dispatch of
    every counter in the rocprofv3 --pmc databases under `dirs` (instances summed)."""
    import sqlite3
    per = {}
    for d in dirs:
        for f in _db_files(d):
            c = sqlite3.connect(f)
            q = ("select k.name, p.dispatch_id, p.counter_name, sum(p.counter_value) from pmc_events p "
                 "join kernels k on p.dispatch_id = k.dispatch_id group by p.dispatch_id, p.counter_name")
            for name, disp, ctr, v in c.execute(q).fetchall():
                if key in name:
                    per.setdefault(name, {}).setdefault(ctr, []).append(float(v))
    out = {}
    for name, ctrs in per.items():
        out[name] = {ctr: {"dispatches": len(v), "mean": sum(v) / len(v)} for ctr, v in sorted(ctrs.items())}
    return out


def pmc_summary(workload, rows, fetch_dir, write_dir, cfetch_dir, cwrite_dir):
    """HBM bytes per sweep launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    scaled by the same counters' reading for the plain copy kernel.  Merged
    into the summary file by strip height while the kernel source is unchanged."""
    def per_kernel(d, counter, key):
        rows = [(n, x) for n, x in _pmc_rows(d, counter) if key in n]
        if not rows:
            return None
        names = [n for n, _ in rows]
        top = max(set(names), key=names.count)  # the variant the timed steps ran
        v = [x for n, x in rows if n == top]
        return sum(v) / len(v)
    f_sweep = per_kernel(fetch_dir, "FETCH_SIZE", "rts_sweep")
    w_sweep = per_kernel(write_dir, "WRITE_SIZE", "rts_sweep")
    rows_cf = [x for n, x in _pmc_rows(cfetch_dir, "FETCH_SIZE") if "copyBuffer" in n]
    rows_cw = [x for n, x in _pmc_rows(cwrite_dir, "WRITE_SIZE") if "copyBuffer" in n]
    cf = max(rows_cf) if rows_cf else None
    cw = max(rows_cw) if rows_cw else None
    kf = COPY_BYTES / (cf * 1024) if cf else None
    kw = COPY_BYTES / (cw * 1024) if cw else None
    entry = {"fetch_kib_per_dispatch": f_sweep, "write_kib_per_dispatch": w_sweep}
    if f_sweep and w_sweep and kf and kw:
        entry["hbm_bytes_per_launch"] = f_sweep * 1024 * kf + w_sweep * 1024 * kw
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    path = os.path.join(ROOT, "profiles", f"rts_sweep_{workload}_pmc.json")
    by_rows = {}
    if os.path.exists(path):
        try:
            old = json.load(open(path))
            if old.get("kernel_hash") == kernel_hash():
                by_rows = old.get("by_rows", {})
        except ValueError:
            pass
    by_rows[str(rows)] = entry
    out = {"workload": workload, "kernel": "rts_sweep", "kernel_hash": kernel_hash(),
           "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes": COPY_BYTES,
           "fetch_scale": kf, "write_scale": kw,
           "by_rows": dict(sorted(by_rows.items(), key=lambda kv: int(kv[0])))}
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p_full):
    """The FP64 oracle on this host's cores: all cores (at most 16, the host
    share of one GPU) on the whole workload (every band, ray and boundary
    iteration, the same synthetic inputs), and one thread on a bounded sample
    of it (the grey band on the bottom third of the layers)."""
    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(16, cores))
    q = p_full.astype(np.float64)
    oracle._load()
    t0 = time.perf_counter()
    ref = oracle.solve(q, threads=threads)
    dt = time.perf_counter() - t0
    nominal = q.ncells * q.nrays * q.nbands
    # single-thread sample: band nbands-1 (grey) of layers 0 .. nz/3
    from paper_2107_08145_amd import inputs
    nz1 = max(2, q.nz // 3)
    b = q.nbands - 1
    s1 = inputs.Problem(q.nx, q.ny, nz1, q.dx, q.dy, q.dz, q.mu, q.w,
                        np.ascontiguousarray(q.kappa[b:b + 1, :nz1]),
                        np.ascontiguousarray(q.rho[:nz1]),
                        np.ascontiguousarray(q.S[b:b + 1, :nz1]), np.ones(1),
                        q.bot, q.top, q.i_bot, q.n_iter)
    t0 = time.perf_counter()
    oracle.solve(s1, threads=1)
    dt1 = time.perf_counter() - t0
    nominal1 = s1.ncells * s1.nrays * s1.nbands
    return ref, {"value": nominal / dt, "unit": "cell-ray-band updates/s", "cores": threads,
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"FP64 oracle, the whole workload: {q.nx}x{q.ny}x{q.nz}, {q.nbands} bands, "
                      f"{q.nrays} rays, n_iter {q.n_iter} (OpenMP over the cells of a plane)",
            "nproc": os.cpu_count(), "affinity_cores": cores, "cpu_model": _cpu_model(),
            "single_thread": {"value": nominal1 / dt1, "unit": "cell-ray-band updates/s",
                              "cores": 1, "seconds": round(dt1, 2),
                              "sample": f"FP64 oracle, one thread: the grey band on layers "
                                        f"0..{nz1 - 1} ({q.nx}x{q.ny}x{nz1}, {q.nrays} rays, "
                                        f"n_iter {q.n_iter})"}}


def error_report(got, ref):
    """Errors of (Q, J, I_top) against the FP64 oracle: the paper's per-value
    validation rule (relative 1e-5 or absolute 1e-7, the latter taken of the
    array's largest magnitude: arbitrary units), its failing values, the
    normwise max|d|/max|ref| and the largest relative error over the values
    with |ref| >= 1e-3 max|ref|."""
    rep = {}
    for name, g, r in zip(("Q", "J", "I_top"), got, ref):
        d = np.abs(g - r)
        a = np.abs(r)
        m = a.max()
        ok = (d <= 1e-5 * a) | (d <= 1e-7 * m)
        big = a >= 1e-3 * m
        rep[name] = {"per_value_failures": int((~ok).sum()), "values": int(ok.size),
                     "normwise": float(d.max() / m),
                     "max_rel_over_1e-3_max": float((d[big] / a[big]).max())}
    return rep


def _time_calls(fn, steps, warmup):
    """Mean wall time (ms) of `steps` enqueued calls, synchronised on both sides."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def adjoint_measure(name, size, prec_name, steps, warmup):
    """Adjoint vs forward on the adjoint workload (128^3 grey by default).

    Loss: L = sum over the top layer and upward rays of (I_top - I_target)^2 +
    sum(g Q), I_target from the same solver on a 5 % perturbed S.  One adjoint
    call re-runs the forward sweep (storing D of every plane) and the reverse
    sweep; the forward reference is one rts_solve.  Also the training-step
    split: a forward that keeps D (rts_solve_for_adjoint) and a backward that
    only sweeps in reverse (rts_adjoint_from_solve)."""
    import torch
    from paper_2107_08145_amd import inputs, rts
    p = inputs.workload(name, size=size)
    prec = rts.RTS_FP32 if prec_name == "fp32" else rts.RTS_FP64
    pd = p.astype(np.float32 if prec == rts.RTS_FP32 else np.float64)
    s_target, g = inputs.adjoint_seeds(p, 4000)
    torch.cuda.set_device(0)
    plan = rts.Plan(pd, prec)
    ins = plan.device_inputs(pd)
    outs = plan.new_outputs(pd)
    tgt = pd.astype(pd.S.dtype)
    tgt.S = s_target.astype(pd.S.dtype)
    _, _, it_target = rts.solve(tgt, prec)
    plan.solve_into([ins], [outs])
    torch.cuda.synchronize()
    gI = (2 * (outs[2] - torch.as_tensor(it_target, device="cuda").to(outs[2].dtype))).contiguous()
    gQ = torch.as_tensor(g, device="cuda", dtype=torch.float64)
    dS = torch.empty_like(ins[2])
    dchi = torch.empty_like(ins[2])
    fwd_ms = _time_calls(lambda: plan.solve_into([ins], [outs]), steps, warmup)
    adj_ms = _time_calls(lambda: plan.adjoint_into([ins], [(gQ, None, gI)], [(dS, dchi)]),
                         steps, warmup)
    plan.check_status()
    keep_ms = _time_calls(lambda: plan.solve_for_adjoint_into([ins], [outs]), steps, warmup)
    back_ms = _time_calls(lambda: plan.adjoint_from_solve_into([ins], [(gQ, None, gI)], [(dS, dchi)]),
                          steps, warmup)
    plan.check_status()
    nominal = p.ncells * p.nrays * p.nbands
    return {"ratio": round(adj_ms / fwd_ms, 4), "adjoint_ms": round(adj_ms, 4),
            "forward_ms": round(fwd_ms, 4), "dtype": "f32" if prec == rts.RTS_FP32 else "f64",
            "adjoint_updates_per_s": nominal / (adj_ms * 1e-3),
            "workspace_bytes": plan.workspace_bytes(rts.RTS_OP_ADJOINT),
            "training_step": {"forward_keeping_d_ms": round(keep_ms, 4), "backward_ms": round(back_ms, 4),
                              "backward_over_forward": round(back_ms / fwd_ms, 3),
                              "step_over_forward": round((keep_ms + back_ms) / fwd_ms, 3)},
            "workload": f"{name}: {p.nx}x{p.ny}x{p.nz}, {p.nbands} band(s), {p.nrays} rays, "
                        f"n_iter {p.n_iter}; L = sum (I_top - I_target)^2 + sum g Q"}


def bench_adjoint(args):
    name = args.workload if args.workload != "bands288" else "adjoint128"
    a = adjoint_measure(name, args.size, args.prec, args.steps, args.warmup)
    out = {"metric": "adjoint time / forward time (RTS, reverse-mode dL/dS and dL/dchi)",
           "value": a["ratio"], "unit": "ratio", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": a["adjoint_ms"], "forward_ms": a["forward_ms"],
           "higher_is_better": False, "dtype": a["dtype"], "data": "synthetic",
           "adjoint_updates_per_s": a["adjoint_updates_per_s"],
           "workspace_bytes": a["workspace_bytes"], "training_step": a["training_step"],
           "config": {"workload": a["workload"]}}
    print(json.dumps(out), flush=True)


def bench_flux(args):
    """The radiative flux vector F and its divergence heating QF on the
    benchmark workload: one flux plan, autotuned with the flux outputs, timed
    with (F, QF) and without them (F = QF = NULL: the same kernels as the plain
    solve).  The flux's own kernels are timed with HIP events on the stream."""
    import torch
    from paper_2107_08145_amd import inputs, rts
    p = inputs.workload(args.workload, size=args.size)
    prec = rts.RTS_FP32 if args.prec == "fp32" else rts.RTS_FP64
    pd = p.astype(np.float32 if prec == rts.RTS_FP32 else np.float64)
    torch.cuda.set_device(0)
    plan = rts.Plan(pd, prec, flux=True)
    ins = plan.device_inputs(pd)
    outs = plan.new_outputs(pd, want_flux=True)
    if args.rows:
        plan.set_schedule(rows_per_strip=args.rows)
    else:
        plan.autotune([ins], [outs], reps=1)
    print(f"# flux plan schedule {plan.schedule()}", file=sys.stderr, flush=True)

    def timed(o):
        plan.enable_timing(True)
        ms = _time_calls(lambda: plan.solve_into([ins], [o]), args.steps, args.warmup)
        sweep_ms, call_ms = plan.last_timing()
        plan.enable_timing(False)
        plan.check_status()
        return ms, sweep_ms, call_ms
    ms_f, sw_f, call_f = timed(outs)
    ms_0, sw_0, call_0 = timed(outs[:3])
    print(f"# with flux {ms_f:.3f} ms (sweep {sw_f:.3f}), without {ms_0:.3f} ms (sweep {sw_0:.3f})",
          file=sys.stderr, flush=True)
    N = p.ncells
    nominal = N * p.nrays * p.nbands
    out = {"metric": "cell-ray-band updates/sec with the flux vector F and -div F "
                     "(288^3 4-band+grey 24-ray RTS)",
           "value": nominal / (ms_f * 1e-3), "unit": "cell-ray-band updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_f, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == rts.RTS_FP32 else "f64", "data": "synthetic",
           "sweep_ms": round(sw_f, 4), "call_ms": round(call_f, 4),
           "without_flux": {"ms_per_step": round(ms_0, 4), "sweep_ms": round(sw_0, 4),
                            "call_ms": round(call_0, 4)},
           "flux_overhead": round(ms_f / ms_0 - 1, 4),
           # flux partial writes: 3 x esz per cell, task and last lap; reduce_flux reads
           # them and S and writes F (3 x 8 B); the divergence reads F, writes QF
           "config": {"workload": f"{args.workload}: {p.nx}x{p.ny}x{p.nz}, {p.nbands} bands, "
                                  f"{p.nrays} rays, n_iter {p.n_iter}; outputs Q, J, I_top, F, QF",
                      "schedule": plan.schedule()}}
    if args.errors:
        import oracle
        plan.solve_into([ins], [outs])
        torch.cuda.synchronize()
        got = [o.double().cpu().numpy() for o in outs]
        ref = oracle.flux(pd.astype(np.float64), threads=16)
        scale = 4 * np.pi * np.abs(ref[1]).max()
        out["errors_vs_oracle"] = {
            "F_of_4pi_max_J": float(np.abs(got[3] - ref[3]).max() / scale),
            "F_of_max_F": float(np.abs(got[3] - ref[3]).max() / np.abs(ref[3]).max()),
            "QF_of_max_QF": float(np.abs(got[4] - ref[4]).max() / np.abs(ref[4]).max()),
            "Q": float(np.abs(got[0] - ref[0]).max() / np.abs(ref[0]).max())}
    print(json.dumps(out), flush=True)


def bench_gs(args):
    """Scattering with Gauss-Seidel source updates (FP64): the benchmark
    atmosphere (at --size, default 128^3) with a seeded photon destruction
    probability per cell, log-uniform in [1e-3, 1e-1], and --gs iterations.
    Timed eagerly and as graph replays (per iteration one launch per step over
    the groups, then one per plane of the last group's last lap); `value`
    counts the cell-ray-band updates of the iterations."""
    import torch
    from paper_2107_08145_amd import inputs, rts
    size = args.size or 128
    p = inputs.workload(args.workload, size=size).astype(np.float64)
    eps = 10 ** np.random.default_rng(9100).uniform(-3, -1, p.S.shape)
    torch.cuda.set_device(0)
    plan = rts.Plan(p, rts.RTS_FP64, gs_iter=args.gs)
    k, r, s = plan.device_inputs(p)
    e = torch.as_tensor(eps, device="cuda")
    Q, J, It = plan.new_outputs(p)
    S = torch.empty_like(J)
    ins, outs = [(k, r, s, e)], [(Q, J, It, None, None, S)]
    eager_ms = _time_calls(lambda: plan.solve_into(ins, outs), max(1, args.steps // 4), 1)
    plan.set_schedule(use_graph=1)
    plan.enable_timing(True)
    ms = _time_calls(lambda: plan.solve_into(ins, outs), args.steps, max(1, args.warmup))
    iter_ms, call_ms = plan.last_timing()
    plan.enable_timing(False)
    plan.check_status()
    tasks = task_list(p)
    executed = sum(p.ncells * nr * laps for laps, nr in tasks) * args.gs
    nominal = p.ncells * p.nrays * p.nbands * args.gs
    out = {"metric": "cell-ray-band updates/sec (Gauss-Seidel scattering, FP64)",
           "value": nominal / (ms * 1e-3), "unit": "cell-ray-band updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "graph_replay": True, "eager_ms_per_step": round(eager_ms, 4),
           "iterations_ms": round(iter_ms, 4), "ms_per_gs_iteration": round(iter_ms / args.gs, 4),
           "executed_updates_per_s": executed / (iter_ms * 1e-3),
           "config": {"workload": f"{args.workload} atmosphere at {p.nx}x{p.ny}x{p.nz}, {p.nbands} "
                                  f"bands, {p.nrays} rays, n_iter {p.n_iter}; eps log-uniform "
                                  f"in [1e-3, 1e-1]", "gs_iter": args.gs}}
    if args.errors:
        import oracle
        got = rts.solve_gs(p, eps, args.gs, plan=plan)
        ref = oracle.solve_gs(p, eps, args.gs)
        out["errors_vs_oracle"] = {n: float(np.abs(g - o).max() / np.abs(o).max())
                                   for n, g, o in zip(("Q", "J", "I_top", "S"), got, ref)}
    print(json.dumps(out), flush=True)


def bench_sub(args):
    """The subdomain decomposition with lagged exchange (the paper's domain-
    decomposed solver, emulated on one GPU): the benchmark workload cut into
    --sub MX MY MZ blocks, n_iter iterations (or until --tol), graph replay;
    the undivided solve of the same plan precision timed beside it.  `value`
    counts the nominal cell-ray-band updates per solve, as the headline."""
    import torch
    from paper_2107_08145_amd import inputs, rts
    p = inputs.workload(args.workload, size=args.size)
    prec = rts.RTS_FP32 if args.prec == "fp32" else rts.RTS_FP64
    pd = p.astype(np.float32 if prec == rts.RTS_FP32 else np.float64)
    torch.cuda.set_device(0)
    sub = tuple(args.sub)
    plan = rts.Plan(pd, prec, sub=sub, tol=args.tol)
    plan.set_schedule(use_graph=1)
    ins = plan.device_inputs(pd)
    outs = plan.new_outputs(pd)
    plan.enable_timing(True)
    ms = _time_calls(lambda: plan.solve_into([ins], [outs]), args.steps, args.warmup)
    iter_ms, call_ms = plan.last_timing()
    plan.enable_timing(False)
    plan.check_status()
    whole = rts.Plan(pd, prec)
    whole.set_schedule(use_graph=1)
    w_ms = _time_calls(lambda: whole.solve_into([ins], [whole.new_outputs(pd)]), args.steps, args.warmup)
    nominal = p.ncells * p.nrays * p.nbands
    out = {"metric": f"cell-ray-band updates/sec (RTS, {sub[0]}x{sub[1]}x{sub[2]} subdomains with "
                     "lagged exchange)",
           "value": nominal / (ms * 1e-3), "unit": "cell-ray-band updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == rts.RTS_FP32 else "f64", "data": "synthetic",
           "graph_replay": True, "iterations_ms": round(iter_ms, 4),
           "executed_updates_per_s": nominal * p.n_iter / (iter_ms * 1e-3),
           "undivided_ms_per_step": round(w_ms, 4),
           "config": {"workload": f"{args.workload}: {p.nx}x{p.ny}x{p.nz}, {p.nbands} bands, "
                                  f"{p.nrays} rays, n_iter {p.n_iter}", "sub": list(sub),
                      "tol": args.tol}}
    if args.errors:
        import oracle
        got = [t.double().cpu().numpy() for t in outs]
        ref = oracle.solve_sub(pd.astype(np.float64), sub, tol=args.tol, threads=16)
        out["errors_vs_oracle"] = error_report(got, ref[:3])
    print(json.dumps(out), flush=True)


def bench_warm(args):
    """Warm start under a tolerance: the benchmark workload and a copy whose
    S is perturbed by 1 % (seeded) alternate from call to call, as successive
    time steps would, each call either cold (initial ghost planes I = S) or
    started from the previous call's final ghost planes.  Eager calls (the
    ghost buffers alternate), same plan and tolerance."""
    import torch
    from paper_2107_08145_amd import inputs, rts
    p = inputs.workload(args.workload, size=args.size)
    prec = rts.RTS_FP32 if args.prec == "fp32" else rts.RTS_FP64
    dt = np.float32 if prec == rts.RTS_FP32 else np.float64
    q = p.astype(np.float64)
    q.S = p.S * (1 + 0.01 * np.random.default_rng(9200).standard_normal(p.S.shape))
    pd, qd = p.astype(dt), q.astype(dt)
    torch.cuda.set_device(0)
    plan = rts.Plan(pd, prec, tol=args.tol)
    ins = [plan.device_inputs(pd), plan.device_inputs(qd)]
    if args.rows:
        plan.set_schedule(rows_per_strip=args.rows)
    else:
        plan.autotune([ins[0]], [plan.new_outputs(pd)], reps=1)
    outs = plan.new_outputs(pd)
    shape = (p.nbands, p.nrays, p.nz, max(p.nx, p.ny))
    ghosts = [torch.zeros(shape, dtype=plan.dtype, device="cuda") for _ in range(2)]
    state = {"k": 0}

    def call(warm):
        k = state["k"]
        gin = ghosts[(k + 1) % 2] if warm and k > 0 else None
        plan.solve_into([tuple(ins[k % 2]) + (None, gin)],
                        [tuple(outs) + (None, None, None, ghosts[k % 2])])
        state["k"] = k + 1
    cold_ms = _time_calls(lambda: call(False), args.steps, args.warmup)
    state["k"] = 0
    warm_ms = _time_calls(lambda: call(True), args.steps, args.warmup)
    plan.check_status()
    nominal = p.ncells * p.nrays * p.nbands
    out = {"metric": "cell-ray-band updates/sec, tolerance-driven iteration with a warm start "
                     "(288^3 4-band+grey 24-ray RTS, 1 % perturbed atmospheres alternating)",
           "value": nominal / (warm_ms * 1e-3), "unit": "cell-ray-band updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(warm_ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == rts.RTS_FP32 else "f64", "data": "synthetic",
           "cold_ms_per_step": round(cold_ms, 4), "warm_over_cold": round(warm_ms / cold_ms, 4),
           "config": {"workload": f"{args.workload}: {p.nx}x{p.ny}x{p.nz}, {p.nbands} bands, "
                                  f"{p.nrays} rays, n_iter {p.n_iter} at most", "tol": args.tol,
                      "schedule": plan.schedule(), "graph_replay": False}}
    print(json.dumps(out), flush=True)


def bench_batched(args):
    """All boxes of the six-box workload in one rts_solve_batched call (graph replay)."""
    import torch
    from paper_2107_08145_amd import inputs, rts
    ps = inputs.workload("boxes6", size=args.size)
    prec = rts.RTS_FP32 if args.prec == "fp32" else rts.RTS_FP64
    pds = [p.astype(np.float32 if prec == rts.RTS_FP32 else np.float64) for p in ps]
    torch.cuda.set_device(0)
    plan = rts.Plan(pds, prec)
    ins = [plan.device_inputs(p) for p in pds]
    outs = [plan.new_outputs(p) for p in pds]
    if args.rows:
        plan.set_schedule(rows_per_strip=args.rows)
    else:
        plan.autotune(ins, outs, reps=1)
    plan.set_schedule(use_graph=1)
    if args.launch_form != "auto":
        plan.set_schedule(single_launch=int(args.launch_form == "single"))
    ms = _time_calls(lambda: plan.solve_into(ins, outs, batched=True), args.steps, args.warmup)
    plan.check_status()
    print(f"# batched forward {ms:.3f} ms", file=sys.stderr, flush=True)
    chosen = plan.schedule()
    other = None
    if args.launch_form == "auto":
        # the other launch form at the same strip height, for comparison
        plan.set_schedule(single_launch=1 - chosen["single_launch"])
        other_ms = _time_calls(lambda: plan.solve_into(ins, outs, batched=True), args.steps, 1)
        plan.check_status()
        plan.set_schedule(**chosen)
        other = {"single_launch": 1 - chosen["single_launch"], "ms_per_step": round(other_ms, 4)}
        print(f"# with single_launch={other['single_launch']}: {other_ms:.3f} ms",
              file=sys.stderr, flush=True)
    nominal = sum(p.ncells * p.nrays * p.nbands for p in ps)
    out = {"metric": "cell-ray-band updates/sec (six uneven boxes, 4-band+grey, 24 rays, batched)",
           "value": nominal / (ms * 1e-3), "unit": "cell-ray-band updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == rts.RTS_FP32 else "f64", "data": "synthetic",
           "config": {"workload": "boxes6: " + ", ".join(f"{p.nx}x{p.ny}x{p.nz}" for p in ps),
                      "schedule": chosen}}
    if other:
        out["other_launch_form"] = other
    if args.adjoint:
        # one rts_adjoint call over every box
        fwd_ms = ms
        seeds, grads, host = [], [], []
        for i, p in enumerate(ps):
            r = np.random.default_rng(5000 + i + 2)
            gq = r.random((p.nz, p.ny, p.nx))
            host.append(gq)
            seeds.append((torch.as_tensor(gq, device="cuda"), None, None))
            grads.append((torch.empty(p.S.shape, dtype=plan.dtype, device="cuda"),
                          torch.empty(p.S.shape, dtype=plan.dtype, device="cuda")))
        adj_ms = _time_calls(lambda: plan.adjoint_into(ins, seeds, grads), max(1, args.steps // 2), 1)
        plan.check_status()
        print(f"# adjoint of {len(ps)} boxes {adj_ms:.3f} ms, forward {fwd_ms:.3f} ms",
              file=sys.stderr, flush=True)
        out["adjoint"] = {"boxes": [f"{p.nx}x{p.ny}x{p.nz}" for p in ps],
                          "ms": round(adj_ms, 3), "forward_ms": round(fwd_ms, 3),
                          "ratio_to_forward": round(adj_ms / fwd_ms, 3),
                          "workspace_bytes": plan.workspace_bytes(rts.RTS_OP_ADJOINT)}
        if args.errors:
            # every box: <dL/dS, S> = L (L is linear in S) and the derivative
            # along rho -> rho (1 + h) (every band's chi) by central differences
            # of the FP64 forward; the two smallest boxes also against the
            # oracle's reverse mode (it keeps every sweep)
            import oracle
            got = [tuple(t.double().cpu().numpy() for t in g) for g in grads]
            # (the adjoint workspace fills most of HBM: the checks' own plans need it back)
            plan.release_workspace()
            del grads
            torch.cuda.empty_cache()
            errs = []
            for n, (p, pd, gq) in enumerate(zip(ps, pds, host)):
                q = pd.astype(np.float64)

                def loss(scale):
                    qq = q.astype(np.float64)
                    qq.rho = q.rho * scale
                    pl64 = rts.Plan(qq, rts.RTS_FP64)
                    pl64.set_schedule(rows_per_strip=4)
                    return float((gq * rts.solve(qq, rts.RTS_FP64, plan=pl64)[0]).sum())
                dS, dchi = got[n]
                L0, h = loss(1.0), 1e-3
                fd = (loss(1 + h) - loss(1 - h)) / (2 * h)
                chi = oracle.chi_of(q)
                e = {"box": f"{p.nx}x{p.ny}x{p.nz}",
                     "S_identity": abs(float((dS * q.S).sum()) - L0) / float(np.abs(dS * q.S).sum()),
                     "rho_derivative": abs(fd - float((dchi * chi).sum()))
                     / float(np.abs(dchi * chi).sum())}
                if p.ncells <= 5_000_000:
                    ref = oracle.adjoint(q, gq, threads=16)
                    e["dS_vs_oracle"] = float(np.abs(dS - ref[0]).max() / np.abs(ref[0]).max())
                    e["dchi_vs_oracle"] = float(np.abs(dchi - ref[1]).max() / np.abs(ref[1]).max())
                errs.append(e)
                print(f"# adjoint box {e}", file=sys.stderr, flush=True)
            out["adjoint"]["errors"] = errs
    if args.errors:
        import oracle
        plan.solve_into(ins, outs, batched=True)
        torch.cuda.synchronize()
        errs = []
        for p, pd, o in zip(ps, pds, outs):
            ref = oracle.solve(pd.astype(np.float64), threads=16)
            got = [t.double().cpu().numpy() for t in o]
            errs.append({"box": f"{p.nx}x{p.ny}x{p.nz}"} | error_report(got, ref))
            print(f"# box {errs[-1]}", file=sys.stderr, flush=True)
        out["errors_vs_oracle"] = errs
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bands288",
                    choices=["bands288", "grey288", "adjoint128", "boxes6"])
    ap.add_argument("--adjoint", action="store_true",
                    help="time rts_adjoint against rts_solve (default workload adjoint128)")
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=0.0,
                    help="tolerance-driven boundary iteration (n_iter sweeps at most)")
    ap.add_argument("--warm", action="store_true",
                    help="with --tol: successive calls on 1 %% perturbed atmospheres, cold against "
                         "warm-started from the previous call's final ghost planes")
    ap.add_argument("--sub", type=int, nargs=3, metavar=("MX", "MY", "MZ"),
                    help="subdomains with lagged exchange: blocks along x, y, z")
    ap.add_argument("--gs", type=int, default=0,
                    help="scattering with Gauss-Seidel source updates: this many iterations "
                         "(FP64; default size 128)")
    ap.add_argument("--flux", action="store_true",
                    help="time the solve with the flux vector F and -div F (flux plan)")
    ap.add_argument("--errors", action="store_true",
                    help="boxes6 and --flux: also the max relative errors against the oracle")
    ap.add_argument("--size", type=int, default=None, help="cube edge override (debug)")
    ap.add_argument("--rows", type=int, default=0,
                    help="rows per strip (0: chosen by the library's autotuner)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="default workload: skip the adjoint / forward measurement")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager calls instead of graph replays")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (scales rocprofv3 byte counters)")
    ap.add_argument("--trace-summary", metavar="TRACE_DIR",
                    help="print per-kernel mean durations of a rocprofv3 --kernel-trace run")
    ap.add_argument("--by-workgroup", action="store_true",
                    help="with --trace-summary: one line per kernel and workgroup size")
    ap.add_argument("--launch-form", choices=("auto", "per-width", "single"), default="auto",
                    help="boxes6: sweep launches per workgroup width or one launch (auto: the "
                         "plan's choice, and the other form timed beside it)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE runs into profiles/")
    ap.add_argument("--counter-summary", nargs="+", metavar="PMC_DIR",
                    help="print the mean per dispatch of every counter of rocprofv3 --pmc runs "
                         "for the kernels named by --kernel")
    ap.add_argument("--kernel", default="rts_", help="with --counter-summary: kernel name substring")
    ap.add_argument("--source-hash", metavar="PREFIX",
                    help="print the hash of the device sources of a kernel (rts_sweep, rts_reverse)")
    args = ap.parse_args()
    if args.source_hash:
        print(kernel_hash(args.source_hash))
        return
    if args.counter_summary:
        print(json.dumps(counter_summary(args.counter_summary, args.kernel), indent=1))
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.pmc_summary:
        pmc_summary(args.workload, args.rows, *args.pmc_summary)
        return
    if args.trace_summary:
        for n, k, avg_us, tot_ms in trace_summary(args.trace_summary, args.by_workgroup):
            if args.by_workgroup and "(" in n:   # drop the argument list
                n = n.split("(")[0] + " " + n[n.rfind("[workgroup"):]
            print(f"{avg_us:12.1f} us  x{k:4d}  {tot_ms:10.3f} ms  {n[:110]}")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2107_08145_amd import inputs, rts

    if args.workload == "boxes6":
        bench_batched(args)
        return
    if args.adjoint:
        bench_adjoint(args)
        return
    if args.flux:
        bench_flux(args)
        return
    if args.gs:
        bench_gs(args)
        return
    if args.sub:
        bench_sub(args)
        return
    if args.warm:
        if not args.tol > 0:
            print("--warm needs --tol > 0", file=sys.stderr)
            sys.exit(2)
        bench_warm(args)
        return
    t_gen = time.perf_counter()
    p = inputs.workload(args.workload, size=args.size)
    prec = rts.RTS_FP32 if args.prec == "fp32" else rts.RTS_FP64
    dt_np = np.float32 if prec == rts.RTS_FP32 else np.float64
    pd = p.astype(dt_np)
    print(f"# inputs generated in {time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    plan = rts.Plan(pd, prec, tol=args.tol)
    ins = plan.device_inputs(pd)
    outs = plan.new_outputs(pd)
    if args.rows:
        plan.set_schedule(rows_per_strip=args.rows)
        tuned = False
    else:
        t_tune = time.perf_counter()
        plan.autotune([ins], [outs], reps=2)
        tuned = True
        print(f"# autotuned in {time.perf_counter() - t_tune:.1f}s: {plan.schedule()}",
              file=sys.stderr, flush=True)
    # the whole call (prep, every sweep launch, reduce) replayed from one
    # captured hipGraph; timed calls record HIP events through event-record
    # nodes of the graph around the sweep launches and the call
    if not args.no_graph:
        plan.set_schedule(use_graph=1)
    torch.cuda.synchronize()
    plan.enable_timing(True)   # (the timed graph is captured during the warm-up)
    for _ in range(args.warmup):
        plan.solve_into([ins], [outs])
    plan.check_status()
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)

    plan.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve_into([ins], [outs])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms, call_ms = plan.last_timing()
    plan.enable_timing(False)
    plan.check_status()
    ms = (t1 - t0) * 1e3 / args.steps

    N = p.ncells
    nominal = N * p.nrays * p.nbands
    esz = 4 if prec == rts.RTS_FP32 else 8
    executed, alg_bytes = sweep_model(p, task_list(p), esz)
    sw_s = sweep_ms * 1e-3
    gbs = alg_bytes / sw_s / 1e9
    tflops = executed * FLOPS_PER_UPDATE / sw_s / 1e12
    peak_alu = PEAK_FP32_TFLOPS if prec == rts.RTS_FP32 else PEAK_FP64_TFLOPS
    traffic = (traffic_from_profile(args.workload, plan.schedule()["rows_per_strip"])
               if args.size is None else None)
    # The sweep is bound by vector ALU issue (VALU busy in the counters; its
    # HBM rate is a fraction of the peak): the roofline is the published FP32
    # (FP64) vector peak.  The HBM side is reported beside it.
    roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(peak_alu, 1),
            "unit": "TFLOP/s", "frac": round(tflops / peak_alu, 4)}
    if prec == rts.RTS_FP32:
        # the kernels issue no packed FP32 instructions: their own issue
        # rate is half the published vector peak
        roof["peak_nonpacked_fp32"] = round(PEAK_FP32_NONPACKED_TFLOPS, 1)
        roof["frac_of_nonpacked_peak"] = round(tflops / PEAK_FP32_NONPACKED_TFLOPS, 4)
    roof["traffic"] = traffic
    # measured HBM rate of the sweep: counter bytes per launch over the timed launch
    roof["traffic_GBs"] = round(traffic / sw_s / 1e9, 1) if traffic else None
    roof["kernel"] = "rts_sweep"
    roof["kernel_ms"] = round(sweep_ms, 4)
    roof["alg_bytes_per_launch"] = alg_bytes
    roof["alg_GBs"] = round(gbs, 1)
    roof["alg_hbm_frac"] = round(gbs / PEAK_HBM_GBS, 4)
    roof["alg_TFLOPs"] = round(tflops, 3)
    roof["executed_updates_per_launch"] = executed

    cfg = {"workload": f"{args.workload}: {p.nx}x{p.ny}x{p.nz}, {p.nbands} bands "
                       f"({'4 opacity bins + grey' if p.nbands == 5 else 'grey'}), "
                       f"{p.nrays} rays S4, n_iter {p.n_iter}, seeded stratified atmosphere",
           "grid": [p.nx, p.ny, p.nz], "bands": p.nbands, "rays": p.nrays, "n_iter": p.n_iter,
           "schedule": plan.schedule(), "autotuned": tuned, "sweep_ms": round(sweep_ms, 4),
           "tol": args.tol, "graph_replay": not args.no_graph,
           "call_ms": round(call_ms, 4), "executed_updates_per_s": executed / (ms * 1e-3)}
    out = {"metric": "cell-ray-band updates/sec (288^3 4-band+grey 24-ray RTS)",
           "value": nominal / (ms * 1e-3), "unit": "cell-ray-band updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if prec == rts.RTS_FP32 else "f64", "data": "synthetic",
           "config": cfg, "roofline": roof}
    if not args.no_adjoint and args.size is None:
        # adjoint / forward time on the 128^3 adjoint workload, same precision
        print("# adjoint (adjoint128)...", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_measure("adjoint128", None, args.prec, args.steps, args.warmup)
    if not args.no_cpu and args.size is None:
        print("# cpu baseline (oracle)...", file=sys.stderr, flush=True)
        # the oracle on the inputs the GPU solved (FP32-rounded in an FP32
        # plan); its result also gives the errors of the timed calls' outputs
        got = [o.double().cpu().numpy() for o in outs]
        ref, out["cpu_baseline"] = cpu_baseline(pd)
        out["errors_vs_oracle"] = error_report(got, ref)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
