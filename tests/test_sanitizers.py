"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle, rebuilt with -fsanitize=address,undefined (every finding
  fatal), runs each of its entry points on small problems in a subprocess
  with the ASan runtime preloaded.
* The library's host planner (rts_host.cpp: validation, task building,
  workspace layout, schedules, the refusals before any device call), rebuilt
  with the sanitizers on its host code only, runs plan creation over a range
  of problems and schedules in a subprocess; no GPU is touched (the device
  objects are linked but never launched).
"""
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _asan_runtime():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    p = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("no ASan runtime")
    return p


def _run(script, env_extra, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env,
                       timeout=timeout, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-fno-fast-math", "-fopenmp", *SAN, "-o", str(lib),
                    os.path.join(ROOT, "oracle", "rts_oracle.cpp")], check=True)
    script = textwrap.dedent(f"""
        import numpy as np, oracle
        from paper_2107_08145_amd import inputs
        oracle._LIB = {str(lib)!r}
        oracle._lib = None
        p = inputs.random_problem(7, 6, 5, seed=3, bands=2, n_iter=2)
        oracle.solve(p, threads=2)
        oracle.solve_dform(p)
        oracle.flux(p, threads=2)
        oracle.solve_tol(p, 1e-3, threads=2)
        oracle.solve_sub(p, (2, 3, 2), threads=2)
        oracle.solve_sub(p, (2, 1, 1), tol=1e-3, threads=2)
        oracle.solve_warm(p, oracle.solve_warm(p)[3], tol=1e-3)
        oracle.solve_gs(p, np.full(p.S.shape, 0.3), 2)
        r = np.random.default_rng(1)
        oracle.adjoint(p, r.random((p.nz, p.ny, p.nx)), r.random(p.S.shape),
                       r.random((p.nbands, p.n_up, p.ny, p.nx)), threads=2)
        oracle.complex_step(p, "chi", 11, threads=2)
        q = inputs.random_problem(2, 2, 2, seed=4)
        oracle.solve(q)
        print("oracle ok")
    """)
    out = _run(script, {"LD_PRELOAD": rt})
    assert "oracle ok" in out


def test_host_planner_under_asan_and_ubsan(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = os.path.join(ROOT, "paper_2107_08145_amd", "_build")
    if not os.path.exists(hipcc) or not os.path.isdir(objs):
        pytest.skip("hipcc or the library's objects are missing")
    # hipcc's host compiler is clang: its own ASan runtime (which carries the
    # UBSan handlers) is preloaded, not gcc's
    rt = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip().splitlines()[-1:]
    rt = rt[0] if rt else ""
    if not os.path.isabs(rt) or not os.path.exists(rt):
        import glob
        cands = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not cands:
            pytest.skip("no clang ASan runtime")
        rt = cands[0]
    dev = sorted(os.path.join(objs, f) for f in os.listdir(objs)
                 if f.endswith(".o") and f != "rts_host.o")
    host_o = tmp_path / "rts_host_san.o"
    lib = tmp_path / "librts_san.so"
    xh = [a for s in SAN for a in ("-Xarch_host", s)]  # sanitize the host code only
    subprocess.run([hipcc, "-O1", "-g", "-std=c++17", "-fPIC", *xh, "-c", "-o", str(host_o),
                    os.path.join(ROOT, "paper_2107_08145_amd", "csrc", "rts_host.cpp")], check=True)
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *xh, "-Xarch_host",
                    "-shared-libsan", "-o", str(lib),
                    str(host_o), *dev], check=True)
    script = textwrap.dedent(f"""
        import ctypes, numpy as np
        from paper_2107_08145_amd import inputs, rts
        rts.LIB_PATH = {str(lib)!r}
        rts._lib = None
        L = rts.lib()
        n = 0
        for shape, kw in [((8, 6, 5), {{}}), ((17, 9, 12), dict(bands=3, n_iter=4)),
                          ((2, 2, 2), {{}}), ((600, 3, 4), {{}}), ((33, 577, 3), dict(bands=2))]:
            p = inputs.random_problem(*shape, seed=n, **kw)
            for prec in (rts.RTS_FP64, rts.RTS_FP32):
                for extra in ({{}}, dict(flux=True), dict(tol=1e-3), dict(sub=(2, 1, 2))):
                    try:
                        pl = rts.Plan(p, prec, **extra)
                    except rts.RTSError:
                        continue
                    for op in (rts.RTS_OP_SOLVE, rts.RTS_OP_ADJOINT, rts.RTS_OP_AUTOTUNE):
                        pl.workspace_bytes(op)
                    for rows in ((2, 4, 6, 8) if prec == rts.RTS_FP32 else (2, 4)):
                        pl.set_schedule(rows_per_strip=rows, split_reverse=rows % 4 == 0,
                                        single_launch=rows == 2)
                        pl.workspace_bytes(rts.RTS_OP_ADJOINT)
                    ci, co = rts.Inputs(256, 256, 256), rts.Outputs(256, None, None)
                    assert L.rts_solve(pl.handle, ctypes.byref(ci), ctypes.byref(co), None, 0,
                                       None) == rts.RTS_E_WORKSPACE
                    n += 1
            try:
                rts.Plan(p, rts.RTS_FP64, gs_iter=2)
                n += 1
            except rts.RTSError:
                pass
        # a multi-box plan and rejected descriptions
        rts.Plan([inputs.random_problem(9, 7, 5, seed=8), inputs.random_problem(12, 5, 6, seed=9)],
                 rts.RTS_FP32)
        bad = inputs.random_problem(5, 5, 5, seed=10)
        bad.mu = bad.mu.copy(); bad.mu[3, 2] = 0.0
        try:
            rts.Plan(bad)
        except rts.RTSError:
            pass
        print("planner ok", n)
    """)
    out = _run(script, {"LD_PRELOAD": rt})
    assert "planner ok" in out
