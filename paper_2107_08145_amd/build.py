"""Build librts.so (gfx950) in-tree with hipcc: every translation unit is
compiled in parallel into paper_2107_08145_amd/_build, then linked."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "librts.so")
# the heaviest units first
SOURCES = ["rts_sweep_f8.hip", "rts_sweep_f6.hip", "rts_sweep_f4.hip", "rts_sweep_f2.hip",
           "rts_sweep_d4.hip", "rts_sweep_d2.hip", "rts_reverse_f.hip", "rts_reverse_d.hip",
           "rts_block.hip", "rts_gs.hip", "rts_misc.hip", "rts_static.hip", "rts_host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # every fused multiply-add is explicit in the source
         "-ffp-contract=off",
         # no packed FP32 instructions in any device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", "-o", obj, os.path.join(CSRC, src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n" + r.stdout + r.stderr)
    return obj


def build_librts(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    if verbose:
        print(f"{HIPCC} {' '.join(FLAGS)} -c <unit> ({len(SOURCES)} units, {jobs} jobs)", flush=True)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build_librts(verbose=True))
