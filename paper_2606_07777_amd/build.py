"""Builds libdualip.so for gfx950 with hipcc, in-tree next to this file."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdualip.so")
SOURCES = ["dl_problem.hip", "dl_grad.hip", "dl_solver.hip", "dl_batch.hip", "dl_mlp.hip", "dl_measure.hip"]
# The gradient-pass kernels are compiled once per variant (families class,
# stored a, BF16 storage), each build its own object, so they compile in parallel.
GRAD_VARIANTS = [(1, 0, 0), (1, 0, 1), (1, 1, 0), (1, 1, 1), (2, 1, 0), (2, 1, 1), (4, 1, 0), (4, 1, 1)]
# The gradient pass never forms a NaN (its inputs are checked finite and its
# padding lanes are kept at -inf / 0), so its float min / max need no NaN
# quieting; the other sources keep IEEE NaN semantics (their divergence checks
# test for NaN).
GRAD_FLAGS = ["-fno-honor-nans"]


def _units():
    units = [(src, src.replace(".hip", ".o"), [], []) for src in SOURCES]
    for mf, a, bf in GRAD_VARIANTS:
        units.append(("dl_grad_variant.hip", f"dl_grad_v_{mf}_{a}_{bf}.o",
                      [f"DL_GV_MF={mf}", f"DL_GV_A={a}", f"DL_GV_BF16={bf}"], GRAD_FLAGS))
    return units


HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 (v_pk_*_f32) stays off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, out: str = LIB, defines=(), objdir: str = None) -> str:
    """Compiles every source to an object, then links the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = objdir or os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src, oname, unit_defs, unit_flags in _units():
        obj = os.path.join(objdir, oname)
        objs.append(obj)
        cmd = [hipcc, *HIPCC_FLAGS, *unit_flags, *[f"-D{d}" for d in (*defines, *unit_defs)], "-I", INCLUDE, "-I", CSRC,
               "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((oname, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    failed = []
    for src, p in procs:
        log, _ = p.communicate()
        log = "\n".join(l for l in log.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(log + "\n")
        elif verbose and log.strip():
            print(log)
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = out + ".tmp"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
