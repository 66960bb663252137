"""Build libboxtile.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1604_03570_amd.build          # full rebuild
    python -m paper_1604_03570_amd.build --quick  # recompile changed sources only
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libboxtile.so")
SOURCES = ["bl_meta.cpp", "bl_api.cpp", "bl_kernels.hip"]
HEADERS = ["bl_internal.h", "bl_launch.h"]
ARCH = os.environ.get("BOXTILE_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags() -> list:
    return [
        f"--offload-arch={ARCH}",
        "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
        # every cell update is one fixed expression: no FMA contraction anywhere
        "-ffp-contract=off",
        # keep the compiler from forming packed-FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        f"-I{INCLUDE}",
    ]


def _obj(src: str) -> str:
    return os.path.join(BUILD, os.path.splitext(src)[0] + ".o")


def _stale(src: str) -> bool:
    o = _obj(src)
    if not os.path.exists(o):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in HEADERS] + \
        [os.path.join(INCLUDE, "boxtile.h")]
    return any(os.path.getmtime(d) > os.path.getmtime(o) for d in deps)


def _compile(src: str) -> str:
    cmd = [hipcc()] + common_flags() + ["-c", os.path.join(CSRC, src), "-o", _obj(src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    noise = "'-packed-fp32-ops' is not a recognized feature"
    return "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)


def build(quick: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    todo = [s for s in SOURCES if not quick or _stale(s)]
    with cf.ThreadPoolExecutor(max_workers=min(4, max(1, len(todo)))) as ex:
        for src, warn in zip(todo, ex.map(_compile, todo)):
            if verbose and warn.strip():
                print(f"[{src}]\n{warn}", file=sys.stderr)
    if todo or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [_obj(s) for s in SOURCES]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}" + (f" (recompiled {', '.join(todo)})" if todo else " (up to date)"))
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true")
    args = ap.parse_args()
    build(quick=args.quick)
