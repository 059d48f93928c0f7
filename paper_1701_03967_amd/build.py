"""Build libfftfem.so in-tree for gfx950.

    python -m paper_1701_03967_amd.build

The plan builder (113-bit host arithmetic) is compiled by g++; the C ABI and
the kernels by hipcc.  Packed-FP32 instructions are disabled for all device
code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfftfem.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# extra defines of the objects for element counts that are not powers of two
ANY_DEFINES = ()


def _run(cmd):
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {cmd[0]} ({r.returncode})")
    return time.time() - t


def _fresh(obj: str, srcs) -> bool:
    """The object exists and is newer than every source and header."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(x) < t for x in srcs)


def build(verbose: bool = True, lib: str = LIB, build_dir: str = BUILD, defines=(), any_defines=None,
          incremental: bool = False) -> str:
    """Compile and link the library.  `defines` (``NAME=VALUE`` strings) are
    passed to the kernel compiles, `any_defines` additionally to the objects
    for element counts that are not powers of two (default ANY_DEFINES),
    `lib` and `build_dir` place the outputs.  `incremental` keeps objects
    newer than every source and header of the library (same defines
    assumed); by default everything is compiled."""
    BUILD = build_dir
    LIB = lib
    dflags = [f"-D{d}" for d in defines]
    os.makedirs(BUILD, exist_ok=True)
    def deps(src):
        """The source and the project headers it includes, transitively."""
        seen, todo = set(), [os.path.join(CSRC, src)]
        while todo:
            f = todo.pop()
            if f in seen or not os.path.exists(f):
                continue
            seen.add(f)
            with open(f) as fh:
                for line in fh:
                    line = line.strip()
                    if line.startswith('#include "'):
                        h = line.split('"')[1]
                        todo += [os.path.join(CSRC, h), os.path.join(INCLUDE, h)]
        return sorted(seen)

    def keep(obj, src):
        return incremental and _fresh(obj, deps(src))

    objs = []
    plan_o = os.path.join(BUILD, "plan.o")
    if not keep(plan_o, "plan.cpp"):
        dt = _run(["g++", "-O2", "-std=gnu++17", "-fPIC", "-pthread", "-Wall", "-I", CSRC, "-I", INCLUDE,
                   "-c", os.path.join(CSRC, "plan.cpp"), "-o", plan_o])
        if verbose:
            print(f"[build] plan.cpp {dt:.1f}s", flush=True)
    objs.append(plan_o)
    for src in ("api.cpp", "batch.cpp"):
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        objs.append(obj)
        if keep(obj, src):
            continue
        dt = _run([HIPCC, "-O2", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", CSRC, "-I", INCLUDE,
                   "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose:
            print(f"[build] {src} {dt:.1f}s", flush=True)
    # kernels: line.hip six times (element counts that are powers of two,
    # other 7-smooth counts (mixed radix), all others (Bluestein); float32 or
    # float64), ops.hip once; compiled in parallel
    extra_any = [f"-D{d}" for d in (ANY_DEFINES if any_defines is None else any_defines)]
    units = [("line.hip", f"line_{name}_{real}.o", [f"-DFFTFEM_LINE_KIND={kind}", f"-DFFTFEM_LINE_REAL={real}"]
              + (extra_any if kind != 0 else []))
             for name, kind in (("p2", 0), ("mr", 1), ("bs", 2)) for real in ("float", "double")]
    units.append(("ops.hip", "ops.o", []))
    units.append(("band.hip", "band.o", []))
    units.append(("lift.hip", "lift.o", []))
    units.append(("long.hip", "long.o", []))

    def compile_unit(u):
        src, o, extra = u
        obj = os.path.join(BUILD, o)
        if keep(obj, src):
            return obj, f"{src} -> {o} (kept)", 0.0
        dt = _run([HIPCC, "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", *DEVICE_FLAGS, *dflags,
                   *extra, "-I", CSRC, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj, f"{src} -> {o}", dt

    with ThreadPoolExecutor(max_workers=len(units)) as ex:
        for obj, what, dt in ex.map(compile_unit, units):
            objs.append(obj)
            if verbose:
                print(f"[build] {what} {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build()
