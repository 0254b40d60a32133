"""Build libmuffin.so in-tree for gfx950.

HIP translation units go through hipcc (one process per file, in parallel);
the host-only C ABI units through g++ against the HIP headers.  The library
lands next to this file, where the Python binding loads it.

    python -m paper_1504_06847_amd.build [--jobs N] [--verbose]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmuffin.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_SOURCES = ["muffin_fft.hip", "muffin_spectral.hip", "muffin_adjoint.hip", "muffin_fused.hip",
               "muffin_wavelet.hip", "muffin_noalloc.hip", "muffin_vis.hip"]
HOST_SOURCES = ["muffin_validate.cpp", "muffin_api.cpp", "muffin_batch.cpp", "muffin_dict.cpp", "muffin_vis.cpp"]

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             # packed FP32 instructions stay disabled on this target
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def _stale(obj: str, src: str) -> bool:
    """An object older than its source or than any header it may include."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    deps += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE)]
    return any(os.path.getmtime(d) > t for d in deps)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit (with ``incremental``, only those whose
    object is older than the source or a header) and link libmuffin.so."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    gxx = shutil.which("g++") or "g++"
    os.makedirs(BUILD, exist_ok=True)
    incs = [f"-I{INCLUDE}", f"-I{CSRC}"]
    cmds = []
    objs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        path = os.path.join(CSRC, src)
        if not incremental or _stale(obj, path):
            cmds.append([hipcc, *HIP_FLAGS, *incs, "-c", path, "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        path = os.path.join(CSRC, src)
        if not incremental or _stale(obj, path):
            cmds.append([gxx, *HOST_FLAGS, *incs, "-c", path, "-o", obj])
        objs.append(obj)
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 4))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for r in ex.map(lambda c: _run(c, verbose), cmds):
            if r.stderr and verbose:
                print(r.stderr, file=sys.stderr)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp,
          f"-L{ROCM}/lib", "-lamdhip64"], verbose)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true",
                    help="recompile only units older than their source or a header")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose, a.incremental))


if __name__ == "__main__":
    main()
