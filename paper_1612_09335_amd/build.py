"""Build ``libcweno.so`` in-tree: host precompute (g++) + gfx950 kernels (hipcc).

Usage: ``python paper_1612_09335_amd/build.py`` (run by path: importing the
package loads the library it builds), or ``__graft_entry__.build()``.
Every call recompiles every source.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcweno.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"

HOST_SOURCES = ["host_geometry.cpp", "host_basis.cpp", "host_operators.cpp", "host_halo.cpp"]
HIP_SOURCES = ["abi.hip", "batch.hip", "server.hip", "moving.hip", "evaluate.hip", "weno.hip"]
# kernels.hip and moving_kernels.hip are compiled once per (precision, dimension, degree)
KERNEL_UNITS = [(tn, d, m) for tn in ("f64", "f32") for d in (2, 3) for m in (1, 2, 3, 4)]
KERNEL_FILES = ["kernels", "moving_kernels"]

# Integer tables depend on exact floating-point comparisons: no contraction.
HOST_FLAGS = ["-std=c++17", "-O3", "-fPIC", "-pthread", "-ffp-contract=off", "-Wall", "-Wextra",
              f"-I{INCLUDE}", f"-I{ROCM}/include", "-D__HIP_PLATFORM_AMD__"]
HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link ``libcweno.so`` next to this file."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    host_objs = [os.path.join(BUILD, src + ".o") for src in HOST_SOURCES]
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_run, [["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
                           for src, obj in zip(HOST_SOURCES, host_objs)]))
    # the universal Sigma matrices become compile-time constants of the kernels
    gen = os.path.join(BUILD, "gen_sigma")
    _run(["g++", *HOST_FLAGS, "-o", gen, os.path.join(CSRC, "gen_sigma.cpp"), *host_objs])
    _run([gen, os.path.join(BUILD, "sigma_tables.hpp")])
    cmds = []
    objs = list(host_objs)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmds.append([HIPCC, *HIP_FLAGS, f"-I{BUILD}", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # the heaviest units first, so that they do not finish last on their own
    units = sorted(((f, tn, d, m) for f in KERNEL_FILES for tn, d, m in KERNEL_UNITS),
                   key=lambda u: (u[0] != "moving_kernels", -u[2], -u[3]))
    for f, tn, d, m in units:
        obj = os.path.join(BUILD, f"{f}_{tn}_d{d}_m{m}.o")
        cmds.append([HIPCC, *HIP_FLAGS, f"-I{BUILD}", f"-DCWENO_TN={tn}", f"-DCWENO_D={d}", f"-DCWENO_M={m}", "-c",
                     os.path.join(CSRC, f + ".hip"), "-o", obj])
        objs.append(obj)
    with cf.ThreadPoolExecutor(jobs) as ex:
        for cmd, out in zip(cmds, ex.map(_run, cmds)):
            if verbose:
                print(" ".join(cmd))
                if out.strip():
                    print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-pthread", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
