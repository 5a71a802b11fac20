"""Build the kmvwave shared library (HIP for gfx950) in-tree.

    python -m paper_2108_10946_amd.build [--jobs N]

Compiles every source under csrc/ with hipcc and links
paper_2108_10946_amd/libkmvwave.so.  Packed-FP32 instructions are disabled for
device code (-packed-fp32-ops).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libkmvwave.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["element.cpp", "mesh.cpp", "problem.cpp", "server.cpp", "capi.cpp", "kernels.hip", "boundary.hip",
           "pml3d.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("KMV_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", BUILD, "-Wall", "-Wno-unused-result", "-pthread"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") or src == "problem.cpp" else []
    cmd = [HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (r.stderr or "").splitlines()
             if "packed-fp32-ops" not in l and l.strip() and "warning generated" not in l]
    return src, r.returncode, "\n".join(noise), obj


def generate_tables():
    """Compile and run gen_tables (host) -> _build/kmv_tables.inc."""
    exe = os.path.join(BUILD, "gen_tables")
    cmd = [os.environ.get("CXX", "g++"), "-O2", "-std=c++17", "-o", exe,
           os.path.join(CSRC, "gen_tables.cpp"), os.path.join(CSRC, "element.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"table generator failed to compile:\n{r.stderr}")
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    with open(os.path.join(BUILD, "kmv_tables.inc"), "w") as f:
        f.write(out)


def build(jobs: int = 0, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    generate_tables()
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, rc, err, obj in ex.map(_compile, SOURCES):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{err}")
            if err and verbose:
                print(f"[{src}]\n{err}", file=sys.stderr)
            objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    a = ap.parse_args()
    print(build(a.jobs))
