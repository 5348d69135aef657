"""Build libarbgpu.so (HIP for gfx950) in-tree.

    python -m paper_1901_04289_amd.build [-j JOBS]

Every .hip translation unit is compiled to an object under _build/, the
limb-kernel instantiations once per (window limbs, operand limbs) shape
listed in csrc/limb_shapes.def, and everything is linked into
paper_1901_04289_amd/libarbgpu.so.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libarbgpu.so")

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I" + os.path.join(ROOT, "include"),
]


def limb_shapes():
    txt = open(os.path.join(CSRC, "limb_shapes.def")).read()
    return [(int(a), int(b)) for a, b in re.findall(r"X\((\d+),\s*(\d+)\)", txt)]


# The limb kernels keep whole multi-limb products in registers: their fully
# unrolled multiply chains exceed the default size limit of requested unrolls.
LIMB_FLAGS = ["-mllvm", "-pragma-unroll-threshold=200000"]


# The FP64 matrix-core loops (radius products, machine-limit probes) keep
# their accumulators in ordinary vector registers; without this the
# loop-carried accumulators are copied to and from the accumulation
# registers around every multiply.
FILE_FLAGS = {"peaks.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
              "radius.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str, obj: str, defines=()):
    extra = (LIMB_FLAGS if defines else []) + FILE_FLAGS.get(os.path.basename(src), [])
    cmd = [HIPCC] + CFLAGS + extra + [f"-D{d}" for d in defines] + ["-c", src, "-o", obj]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, time.time() - t


def build(jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    units = []
    for name in sorted(os.listdir(CSRC)):
        if not name.endswith(".hip") or name == "limb_inst.hip":
            continue
        units.append((os.path.join(CSRC, name), os.path.join(BUILD, name[:-4] + ".o"), ()))
    for ns, na in limb_shapes():
        units.append((os.path.join(CSRC, "limb_inst.hip"),
                      os.path.join(BUILD, f"limb_inst_{ns}_{na}.o"), (f"ARB_NS={ns}", f"ARB_NA={na}")))
    # slowest (widest) shapes first
    units.sort(key=lambda u: -sum(int(x.split("=")[1]) for x in u[2]) if u[2] else 0)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, *u) for u in units]
        for f in cf.as_completed(futs):
            obj, dt = f.result()
            objs.append(obj)
            if verbose:
                print(f"  {os.path.basename(obj)} {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + sorted(objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=0)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    t = time.time()
    path = build(a.jobs, a.verbose)
    print(f"built {path} in {time.time() - t:.1f}s")


if __name__ == "__main__":
    sys.exit(main())
