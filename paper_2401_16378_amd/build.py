"""Build libpauli.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2401_16378_amd.build [-j JOBS]

Each source compiles to an object under _build/, then one shared library is
linked next to this file.  All device code is compiled for gfx950 with packed
FP32 instructions disabled.

The compiler's per-kernel resource report is read for every kernel: a kernel
that needs scratch memory (register spills or a private stack) fails the
build, so a shape that outgrows the register file cannot ship unnoticed.  The
report of the last build is written to _build/resource_usage.txt.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpauli.so")
ARCH = "gfx950"
SOURCES = ["api.cpp", "gray_fp64.hip", "mfma.hip", "mfma_i8.hip", "batched.hip", "strings.hip", "fwht.hip"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]
REMARKS = "-Rpass-analysis=kernel-resource-usage"
_REMARK = re.compile(r"remark:\s+(Function Name|ScratchSize \[bytes/lane\]|VGPRs Spill|SGPRs Spill"
                     r"|VGPRs|AGPRs|Occupancy \[waves/SIMD\]|Dynamic Stack):\s*(\S+)")


def resource_usage(text: str) -> list:
    """Per-kernel records {name, ScratchSize, VGPRs, ...} from the remarks."""
    kernels = []
    for key, val in _REMARK.findall(text):
        if key == "Function Name":
            kernels.append({"name": val})
        elif kernels:
            kernels[-1][key.split(" [")[0]] = val
    return kernels


def _compile(src: str):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *FLAGS, REMARKS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    usage = resource_usage(r.stdout)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l
                    and not re.match(r"^\s*(\d+ \|.*|\|\s*\^)\s*$", l))
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, out))
    if out.strip():
        print(out)
    return obj, usage


def check_no_scratch(usage: dict) -> None:
    bad = ["%s: %s (scratch %s B/lane, VGPR spill %s, SGPR spill %s, dynamic stack %s)"
           % (src, k["name"], k.get("ScratchSize"), k.get("VGPRs Spill"), k.get("SGPRs Spill"),
              k.get("Dynamic Stack"))
           for src, ks in usage.items() for k in ks
           if k.get("ScratchSize", "0") != "0" or k.get("VGPRs Spill", "0") != "0"
           or k.get("SGPRs Spill", "0") != "0" or k.get("Dynamic Stack", "False") != "False"]
    if bad:
        raise RuntimeError("kernels that need scratch memory:\n  " + "\n  ".join(bad))


def build(jobs: int = 4) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    usage = {src: u for src, (_, u) in zip(SOURCES, results)}
    with open(os.path.join(BUILD, "resource_usage.txt"), "w") as f:
        for src, ks in usage.items():
            for k in ks:
                f.write("%s %s\n" % (src, " ".join("%s=%s" % (a.replace(" ", "_"), b) for a, b in k.items())))
    if not any(usage.values()):
        raise RuntimeError("the compiler printed no kernel resource report")
    check_no_scratch(usage)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, *objs]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=4)
    a = ap.parse_args()
    print(build(a.jobs))
    sys.exit(0)
