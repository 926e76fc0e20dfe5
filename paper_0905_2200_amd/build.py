"""Build libfe.so (HIP, gfx950) in place: ``python -m paper_0905_2200_amd.build``."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfe.so")
SOURCES = ["fe_kernels.hip", "fe_tiling.hip", "fe_host.hip"] + ["fe_map_n%d.hip" % n for n in range(1, 9)]
ARCH = os.environ.get("FE_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        jobs.append(([HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj], obj))

    def run(job):
        cmd, _ = job
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return r.returncode, cmd, r.stdout

    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(run, jobs))
    failed = [(cmd, out) for rc, cmd, out in results if rc != 0]
    for _, _, out in results:
        msg = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if msg.strip() and (verbose or failed):
            print(msg, file=sys.stderr)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(c[-3] for c, _ in failed))
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
