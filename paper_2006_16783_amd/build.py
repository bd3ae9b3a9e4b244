"""Builds libsiting.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsiting.so")
ARCH = os.environ.get("SITING_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA results in ordinary VGPRs (no accumulator-register copies)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


# Extra device-pass flags per source, measured with identical results.  The
# LDS-tile VIX kernels (vix.hip; issue-bound integer work with LDS reads in
# blocks) and SITE (one wavefront, latency-bound) are scheduled for
# instruction-level parallelism: at 46400^2, ROI 100, VIX 176.0 ms against
# 176.7 ms with the default scheduler, SITE 16.7 ms against 17.6 ms.  The
# global-read VIX kernels (vix_global.hip, large ROI) keep the default: with
# it 3.23 s against 3.43 s at 16384^2, ROI 500.  VIEWSHED gained nothing from
# it (5.88 / 5.90 ms).
_ILP = ["-Xarch_device", "-mllvm=-misched=gcn-max-ilp"]
FILE_FLAGS = {
    "vix.hip": _ILP,
    "greedy.hip": _ILP,
}


def flags_of(name: str):
    """Every compile flag a source is built with (also keys profile records)."""
    return [*HIPCC_FLAGS, *FILE_FLAGS.get(name, [])]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel, each with its own flags) and link
    them into paper_2006_16783_amd/libsiting.so."""
    import tempfile
    srcs = sources()
    inc = ["-I", os.path.join(HERE, "..", "include")]
    with tempfile.TemporaryDirectory(prefix="siting_build_") as tmpd:
        procs, objs = [], []
        for src in srcs:
            name = os.path.basename(src)
            obj = os.path.join(tmpd, name + ".o")
            cflags = [f for f in flags_of(name) if f != "-shared"]
            cmd = [hipcc(), *cflags, *inc, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((name, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                 stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        failed = False
        for name, pr in procs:
            out, _ = pr.communicate()
            if pr.returncode != 0:
                failed = True
                sys.stderr.write(out)
            elif verbose and out.strip():
                sys.stderr.write(out)
        if failed:
            raise RuntimeError("hipcc failed building libsiting.so")
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}",
               "-Wl,--version-script=" + os.path.join(CSRC, "exports.map"), "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libsiting.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
