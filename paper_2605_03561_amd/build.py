"""Build the HIP shared libraries in-tree for gfx950.

``python -m paper_2605_03561_amd.build`` compiles ``csrc/*.hip`` into
``libta.so`` (the C-ABI library) and ``csrc/synth/*.hip`` into
``libta_synth.so`` (the synthetic-trace generator used by the benchmark).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{os.path.join(ROOT, 'include')}",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _run(cmd, what):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {what}")


def _compile(sources, out, extra=()):
    """Compiles each source to an object in parallel, then links the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in sources]
    jobs = int(os.environ.get("MAX_JOBS", "0")) or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(sources)))) as ex:
        futs = [ex.submit(_run, [_hipcc(), *HIPCC_FLAGS, *extra, "-c", "-o", o, src], src)
                for src, o in zip(sources, objs)]
        for f in futs:
            f.result()
    tmp = out + ".tmp"
    _run([_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], out)
    os.replace(tmp, out)
    return out


def build_ta() -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    return _compile(srcs, os.path.join(HERE, "libta.so"))


def build_synth() -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "synth", "*.hip")))
    if not srcs:
        return ""
    return _compile(srcs, os.path.join(HERE, "libta_synth.so"))


def build_all() -> list[str]:
    return [p for p in (build_ta(), build_synth()) if p]


if __name__ == "__main__":
    for p in build_all():
        print(p)
