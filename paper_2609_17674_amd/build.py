"""Build step for libsmcx.so (hipcc, gfx950) — compiled in-tree."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsmcx.so")
ROOT = os.path.dirname(HERE)

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # rounding is controlled explicitly with fma() where a fused op is wanted
    "-ffp-contract=off",
    # no packed FP32 instructions on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, obj: str) -> subprocess.CompletedProcess:
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    return subprocess.run([hipcc()] + flags + ["-c", "-o", obj, src], capture_output=True,
                          text=True)


def build_library(force: bool = True, verbose: bool = False, jobs: int = 0) -> str:
    """Compile every csrc/*.hip into libsmcx.so (always, unless force=False and up to date).

    The translation units compile in parallel (`jobs` processes, default: the
    CPU count, at most 8) and are then linked into one shared library."""
    srcs = sources()
    deps = srcs + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "smcx.h")]
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(p) for p in deps):
        return LIB
    jobs = jobs or min(8, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="smcx_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in srcs]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_compile, srcs, objs))
        for src, res in zip(srcs, results):
            if res.returncode != 0:
                raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n" + res.stdout +
                                   res.stderr)
            if verbose and res.stderr:
                print(res.stderr)
        tmp = LIB + ".tmp%d" % os.getpid()
        res = subprocess.run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] +
                             objs, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
