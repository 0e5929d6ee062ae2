"""Build the gfx950 HIP library ``libinc.so`` in-tree with hipcc.

Each source is compiled to an object with its own flags (the event kernels
twice: kernels.hip with IEEE arithmetic and precise transcendentals,
kernels_fast.hip with the fast-math flags), then the objects are linked.

Usage: ``python -m paper_1309_7963_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libinc.so")
SOURCES = ["api.hip", "setup.hip", "kernels.hip", "kernels_fast.hip", "server.hip", "ring.hip", "tally.hip"]
HEADERS = ["device.h", "event.h", "kernels.h", "ctx.h", "copy_pool.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions are kept out of generated code on these boxes
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
# fast-math build of the event kernels: approximate library functions, x / y as
# x * rcp(y), no errno, FP32 denormals flushed (no reassociation, and NaN and
# infinity keep their meaning, so input checks still hold)
FAST_FLAGS = ["-fapprox-func", "-freciprocal-math", "-fno-math-errno", "-fgpu-flush-denormals-to-zero"]
EXTRA_FLAGS = {"kernels_fast.hip": FAST_FLAGS}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in SOURCES + HEADERS] + [os.path.join(ROOT, "include", "inc.h")]
    return any(os.path.getmtime(d) > t for d in deps)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    tmpdir = tempfile.mkdtemp(prefix="libinc_build_")
    try:
        inc = ["-I", os.path.join(ROOT, "include")]
        jobs = []
        for f in SOURCES:
            obj = os.path.join(tmpdir, f.replace(".hip", ".o"))
            jobs.append((f, obj, [hipcc()] + HIPCC_FLAGS + EXTRA_FLAGS.get(f, []) + inc +
                         ["-c", os.path.join(CSRC, f), "-o", obj]))
        with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as ex:
            results = list(ex.map(lambda j: _run(j[2], verbose), jobs))
        for (f, _, _), res in zip(jobs, results):
            if res.returncode != 0:
                sys.stderr.write(res.stdout)
                raise RuntimeError("hipcc failed compiling %s" % f)
        tmp = LIB + ".tmp%d" % os.getpid()
        res = _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + [o for _, o, _ in jobs] + ["-o", tmp],
                   verbose)
        if res.returncode != 0:
            sys.stderr.write(res.stdout)
            raise RuntimeError("hipcc failed linking %s" % LIB)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
