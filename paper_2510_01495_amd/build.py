"""Builds libttv.so (the gfx950 HIP kernels and the C ABI) in-tree with hipcc.

Every source is compiled to its own object (in parallel), then the objects
are linked into the shared library.
"""

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libttv.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code (never emitted by
# the compiler); gfx950 only; wave64.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wno-unused-command-line-argument",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _filter(text: str):
    return [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    return r.returncode, _filter(r.stdout + r.stderr)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source into paper_2510_01495_amd/libttv.so (always rebuilds)."""
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), len(os.sched_getaffinity(0)), 16))
    tmpdir = tempfile.mkdtemp(prefix="ttv_build_")
    try:
        objs = [os.path.join(tmpdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
        cmds = [[HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", s, "-o", o]
                for s, o in zip(srcs, objs)]
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        failed = False
        for cmd, (rc, msgs) in zip(cmds, results):
            if verbose:
                print(" ".join(cmd), flush=True)
            if rc != 0:
                failed = True
                sys.stderr.write("\n".join(msgs) + "\n")
            elif verbose and msgs:
                print("\n".join(msgs))
        if failed:
            raise RuntimeError("hipcc failed")
        tmp = LIB + ".tmp"
        rc, msgs = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
        if rc != 0:
            sys.stderr.write("\n".join(msgs) + "\n")
            raise RuntimeError(f"link failed with status {rc}")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
