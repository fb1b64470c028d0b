"""Build libxeng.so (gfx950) in-tree with hipcc.

Each translation unit under csrc/ compiles to its own object in parallel
(the kernel instantiations are split over several units for that), then the
objects link into libxeng.so next to this file.

Usage: python build.py [--incremental]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libxeng.so")
ARCH = os.environ.get("XENG_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-fp32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # early unroll attempts on loops whose bounds become constant only after
    # the enclosing loop is unrolled; every loop ends up fully unrolled
    "-Wno-pass-failed",
]
# Units of the 16-row-tile kernel: the register allocator's default order
# keeps some of the many 4-register accumulator tuples in different registers
# at the top and the bottom of the main loop and moves them around with
# accvgpr copies every iteration; assigning local ranges in reverse order
# keeps every accumulator in place (checked in the generated assembly).
PER_FILE_FLAGS = {
    "k_x16_": ["-mllvm", "-greedy-reverse-local-assignment"],
    "k_batch": ["-mllvm", "-greedy-reverse-local-assignment"],
}
# the host pass warns that it does not know the packed-fp32 feature
_NOISE = ("'-packed-fp32-ops' is not a recognized feature",)


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if not any(n in l for n in _NOISE))
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\nfailed ({res.returncode}):\n{err}")
    return err


def build(verbose: bool = False, incremental: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    headers = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(HERE, "..", "include", "*.h"))
    newest_header = max(os.path.getmtime(h) for h in headers)

    def deps_of(obj):
        """Headers the object was built from (its -MMD file), or None."""
        try:
            with open(obj + ".d") as fh:
                text = fh.read().replace("\\\n", " ")
        except OSError:
            return None
        return [t for t in text.split(":", 1)[1].split() if t.endswith((".h", ".hpp"))]

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.basename(src).replace(".hip", ".o"))
        if incremental and os.path.exists(obj):
            deps = deps_of(obj)
            newest = newest_header if deps is None else max([os.path.getmtime(d) for d in deps if os.path.exists(d)] or [0])
            if os.path.getmtime(obj) > max(os.path.getmtime(src), newest):
                return obj
        extra = [f for key, flags in PER_FILE_FLAGS.items() if os.path.basename(src).startswith(key) for f in flags]
        cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-MMD", "-MF", obj + ".d", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
        return obj

    jobs = jobs or min(len(sources), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, sources))
    tmp = OUT + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
