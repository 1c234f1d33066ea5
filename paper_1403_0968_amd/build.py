"""Build libsem.so (HIP for gfx950) in-tree.

    python -m paper_1403_0968_amd.build

Every source under ``csrc/`` is compiled by hipcc for gfx950 and linked into
``paper_1403_0968_amd/libsem.so``.  Packed-FP32 instructions are disabled
for device code (``-packed-fp32-ops``).  The operator sources are compiled
without machine-level instruction sinking: the element routine issues all of
an element's loads before its first use of them, and sinking moves loads
whose only uses lie past a branch (the LDS stores of a partial workgroup)
down to those uses, which serialises the memory phases of the kernel.  The
DG volume kernel is compiled with the matrix instructions accumulating in
ordinary vector registers.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsem.so")
BUILD = os.path.join(HERE, "_build")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result", "-Wno-unknown-pragmas",
          "-I", os.path.join(HERE, "..", "include")]


PER_FILE = {f: ["-mllvm", "-disable-machine-sink"]
            for f in ("ax.hip", "ax_solve.hip")}
# the DG volume kernel's FP64 matrix instructions accumulate in ordinary
# vector registers (gfx950's register file is unified), which keeps the
# compiler from copying loop-carried accumulators between register files
PER_FILE["dg.hip"] = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc, *COMMON, *PER_FILE.get(os.path.basename(src), []), *lang,
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        # the host pass warns about the device-only target feature; keep the rest
        err = "\n".join(l for l in r.stderr.splitlines()
                        if "packed-fp32-ops" not in l)
        if verbose and err.strip():
            print(err, flush=True)
        return obj

    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = OUT + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(OUT)
