"""Build the HIP shared library libh2ulv.so in-tree (gfx950).

    python -m paper_2208_10907_amd.build

Every source is compiled with hipcc for gfx950; host-only geometry code is
compiled without floating-point contraction so that the cluster tree and the
admissibility decisions are reproducible.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
OUT_DIR = PKG / "_lib"
LIB = OUT_DIR / "libh2ulv.so"
BUILD_DIR = PKG.parent / "_build"

HIP_FLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             # per-kernel register / LDS / scratch report, checked below
             "-Rpass-analysis=kernel-resource-usage"]
SOURCES = [
    # MFMA accumulators in ordinary VGPRs (no copies between register files in the K loop)
    ("h2ulv_kernels.hip", ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]),
    ("h2ulv_learned.hip", []),
    ("h2ulv_noalloc.hip", []),
    ("h2ulv_rankmodel.cpp", ["-x", "hip"]),
    ("h2ulv_dense.cpp", ["-x", "hip"]),
    ("h2ulv_factor.cpp", ["-x", "hip"]),
    ("h2ulv_api.cpp", ["-x", "hip"]),
    ("h2ulv_tree.cpp", ["-x", "hip", "-ffp-contract=off"]),
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def scratch_users(remarks: str) -> list:
    """Kernels whose resource report shows private (scratch) memory per lane:
    register spills or stack arrays, which every kernel here is written to
    avoid (they cost a memory round trip per access and a per-lane scratch
    allocation at launch)."""
    out, name = [], None
    for line in remarks.splitlines():
        if "Function Name:" in line:
            name = line.split("Function Name:", 1)[1].split("[-Rpass")[0].strip()
        elif "ScratchSize [bytes/lane]:" in line and name:
            val = int(line.split("ScratchSize [bytes/lane]:", 1)[1].split("[")[0].strip())
            if val > 0:
                out.append((name, val))
    return out


def build(verbose: bool = False) -> Path:
    from concurrent.futures import ThreadPoolExecutor
    BUILD_DIR.mkdir(exist_ok=True)
    OUT_DIR.mkdir(exist_ok=True)
    cc = hipcc()

    def compile_one(item):
        src, extra = item
        obj = BUILD_DIR / (src.replace(".", "_") + ".o")
        cmd = [cc, *HIP_FLAGS, *extra, "-c", str(CSRC / src), "-o", str(obj)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        bad = scratch_users(r.stderr)
        if bad:
            raise RuntimeError(f"{src}: kernels use scratch memory: " +
                               ", ".join(f"{n} ({v} B/lane)" for n, v in bad))
        return str(obj)

    # the sources compile independently; at most one hipcc per available core
    workers = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = OUT_DIR / "libh2ulv.so.tmp"
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
