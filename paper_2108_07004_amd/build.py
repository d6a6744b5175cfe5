"""Build libdemap.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
LIB = PKG / "libdemap.so"
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 VALU ops stay off: plain float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and Path(cand).exists():
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def sources() -> list[Path]:
    return sorted(CSRC.glob("*.hip"))


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}\n{res.stderr[-6000:]}")


def build(verbose: bool = False, jobs: int | None = None) -> Path:
    """Compile every HIP source (in parallel, one object each) and link
    paper_2108_07004_amd/libdemap.so; always recompiles."""
    cc = hipcc()
    srcs = sources()
    jobs = jobs or max(1, min(len(srcs), 8, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="demap_build_") as d:
        objs = [Path(d) / (s.stem + ".o") for s in srcs]
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda so: _run([cc, *HIPCC_FLAGS, "-c", str(so[0]), "-o", str(so[1])], verbose),
                        zip(srcs, objs)))
        tmp = LIB.with_name(f"libdemap.so.tmp{os.getpid()}")
        _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
