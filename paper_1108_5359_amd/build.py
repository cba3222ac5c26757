"""Build librpca.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed FP32 instructions
disabled (the compiler would otherwise form v_pk_* FP32 ops from ordinary
float code), then linked with rocSOLVER/rocBLAS (used for the FP64 SVD of
the seed block).
"""
from __future__ import annotations

import concurrent.futures
import os
import pathlib
import subprocess
import sys

HERE = pathlib.Path(__file__).resolve().parent
CSRC = HERE / "csrc"
LIB = HERE / "librpca.so"
BUILD = HERE / "_build"
ROCM = pathlib.Path(os.environ.get("ROCM_PATH", "/opt/rocm"))
SOURCES = ["api.cpp", "batch_api.cpp", "server.cpp", "pipeline.cpp", "filter.hip", "reconstruct.hip", "seed.hip", "seed_small.hip", "seed_large.hip", "batch.hip", "rank.cpp"]
# filter_inst.hip is compiled once per tile class (one object each)
FILTER_PT = [1, 2, 3, 4, 5, 7, 8, 10, 13, 16, 19, 26, 32]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{ROCM / 'include'}",
]


def _compile(src: pathlib.Path, obj: pathlib.Path, defines=()) -> None:
    cmd = [str(ROCM / "bin" / "hipcc"), *HIPCC_FLAGS, *defines]
    if src.suffix == ".cpp":
        cmd += ["-x", "hip"]
    cmd += ["-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src.name}:\n{r.stdout}\n{r.stderr}")
    # hipcc's host pass does not know the packed-fp32 feature; drop that note.
    for line in (r.stderr or "").splitlines():
        if "packed-fp32-ops" in line or not line.strip():
            continue
        if "warning" in line or "error" in line:
            print(line, file=sys.stderr)


def build(jobs: int | None = None) -> pathlib.Path:
    """Compile every source and link librpca.so.  Always rebuilds."""
    BUILD.mkdir(exist_ok=True)
    objs = []
    jobs = jobs or min(8, os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = []
        for pt in sorted(FILTER_PT, reverse=True):     # largest first: they take longest
            obj = BUILD / f"filter_inst_pt{pt}.o"
            objs.append(obj)
            # MFMA results in arch VGPRs: the quarter-tile precision kernel
            # otherwise keeps its accumulators in acc VGPRs and spends one
            # VALU move per value reading them back (no other filter kernel
            # changes: they already use arch VGPRs or need both files)
            futs.append(ex.submit(_compile, CSRC / "filter_inst.hip", obj,
                                  (f"-DRPCA_PT={pt}", "-mllvm", "-amdgpu-mfma-vgpr-form")))
        for s in SOURCES:
            obj = BUILD / (s.replace(".", "_") + ".o")
            objs.append(obj)
            futs.append(ex.submit(_compile, CSRC / s, obj))
        for f in futs:
            f.result()
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [str(ROCM / "bin" / "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC",
           *map(str, objs), "-o", str(tmp), f"-L{ROCM / 'lib'}", "-lrocsolver", "-lrocblas",
           f"-Wl,-rpath,{ROCM / 'lib'}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
