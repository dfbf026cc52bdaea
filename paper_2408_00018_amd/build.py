"""Build the gfx950 HIP library in-tree (hipcc, no JIT cache).

The product is ``paper_2408_00018_amd/libsa_hip.so`` exporting the C ABI of
``include/sa.h``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsa_hip.so")
PEAK_LIB = os.path.join(PKG, "libsa_peak.so")

SOURCES = ["sa_kernels.hip", "sa_coupled.hip", "sa_overlay.hip", "sa_api.hip", "sa_batch.hip", "sa_batch_api.hip",
           "sa_mlp.hip", "sa_nm.hip", "sa_variant.hip"]
PEAK_SOURCES = ["peak_probe.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # FP64 runs are compared move for move with a plain FP64 evaluation, so no
    # implicit contraction; FP32 code writes its fused multiply-adds explicitly.
    "-ffp-contract=off",
    # Packed FP32 instructions stay off: every VALU op here is scalar FP32/FP64
    # or integer.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Matrix-core results stay in ordinary VGPRs, where the relu/BF16 packing
    # that follows each product reads them, instead of accumulation registers
    # that need a v_accvgpr_read per value.
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    # Loop headers on 32-byte boundaries.  The plain step loop is one ~1.8 KB
    # block run by a single wave per SIMD; where its header falls inside a
    # fetch line the level ran 2.5% slower (MI355X, same sources, 32-byte
    # alignment measured best against 64 and 128).
    "-falign-loops=32",
    "-Wall",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the gfx950 library cannot be built")


OBJ_DIR = os.path.join(PKG, "_build")


def _compile(sources, out, verbose):
    """Compile each source to its own object in parallel (each translation
    unit holds its kernels and their launchers, so no device-code linking is
    needed), then link the shared library."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]

    def one(src):
        obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *compile_flags, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    jobs = max(1, min(len(sources), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(one, sources))
    tmp = out + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile the library and the issue-rate probe; always rebuilds.
    Returns the library's path."""
    _compile(SOURCES, LIB, verbose)
    _compile(PEAK_SOURCES, PEAK_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
