"""Build the HIP library liblbm_hip.so for gfx950 (hipcc, in-tree).

Usage: python -m paper_2403_18466_amd.build   (or call build()).
The library is rebuilt on every call to build(); loading code never builds.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm_hip.so")
# matrix-core results in VGPRs, read by the activation without
# accumulator-register moves
VGPR_FORM = ("-mllvm", "-amdgpu-mfma-vgpr-form")
# max-ILP instruction scheduler: the learned-collision step ran 1% faster with
# it on every grid measured (D2Q9 8 x 256^2 to 4096^2, D3Q19 256^3), the D2Q9
# adjoint 1.5% faster, the D3Q19 adjoint 1.9% (since its gradient tiles share
# operands; 2% slower before); the other kernels stay on the default
# scheduler, several of which need more registers with it
MAX_ILP = ("-mllvm", "-amdgpu-sched-strategy=max-ilp")
# (source, extra flags): the wide-network kernels use the max-ILP scheduler
# too, which keeps their LDS weight reads ahead of the matrix-core work,
SOURCES = [
    (os.path.join(CSRC, "lbm_api.hip"), VGPR_FORM),
    (os.path.join(CSRC, "nlbm_fwd.hip"), VGPR_FORM + MAX_ILP),
    # and IEEE mode off (LeakyReLU's max then needs no NaN-quieting
    # canonicalisation; the wide step has no NaN tests)
    (os.path.join(CSRC, "wide.hip"), VGPR_FORM + MAX_ILP + ("-mno-amdgpu-ieee", "-fno-honor-nans")),
    (os.path.join(CSRC, "wide_bwd.hip"), VGPR_FORM),
    (os.path.join(CSRC, "nlbm_bwd.hip"), VGPR_FORM + MAX_ILP),
    (os.path.join(CSRC, "nlbm_bwd_d2q9.hip"), VGPR_FORM + MAX_ILP),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def compile_command(src: str, obj: str, extra=()):
    return [
        hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-c",
        # no packed FP32 instructions anywhere in the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        *extra, src, "-o", obj,
    ]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)


def build(verbose: bool = False) -> str:
    # the translation units compile in parallel (hipcc runs as a separate
    # process; the threads only wait for it)
    from concurrent.futures import ThreadPoolExecutor
    objs = [os.path.join(CSRC, os.path.basename(src) + ".o") for src, _ in SOURCES]
    jobs = [compile_command(src, obj, extra) for (src, extra), obj in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        for f in [ex.submit(_run, cmd, verbose) for cmd in jobs]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    for obj in objs:
        os.remove(obj)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
