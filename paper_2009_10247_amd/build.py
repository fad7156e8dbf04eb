"""Build the engine library liblp.so (HIP, gfx950) in-tree.

    python -m paper_2009_10247_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblp.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("lp_build.cpp", "lp_step.hip", "lp_batch.hip", "lp_spmm.hip", "lp_frontier.hip", "lp_dense.hip",
            "lp_runtime.hip", "lp_server.cpp")]
ARCH = os.environ.get("LP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# No packed FP32 instructions (v_pk_add_f32 and its kin) in device code. The
# device pass honours the feature (tests/test_abi.py compiles a float2 kernel
# with these flags and finds none); the host pass does not know it and says so
# once per source, a line the build drops.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_PASS_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def command(out: str) -> list[str]:
    return [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared", *NO_PACKED_FP32,
            "-Wall", "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES, "-o", out]


def run_hipcc(cmd: list[str]) -> None:
    """Run hipcc; forward its output except the host pass's note on the
    packed-FP32 feature; raise on failure."""
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in r.stdout.splitlines() if ln.strip() != HOST_PASS_NOTE)
    if out.strip():
        print(out, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    run_hipcc(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
