"""Build libmsrs.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1807_08848_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "k_local.hip", "k_range.hip", "k_coarse.hip", "serve.hip"]
LIB = os.path.join(HERE, "libmsrs.so")
ARCH = os.environ.get("MSRS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def torch_hip_runtime():
    """The HIP runtime library bundled with torch, if any.

    The library must run on the same HIP runtime instance as torch so that
    torch's streams are valid handles and stream order covers both.
    """
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec is None or not spec.origin:
            return None
        p = os.path.join(os.path.dirname(spec.origin), "lib", "libamdhip64.so")
        return p if os.path.exists(p) else None
    except Exception:
        return None


def command(out: str = LIB) -> list[str]:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-mcode-object-version=5",
           # packed FP32 VALU forms are kept out of every kernel
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-result",
           "-o", out] + [os.path.join(CSRC, s) for s in SOURCES]
    rt = os.environ.get("MSRS_HIP_RUNTIME") or torch_hip_runtime()
    if rt:
        cmd += ["-no-hip-rt", f"-Wl,{rt}", f"-Wl,-rpath,{os.path.dirname(rt)}"]
    return cmd


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{errs}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
