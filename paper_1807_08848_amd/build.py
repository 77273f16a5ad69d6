"""Build libmsrs.so (HIP, gfx950) in-tree with hipcc.

Every source compiles to its own object in parallel (no device code crosses
files), then one link step makes the shared library.

Usage: python -m paper_1807_08848_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "k_local.hip", "k_factor.hip", "k_sweep.hip", "k_range.hip", "k_coarse.hip", "serve.hip",
           "noalloc.hip"]
LIB = os.path.join(HERE, "libmsrs.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build")
ARCH = os.environ.get("MSRS_OFFLOAD_ARCH", "gfx950")

# packed FP32 VALU forms are kept out of every kernel
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-mcode-object-version=5",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


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


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def compile_command(src: str, obj: str) -> list[str]:
    return [hipcc()] + FLAGS + ["-c", "-o", obj, src]


def link_command(objs: list[str], out: str = LIB) -> list[str]:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs
    rt = os.environ.get("MSRS_HIP_RUNTIME") or torch_hip_runtime()
    if rt:
        cmd += ["-no-hip-rt", f"-Wl,{rt}", f"-Wl,-rpath,{os.path.dirname(rt)}"]
    return cmd


def _run(cmd: list[str], verbose: bool):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}): {' '.join(cmd)}\n{errs}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)


def _stale(src: str, obj: str) -> bool:
    """An object older than its source or than any header of the library."""
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    deps.append(os.path.join(os.path.dirname(HERE), "include", "msrs.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def build(verbose: bool = False, incremental: bool | None = None) -> str:
    """Compile every source (incremental=True, or MSRS_BUILD_INCREMENTAL=1:
    only those whose object is out of date) and link libmsrs.so."""
    if incremental is None:
        incremental = os.environ.get("MSRS_BUILD_INCREMENTAL") == "1"
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in srcs]
    todo = [(s, o) for s, o in zip(srcs, objs) if not incremental or _stale(s, o)]
    if todo:
        with ThreadPoolExecutor(max_workers=len(todo)) as ex:
            list(ex.map(lambda so: _run(compile_command(*so), verbose), todo))
    tmp = LIB + ".tmp"
    _run(link_command(objs, tmp), verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
