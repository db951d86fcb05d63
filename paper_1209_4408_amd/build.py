"""Build libgol.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libgol.so")
OBJ = os.path.join(PKG, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall",
          "-Wno-unused-function"]
# Device code: gfx950 only; keep the compiler from forming packed-FP32 ops.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
HOST_SOURCES = ["gol_capi.cpp", "gol_plan.cpp", "gol_serve.cpp", "gol_tune.cpp"]
DEVICE_SOURCES = ["gol_kernels.hip", "gol_probe.hip"]


def _run(cmd: list[str]) -> None:
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))


def _stale(obj: str, src: str) -> bool:
    """The object is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, f) for d in (CSRC, INCLUDE) for f in os.listdir(d)
                    if f.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(save_temps: bool = False, out: str = LIB, defines: tuple = (),
          incremental: bool = False) -> str:
    """Compile every source (or, incremental, those whose object is stale) and
    link libgol.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ, exist_ok=True)
    jobs, objs = [], []
    for s in DEVICE_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        cmd = [HIPCC, *COMMON, *DEVICE, *[f"-D{d}" for d in defines], "-c",
               os.path.join(CSRC, s), "-o", o]
        if save_temps:
            cmd += ["-save-temps=obj"]
        jobs.append((cmd, o, os.path.join(CSRC, s)))
    for s in HOST_SOURCES:
        o = os.path.join(OBJ, s + ".o")
        jobs.append(([HIPCC, *COMMON, "-D__HIP_PLATFORM_AMD__", "-c", os.path.join(CSRC, s),
                      "-o", o], o, os.path.join(CSRC, s)))
    todo = [cmd for cmd, o, src in jobs if not incremental or defines or _stale(o, src)]
    with ThreadPoolExecutor(max_workers=min(8, max(1, len(todo)))) as ex:
        list(ex.map(_run, todo))
    objs = [o for _, o, _ in jobs]
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(save_temps="--save-temps" in sys.argv, incremental="--incremental" in sys.argv))
