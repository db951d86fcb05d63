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


def _includes(path: str, seen: set) -> set:
    """The source and the project headers it includes, recursively."""
    import re
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for line in open(path, encoding="utf-8", errors="replace"):
        m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
        if m:
            for d in (CSRC, INCLUDE):
                cand = os.path.join(d, m.group(1))
                if os.path.exists(cand):
                    _includes(cand, seen)
                    break
    return seen


def _stale(obj: str, src: str) -> bool:
    """The object is missing or older than its source or a header it includes."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _includes(src, set()))


# Host-code sanitizer builds (CPU runs of the scheduler, planner and C ABI
# checks): the host sources instrumented, the device code as always.  Each
# -fsanitize= goes to the host compilation only.
SANITIZERS = {"address": ["address", "undefined"], "thread": ["thread"]}


def sanitized_lib(kind: str) -> str:
    return os.path.join(OBJ + "_" + kind, "libgol.so")


def sanitizer_runtime(kind: str) -> str:
    """The clang runtime a process that loads a sanitized libgol preloads."""
    name = {"address": "asan", "thread": "tsan"}[kind]
    return subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                           f"-print-file-name=libclang_rt.{name}-x86_64.so"],
                          capture_output=True, text=True, check=True).stdout.strip()


def build(save_temps: bool = False, out: str = LIB, defines: tuple = (),
          incremental: bool = False, sanitize: str = "") -> str:
    """Compile every source (or, incremental, those whose object is stale) and
    link libgol.so; sanitize ("address": ASan + UBSan, "thread": TSan)
    instruments the host sources into _build_<kind>/libgol.so instead."""
    from concurrent.futures import ThreadPoolExecutor
    obj_dir = OBJ if not sanitize else OBJ + "_" + sanitize
    if sanitize:
        out = sanitized_lib(sanitize)
    san = []
    for k in SANITIZERS.get(sanitize, []):
        san += ["-Xarch_host", f"-fsanitize={k}"]
    if san:
        san += ["-fno-omit-frame-pointer", "-g"]
    os.makedirs(obj_dir, exist_ok=True)
    jobs, objs = [], []
    for s in DEVICE_SOURCES:
        o = os.path.join(obj_dir, s + ".o")
        cmd = [HIPCC, *COMMON, *DEVICE, *[f"-D{d}" for d in defines], "-c",
               os.path.join(CSRC, s), "-o", o]
        if save_temps:
            cmd += ["-save-temps=obj"]
        jobs.append((cmd, o, os.path.join(CSRC, s)))
    for s in HOST_SOURCES:
        o = os.path.join(obj_dir, s + ".o")
        jobs.append(([HIPCC, *COMMON, *san, "-D__HIP_PLATFORM_AMD__", "-c",
                      os.path.join(CSRC, s), "-o", o], o, os.path.join(CSRC, s)))
    todo = [cmd for cmd, o, src in jobs if not incremental or defines or _stale(o, src)]
    with ThreadPoolExecutor(max_workers=min(8, max(1, len(todo)))) as ex:
        list(ex.map(_run, todo))
    objs = [o for _, o, _ in jobs]
    tmp = out + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    if san:
        link += ["-shared-libsan", *[f for f in san if f.startswith("-fsanitize")]]
    _run(link)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    kind = ""
    for a in sys.argv[1:]:
        if a.startswith("--sanitize="):
            kind = a.split("=", 1)[1]
    print(build(save_temps="--save-temps" in sys.argv, incremental="--incremental" in sys.argv,
                sanitize=kind))
