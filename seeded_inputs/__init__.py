"""Seeded synthetic inputs for the Life step.

This module serves both the oracle side (tests) and the GPU side (tests, bench)
and holds none of the Life arithmetic: it only draws boards and workload
parameters.  Cells come from the counter-based SplitMix64 generator in
``gen.c`` (see its header for the exact definition; ``gen_device.hip`` draws
the same cells straight into device memory); workload parameters of the
batched and served mixes come from ``numpy.random.default_rng(seed)``.

Workloads (synthetic stand-ins for the paper's drawn initial figures, which the
paper does not give):
  * single board: rows x cols, i.i.d. Bernoulli(p) cells from (seed, board_id);
  * batched mix: per board, rows and cols log-uniform integers, density
    uniform, generations uniform integers, drawn in that order per board;
  * served stream: the same per-request draws plus exponential inter-arrival
    gaps (Poisson process).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libseeded_inputs.so")
_DEV_SRC = os.path.join(_HERE, "gen_device.hip")
_DEV_LIB = os.path.join(_HERE, "libseeded_inputs_device.so")
_HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
_lib = None
_dev_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c (host) and gen_device.hip (gfx950) into shared libraries
    next to them."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_DEV_LIB):
        tmp = _DEV_LIB + ".tmp"
        subprocess.check_call([_HIPCC, "-O3", "-shared", "-fPIC", "--offload-arch=gfx950",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               _DEV_SRC, "-o", tmp])
        os.replace(tmp, _DEV_LIB)
    return _LIB


def _load_device():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB):
            raise RuntimeError(f"{_DEV_LIB} is missing: run seeded_inputs.build() first")
        lib = ctypes.CDLL(_DEV_LIB)
        lib.si_gen_packed_device.restype = ctypes.c_int
        lib.si_gen_packed_device.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                             ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                             ctypes.c_void_p]
        _dev_lib = lib
    return _dev_lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64, i64 = ctypes.c_uint64, ctypes.c_int64
        lib.si_mix64.restype = u64
        lib.si_mix64.argtypes = [u64]
        lib.si_splitmix64_nth.restype = u64
        lib.si_splitmix64_nth.argtypes = [u64, u64]
        lib.si_board_key.restype = u64
        lib.si_board_key.argtypes = [u64, u64]
        lib.si_threshold.restype = ctypes.c_uint32
        lib.si_threshold.argtypes = [ctypes.c_double]
        for name in ("si_gen_bytes", "si_gen_packed"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [u64, u64, i64, i64, ctypes.c_double, ctypes.c_void_p]
        _lib = lib
    return _lib


def words_per_row(cols: int) -> int:
    return (int(cols) + 63) // 64


def splitmix64_nth(state: int, i: int) -> int:
    return int(_load().si_splitmix64_nth(state & (2**64 - 1), i))


def board_bytes(seed: int, board_id: int, rows: int, cols: int, p: float,
                out: np.ndarray | None = None) -> np.ndarray:
    """Board as a (rows, cols) uint8 array of 0/1."""
    if out is None:
        out = np.empty((rows, cols), dtype=np.uint8)
    assert out.dtype == np.uint8 and out.flags.c_contiguous and out.size == rows * cols
    rc = _load().si_gen_bytes(seed, board_id, rows, cols, float(p), out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid board size")
    return out


def board_packed(seed: int, board_id: int, rows: int, cols: int, p: float,
                 out: np.ndarray | None = None) -> np.ndarray:
    """Board as a (rows, ceil(cols/64)) uint64 array, LSB-first, padding 0."""
    w = words_per_row(cols)
    if out is None:
        out = np.empty((rows, w), dtype=np.uint64)
    assert out.dtype in (np.uint64, np.int64) and out.flags.c_contiguous
    assert out.size == rows * w
    rc = _load().si_gen_packed(seed, board_id, rows, cols, float(p), out.ctypes.data)
    if rc != 0:
        raise ValueError("invalid board size")
    return out


def board_packed_device(seed: int, board_id: int, rows: int, cols: int, p: float, out):
    """The board of board_packed, drawn on the device into `out`: a contiguous
    int64 / uint64 torch tensor on a GPU with rows * ceil(cols/64) elements,
    on the current stream (asynchronous).  Returns `out`."""
    import torch
    w = words_per_row(cols)
    if not (out.is_cuda and out.is_contiguous() and out.dtype in (torch.int64, torch.uint64)
            and out.numel() == rows * w):
        raise ValueError("out must be a contiguous 64-bit GPU tensor of rows * words_per_row "
                         "elements")
    rc = _load_device().si_gen_packed_device(seed, board_id, rows, cols, float(p),
                                             out.data_ptr(),
                                             torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise ValueError("invalid board size" if rc == -1 else "device generation failed")
    return out


def _log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    v = int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))
    return min(max(v, lo), hi)


@dataclass(frozen=True)
class BoardSpec:
    board_id: int
    rows: int
    cols: int
    p: float
    generations: int


def batch_specs(seed: int, n: int = 4096, side_lo: int = 64, side_hi: int = 2048,
                p_lo: float = 0.1, p_hi: float = 0.6, gen_lo: int = 10,
                gen_hi: int = 1000) -> list[BoardSpec]:
    """The batched mix: n boards, rows/cols log-uniform, p and generations uniform."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        rows = _log_uniform_int(rng, side_lo, side_hi)
        cols = _log_uniform_int(rng, side_lo, side_hi)
        p = float(rng.uniform(p_lo, p_hi))
        g = int(rng.integers(gen_lo, gen_hi + 1))
        out.append(BoardSpec(b, rows, cols, p, g))
    return out


@dataclass(frozen=True)
class RequestSpec:
    board_id: int
    arrival_s: float
    rows: int
    cols: int
    p: float
    generations: int


def serve_specs(seed: int, n: int = 4096, rate_per_s: float = 500.0, side_lo: int = 32,
                side_hi: int = 8192, p_lo: float = 0.05, p_hi: float = 0.7,
                gen_lo: int = 1, gen_hi: int = 10000) -> list[RequestSpec]:
    """The served stream: Poisson arrivals, per-request board and generations."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for b in range(n):
        t += float(rng.exponential(1.0 / rate_per_s))
        rows = _log_uniform_int(rng, side_lo, side_hi)
        cols = _log_uniform_int(rng, side_lo, side_hi)
        p = float(rng.uniform(p_lo, p_hi))
        g = int(rng.integers(gen_lo, gen_hi + 1))
        out.append(RequestSpec(b, t, rows, cols, p, g))
    return out
