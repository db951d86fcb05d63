"""ORACLE -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library under
``paper_1209_4408_amd/`` and its Python binding) never imports, links or calls
anything here, and this package imports nothing from the product.

Contents:
  * ``life(board, G, threads=1)``: the plain C byte-per-cell oracle
    (``gol_oracle.c``), serial or with the paper's row decomposition over
    OpenMP threads;
  * ``ref``: the same definition written with numpy rolls (tiny boards);
  * ``pack`` / ``unpack``: the packed-board layout of the library boundary
    (cell (r, c) is bit c mod 64 of word r * W + c // 64, LSB first,
    W = ceil(C / 64), padding bits 0), written with ``numpy.packbits``;
  * ``torus_window``: a wrapped sub-board, for light-cone checks of large runs;
  * ``population_at``: live cells after chosen generation counts (Table 1);
  * ``life_decomp``: the C oracle with the paper's row, column or 2-D block
    decomposition over OpenMP threads (Sections 2.1-2.2), for the CPU study;
  * ``python -m oracle``: the same from the command line on .npy boards.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import ref  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gol_oracle.c")
# ORACLE_LIB names another build of the oracle (the sanitizer builds below,
# for CPU runs of the pins under ASan / UBSan or TSan); by default liboracle.so.
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None
# Sanitizer builds of build(sanitize=...): the compiler, its flags and the
# runtime a process preloads.  ASan + UBSan with gcc; TSan with LLVM's clang
# and OpenMP runtime, whose tool interface (libarcher, named by
# OMP_TOOL_LIBRARIES) tells TSan about the parallel region's barriers.
_LLVM = "/opt/rocm/llvm"
SANITIZE = {"address": ("gcc", ["-fsanitize=address", "-fsanitize=undefined"]),
            "thread": (_LLVM + "/bin/clang",
                       ["-fsanitize=thread", f"-L{_LLVM}/lib", f"-Wl,-rpath,{_LLVM}/lib"])}
SANITIZER_RUNTIME = {"address": ("gcc", "libasan.so"),
                     "thread": (_LLVM + "/bin/clang", "libclang_rt.tsan-x86_64.so")}
OMP_TOOL_LIBRARY = _LLVM + "/lib/libarcher.so"


def build(force: bool = True, sanitize: str = "") -> str:
    """Compile the C oracle (plain -O2, OpenMP for the row-decomposed variant);
    sanitize ("address": ASan + UBSan, "thread": TSan) builds
    liboracle_<kind>.so with those checks instead."""
    out = _LIB if not sanitize else os.path.join(_HERE, f"liboracle_{sanitize}.so")
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cc, extra = SANITIZE[sanitize] if sanitize else ("gcc", [])
        if sanitize:
            extra = extra + ["-g", "-fno-omit-frame-pointer"]
        subprocess.check_call([cc, "-O2", "-fopenmp", *extra, "-shared", "-fPIC", _SRC,
                               "-o", tmp])
        os.replace(tmp, out)
    return out


def sanitizer_runtime(kind: str) -> str:
    cc, name = SANITIZER_RUNTIME[kind]
    return subprocess.run([cc, f"-print-file-name={name}"], capture_output=True, text=True,
                          check=True).stdout.strip()


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64 = ctypes.c_int64
        lib.oracle_life.restype = ctypes.c_int
        lib.oracle_life.argtypes = [ctypes.c_void_p, i64, i64, i64, ctypes.c_void_p]
        lib.oracle_life_omp.restype = ctypes.c_int
        lib.oracle_life_omp.argtypes = [ctypes.c_void_p, i64, i64, i64, ctypes.c_void_p,
                                        ctypes.c_int]
        lib.oracle_life_decomp.restype = ctypes.c_int
        lib.oracle_life_decomp.argtypes = [ctypes.c_void_p, i64, i64, i64, ctypes.c_void_p,
                                           ctypes.c_int, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def life(board: np.ndarray, generations: int, threads: int = 1) -> np.ndarray:
    """B3/S23 on the torus of ``board`` (2-D, nonzero = alive) -> 0/1 uint8."""
    b = np.ascontiguousarray(board, dtype=np.uint8)
    if b.ndim != 2:
        raise ValueError("board must be 2-D")
    out = np.empty_like(b)
    R, C = b.shape
    if threads > 1:
        rc = _load().oracle_life_omp(b.ctypes.data, R, C, int(generations), out.ctypes.data,
                                     int(threads))
    else:
        rc = _load().oracle_life(b.ctypes.data, R, C, int(generations), out.ctypes.data)
    if rc == -1:
        raise ValueError("invalid arguments")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out


DECOMPOSITIONS = {"rows": 0, "cols": 1, "2d": 2}


def life_decomp(board: np.ndarray, generations: int, threads: int, decomposition: str) -> np.ndarray:
    """The C oracle with each generation split among ``threads`` OpenMP
    threads by rows (Figure 1), columns (Figure 2) or an m x n grid of
    sub-regions (Figure 3, m n = threads, as square as threads allows)."""
    b = np.ascontiguousarray(board, dtype=np.uint8)
    if b.ndim != 2:
        raise ValueError("board must be 2-D")
    out = np.empty_like(b)
    R, C = b.shape
    rc = _load().oracle_life_decomp(b.ctypes.data, R, C, int(generations), out.ctypes.data,
                                    int(threads), DECOMPOSITIONS[decomposition])
    if rc == -1:
        raise ValueError("invalid arguments")
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out


def words_per_row(cols: int) -> int:
    return (int(cols) + 63) // 64


def pack(board: np.ndarray) -> np.ndarray:
    """(R, C) cells -> (R, W) uint64 words of the boundary layout."""
    b = (np.asarray(board) != 0).astype(np.uint8)
    R, C = b.shape
    W = words_per_row(C)
    by = np.packbits(b, axis=1, bitorder="little")          # (R, ceil(C/8))
    padded = np.zeros((R, 8 * W), dtype=np.uint8)
    padded[:, : by.shape[1]] = by
    return padded.view("<u8").reshape(R, W).astype(np.uint64)


def unpack(words: np.ndarray, cols: int) -> np.ndarray:
    """(R, W) words of the boundary layout -> (R, cols) 0/1 uint8."""
    w = np.ascontiguousarray(words).view(np.uint64)
    R, W = w.shape
    by = w.astype("<u8").view(np.uint8).reshape(R, 8 * W)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return bits[:, :cols].copy()


def padding_is_zero(words: np.ndarray, cols: int) -> bool:
    """True when every bit at a column >= cols is 0."""
    w = np.ascontiguousarray(words).view(np.uint64)
    R, W = w.shape
    by = w.astype("<u8").view(np.uint8).reshape(R, 8 * W)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return not bits[:, cols:].any()


def torus_window(board: np.ndarray, r0: int, c0: int, h: int, w: int) -> np.ndarray:
    """Rows r0..r0+h-1 and cols c0..c0+w-1 of the board, indices taken mod R, C."""
    R, C = board.shape
    rows = np.arange(r0, r0 + h) % R
    cols = np.arange(c0, c0 + w) % C
    return np.ascontiguousarray(board[np.ix_(rows, cols)])


def torus_window_packed(words: np.ndarray, cols: int, r0: int, c0: int, h: int,
                        w: int) -> np.ndarray:
    """Like ``torus_window`` but reads a packed board without unpacking all of it."""
    R, W = words.shape
    rows = np.arange(r0, r0 + h) % R
    cidx = np.arange(c0, c0 + w) % cols
    sub = np.asarray(words)[rows][:, np.unique(cidx // 64)]
    # map each wanted column to (word position within sub, bit)
    uw = np.unique(cidx // 64)
    pos = np.searchsorted(uw, cidx // 64)
    bit = (cidx % 64).astype(np.uint64)
    vals = (sub[:, pos].astype(np.uint64) >> bit[None, :]) & np.uint64(1)
    return vals.astype(np.uint8)


def light_cone_check(gpu_out_window: np.ndarray, board_in, cols_or_none, r0: int,
                     c0: int, k_rows: int, k_cols: int, generations: int,
                     threads: int = 1, packed: bool = False) -> bool:
    """Check a k_rows x k_cols output window at (r0, c0) after G generations.

    The window's value depends only on the input within Chebyshev distance G,
    so the oracle runs on the (k + 2G)-wide wrapped input window, itself treated
    as a torus: wrong values from its own seam move at most one cell per
    generation and never reach the centre.
    """
    G = int(generations)
    h, w = k_rows + 2 * G, k_cols + 2 * G
    if packed:
        win = torus_window_packed(board_in, cols_or_none, r0 - G, c0 - G, h, w)
    else:
        win = torus_window(board_in, r0 - G, c0 - G, h, w)
    res = life(win, G, threads=threads)
    centre = res[G:G + k_rows, G:G + k_cols]
    return bool(np.array_equal(centre, np.asarray(gpu_out_window, dtype=np.uint8)))


def population_at(board: np.ndarray, checks, threads: int = 1) -> list[int]:
    """Live cells after each generation count in ``checks`` (non-decreasing):
    the quantity the paper tabulates at chosen iteration counts (Table 1).
    The board is evolved with ``life`` from one check to the next and its live
    cells counted."""
    out, cur, g = [], board, 0
    for c in checks:
        c = int(c)
        if c < g:
            raise ValueError("checks must be non-decreasing")
        cur = life(cur, c - g, threads)
        g = c
        out.append(int(np.count_nonzero(cur)))
    return out
