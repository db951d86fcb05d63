"""Python binding of libgol (the C ABI in include/gol.h): argument marshalling only.

Every step of the Life computation runs in the library's HIP kernels; torch
only supplies device memory (packed boards are int64 tensors of shape
(rows, ceil(cols / 64)), reinterpreted as uint64 words) and HIP streams.
If libgol.so is missing this module raises on first use: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Iterable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GOL_LIB names another build of the same library (the host-sanitizer builds
# of build.py for CPU test runs); by default the in-tree libgol.so.
LIB_PATH = os.environ.get("GOL_LIB") or os.path.join(_HERE, "libgol.so")

GOL_OK = 0
GOL_EINVAL = -1
GOL_ENOMEM = -2
GOL_EDEVICE = -3
GOL_EAGAIN = -4
GOL_ENOTFOUND = -5
GOL_ECANCELED = -6

_lib = None


class GolError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class Board(ctypes.Structure):
    _fields_ = [("d_in", ctypes.c_void_p), ("d_out", ctypes.c_void_p), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("generations", ctypes.c_int64)]


class PassConfig(ctypes.Structure):
    _fields_ = [("t_block", ctypes.c_int32), ("band_rows", ctypes.c_int32),
                ("prefetch", ctypes.c_int32), ("layout", ctypes.c_int32)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("chunk_generations", ctypes.c_int32),
                ("device", ctypes.c_int32), ("max_resident", ctypes.c_int32),
                ("t_block", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("retired", ctypes.c_int64),
                ("plan_host_s", ctypes.c_double), ("device_busy_s", ctypes.c_double),
                ("cell_updates", ctypes.c_double), ("max_resident", ctypes.c_int64),
                ("mean_resident", ctypes.c_double), ("resident_bytes", ctypes.c_int64),
                ("peak_resident_bytes", ctypes.c_int64), ("t_block", ctypes.c_int64),
                ("last_chunk_generations", ctypes.c_int64), ("last_band_rows", ctypes.c_int64),
                ("busy_band_rows", ctypes.c_int64), ("admit_host_s", ctypes.c_double),
                ("retire_host_s", ctypes.c_double), ("starved_s", ctypes.c_double),
                ("chunk_gap_s", ctypes.c_double)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("generations_done", ctypes.c_int64), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


def lib():
    """Load libgol.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        # torch loads its own copy of the HIP runtime (same soname, requested
        # by file name); loading torch first makes libgol bind to that copy,
        # so the process holds one HIP runtime whichever module asks first.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        sig = {
            "gol_last_error": (ctypes.c_char_p, []),
            "gol_version": (ctypes.c_char_p, []),
            "gol_step": (c_int, [vp, i64, i64, i64, vp]),
            "gol_step_packed": (c_int, [vp, i64, i64, i64, vp, vp]),
            "gol_step_packed_ex": (c_int, [vp, i64, i64, i64, vp, vp, c_int]),
            "gol_step_packed_noalloc": (c_int, [vp, i64, i64, i64, vp, vp]),
            "gol_tune": (c_int, [i64, i64, vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
            "gol_step_packed_cfg": (c_int, [vp, i64, i64, i64, vp, vp,
                                            ctypes.POINTER(PassConfig)]),
            "gol_step_packed_population": (c_int, [vp, i64, i64, i64, vp, vp,
                                                   ctypes.POINTER(PassConfig), vp, i64, vp]),
            "gol_population": (c_int, [vp, i64, i64, vp, vp]),
            "gol_step_packed_bounded": (c_int, [vp, i64, i64, i64, vp, vp,
                                                ctypes.POINTER(PassConfig)]),
            "gol_strip_pass": (c_int, [vp, vp, vp, i64, i64, i64, vp, vp,
                                       ctypes.POINTER(PassConfig)]),
            "gol_tune_cfg": (c_int, [i64, i64, vp, ctypes.POINTER(PassConfig)]),
            "gol_pack": (c_int, [vp, i64, i64, vp, vp]),
            "gol_unpack": (c_int, [vp, i64, i64, vp, vp]),
            "gol_batch_run": (c_int, [vp, i64, vp]),
            "gol_plan_create": (c_int, [vp, i64, c_int, ctypes.POINTER(vp)]),
            "gol_plan_create_cfg": (c_int, [vp, i64, ctypes.POINTER(PassConfig),
                                            ctypes.POINTER(vp)]),
            "gol_plan_config": (c_int, [vp, ctypes.POINTER(PassConfig)]),
            "gol_debug_plan_queue_gave_up": (c_int, [vp, ctypes.POINTER(ctypes.c_int32)]),
            "gol_plan_run": (c_int, [vp, vp]),
            "gol_plan_info": (c_int, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double)]),
            "gol_plan_destroy": (c_int, [vp]),
            "gol_serve_create": (c_int, [ctypes.POINTER(ServeConfig), ctypes.POINTER(vp)]),
            "gol_serve_submit": (c_int, [vp, vp, i64, i64, i64, ctypes.POINTER(ctypes.c_uint64)]),
            "gol_serve_poll": (c_int, [vp, ctypes.c_uint64, vp, ctypes.POINTER(RequestInfo)]),
            "gol_serve_wait": (c_int, [vp, ctypes.c_uint64, vp, ctypes.POINTER(RequestInfo)]),
            "gol_serve_cancel": (c_int, [vp, ctypes.c_uint64]),
            "gol_serve_now": (ctypes.c_double, [vp]),
            "gol_serve_get_stats": (c_int, [vp, ctypes.POINTER(ServeStats)]),
            "gol_serve_destroy": (c_int, [vp]),
            "gol_set_allocator": (c_int, [vp, vp, vp]),
            "gol_debug_serve_create_host": (c_int, [ctypes.POINTER(ServeConfig), i64,
                                                    ctypes.POINTER(vp)]),
            "gol_debug_serve_host_peak_bytes": (i64, [vp]),
            "gol_debug_valu_rate": (c_int, [c_int, vp, ctypes.POINTER(ctypes.c_double)]),
            "gol_debug_plan_tables": (c_int, [vp, vp, vp, i64, c_int, c_int, vp, i64, vp, i64, vp,
                                              i64, vp, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(i64), ctypes.POINTER(i64),
                                              ctypes.POINTER(i64)]),
            "gol_debug_chunk_plan_tables": (c_int, [vp, vp, vp, i64, c_int, c_int, vp, i64, vp,
                                                    i64, vp, i64, vp,
                                                    ctypes.POINTER(ctypes.c_int32),
                                                    ctypes.POINTER(i64), ctypes.POINTER(i64),
                                                    ctypes.POINTER(i64),
                                                    ctypes.POINTER(ctypes.c_int32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != GOL_OK:
        raise GolError(rc, lib().gol_last_error().decode(errors="replace"))
    return rc


def version() -> str:
    return lib().gol_version().decode()


def words_per_row(cols: int) -> int:
    return (int(cols) + 63) // 64


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> int:
    return int(t.data_ptr())


def _dev_words(t, rows: int, cols: int, name: str, nrows: int | None = None,
               at_least: bool = False):
    """A device tensor of packed words: CUDA, C-contiguous, 8-byte elements,
    exactly (or, with at_least, at least) (nrows or rows) * W of them."""
    import torch
    n = (rows if nrows is None else nrows) * words_per_row(cols)
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype not in (torch.int64, getattr(torch, "uint64", torch.int64)):
        raise ValueError(f"{name} must hold 64-bit words (int64), got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n and not (at_least and t.numel() >= n):
        raise ValueError(f"{name} holds {t.numel()} words, expected {n}")
    return t


def _host_array(a, size: int, dtypes, name: str, writable: bool):
    """A host numpy array the library reads or writes `size` elements of."""
    if not isinstance(a, np.ndarray):
        raise ValueError(f"{name} must be a numpy array")
    if a.dtype not in dtypes:
        raise ValueError(f"{name} must have dtype {' or '.join(str(d) for d in dtypes)}, "
                         f"got {a.dtype}")
    if not a.flags.c_contiguous:
        raise ValueError(f"{name} must be C-contiguous")
    if writable and not a.flags.writeable:
        raise ValueError(f"{name} must be writable")
    if a.size != size:
        raise ValueError(f"{name} holds {a.size} elements, expected {size}")
    return a


_WORD_DTYPES = (np.dtype(np.uint64), np.dtype(np.int64))


# ---------------------------------------------------------------------------
# Single board
# ---------------------------------------------------------------------------
def step(board: np.ndarray, generations: int, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Host byte board (rows, cols), nonzero = alive -> 0/1 uint8 after G generations."""
    b = np.ascontiguousarray(board, dtype=np.uint8)
    if b.ndim != 2:
        raise ValueError("board must be 2-D")
    if out is None:
        out = np.empty_like(b)
    rows, cols = b.shape
    _host_array(out, rows * cols, (np.dtype(np.uint8),), "out", writable=True)
    _check(lib().gol_step(b.ctypes.data, rows, cols, int(generations), out.ctypes.data))
    return out


def empty_packed(rows: int, cols: int, device="cuda"):
    import torch
    return torch.empty((rows, words_per_row(cols)), dtype=torch.int64, device=device)


LAYOUT_BAND = 1
LAYOUT_PAIRED = 2
LAYOUT_RESIDENT = 3  # whole board in one workgroup's LDS for a run (small boards)
LAYOUT_QUEUE = 4  # batch plans: the persistent work-queue form


def step_packed(d_in, rows: int, cols: int, generations: int, d_out=None, stream=None,
                t_block: int = 0, config: dict | None = None):
    """Packed device board -> packed device board (asynchronous on `stream`).

    config: gol_pass_config fields as a dict (t_block, band_rows, prefetch,
    layout; missing or 0 = automatic); when given, t_block is ignored."""
    _dev_words(d_in, rows, cols, "d_in")
    if d_out is None:
        d_out = empty_packed(rows, cols, d_in.device)
    _dev_words(d_out, rows, cols, "d_out")
    if config is not None:
        c = PassConfig(**{k: int(v) for k, v in config.items()})
        _check(lib().gol_step_packed_cfg(_ptr(d_in), rows, cols, int(generations), _ptr(d_out),
                                         _stream_handle(stream), ctypes.byref(c)))
    else:
        _check(lib().gol_step_packed_ex(_ptr(d_in), rows, cols, int(generations), _ptr(d_out),
                                        _stream_handle(stream), int(t_block)))
    return d_out


# Largest packed board (bytes) gol_step_packed_noalloc takes: its fixed scratch.
NOALLOC_MAX_BYTES = 64 << 20


def step_packed_noalloc(d_in, rows: int, cols: int, generations: int, d_out, stream=None):
    """step_packed through gol_step_packed_noalloc: the library allocates
    nothing (its ping-pong board is a fixed device array), so d_out must be
    given; boards above NOALLOC_MAX_BYTES raise GolError (GOL_EINVAL)."""
    _dev_words(d_in, rows, cols, "d_in")
    _dev_words(d_out, rows, cols, "d_out")
    _check(lib().gol_step_packed_noalloc(_ptr(d_in), rows, cols, int(generations), _ptr(d_out),
                                         _stream_handle(stream)))
    return d_out


def step_packed_bounded(d_in, rows: int, cols: int, generations: int, d_out=None, stream=None,
                        config: dict | None = None):
    """step_packed on a bounded board: every cell beyond the edges is dead
    (no torus).  config as for step_packed (band layout only)."""
    _dev_words(d_in, rows, cols, "d_in")
    if d_out is None:
        d_out = empty_packed(rows, cols, d_in.device)
    _dev_words(d_out, rows, cols, "d_out")
    c = PassConfig(**{k: int(v) for k, v in (config or {}).items()})
    _check(lib().gol_step_packed_bounded(_ptr(d_in), rows, cols, int(generations), _ptr(d_out),
                                         _stream_handle(stream), ctypes.byref(c)))
    return d_out


def strip_pass(d_strip, d_top, d_bottom, rows: int, cols: int, t: int, d_out=None, stream=None,
               config: dict | None = None):
    """t generations of a row strip of a larger torus: d_top holds the t rows
    above the strip (farthest first), d_bottom the t rows below it (nearest
    first); columns wrap.  Returns d_out (the strip at generation + t)."""
    _dev_words(d_strip, rows, cols, "d_strip")
    _dev_words(d_top, rows, cols, "d_top", nrows=int(t), at_least=True)
    _dev_words(d_bottom, rows, cols, "d_bottom", nrows=int(t), at_least=True)
    if d_out is None:
        d_out = empty_packed(rows, cols, d_strip.device)
    _dev_words(d_out, rows, cols, "d_out")
    c = PassConfig(**{k: int(v) for k, v in (config or {}).items()})
    _check(lib().gol_strip_pass(_ptr(d_strip), _ptr(d_top), _ptr(d_bottom), rows, cols, int(t),
                                _ptr(d_out), _stream_handle(stream), ctypes.byref(c)))
    return d_out


VALU_KINDS = ("v_xor_b32", "v_bitop3_b32", "v_alignbit_b32", "v_mov_b32_dpp", "v_add_u32")


def valu_rate(kind: int, stream=None) -> float:
    """Lane operations per second of one VALU instruction kind (VALU_KINDS[kind])
    on the current device, from the issue-rate probe (synchronous)."""
    r = ctypes.c_double()
    _check(lib().gol_debug_valu_rate(int(kind), _stream_handle(stream), ctypes.byref(r)))
    return r.value


def population(d_packed, rows: int, cols: int, stream=None) -> int:
    """Live cells of a packed device board (waits for the result)."""
    import torch
    _dev_words(d_packed, rows, cols, "d_packed")
    cnt = torch.zeros(1, dtype=torch.int64, device=d_packed.device)
    _check(lib().gol_population(_ptr(d_packed), rows, cols, _ptr(cnt), _stream_handle(stream)))
    return int(cnt.item())


def step_packed_population(d_in, rows: int, cols: int, generations: int, checks, d_out=None,
                           stream=None, config: dict | None = None):
    """step_packed that also records the population after each generation count
    in `checks` (non-decreasing, each in 0..generations).  Returns (d_out, counts),
    counts a device int64 tensor with one entry per check (asynchronous)."""
    import torch
    _dev_words(d_in, rows, cols, "d_in")
    if d_out is None:
        d_out = empty_packed(rows, cols, d_in.device)
    _dev_words(d_out, rows, cols, "d_out")
    ch = np.ascontiguousarray(list(checks), dtype=np.int64)
    counts = torch.empty(max(1, len(ch)), dtype=torch.int64, device=d_in.device)
    c = PassConfig(**{k: int(v) for k, v in (config or {}).items()})
    _check(lib().gol_step_packed_population(_ptr(d_in), rows, cols, int(generations), _ptr(d_out),
                                            _stream_handle(stream), ctypes.byref(c),
                                            ch.ctypes.data if len(ch) else None, len(ch),
                                            _ptr(counts)))
    return d_out, counts[:len(ch)]


def tune(rows: int, cols: int, stream=None) -> tuple[int, int]:
    """Autotune the single-board path for this size; returns (t_block, band_rows)."""
    t, h = ctypes.c_int(), ctypes.c_int()
    _check(lib().gol_tune(rows, cols, _stream_handle(stream), ctypes.byref(t), ctypes.byref(h)))
    return t.value, h.value


def tune_config(rows: int, cols: int, stream=None) -> dict:
    """Autotune the single-board path for this size; returns the chosen
    gol_pass_config as a dict."""
    c = PassConfig()
    _check(lib().gol_tune_cfg(rows, cols, _stream_handle(stream), ctypes.byref(c)))
    return {f: getattr(c, f) for f, _ in PassConfig._fields_}


def _dev_bytes(t, rows: int, cols: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.uint8 or \
            not t.is_contiguous() or t.numel() != rows * cols:
        raise ValueError(f"{name} must be a contiguous uint8 device tensor of {rows * cols} "
                         "cells")
    return t


def pack(d_bytes, rows: int, cols: int, d_out=None, stream=None):
    _dev_bytes(d_bytes, rows, cols, "d_bytes")
    if d_out is None:
        d_out = empty_packed(rows, cols, d_bytes.device)
    _dev_words(d_out, rows, cols, "d_out")
    _check(lib().gol_pack(_ptr(d_bytes), rows, cols, _ptr(d_out), _stream_handle(stream)))
    return d_out


def unpack(d_packed, rows: int, cols: int, d_out=None, stream=None):
    import torch
    _dev_words(d_packed, rows, cols, "d_packed")
    if d_out is None:
        d_out = torch.empty((rows, cols), dtype=torch.uint8, device=d_packed.device)
    _dev_bytes(d_out, rows, cols, "d_out")
    _check(lib().gol_unpack(_ptr(d_packed), rows, cols, _ptr(d_out), _stream_handle(stream)))
    return d_out


# ---------------------------------------------------------------------------
# Many boards
# ---------------------------------------------------------------------------
@dataclass
class BatchBoard:
    d_in: object
    d_out: object
    rows: int
    cols: int
    generations: int


def _board_array(boards: Sequence[BatchBoard]):
    arr = (Board * max(1, len(boards)))()
    for i, b in enumerate(boards):
        _dev_words(b.d_in, b.rows, b.cols, f"boards[{i}].d_in")
        _dev_words(b.d_out, b.rows, b.cols, f"boards[{i}].d_out")
        arr[i] = Board(_ptr(b.d_in), _ptr(b.d_out), b.rows, b.cols, b.generations)
    return arr


def batch_run(boards: Sequence[BatchBoard], stream=None) -> None:
    arr = _board_array(boards)
    _check(lib().gol_batch_run(ctypes.cast(arr, ctypes.c_void_p), len(boards),
                               _stream_handle(stream)))


class Plan:
    """A batch schedule built once and replayed (HIP graph) on the same buffers."""

    def __init__(self, boards: Sequence[BatchBoard], t_block: int = 0, band_rows: int = 0,
                 queue: bool = False):
        """t_block / band_rows 0: tuned at creation (gol_plan_create_cfg);
        queue=True: the persistent work-queue form (GOL_LAYOUT_QUEUE)."""
        self._boards = list(boards)  # keep the tensors alive
        arr = _board_array(self._boards)
        h = ctypes.c_void_p()
        c = PassConfig(t_block=int(t_block), band_rows=int(band_rows),
                       layout=LAYOUT_QUEUE if queue else 0)
        _check(lib().gol_plan_create_cfg(ctypes.cast(arr, ctypes.c_void_p), len(self._boards),
                                         ctypes.byref(c), ctypes.byref(h)))
        self._h = h

    def config(self) -> dict:
        """The plan's generations per pass and band height (tuned or given)."""
        c = PassConfig()
        _check(lib().gol_plan_config(self._h, ctypes.byref(c)))
        return {"t_block": c.t_block, "band_rows": c.band_rows,
                **({"layout": "queue"} if c.layout == LAYOUT_QUEUE else {})}

    def queue_gave_up(self) -> bool:
        """Queue form: whether a wave of the last run gave up waiting (waits
        for the plan's runs)."""
        v = ctypes.c_int32()
        _check(lib().gol_debug_plan_queue_gave_up(self._h, ctypes.byref(v)))
        return bool(v.value)

    def run(self, stream=None) -> None:
        _check(lib().gol_plan_run(self._h, _stream_handle(stream)))

    def info(self):
        w, lv, cu = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().gol_plan_info(self._h, ctypes.byref(w), ctypes.byref(lv), ctypes.byref(cu)))
        return {"waves_level0": w.value, "levels": lv.value, "cell_updates": cu.value}

    def close(self) -> None:
        if self._h:
            lib().gol_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
class Server:
    """Continuous-batching request loop (gol_serve_*).

    host_executor=True builds the scheduler over host memory instead of the
    GPU (gol_debug_serve_create_host): for testing the scheduling policy; it
    does not compute the Life rule."""

    def __init__(self, hbm_budget_bytes: int = 64 << 30, chunk_generations: int = 0,
                 device: int = 0, max_resident: int = 0, t_block: int = 0,
                 host_executor: bool = False, fail_at_chunk: int = 0):
        cfg = ServeConfig(hbm_budget_bytes, chunk_generations, device, max_resident, t_block)
        h = ctypes.c_void_p()
        if host_executor:
            _check(lib().gol_debug_serve_create_host(ctypes.byref(cfg), fail_at_chunk,
                                                     ctypes.byref(h)))
        else:
            _check(lib().gol_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._shapes: dict[int, tuple[int, int]] = {}  # ticket -> (rows, cols)

    def host_peak_bytes(self) -> int:
        return int(lib().gol_debug_serve_host_peak_bytes(self._h))

    def submit(self, packed: np.ndarray, rows: int, cols: int, generations: int) -> int:
        a = np.ascontiguousarray(packed)
        if a.dtype not in _WORD_DTYPES:
            raise ValueError(f"packed board must hold 64-bit words, got {a.dtype}")
        a = a.view(np.uint64)
        if a.size != rows * words_per_row(cols):
            raise ValueError("packed board has the wrong size")
        t = ctypes.c_uint64()
        _check(lib().gol_serve_submit(self._h, a.ctypes.data, rows, cols, int(generations),
                                      ctypes.byref(t)))
        self._shapes[t.value] = (int(rows), int(cols))
        return t.value

    def _out(self, ticket: int, out: np.ndarray) -> np.ndarray:
        """The result buffer must hold exactly the ticket's rows * W words."""
        shape = self._shapes.get(int(ticket))
        if shape is None:  # never submitted here, or already retired
            raise GolError(GOL_ENOTFOUND, f"unknown or retired ticket {ticket}")
        return _host_array(out, shape[0] * words_per_row(shape[1]), _WORD_DTYPES, "out",
                           writable=True)

    def poll(self, ticket: int, out: np.ndarray):
        self._out(ticket, out)
        info = RequestInfo()
        rc = lib().gol_serve_poll(self._h, ticket, out.ctypes.data, ctypes.byref(info))
        if rc == GOL_EAGAIN:
            return None
        self._shapes.pop(int(ticket), None)  # retired, failed or cancelled
        _check(rc)
        return info

    def wait(self, ticket: int, out: np.ndarray) -> RequestInfo:
        self._out(ticket, out)
        info = RequestInfo()
        rc = lib().gol_serve_wait(self._h, ticket, out.ctypes.data, ctypes.byref(info))
        self._shapes.pop(int(ticket), None)
        _check(rc)
        return info

    def cancel(self, ticket: int) -> None:
        _check(lib().gol_serve_cancel(self._h, ticket))

    def now(self) -> float:
        return float(lib().gol_serve_now(self._h))

    def stats(self) -> dict:
        st = ServeStats()
        _check(lib().gol_serve_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}

    def close(self) -> None:
        if self._h:
            lib().gol_serve_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Host-only view of the batch planner (no device work)
# ---------------------------------------------------------------------------
SEGMENT_DTYPE = np.dtype([("board", "<i4"), ("p0", "<i4"), ("r0", "<i4"), ("h", "<u2"),
                          ("lane0", "u1"), ("nlanes", "u1")])
WAVEITEM_DTYPE = np.dtype([("seg_begin", "<i4"), ("nseg", "<i2"), ("h", "<u2"), ("maxK", "<i4"),
                           ("flags", "<i4")])


def plan_tables(rows: Iterable[int], cols: Iterable[int], generations: Iterable[int],
                t_block: int = 8, band_rows: int = 64, chunk: bool = False):
    """The batch schedule the library would build for these boards (host only).

    Returns (segs, items, levels, late_begin, starts): levels[L] = (early, late)
    wave counts of level L, which launches items[:early] and
    items[late_begin:late_begin + late]; starts[b] = level of board b's first
    pass.  chunk=True: the schedule of a served chunk (each board tiled on
    its own; band_rows 0 = the server's model choice), and a sixth element,
    the band height used."""
    r = np.ascontiguousarray(list(rows), dtype=np.int64)
    c = np.ascontiguousarray(list(cols), dtype=np.int64)
    g = np.ascontiguousarray(list(generations), dtype=np.int64)
    ns, ni, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    lb, band = ctypes.c_int32(), ctypes.c_int32()

    def call(segs, items, levels, starts):
        args = [r.ctypes.data, c.ctypes.data, g.ctypes.data, len(r), t_block, band_rows,
                segs.ctypes.data if segs is not None else None, 0 if segs is None else len(segs),
                items.ctypes.data if items is not None else None,
                0 if items is None else len(items),
                levels.ctypes.data if levels is not None else None,
                0 if levels is None else len(levels),
                starts.ctypes.data if starts is not None else None, ctypes.byref(lb),
                ctypes.byref(ns), ctypes.byref(ni), ctypes.byref(nl)]
        if chunk:
            _check(lib().gol_debug_chunk_plan_tables(*args, ctypes.byref(band)))
        else:
            _check(lib().gol_debug_plan_tables(*args))
    call(None, None, None, None)
    segs = np.zeros(ns.value, dtype=SEGMENT_DTYPE)
    items = np.zeros(ni.value, dtype=WAVEITEM_DTYPE)
    levels = np.zeros((nl.value, 2), dtype=np.int32)
    starts = np.zeros(len(r), dtype=np.int32)
    call(segs, items, levels, starts)
    if chunk:
        return segs, items, levels, int(lb.value), starts, int(band.value)
    return segs, items, levels, int(lb.value), starts
