"""ORACLE (numpy form) -- test infrastructure only; the product path never imports it.

The same definition as ``gol_oracle.c``, written a second way: the eight
neighbour counts are sums of the board rolled by each of the eight offsets of
the Moore neighbourhood (Section 1, Introduction), rolling wraps around both
axes, which is the torus of Section 2.2, and the whole board is replaced at
once each generation (Section 1).  A leading batch axis is allowed, so every
board of a tiny torus can be stepped in one call.
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dr, dc) for dr in (-1, 0, 1) for dc in (-1, 0, 1) if (dr, dc) != (0, 0)]


def neighbour_count(board: np.ndarray) -> np.ndarray:
    """Live-neighbour count of every cell; board shape (..., R, C), cells 0/1."""
    b = (np.asarray(board) != 0).astype(np.int16)
    n = np.zeros_like(b)
    for dr, dc in OFFSETS:
        # value at (r, c) of the rolled array is b[(r - dr) mod R, (c - dc) mod C]
        n += np.roll(b, shift=(dr, dc), axis=(-2, -1))
    return n


def life_step(board: np.ndarray) -> np.ndarray:
    """One B3/S23 generation on the torus (Section 1 transitions)."""
    alive = np.asarray(board) != 0
    n = neighbour_count(board)
    born = (~alive) & (n == 3)
    survive = alive & ((n == 2) | (n == 3))
    return (born | survive).astype(np.uint8)


def life(board: np.ndarray, generations: int) -> np.ndarray:
    if generations < 0:
        raise ValueError("generations must be >= 0")
    cur = (np.asarray(board) != 0).astype(np.uint8)
    for _ in range(generations):
        cur = life_step(cur)
    return cur


def population(board: np.ndarray) -> int:
    """Live-cell count (the quantity of the paper's Table 1)."""
    return int(np.count_nonzero(board))


def neighbour_count_bounded(board: np.ndarray) -> np.ndarray:
    """Live-neighbour count when every cell beyond the board's edges is dead:
    the board is surrounded by one ring of dead cells and each of the eight
    offsets is a slice of the ringed board (no wrap)."""
    b = (np.asarray(board) != 0).astype(np.int16)
    R, C = b.shape[-2], b.shape[-1]
    pad = np.zeros(b.shape[:-2] + (R + 2, C + 2), dtype=np.int16)
    pad[..., 1:R + 1, 1:C + 1] = b
    n = np.zeros_like(b)
    for dr, dc in OFFSETS:
        n += pad[..., 1 + dr:1 + dr + R, 1 + dc:1 + dc + C]
    return n


def life_bounded(board: np.ndarray, generations: int) -> np.ndarray:
    """B3/S23 (Section 1 transitions, every cell at once) on a finite board in
    a dead surrounding: cells beyond the edges are dead at every generation
    and are not evolved."""
    if generations < 0:
        raise ValueError("generations must be >= 0")
    cur = (np.asarray(board) != 0).astype(np.uint8)
    for _ in range(generations):
        alive = cur != 0
        n = neighbour_count_bounded(cur)
        cur = (((~alive) & (n == 3)) | (alive & ((n == 2) | (n == 3)))).astype(np.uint8)
    return cur


def strip_pass(strip: np.ndarray, top: np.ndarray, bottom: np.ndarray,
               generations: int) -> np.ndarray:
    """A row strip of a larger torus after ``generations`` (= t) generations,
    given the t rows above it (``top``, farthest first) and the t rows below
    it (``bottom``, nearest first) at the start: the unit of the row
    decomposition of Section 2.1.  Rows are whole torus rows, so columns wrap.

    A cell's state after t generations depends only on cells within t rows of
    it (one row per generation), so the strip's rows follow from the stacked
    rows top | strip | bottom alone.  The stack is evolved with nothing above
    or below it (those rows read as dead) and columns wrapping; whatever that
    cut changes spreads inwards one row per generation and stays inside the
    t halo rows, which are dropped."""
    t = int(generations)
    if t < 0:
        raise ValueError("generations must be >= 0")
    s = (np.asarray(strip) != 0).astype(np.uint8)
    a = (np.asarray(top) != 0).astype(np.uint8)
    b = (np.asarray(bottom) != 0).astype(np.uint8)
    if a.shape != (t, s.shape[1]) or b.shape != (t, s.shape[1]):
        raise ValueError("top and bottom must hold t rows of the strip's width")
    cur = np.concatenate([a, s, b], axis=0)
    H, C = cur.shape
    for _ in range(t):
        pad = np.zeros((H + 2, C), dtype=np.int16)
        pad[1:H + 1] = cur
        n = np.zeros((H, C), dtype=np.int16)
        for dr, dc in OFFSETS:
            # rows: no wrap (slice of the padded stack); columns: wrap (roll)
            n += np.roll(pad[1 + dr:1 + dr + H], shift=-dc, axis=1)
        alive = cur != 0
        cur = (((~alive) & (n == 3)) | (alive & ((n == 2) | (n == 3)))).astype(np.uint8)
    return cur[t:t + s.shape[0]]
