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
