"""Readers for the text fixtures under tests/golden/."""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def patterns():
    """{name: (kind, period, (dr, dc), cells as uint8 array)}"""
    out = {}
    with open(os.path.join(GOLDEN, "patterns.txt")) as f:
        blocks = [b for b in f.read().split("\n\n")]
    for blk in blocks:
        lines = [ln for ln in blk.splitlines() if ln and not ln.startswith("#")]
        if not lines:
            continue
        head = lines[0].split()
        name, kind, period = head[0], head[1], int(head[2])
        shift = (int(head[3]), int(head[4])) if kind == "ship" else (0, 0)
        rows = lines[1:]
        w = max(len(r) for r in rows)
        cells = np.array([[1 if ch == "O" else 0 for ch in r.ljust(w, ".")] for r in rows],
                         dtype=np.uint8)
        out[name] = (kind, period, shift, cells)
    return out


def splitmix64_answers():
    out = []
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                s, i, v = ln.split()
                out.append((int(s), int(i), int(v)))
    return out


def place(cells: np.ndarray, R: int, C: int, r0: int, c0: int) -> np.ndarray:
    """Pattern on an empty R x C torus with its top-left corner at (r0, c0), wrapped."""
    b = np.zeros((R, C), dtype=np.uint8)
    h, w = cells.shape
    for i in range(h):
        for j in range(w):
            if cells[i, j]:
                b[(r0 + i) % R, (c0 + j) % C] = 1
    return b
