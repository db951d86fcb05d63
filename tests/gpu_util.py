"""Helpers for GPU tests: device tensors of packed boards, oracle comparisons."""
from __future__ import annotations

import sys

import numpy as np

import oracle
import seeded_inputs


def say(*a):
    """Print (and flush) what names the case before each GPU step."""
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(words: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(words).view(np.int64)).cuda()


def from_dev(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def rand_bytes(seed, bid, R, C, p=0.4):
    return seeded_inputs.board_bytes(seed, bid, R, C, p)


def expect_words(board_bytes: np.ndarray, G: int, threads: int = 1) -> np.ndarray:
    return oracle.pack(oracle.life(board_bytes, G, threads=threads))


def first_diff(a: np.ndarray, b: np.ndarray, cols: int) -> str:
    ua, ub = oracle.unpack(a, cols), oracle.unpack(b, cols)
    idx = np.argwhere(ua != ub)
    return f"{len(idx)} cells differ, first at {idx[:5].tolist()}"
