"""Boards at the size limits (GPU).

A board that repeats a p x q tile (p | rows, q | cols) stays a tiling of that
tile's own evolution on the p x q torus: every cell's eight neighbour offsets
land, modulo (p, q), on the tile's neighbours.  So a board of several GiB can
be checked cell for cell against the oracle run on the tile alone.  These
cases reach the largest row and column counts the interface accepts (2^30),
boards above 4 GiB (byte offsets past 32 bits), and the paired layout just
below its 2 GiB limit.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol

from gpu_util import expect_words, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu


def tiled_board(tile_bytes: np.ndarray, R: int, C: int):
    """Packed device board of R x C cells repeating tile_bytes (q % 64 == 0)."""
    p, q = tile_bytes.shape
    assert R % p == 0 and C % q == 0 and q % 64 == 0
    small = to_dev(oracle.pack(tile_bytes))          # p x q/64 words
    return small.repeat(R // p, C // q).contiguous()


def assert_tiled(d_out, want_words: np.ndarray, R: int, C: int):
    import torch
    p, ws = want_words.shape
    exp = to_dev(want_words).view(1, p, 1, ws)
    same = d_out.view(R // p, p, (C // 64) // ws, ws) == exp
    ok = bool(same.all())
    if not ok:
        bad = torch.nonzero(~same)[:5].tolist()
        pytest.fail(f"tiling broken at (row block, row, col block, word) {bad}")


def free():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# (rows, cols, tile rows, tile cols, generations)
EXTREME = [
    (1 << 30, 64, 16, 64, 13),    # most rows: 8 GiB, one word per row
    (40, 1 << 30, 8, 128, 13),    # most columns: 5 GiB, 2^24 words per row
]


@pytest.mark.parametrize("R,C,p,q,G", EXTREME, ids=["rows_2^30", "cols_2^30"])
def test_largest_boards_default_path(R, C, p, q, G):
    tile = rand_bytes(1230, p + q, p, q, 0.4)
    say(f"extreme R={R} C={C} tile {p}x{q} G={G}")
    d_in = tiled_board(tile, R, C)
    d_out = gol.step_packed(d_in, R, C, G)
    assert_tiled(d_out, expect_words(tile, G), R, C)
    del d_in, d_out
    free()


def test_paired_layout_just_below_2_gib():
    R, C, p, q, G = 16376, 1 << 20, 8, 128, 25  # 16376 x 2^14 words x 8 B < 2^31
    assert R * (C // 64) * 8 < 1 << 31
    tile = rand_bytes(1231, 1, p, q, 0.4)
    say(f"paired near 2 GiB R={R} C={C} G={G}")
    d_in = tiled_board(tile, R, C)
    d_out = gol.step_packed(d_in, R, C, G,
                            config=dict(t_block=12, layout=gol.LAYOUT_PAIRED, band_rows=30))
    assert_tiled(d_out, expect_words(tile, G), R, C)
    del d_in, d_out
    free()


def test_batch_with_a_board_above_4_gib():
    """One 5 GiB board among small ones in one batched schedule."""
    R, C, p, q, G = 40, 1 << 30, 8, 128, 29
    tile = rand_bytes(1232, 2, p, q, 0.35)
    say(f"batch with R={R} C={C} G={G}")
    d_big = tiled_board(tile, R, C)
    big_out = gol.empty_packed(R, C)
    boards = [gol.BatchBoard(d_big, big_out, R, C, G)]
    small = []
    for i, (r, c, g) in enumerate([(37, 100, 17), (5, 3, 29), (130, 2049, 12)]):
        b = rand_bytes(1233, i, r, c, 0.4)
        d = to_dev(oracle.pack(b))
        o = gol.empty_packed(r, c)
        boards.append(gol.BatchBoard(d, o, r, c, g))
        small.append((o, expect_words(b, g)))
    gol.batch_run(boards)
    assert_tiled(big_out, expect_words(tile, G), R, C)
    for o, want in small:
        got = o.cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want)
    del d_big, big_out, boards
    free()
