"""Population (live-cell count) on the GPU against the oracle.

The paper tabulates the population of its patterns at chosen iteration counts
(Table 1: 100, 200, 500, 1000, 2000).  gol_population counts a packed board;
gol_step_packed_population advances a board and records the population after
each chosen generation count, counted after the pass that ends at each of them.
"""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
from gpu_util import expect_words, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu


def dirty(w: np.ndarray, C: int) -> np.ndarray:
    """Every padding bit set (they are not cells)."""
    w = w.copy()
    if C % 64:
        w[:, -1] |= ~np.uint64((1 << (C % 64)) - 1)
    return w


@pytest.mark.parametrize("R,C", [(1, 1), (1, 64), (3, 5), (7, 63), (40, 100), (33, 129),
                                 (257, 4095), (64, 4096), (1000, 1), (300, 2049)])
def test_population_matches_oracle(R, C):
    b = rand_bytes(77, R + C, R, C, 0.45)
    say("population", R, C)
    got = gol.population(to_dev(dirty(oracle.pack(b), C)), R, C)
    assert got == int(np.count_nonzero(b))


def test_population_of_a_board_above_4_gib():
    """2^30 rows x 64 columns repeating a 16 x 64 tile: tile count x 2^26."""
    R, C = 1 << 30, 64
    tile = rand_bytes(78, 0, 16, 64, 0.4)
    d = to_dev(oracle.pack(tile)).repeat(R // 16, 1).contiguous()
    say("population 8 GiB")
    assert gol.population(d, R, C) == int(np.count_nonzero(tile)) * (R // 16)
    del d
    import torch
    torch.cuda.empty_cache()


# (rows, cols, generations, checks, config): every layout and pass length,
# checks at 0, repeated, inside and at the end of remainder passes
CASES = [
    (96, 2048, 40, [0, 5, 5, 13, 37, 40], None),
    (100, 300, 37, [1, 2, 16, 36], dict(t_block=8)),
    (70, 3969, 33, [12, 24, 33], dict(t_block=12, layout=gol.LAYOUT_BAND, band_rows=7)),
    # paired layouts whose last pair overlaps the first (2 H x pairs > rows)
    (40, 64, 37, [12, 24, 36, 37], dict(t_block=12, layout=gol.LAYOUT_PAIRED, band_rows=20)),
    (41, 32, 24, [8, 16, 24], dict(t_block=8, layout=gol.LAYOUT_PAIRED, band_rows=10)),
    (130, 160, 50, [0, 16, 48, 50], dict(t_block=16, layout=gol.LAYOUT_PAIRED, band_rows=65)),
    (257, 4096, 30, [12, 29, 30], dict(t_block=12, layout=gol.LAYOUT_PAIRED, band_rows=22)),
    (5, 5, 20, [3, 20], None),
    (33, 100, 0, [0, 0], None),
]


@pytest.mark.parametrize("R,C,G,checks,cfg", CASES)
def test_step_population_matches_oracle(R, C, G, checks, cfg):
    b = rand_bytes(4410, R * 3 + C, R, C, 0.4)
    say(f"step population R={R} C={C} G={G} checks={checks} cfg={cfg}")
    d_in = to_dev(dirty(oracle.pack(b), C))
    d_out, counts = gol.step_packed_population(d_in, R, C, G, checks, config=cfg)
    got = from_dev(d_out)
    assert np.array_equal(got, expect_words(b, G))
    assert counts.cpu().tolist() == oracle.population_at(b, checks)


def test_step_population_in_place_odd_pass_count():
    R, C, G = 64, 256, 21  # passes 1, 4, 16 under t_block 16
    b = rand_bytes(4411, 0, R, C, 0.5)
    d = to_dev(oracle.pack(b))
    checks = [1, 5, 21]
    _, counts = gol.step_packed_population(d, R, C, G, checks, d_out=d, config=dict(t_block=16))
    assert np.array_equal(from_dev(d), expect_words(b, G))
    assert counts.cpu().tolist() == oracle.population_at(b, checks)


def test_table1_iteration_counts_on_a_16384_board():
    """The benchmark board's size with the paper's Table 1 iteration counts, in
    the tuned launch configuration: a 16384 x 16384 board repeating a 128 x 256
    tile has, at every generation, (16384 / 128) x (16384 / 256) times the
    tile's own population on its 128 x 256 torus."""
    R = C = 16384
    tile = rand_bytes(1209, 3, 128, 256, 0.3)
    d = to_dev(oracle.pack(tile)).repeat(R // 128, C // 256).contiguous()
    checks = [100, 200, 500, 1000]
    say("table 1 checks on 16384^2")
    cfg = gol.tune_config(R, C)
    d_out, counts = gol.step_packed_population(d, R, C, 1000, checks, config=cfg)
    reps = (R // 128) * (C // 256)
    assert counts.cpu().tolist() == [reps * p for p in oracle.population_at(tile, checks)]
