"""Bounded boards (cells beyond the edges dead at every generation) on the GPU
against the oracle's bounded form (``oracle.ref.life_bounded``), bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
from gpu_util import first_diff, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu


def want_words(b, G):
    return oracle.pack(oracle.ref.life_bounded(b, G))


def dirty(w: np.ndarray, C: int) -> np.ndarray:
    w = w.copy()
    if C % 64:
        w[:, -1] |= ~np.uint64((1 << (C % 64)) - 1)
    return w


# shapes: tiny, odd widths around 32 / 64, several strips (> 62 dwords) and
# bands, a single row / column
SHAPES = [(1, 1), (1, 100), (100, 1), (3, 3), (5, 31), (7, 33), (40, 64), (41, 95),
          (70, 2049), (257, 4095), (130, 4096), (300, 1000)]


@pytest.mark.parametrize("T", [1, 2, 4, 8, 12, 16])
def test_bounded_matches_oracle(T):
    for i, (R, C) in enumerate(SHAPES):
        G = 2 * T + 3  # remainder passes too
        b = rand_bytes(4412, 100 * T + i, R, C, 0.4)
        say(f"bounded T={T} R={R} C={C} G={G}")
        d_out = gol.step_packed_bounded(to_dev(dirty(oracle.pack(b), C)), R, C, G,
                                        config=dict(t_block=T))
        got = from_dev(d_out)
        want = want_words(b, G)
        assert oracle.padding_is_zero(got, C)
        assert np.array_equal(got, want), (R, C, T, first_diff(got, want, C))


def test_bounded_band_heights_and_in_place():
    R, C, G = 150, 700, 37
    b = rand_bytes(4413, 0, R, C, 0.45)
    for h in (1, 7, 40, 150, 400):
        say("bounded band rows", h)
        got = from_dev(gol.step_packed_bounded(to_dev(oracle.pack(b)), R, C, G,
                                               config=dict(t_block=12, band_rows=h)))
        assert np.array_equal(got, want_words(b, G)), h
    d = to_dev(oracle.pack(b))
    gol.step_packed_bounded(d, R, C, 25, d_out=d, config=dict(t_block=8))  # 4 passes
    assert np.array_equal(from_dev(d), want_words(b, 25))
    d = to_dev(oracle.pack(b))
    gol.step_packed_bounded(d, R, C, 24, d_out=d, config=dict(t_block=8))  # 3 passes: odd
    assert np.array_equal(from_dev(d), want_words(b, 24))


def test_bounded_differs_from_torus():
    """A glider heading off the bottom-right edge: on the torus it comes back,
    on a bounded board it does not."""
    b = np.zeros((12, 12), dtype=np.uint8)
    b[8, 9] = b[9, 10] = b[10, 8] = b[10, 9] = b[10, 10] = 1
    d = to_dev(oracle.pack(b))
    bounded = from_dev(gol.step_packed_bounded(d, 12, 12, 24))
    torus = from_dev(gol.step_packed(d, 12, 12, 24))
    assert np.array_equal(bounded, want_words(b, 24))
    assert np.array_equal(torus, oracle.pack(oracle.life(b, 24)))
    assert not np.array_equal(bounded, torus)


def test_bounded_16384_board_corners():
    """The benchmark board's size, 100 generations: each corner's 64 x 64 cells
    depend only on the 164 x 164 corner region (the edges are dead, and cells
    farther than 100 from the window cannot reach it), which the oracle runs."""
    R = C = 16384
    G, w = 100, 64
    import seeded_inputs
    full = seeded_inputs.board_packed(1209, 0, R, C, 0.3)
    say("bounded 16384^2")
    got = from_dev(gol.step_packed_bounded(to_dev(full), R, C, G))
    cells = oracle.unpack
    k = w + G
    for rs, cs in ((slice(0, k), slice(0, k)), (slice(R - k, R), slice(0, k)),
                   (slice(0, k), slice(C - k, C)), (slice(R - k, R), slice(C - k, C))):
        rows = full[rs]
        region = cells(rows, C)[:, cs]
        want = oracle.ref.life_bounded(region, G)
        out = cells(got[rs], C)[:, cs]
        # the window at the board's corner: rows / cols within w of the true edges
        r_in = slice(0, w) if rs.start == 0 else slice(k - w, k)
        c_in = slice(0, w) if cs.start == 0 else slice(k - w, k)
        assert np.array_equal(out[r_in, c_in], want[r_in, c_in]), (rs, cs)
