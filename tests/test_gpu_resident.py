"""Resident layout (the whole board in one workgroup's LDS for a run) on the GPU
against the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
from gpu_util import expect_words, first_diff, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu

RES = dict(layout=gol.LAYOUT_RESIDENT)


def dirty(w: np.ndarray, C: int) -> np.ndarray:
    """Every padding bit set (they are not cells)."""
    w = w.copy()
    if C % 64:
        w[:, -1] |= ~np.uint64((1 << (C % 64)) - 1)
    return w


# tiny tori, widths around 32 / 64, Table 2's boards, and boards at the
# layout's limits: 7168 rows of one dword, rows of 1024 dwords (the widest),
# 248 x 1024 (two generations plus their segment pads just under 64 KiB)
SHAPES = [(1, 1), (2, 3), (3, 2), (1, 100), (100, 1), (5, 31), (7, 33), (40, 64), (41, 95),
          (60, 120), (120, 240), (256, 256), (130, 1000), (7168, 32), (1, 32768), (7, 32768),
          (3, 32767), (248, 1024)]


@pytest.mark.parametrize("R,C", SHAPES)
def test_resident_matches_oracle(R, C):
    b = rand_bytes(4430, R + C, R, C, 0.4)
    for G in (1, 7, 30):
        say(f"resident R={R} C={C} G={G}")
        got = from_dev(gol.step_packed(to_dev(dirty(oracle.pack(b), C)), R, C, G, config=RES))
        want = expect_words(b, G)
        assert oracle.padding_is_zero(got, C)
        assert np.array_equal(got, want), (R, C, G, first_diff(got, want, C))


def test_every_tiny_torus_shape():
    for R in range(1, 6):
        for C in range(1, 6):
            b = rand_bytes(4431, 10 * R + C, R, C, 0.5)
            got = from_dev(gol.step_packed(to_dev(oracle.pack(b)), R, C, 9, config=RES))
            assert np.array_equal(got, expect_words(b, 9)), (R, C)


def test_long_runs_and_default_choice():
    """Table 2's largest case (2000 iterations) and a 64^2 board through the
    default configuration, which takes this layout for boards that small, and
    the 256^2 board asked for explicitly."""
    for R, C, G, cfg in ((120, 240, 2000, None), (64, 64, 1000, None), (256, 256, 100, RES)):
        b = rand_bytes(4432, G, R, C, 0.3)
        say(f"resident R={R} C={C} G={G} cfg={cfg}")
        got = from_dev(gol.step_packed(to_dev(oracle.pack(b)), R, C, G, config=cfg))
        assert np.array_equal(got, expect_words(b, G)), (R, C, G)


def test_in_place_population_and_host_api():
    R, C, G = 100, 300, 45
    b = rand_bytes(4433, 0, R, C, 0.4)
    d = to_dev(oracle.pack(b))
    gol.step_packed(d, R, C, G, d_out=d, config=RES)
    assert np.array_equal(from_dev(d), expect_words(b, G))
    checks = [0, 1, 20, 20, 45]
    d_out, counts = gol.step_packed_population(to_dev(oracle.pack(b)), R, C, G, checks,
                                               config=RES)
    assert np.array_equal(from_dev(d_out), expect_words(b, G))
    assert counts.cpu().tolist() == oracle.population_at(b, checks)
    # the host byte API on a board the default sends to this layout
    b2 = rand_bytes(4433, 1, 60, 120, 0.5)
    assert np.array_equal(gol.step(b2, 500), oracle.life(b2, 500))


def test_runs_longer_than_one_launch():
    """A run of more than 65536 generations is split into several launches."""
    R, C, G = 8, 40, 65536 * 2 + 7
    b = rand_bytes(4434, 0, R, C, 0.5)
    say(f"resident R={R} C={C} G={G}")
    got = from_dev(gol.step_packed(to_dev(oracle.pack(b)), R, C, G, config=RES))
    assert np.array_equal(got, expect_words(b, G))


def test_resident_rejects_a_board_too_large():
    import torch
    d = torch.zeros((257, 16), dtype=torch.int64, device="cuda")
    with pytest.raises(gol.GolError):
        gol.step_packed(d, 257, 1024, 3, config=RES)
    d = torch.zeros((1, 513), dtype=torch.int64, device="cuda")
    with pytest.raises(gol.GolError):
        gol.step_packed(d, 1, 32769, 3, config=RES)  # a row of 1025 dwords
