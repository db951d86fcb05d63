"""The seeded input generator: known answers and layout agreement."""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs
from golden_io import splitmix64_answers


def test_splitmix64_known_answers():
    for state, i, want in splitmix64_answers():
        assert seeded_inputs.splitmix64_nth(state, i) == want


@pytest.mark.parametrize("R,C", [(1, 1), (3, 63), (4, 64), (5, 65), (17, 300)])
def test_bytes_and_packed_agree(R, C):
    b = seeded_inputs.board_bytes(1209, 3, R, C, 0.37)
    w = seeded_inputs.board_packed(1209, 3, R, C, 0.37)
    assert np.array_equal(oracle.pack(b), w)
    assert oracle.padding_is_zero(w, C)


def test_cell_definition_small():
    """Cell (r, c) is alive iff the high 32 bits of the (r*C + c + 1)-th output of
    the stream keyed by (seed, board) fall below floor(p * 2^32)."""
    seed, bid, R, C, p = 4408, 7, 3, 5, 0.3
    b = seeded_inputs.board_bytes(seed, bid, R, C, p)
    M = 2 ** 64 - 1
    G = 0x9E3779B97F4A7C15
    mix = seeded_inputs._load().si_mix64
    key = (mix((seed + G) & M) ^ mix((bid + 2 * G) & M)) & M
    thr = math.floor(p * 2 ** 32)
    for r in range(R):
        for c in range(C):
            h = seeded_inputs.splitmix64_nth(key, r * C + c + 1)
            assert b[r, c] == int((h >> 32) < thr)


@pytest.mark.parametrize("p", [0.1, 0.3, 0.5, 0.6])
def test_density(p):
    b = seeded_inputs.board_bytes(1209, 0, 512, 512, p)
    n = b.size
    sd = math.sqrt(n * p * (1 - p))
    assert abs(int(b.sum()) - n * p) < 6 * sd


def test_extreme_densities():
    assert not seeded_inputs.board_bytes(1, 1, 9, 9, 0.0).any()
    assert seeded_inputs.board_bytes(1, 1, 9, 9, 1.0).all()


def test_boards_differ_by_id_and_seed():
    a = seeded_inputs.board_bytes(1, 1, 32, 32, 0.5)
    assert not np.array_equal(a, seeded_inputs.board_bytes(1, 2, 32, 32, 0.5))
    assert not np.array_equal(a, seeded_inputs.board_bytes(2, 1, 32, 32, 0.5))


def test_batch_specs_ranges():
    specs = seeded_inputs.batch_specs(1209, n=4096)
    assert len(specs) == 4096
    assert all(64 <= s.rows <= 2048 and 64 <= s.cols <= 2048 for s in specs)
    assert all(0.1 <= s.p <= 0.6 and 10 <= s.generations <= 1000 for s in specs)
    assert specs == seeded_inputs.batch_specs(1209, n=4096)
    # log-uniform sides: the median side is close to sqrt(64 * 2048)
    med = np.median([s.rows for s in specs])
    assert 300 < med < 420


def test_serve_specs_poisson():
    specs = seeded_inputs.serve_specs(1209, n=4096, rate_per_s=500.0)
    t = np.array([s.arrival_s for s in specs])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 500.0) < 0.1 / 500.0
    assert all(32 <= s.rows <= 8192 and 1 <= s.generations <= 10000 for s in specs)


def test_device_generator_library_exports_its_entry_point():
    """The device form (gen_device.hip) loads on a machine without a GPU and
    exports its one entry point; its output is checked on the GPU."""
    lib = seeded_inputs._load_device()
    assert hasattr(lib, "si_gen_packed_device")
