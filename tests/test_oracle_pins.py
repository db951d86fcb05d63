"""Pins of the oracle against what the paper and the mathematics fix.

Each test would fail for a plausible slip in the oracle: a missing or doubled
neighbour offset, a wrong wrap index, a swapped survive/birth count, an
in-place (non-simultaneous) update, an off-by-one generation loop.
Both forms of the oracle (C loops and numpy rolls) are pinned.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import seeded_inputs
from golden_io import patterns, place

IMPLS = {
    "c": lambda b, g: oracle.life(b, g),
    "c_omp": lambda b, g: oracle.life(b, g, threads=3),
    "numpy": lambda b, g: oracle.ref.life(b, g),
}


@pytest.fixture(params=sorted(IMPLS))
def life(request):
    return IMPLS[request.param]


def expected_centre(pattern9: int) -> int:
    """Section 1's four transitions, applied to a 3x3 neighbourhood given as 9 bits
    (bit 4 is the centre)."""
    alive = (pattern9 >> 4) & 1
    n = sum((pattern9 >> k) & 1 for k in range(9) if k != 4)
    if alive:
        if n < 2:
            return 0  # under-population
        if n in (2, 3):
            return 1  # lives on
        return 0      # overcrowding
    return 1 if n == 3 else 0  # reproduction


def test_rule_all_512_neighbourhoods(life):
    live = 0
    for pat in range(512):
        b = np.zeros((5, 5), dtype=np.uint8)
        for k in range(9):
            b[1 + k // 3, 1 + k % 3] = (pat >> k) & 1
        got = int(life(b, 1)[2, 2])
        assert got == expected_centre(pat), pat
        live += got
    # closed form: C(8,3) births + C(8,2) + C(8,3) survivals
    assert live == math.comb(8, 3) + math.comb(8, 2) + math.comb(8, 3) == 140


@pytest.mark.parametrize("name", ["block", "beehive", "loaf", "boat", "tub"])
@pytest.mark.parametrize("R,C,r0,c0", [(8, 8, 2, 2), (9, 11, 7, 9), (10, 7, 0, 5)])
def test_still_lifes(life, name, R, C, r0, c0):
    kind, period, _, cells = patterns()[name]
    assert kind == "still"
    b = place(cells, R, C, r0, c0)  # some placements straddle the torus seam
    for g in (1, 2, 5):
        assert np.array_equal(life(b, g), b)


@pytest.mark.parametrize("name", ["blinker", "toad", "beacon", "pulsar"])
def test_oscillators(life, name):
    kind, period, _, cells = patterns()[name]
    R, C = cells.shape[0] + 6, cells.shape[1] + 7
    for r0, c0 in [(3, 3), (R - 2, C - 3)]:
        b = place(cells, R, C, r0, c0)
        for g in range(1, period):
            assert not np.array_equal(life(b, g), b), (name, g)
        assert np.array_equal(life(b, period), b)
        assert np.array_equal(life(b, 3 * period), b)


@pytest.mark.parametrize("name", ["glider", "lwss"])
def test_spaceships_translate(life, name):
    kind, period, (dr, dc), cells = patterns()[name]
    R, C = 13, 17
    b = place(cells, R, C, 5, 6)
    for k in (1, 2, 5):
        assert np.array_equal(life(b, k * period), np.roll(b, (k * dr, k * dc), axis=(0, 1)))


@pytest.mark.parametrize("R,C", [(6, 6), (6, 8), (7, 5), (10, 13)])
def test_glider_returns_after_lcm(R, C):
    """On an R x C torus a glider moving (+1, +1) per 4 generations first comes
    back to its start after 4 * lcm(R, C) generations."""
    _, _, _, cells = patterns()["glider"]
    b = place(cells, R, C, 1, 1)
    L = math.lcm(R, C)
    assert np.array_equal(oracle.life(b, 4 * L), b)
    cur = b
    for k in range(1, L):
        cur = oracle.life(cur, 4)
        assert not np.array_equal(cur, b), k
        assert np.array_equal(cur, np.roll(b, (k, k), axis=(0, 1)))


def test_empty_board_is_fixed(life):
    """Table 1's second figure dies out and its population stays 0 afterwards."""
    for R, C in [(1, 1), (3, 5), (32, 64)]:
        z = np.zeros((R, C), dtype=np.uint8)
        for g in (0, 1, 7):
            assert not life(z, g).any()


@pytest.mark.parametrize("R", range(1, 6))
@pytest.mark.parametrize("C", range(1, 6))
def test_full_board_dies(life, R, C):
    """Every cell of a full torus has eight live neighbours (counted per offset,
    also where offsets alias on tiny tori) and dies of overcrowding."""
    full = np.ones((R, C), dtype=np.uint8)
    assert not life(full, 1).any()


def test_generation_zero_normalises(life):
    b = np.array([[0, 7, 255], [1, 0, 2]], dtype=np.uint8)
    assert np.array_equal(life(b, 0), (b != 0).astype(np.uint8))


def _rand(R, C, seed, p=0.4):
    return seeded_inputs.board_bytes(seed, R * 1000 + C, R, C, p)


@pytest.mark.parametrize("R,C", [(7, 9), (16, 16), (5, 23)])
def test_symmetries(life, R, C):
    """The rule and the torus are invariant under translations, transposition and
    reflections, so the step commutes with them."""
    b = _rand(R, C, 11)
    g = 6
    ref = life(b, g)
    for sh in [(1, 0), (0, 1), (3, -2), (R - 1, C - 1)]:
        assert np.array_equal(life(np.roll(b, sh, axis=(0, 1)), g), np.roll(ref, sh, axis=(0, 1)))
    assert np.array_equal(life(np.ascontiguousarray(b.T), g), ref.T)
    assert np.array_equal(life(np.ascontiguousarray(b[::-1]), g), ref[::-1])
    assert np.array_equal(life(np.ascontiguousarray(b[:, ::-1]), g), ref[:, ::-1])


def test_tiling_periodicity(life):
    """A board tiled a x b times stays tiled: step(tile(x)) == tile(step(x))."""
    x = _rand(6, 10, 3)
    for a, bb in [(2, 1), (1, 3), (3, 2)]:
        assert np.array_equal(life(np.tile(x, (a, bb)), 5), np.tile(life(x, 5), (a, bb)))


def test_composition(life):
    x = _rand(12, 20, 5)
    assert np.array_equal(life(x, 7), life(life(x, 3), 4))
    assert np.array_equal(life(x, 7), life(life(life(x, 1), 1), 5))


def test_simultaneous_update_not_in_place():
    """A blinker only oscillates if all cells change at once; an in-place
    row-major sweep would not give the period-2 pattern."""
    _, _, _, cells = patterns()["blinker"]
    b = place(cells, 5, 5, 2, 1)
    one = oracle.life(b, 1)
    assert np.array_equal(one, b.T)  # horizontal blinker becomes vertical


def _all_boards(R, C):
    n = R * C
    idx = np.arange(2 ** n, dtype=np.int64)
    bits = ((idx[:, None] >> np.arange(n)[None, :]) & 1).astype(np.uint8)
    return bits.reshape(-1, R, C)


def _by_table(boards):
    """Independent evaluation: for every cell gather its 3x3 wrapped
    neighbourhood as 9 bits and look the next state up in the table of
    Section 1's transitions."""
    table = np.array([expected_centre(p) for p in range(512)], dtype=np.uint8)
    B, R, C = boards.shape
    code = np.zeros((B, R, C), dtype=np.int64)
    for k in range(9):
        dr, dc = k // 3 - 1, k % 3 - 1
        rr = (np.arange(R) + dr) % R
        cc = (np.arange(C) + dc) % C
        code |= boards[:, rr][:, :, cc].astype(np.int64) << k
    return table[code]


@pytest.mark.parametrize("R,C", [(R, C) for R in range(1, 17) for C in range(1, 17)
                                 if R * C <= 16])
def test_exhaustive_tiny_tori(R, C):
    """Every board of every torus with R * C <= 16 cells, generations 1..3."""
    boards = _all_boards(R, C)
    cur_t = boards
    cur_n = boards
    for g in range(1, 4):
        cur_t = _by_table(cur_t)
        cur_n = oracle.ref.life_step(cur_n)
        assert np.array_equal(cur_t, cur_n), (R, C, g)
    # the C oracle on every board of the small tori, a sample of the larger ones
    rng = np.random.default_rng(R * 100 + C)
    pick = range(len(boards)) if len(boards) <= 512 else rng.choice(len(boards), 256, replace=False)
    for i in pick:
        assert np.array_equal(oracle.life(boards[i], 3), cur_t[i]), (R, C, i)


def test_light_cone_window():
    """A window of a run depends only on the input within distance G."""
    b = _rand(60, 70, 9, 0.35)
    G = 9
    full = oracle.life(b, G)
    for r0, c0 in [(0, 0), (55, 66), (20, 31)]:
        k = 8
        want = oracle.torus_window(full, r0, c0, k, k)
        assert oracle.light_cone_check(want, b, None, r0, c0, k, k, G)
        packed = oracle.pack(b)
        assert oracle.light_cone_check(want, packed, 70, r0, c0, k, k, G, packed=True)
    bad = oracle.torus_window(full, 3, 4, 8, 8).copy()
    bad[0, 0] ^= 1
    assert not oracle.light_cone_check(bad, b, None, 3, 4, 8, 8, G)


@pytest.mark.parametrize("R,C", [(1, 1), (1, 64), (3, 65), (5, 127), (2, 128), (4, 200)])
def test_pack_layout(R, C):
    b = _rand(R, C, 2, 0.5)
    w = oracle.pack(b)
    W = (C + 63) // 64
    assert w.shape == (R, W) and w.dtype == np.uint64
    for r in range(R):
        for c in range(C):
            assert int(w[r, c // 64] >> np.uint64(c % 64)) & 1 == b[r, c]
    assert oracle.padding_is_zero(w, C)
    assert np.array_equal(oracle.unpack(w, C), b)


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.life(np.zeros((2, 2), np.uint8), -1)
    with pytest.raises(ValueError):
        oracle.ref.life(np.zeros((2, 2), np.uint8), -1)


# ---------------------------------------------------------------------------
# Population at chosen generation counts (the quantity of Table 1)
# ---------------------------------------------------------------------------
def test_population_at_pins():
    """Still lifes keep their count, a blinker keeps 3, a glider keeps 5 while it
    crosses the seams, the full 4x4 torus dies at once, and checks may repeat."""
    pats = patterns()
    block = place(pats["block"][3], 16, 16, 3, 4)
    assert oracle.population_at(block, [0, 1, 50]) == [4, 4, 4]
    blinker = place(pats["blinker"][3], 9, 11, 4, 4)
    assert oracle.population_at(blinker, [0, 1, 2, 2, 101]) == [3, 3, 3, 3, 3]
    glider = place(pats["glider"][3], 12, 10, 10, 8)  # crosses both seams
    assert oracle.population_at(glider, [0, 4, 40, 120]) == [5, 5, 5, 5]
    full = np.ones((4, 4), dtype=np.uint8)
    assert oracle.population_at(full, [0, 1, 2]) == [16, 0, 0]
    with pytest.raises(ValueError):
        oracle.population_at(block, [3, 2])


def test_population_at_matches_numpy_form():
    """The C oracle's counts against the numpy-roll form, step by step."""
    b = seeded_inputs.board_bytes(1209, 77, 37, 53, 0.4)
    checks = [0, 1, 2, 5, 5, 17, 40]
    want = [oracle.ref.population(oracle.ref.life(b, g)) for g in checks]
    assert oracle.population_at(b, checks) == want
    assert oracle.population_at(b, checks, threads=3) == want


# ---------------------------------------------------------------------------
# Bounded boards (cells beyond the edges dead at every generation)
# ---------------------------------------------------------------------------
def bounded_brute(board, generations):
    """Cell by cell: count the in-board neighbours with explicit loops."""
    cur = [[int(v != 0) for v in row] for row in board]
    R, C = len(cur), len(cur[0])
    for _ in range(generations):
        nxt = [[0] * C for _ in range(R)]
        for r in range(R):
            for c in range(C):
                n = 0
                for dr in (-1, 0, 1):
                    for dc in (-1, 0, 1):
                        if (dr or dc) and 0 <= r + dr < R and 0 <= c + dc < C:
                            n += cur[r + dr][c + dc]
                nxt[r][c] = 1 if n == 3 or (cur[r][c] and n == 2) else 0
        cur = nxt
    return np.array(cur, dtype=np.uint8)


@pytest.mark.parametrize("R,C", [(1, 1), (1, 7), (2, 2), (3, 3), (4, 9), (7, 5), (9, 12)])
def test_bounded_brute_force(R, C):
    for k in range(6):
        b = seeded_inputs.board_bytes(555, 10 * R + C + k, R, C, 0.45)
        for g in (0, 1, 2, 5):
            assert np.array_equal(oracle.ref.life_bounded(b, g), bounded_brute(b, g)), (R, C, k, g)


@pytest.mark.parametrize("R,C", [(3, 3), (4, 7), (10, 6), (16, 16)])
def test_bounded_full_board(R, C):
    """Closed form: a full board keeps only its four corners (3 neighbours each;
    edge cells have 5, inner cells 8), which then die alone."""
    full = np.ones((R, C), dtype=np.uint8)
    g1 = oracle.ref.life_bounded(full, 1)
    corners = np.zeros((R, C), dtype=np.uint8)
    corners[0, 0] = corners[0, -1] = corners[-1, 0] = corners[-1, -1] = 1
    assert np.array_equal(g1, corners)
    assert not oracle.ref.life_bounded(full, 2).any()
    # 2 x 2: every cell has three neighbours, a block
    assert oracle.ref.life_bounded(np.ones((2, 2), dtype=np.uint8), 5).all()


@pytest.mark.parametrize("C", [1, 2, 5, 12])
def test_bounded_line_shrinks(C):
    """A full 1 x C line loses its two end cells every generation."""
    line = np.ones((1, C), dtype=np.uint8)
    for g in range(0, C + 2):
        want = np.zeros((1, C), dtype=np.uint8)
        want[0, g:C - g] = 1
        assert np.array_equal(oracle.ref.life_bounded(line, g), want), (C, g)


def test_bounded_equals_torus_away_from_the_edges():
    """Live cells kept more than G cells from every edge never meet the
    boundary within G generations, so both boundaries give the same board."""
    inner = seeded_inputs.board_bytes(556, 0, 20, 30, 0.4)
    b = np.zeros((20 + 2 * 13, 30 + 2 * 13), dtype=np.uint8)
    b[13:33, 13:43] = inner
    for g in (1, 6, 12):
        assert np.array_equal(oracle.ref.life_bounded(b, g), oracle.life(b, g))


def test_bounded_block_in_a_corner():
    b = np.zeros((6, 6), dtype=np.uint8)
    b[:2, :2] = 1
    assert np.array_equal(oracle.ref.life_bounded(b, 9), b)


# ---------------------------------------------------------------------------
# Strip pass (a row strip of a larger torus with t halo rows on each side)
# ---------------------------------------------------------------------------
def torus_strip(board, a, rows, t):
    """Strip rows a .. a + rows - 1 of a torus and its t halo rows each side,
    every index taken modulo the torus's row count."""
    R = board.shape[0]
    idx = lambda lo, n: [(lo + k) % R for k in range(n)]
    return board[idx(a, rows)], board[idx(a - t, t)], board[idx(a + rows, t)]


@pytest.mark.parametrize("R,C,a,rows,t", [(12, 9, 3, 4, 1), (12, 9, 3, 4, 3), (10, 7, 8, 5, 2),
                                          (9, 5, 0, 9, 4), (16, 11, 5, 2, 6), (7, 3, 6, 1, 9),
                                          (20, 64, 17, 6, 5)])
def test_strip_pass_is_a_slice_of_the_torus(R, C, a, rows, t):
    """With halo rows taken from the torus, the strip after t generations is
    the torus's own rows a .. a + rows - 1 (mod R) after t generations, also
    where the strip or its halos cross row 0 and where t exceeds the strip's
    height or the torus's."""
    for k in range(4):
        b = seeded_inputs.board_bytes(557, 100 * k + R + C + a, R, C, 0.4)
        strip, top, bottom = torus_strip(b, a, rows, t)
        want = oracle.ref.life(b, t)[[(a + i) % R for i in range(rows)]]
        assert np.array_equal(oracle.ref.strip_pass(strip, top, bottom, t), want), (k,)


def test_strip_pass_one_generation_cell_by_cell():
    """t = 1 with unrelated halo rows, against an explicit loop: row -1 is
    top, row rows is bottom, columns wrap."""
    rows, C = 5, 7
    for k in range(6):
        s = seeded_inputs.board_bytes(558, k, rows, C, 0.5)
        top = seeded_inputs.board_bytes(558, 100 + k, 1, C, 0.5)
        bot = seeded_inputs.board_bytes(558, 200 + k, 1, C, 0.5)

        def cell(r, c):
            if r < 0:
                return int(top[0, c % C])
            if r >= rows:
                return int(bot[0, c % C])
            return int(s[r, c % C])
        want = np.zeros((rows, C), dtype=np.uint8)
        for r in range(rows):
            for c in range(C):
                n = sum(cell(r + dr, c + dc) for dr in (-1, 0, 1) for dc in (-1, 0, 1)
                        if dr or dc)
                want[r, c] = 1 if n == 3 or (s[r, c] and n == 2) else 0
        assert np.array_equal(oracle.ref.strip_pass(s, top, bot, 1), want), k


def test_strip_pass_light_cone():
    """The farthest halo row (t rows away) reaches only the strip's edge row:
    changing it leaves every other row as it was, and changes the edge row for
    some boards."""
    rows, C, t = 8, 20, 3
    changed = 0
    for k in range(20):
        s = seeded_inputs.board_bytes(559, k, rows, C, 0.45)
        top = seeded_inputs.board_bytes(559, 100 + k, t, C, 0.45)
        bot = seeded_inputs.board_bytes(559, 200 + k, t, C, 0.45)
        base = oracle.ref.strip_pass(s, top, bot, t)
        top2 = top.copy()
        top2[0] ^= 1
        bot2 = bot.copy()
        bot2[-1] ^= 1
        up = oracle.ref.strip_pass(s, top2, bot, t)
        down = oracle.ref.strip_pass(s, top, bot2, t)
        assert np.array_equal(up[1:], base[1:]) and np.array_equal(down[:-1], base[:-1])
        changed += int(not np.array_equal(up[0], base[0])) + int(not np.array_equal(down[-1], base[-1]))
    assert changed > 0
