"""Strip pass (a row strip of a larger torus, halo rows in separate buffers) on
the GPU against the oracle (``oracle.ref.strip_pass``, ``oracle.life``), bit
for bit."""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
import seeded_inputs
from gpu_util import first_diff, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu

T_ALL = [1, 2, 4, 8, 12, 16]


def dirty(w: np.ndarray, C: int) -> np.ndarray:
    """Every padding bit set (they are not cells)."""
    w = w.copy()
    if C % 64:
        w[:, -1] |= ~np.uint64((1 << (C % 64)) - 1)
    return w


def run_strip(strip, top, bottom, t, config=None):
    """Byte boards in, packed words of the GPU result out (dirty padding in)."""
    rows, C = strip.shape
    d = [to_dev(dirty(oracle.pack(x), C)) for x in (strip, top, bottom)]
    return from_dev(gol.strip_pass(d[0], d[1], d[2], rows, C, t, config=config))


SHAPES = [(1, 1), (3, 5), (1, 100), (40, 33), (41, 64), (130, 95), (70, 2049), (257, 4096),
          (300, 1000)]


@pytest.mark.parametrize("t", T_ALL)
def test_strip_matches_oracle(t):
    """Strip and halo rows drawn independently (no torus behind them)."""
    for i, (rows, C) in enumerate(SHAPES):
        s = rand_bytes(4420, 100 * t + i, rows, C, 0.4)
        top = rand_bytes(4421, 100 * t + i, t, C, 0.4)
        bot = rand_bytes(4422, 100 * t + i, t, C, 0.4)
        say(f"strip t={t} rows={rows} C={C}")
        got = run_strip(s, top, bot, t)
        want = oracle.pack(oracle.ref.strip_pass(s, top, bot, t))
        assert oracle.padding_is_zero(got, C)
        assert np.array_equal(got, want), (t, rows, C, first_diff(got, want, C))


def test_strip_band_heights_and_prefetch():
    rows, C, t = 150, 700, 12
    s = rand_bytes(4423, 0, rows, C, 0.45)
    top = rand_bytes(4423, 1, t, C, 0.45)
    bot = rand_bytes(4423, 2, t, C, 0.45)
    want = oracle.pack(oracle.ref.strip_pass(s, top, bot, t))
    for h, pd in ((1, 9), (7, 6), (40, 9), (150, 6), (400, 9)):
        say("strip band rows", h, "prefetch", pd)
        got = run_strip(s, top, bot, t, config=dict(band_rows=h, prefetch=pd))
        assert np.array_equal(got, want), (h, pd)


def ring_run(board, heights, G, t):
    """A torus cut into strips of the given heights, each in its own buffer,
    advanced G generations in passes of t: before each pass every strip's
    halo buffers are filled from its neighbours' rows (the exchange a ring of
    devices would make), then every strip runs one pass."""
    import torch
    R, C = board.shape
    assert sum(heights) == R and G % t == 0
    starts = np.cumsum([0] + heights[:-1])
    words = oracle.pack(board)
    cur = [to_dev(words[a:a + h]) for a, h in zip(starts, heights)]
    nxt = [torch.empty_like(x) for x in cur]
    W = words.shape[1]
    top = [torch.empty((t, W), dtype=torch.int64, device="cuda") for _ in heights]
    bot = [torch.empty((t, W), dtype=torch.int64, device="cuda") for _ in heights]
    for _ in range(G // t):
        whole = torch.cat(cur, 0)  # the exchange: rows of the neighbours, modulo R
        for k, (a, h) in enumerate(zip(starts, heights)):
            top[k].copy_(whole[torch.arange(a - t, a, device="cuda") % R])
            bot[k].copy_(whole[torch.arange(a + h, a + h + t, device="cuda") % R])
        for k, h in enumerate(heights):
            gol.strip_pass(cur[k], top[k], bot[k], h, C, t, d_out=nxt[k])
        cur, nxt = nxt, cur
    return from_dev(torch.cat(cur, 0))


@pytest.mark.parametrize("R,C,heights,G,t", [
    (96, 200, [32, 32, 32], 48, 16),
    (100, 64, [1, 60, 7, 32], 36, 12),   # a strip thinner than t
    (40, 33, [40], 24, 8),                # one strip: its halos are its own rows
    (64, 4096, [16, 16, 16, 16], 40, 4),
])
def test_ring_of_strips_equals_the_torus(R, C, heights, G, t):
    b = rand_bytes(4424, R + C, R, C, 0.4)
    say(f"ring R={R} C={C} heights={heights} G={G} t={t}")
    got = ring_run(b, heights, G, t)
    want = oracle.pack(oracle.life(b, G))
    assert np.array_equal(got, want), first_diff(got, want, C)


def test_strip_at_one_gpus_share_of_the_65536_board():
    """The strip one of eight GPUs would hold of the 65536^2 board (8192 x
    65536), one pass of t = 16 with independent random halos, in the launch
    configuration the benchmark times.  Rows 0 .. h - 1 of the result follow
    from the top halo and strip rows 0 .. h + t - 1; the oracle runs that full
    width region, and the same near the bottom edge and in the middle."""
    rows, C, t, h = 8192, 65536, 16, 24
    s = seeded_inputs.board_packed(1209, 8, rows, C, 0.5)
    top = seeded_inputs.board_packed(1209, 9, t, C, 0.5)
    bot = seeded_inputs.board_packed(1209, 10, t, C, 0.5)
    say("strip 8192 x 65536, t 16")
    got = from_dev(gol.strip_pass(to_dev(s), to_dev(top), to_dev(bot), rows, C, t))
    cells = lambda w: oracle.unpack(w, C)
    cases = [
        (0, cells(top), cells(s[h:h + t])),                        # top edge
        (rows - h, cells(s[rows - h - t:rows - h]), cells(bot)),   # bottom edge
        (4000, cells(s[4000 - t:4000]), cells(s[4000 + h:4000 + h + t])),
    ]
    for r0, above, below in cases:
        want = oracle.ref.strip_pass(cells(s[r0:r0 + h]), above, below, t)
        assert np.array_equal(cells(got[r0:r0 + h]), want), r0
