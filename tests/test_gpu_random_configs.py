"""Seeded random cases on the GPU against the oracle: board shapes, generation
counts and launch configurations drawn together, so that combinations no
hand-picked case names (odd widths with short bands, remainder passes after
paired passes, resident boards at odd sizes, bounded and strip passes of
random shape) are still compared bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
from gpu_util import expect_words, first_diff, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu

BAND_PD = {1: (3, 6), 2: (3, 6), 4: (3, 6), 8: (6, 9), 12: (6, 9), 16: (9, 12)}


def draw_case(rng):
    R = int(rng.integers(1, 300))
    C = int(rng.integers(1, 700))
    G = int(rng.integers(0, 60))
    kind = rng.choice(["default", "band", "paired", "resident"])
    if kind == "paired" and (C % 32 or R < 2):
        kind = "band"
    if kind == "resident" and R * ((C + 31) // 32) > 7168:
        kind = "band"
    if kind == "default":
        return R, C, G, None
    if kind == "resident":
        return R, C, G, dict(layout=gol.LAYOUT_RESIDENT)
    if kind == "band":
        T = int(rng.choice(list(BAND_PD)))
        return R, C, G, dict(t_block=T, layout=gol.LAYOUT_BAND, prefetch=int(rng.choice(BAND_PD[T])),
                             band_rows=int(rng.integers(1, R + 20)))
    T = int(rng.choice([8, 12, 16]))
    H = int(rng.integers(T, max(T + 1, R // 2 + 1)))  # bands of at least t_block rows
    return R, C, G, dict(t_block=T, layout=gol.LAYOUT_PAIRED, prefetch=int(rng.choice([9, 12])),
                         band_rows=H)


def test_random_single_board_cases():
    rng = np.random.default_rng(4440)
    ran = 0
    for k in range(60):
        R, C, G, cfg = draw_case(rng)
        b = rand_bytes(4441, k, R, C, float(rng.uniform(0.1, 0.7)))
        say(f"case {k}: R={R} C={C} G={G} cfg={cfg}")
        try:
            d_out = gol.step_packed(to_dev(oracle.pack(b)), R, C, G, config=cfg)
        except gol.GolError as e:
            # only a paired geometry the layout cannot hold may be refused
            assert cfg is not None and cfg.get("layout") == gol.LAYOUT_PAIRED, (cfg, e)
            continue
        got = from_dev(d_out)
        want = expect_words(b, G)
        assert np.array_equal(got, want), (k, R, C, G, cfg, first_diff(got, want, C))
        ran += 1
    assert ran >= 50


def test_random_bounded_and_strip_cases():
    rng = np.random.default_rng(4442)
    for k in range(25):
        R = int(rng.integers(1, 200))
        C = int(rng.integers(1, 500))
        G = int(rng.integers(0, 40))
        T = int(rng.choice([1, 2, 4, 8, 12, 16]))
        b = rand_bytes(4443, k, R, C, 0.4)
        say(f"bounded {k}: R={R} C={C} G={G} T={T}")
        got = from_dev(gol.step_packed_bounded(to_dev(oracle.pack(b)), R, C, G,
                                               config=dict(t_block=T)))
        assert np.array_equal(got, oracle.pack(oracle.ref.life_bounded(b, G))), (k, R, C, G, T)
        top = rand_bytes(4444, k, T, C, 0.4)
        bot = rand_bytes(4445, k, T, C, 0.4)
        say(f"strip {k}: R={R} C={C} t={T}")
        d = [to_dev(oracle.pack(x)) for x in (b, top, bot)]
        got = from_dev(gol.strip_pass(d[0], d[1], d[2], R, C, T))
        assert np.array_equal(got, oracle.pack(oracle.ref.strip_pass(b, top, bot, T))), (k, R, C, T)
