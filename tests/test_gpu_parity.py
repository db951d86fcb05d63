"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for bit.

Life is a deterministic integer map, so every comparison is exact equality of
all cells (and of the padding bits, which must be 0).
"""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
import seeded_inputs
from golden_io import patterns, place
from gpu_util import expect_words, first_diff, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu

T_BLOCKS = [1, 2, 4, 8, 12, 16]


def run_packed(b, G, T=0, inplace=False):
    R, C = b.shape
    d_in = to_dev(oracle.pack(b))
    d_out = d_in if inplace else gol.empty_packed(R, C)
    gol.step_packed(d_in, R, C, G, d_out, t_block=T)
    return from_dev(d_out)


def check(b, G, T=0, inplace=False, threads=1):
    R, C = b.shape
    say(f"case R={R} C={C} G={G} T={T} inplace={inplace}")
    got = run_packed(b, G, T, inplace)
    want = expect_words(b, G, threads)
    assert oracle.padding_is_zero(got, C)
    assert np.array_equal(got, want), first_diff(got, want, C)


@pytest.mark.parametrize("T", T_BLOCKS)
def test_tiny_tori_all_T(T):
    for R in range(1, 6):
        for C in range(1, 6):
            b = rand_bytes(7, 100 * R + C, R, C, 0.5)
            check(b, 5, T)


@pytest.mark.parametrize("C", [1, 2, 3, 31, 32, 33, 63, 64, 65, 95, 96, 97, 127, 128, 129, 130])
def test_odd_widths(C):
    b = rand_bytes(4408, C, 37, C, 0.45)
    for T in (1, 8):
        check(b, 11, T)


@pytest.mark.parametrize("R,C", [(1, 128), (2, 256), (3, 384), (5, 128), (37, 640), (300, 8192),
                                 (129, 16384 + 128), (64, 8064), (1000, 33 * 128)])
def test_one_generation_kernel_on_128_aligned_rows(R, C):
    """Rows of whole 128-bit words take the one-generation kernel (256-dword
    strips, four dwords per lane): single passes, a pass count in place, and
    every remainder pass of 1 generation, against the oracle."""
    b = rand_bytes(2024, R + C, R, C, 0.45)
    for G in (1, 2, 5):
        check(b, G, 1)
    check(b, 3, 1, inplace=True)
    check(b, 17, 8)  # 2 passes of 8 and one of 1


@pytest.mark.parametrize("R,C", [(1, 200), (2, 77), (3, 4097), (257, 4095), (200, 8191), (70, 3969),
                                 (64, 3968), (33, 2047)])
def test_shapes_spanning_several_tiles(R, C):
    b = rand_bytes(1209, R * 7 + C, R, C, 0.35)
    for T in (4, 8, 16):
        check(b, 19, T)


@pytest.mark.parametrize("G", [0, 1, 2, 3, 7, 8, 9, 15, 16, 17, 100])
def test_generation_counts(G):
    b = rand_bytes(3, G, 150, 300, 0.5)
    check(b, G, 8)


def test_inplace_odd_and_even_pass_counts():
    b = rand_bytes(11, 0, 96, 200, 0.4)
    for G in (8, 16, 24, 5, 13):  # pass counts 1, 2, 3, and binary remainders
        check(b, G, 8, inplace=True)


def dirty_padding(w: np.ndarray, C: int, seed: int) -> np.ndarray:
    """Packed words with random bits at every column >= C."""
    w = w.copy()
    if C % 64:
        rng = np.random.default_rng(seed)
        junk = rng.integers(0, 1 << 63, size=w.shape[0], dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        w[:, -1] |= junk & ~np.uint64((1 << (C % 64)) - 1)
    return w


@pytest.mark.parametrize("C", [1, 5, 31, 33, 47, 63, 65, 70, 100, 127])
def test_input_padding_bits_ignored(C):
    R = 40
    b = rand_bytes(5, C, R, C, 0.5)
    w = dirty_padding(oracle.pack(b), C, C)
    assert not np.array_equal(w, oracle.pack(b)) or C % 64 == 0
    for T in (1, 8, 16):
        say("dirty padding C", C, "T", T)
        d_in = to_dev(w)
        d_out = gol.empty_packed(R, C)
        gol.step_packed(d_in, R, C, 9 + T, d_out, t_block=T)
        got = from_dev(d_out)
        assert np.array_equal(got, expect_words(b, 9 + T)), (C, T)


def test_patterns_on_gpu():
    for name, (kind, period, (dr, dc), cells) in patterns().items():
        R, C = cells.shape[0] + 9, cells.shape[1] + 70
        b = place(cells, R, C, R - 2, C - 3)  # straddles both seams
        say("pattern", name)
        got = oracle.unpack(run_packed(b, 4 * period), C)
        if kind == "ship":
            want = np.roll(b, (4 * dr, 4 * dc), axis=(0, 1))
        else:
            want = b
        assert np.array_equal(got, want), name


def test_glider_wraps_torus_on_gpu():
    _, _, _, cells = patterns()["glider"]
    R, C = 10, 13
    b = place(cells, R, C, 1, 1)
    assert np.array_equal(oracle.unpack(run_packed(b, 4 * 130), C), b)


@pytest.mark.parametrize("seed", [1209, 4408, 7])
def test_host_byte_api_256(seed):
    """The 256 x 256, p = 0.5, 100-generation byte-board workload."""
    b = seeded_inputs.board_bytes(seed, 0, 256, 256, 0.5)
    say("gol_step 256x256 seed", seed)
    got = gol.step(b, 100)
    assert np.array_equal(got, oracle.life(b, 100))


def test_host_byte_api_inplace_and_values():
    b = rand_bytes(9, 9, 50, 77, 0.5) * 7  # nonzero = alive
    want = oracle.life(b, 6)
    gol.step(b, 6, out=b)
    assert np.array_equal(b, want)


def test_host_byte_api_from_several_threads():
    """Concurrent gol_step calls each hold their own library stream and pinned
    staging buffer; boards of growing sizes make the buffers grow too."""
    import threading
    boards = [rand_bytes(10, k, 40 + 37 * k, 50 + 61 * k, 0.4) for k in range(8)]
    want = [oracle.life(b, 13) for b in boards]
    errors = []

    def worker(t):
        try:
            for rep in range(3):
                for k in range(t % 2, len(boards), 2):
                    if not np.array_equal(gol.step(boards[k], 13), want[k]):
                        errors.append((t, rep, k))
        except Exception as exc:  # reported below
            errors.append((t, repr(exc)))
    say("gol_step from 4 threads")
    threads = [threading.Thread(target=worker, args=(t,)) for t in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors


def test_device_pack_unpack_roundtrip():
    import torch
    R, C = 70, 333
    b = rand_bytes(2, 2, R, C, 0.5) * 3
    d = torch.from_numpy(b).cuda()
    w = gol.pack(d, R, C)
    assert np.array_equal(from_dev(w), oracle.pack(b))
    u = gol.unpack(w, R, C)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), (b != 0).astype(np.uint8))


def test_repeat_determinism():
    b = rand_bytes(1, 1, 300, 1000, 0.5)
    a1 = run_packed(b, 40)
    a2 = run_packed(b, 40)
    assert np.array_equal(a1, a2)


def test_tiling_periodicity_on_gpu():
    """A tiled board stays tiled: step(tile(x)) == tile(step(x)), all cells checked."""
    x = rand_bytes(21, 0, 48, 96, 0.4)
    big = np.tile(x, (7, 5))
    R, C = big.shape
    say("tiled", R, C)
    got = oracle.unpack(run_packed(big, 33), C)
    assert np.array_equal(got, np.tile(oracle.life(x, 33), (7, 5)))


def test_autotuned_choice_is_used_and_exact():
    for R, C, G in ((700, 3000, 37), (600, 2048, 45)):  # the second allows the paired layout
        cfg = gol.tune_config(R, C)
        assert cfg["t_block"] in (8, 12, 16) and 1 <= cfg["band_rows"] <= R
        assert cfg["layout"] in (gol.LAYOUT_BAND, gol.LAYOUT_PAIRED)
        b = rand_bytes(77, 1, R, C, 0.4)
        check(b, G, 0)  # t_block 0 takes the tuned choice


def test_autotuner_times_the_resident_layout_on_small_boards():
    """On a board the resident layout fits, it is one of the timed candidates;
    whatever wins is then the default for that size and stays exact."""
    for R, C, G in ((64, 64, 101), (200, 300, 50)):
        cfg = gol.tune_config(R, C)
        say("tuned", R, C, cfg)
        assert cfg["layout"] in (gol.LAYOUT_BAND, gol.LAYOUT_PAIRED, gol.LAYOUT_RESIDENT)
        b = rand_bytes(78, R, R, C, 0.4)
        check(b, G, 0)
        got = from_dev(gol.step_packed(to_dev(oracle.pack(b)), R, C, G, config=cfg))
        assert np.array_equal(got, expect_words(b, G)), cfg


# ---------------------------------------------------------------------------
# Explicit launch configurations (gol_step_packed_cfg)
# ---------------------------------------------------------------------------
PAIRED = [dict(t_block=8, prefetch=9), dict(t_block=8, prefetch=12), dict(t_block=12, prefetch=9),
          dict(t_block=12, prefetch=12), dict(t_block=16, prefetch=9),
          dict(t_block=16, prefetch=12)]

# (rows, cols, generations, band_rows): pairs overlapping the first pair
# (2 H x pairs > rows), boards whose cone wraps the torus, bands taller than
# the board, C % 64 == 32 (a padding dword), one pair covering the whole
# board, strips narrower than 30 dwords, several strips
PAIRED_SHAPES = [(40, 64, 37, 20), (41, 32, 24, 10), (100, 96, 50, 25), (257, 4096, 30, 22),
                 (300, 1984, 41, 37), (64, 2048, 33, 16), (33, 4064, 26, 16), (16, 320, 40, 8),
                 (95, 1952, 29, 24), (130, 160, 17, 65), (7, 64, 30, 1), (1, 32, 20, 1),
                 (23, 128, 19, 40)]


def run_cfg(b, G, cfg, inplace=False):
    R, C = b.shape
    d_in = to_dev(oracle.pack(b))
    d_out = d_in if inplace else gol.empty_packed(R, C)
    gol.step_packed(d_in, R, C, G, d_out, config=cfg)
    return from_dev(d_out)


@pytest.mark.parametrize("cfg", PAIRED, ids=lambda c: f"T{c['t_block']}pd{c['prefetch']}")
def test_paired_layout(cfg):
    for R, C, G, h in PAIRED_SHAPES:
        full = dict(cfg, layout=gol.LAYOUT_PAIRED, band_rows=h)
        b = rand_bytes(4408, R * 7 + C, R, C, 0.4)
        say(f"paired R={R} C={C} G={G} {full}")
        got = run_cfg(b, G, full)
        want = expect_words(b, G)
        assert oracle.padding_is_zero(got, C)
        assert np.array_equal(got, want), first_diff(got, want, C)


def test_paired_layout_inplace_and_every_pass_count():
    b = rand_bytes(12, 3, 96, 2048, 0.45)
    for G in (12, 24, 36, 25, 47):  # 1, 2, 3 passes, with remainders
        say("paired in place G", G)
        got = run_cfg(b, G, dict(t_block=12, layout=gol.LAYOUT_PAIRED, band_rows=24), True)
        assert np.array_equal(got, expect_words(b, G))


@pytest.mark.parametrize("cfg", [dict(t_block=8, prefetch=6), dict(t_block=12, prefetch=6),
                                 dict(t_block=12, prefetch=9), dict(t_block=16, prefetch=9),
                                 dict(t_block=16, prefetch=12), dict(t_block=4, prefetch=6)],
                         ids=lambda c: f"T{c['t_block']}pd{c['prefetch']}")
def test_band_layout_configs(cfg):
    for R, C, G, h in [(37, 100, 41, 9), (257, 4095, 30, 40), (70, 3969, 33, 7), (5, 5, 24, 2),
                       (300, 2048, 50, 73)]:
        full = dict(cfg, layout=gol.LAYOUT_BAND, band_rows=h)
        b = rand_bytes(77, R + C, R, C, 0.4)
        say(f"band R={R} C={C} G={G} {full}")
        got = run_cfg(b, G, full)
        assert np.array_equal(got, expect_words(b, G)), first_diff(got, expect_words(b, G), C)


def test_config_errors():
    R, C = 64, 100
    d = gol.empty_packed(R, C)
    for cfg in (dict(t_block=12, layout=gol.LAYOUT_PAIRED),          # C % 32 != 0
                dict(t_block=4, layout=gol.LAYOUT_PAIRED),           # T not 8, 12, 16
                dict(t_block=16, prefetch=3),                         # prefetch not built
                dict(t_block=5), dict(layout=4), dict(band_rows=-1)):
        with pytest.raises(gol.GolError) as e:
            gol.step_packed(d, R, C, 5, config=cfg)
        assert e.value.code == -1, cfg


def test_valu_probe_reports_a_rate_for_every_kind():
    """The issue-rate probe behind the ALU roofline: every instruction kind
    gives a finite positive rate, no kind above twice the 78.6 T lane-ops/s
    peak (64 lanes per SIMD per clock would be), and bad kinds are refused."""
    for k in range(len(gol.VALU_KINDS)):
        r = gol.valu_rate(k)
        say("valu probe", gol.VALU_KINDS[k], r)
        assert 0 < r < 2 * 78.6432e12
    with pytest.raises(gol.GolError):
        gol.valu_rate(5)
