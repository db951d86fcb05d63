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

T_BLOCKS = [1, 2, 4, 8, 16]


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


def test_input_padding_bits_ignored():
    R, C = 40, 100
    b = rand_bytes(5, 5, R, C, 0.5)
    w = oracle.pack(b)
    w[:, -1] |= np.uint64(0xFFFFFFF000000000)  # set bits at columns >= 100
    d_in = to_dev(w)
    d_out = gol.empty_packed(R, C)
    gol.step_packed(d_in, R, C, 9, d_out)
    got = from_dev(d_out)
    assert np.array_equal(got, expect_words(b, 9))


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
    R, C, G = 700, 3000, 37
    T, band = gol.tune(R, C)
    assert T in (4, 8, 16) and 1 <= band <= R
    b = rand_bytes(77, 1, R, C, 0.4)
    check(b, G, 0)  # t_block 0 takes the tuned choice
