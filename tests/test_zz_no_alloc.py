"""gol_step_packed_noalloc, the entry point that allocates nothing (its
ping-pong board is a fixed device array), against gol_step_packed on the
same seeded boards: bit for bit, on calls in a row whose later boards are
smaller, so each call runs over what the last one left in the array."""
import ctypes

import numpy as np
import pytest

import seeded_inputs

pytestmark = pytest.mark.gpu


def _pair(gol, torch, seed, R, C, G, p, in_place=False):
    w = seeded_inputs.board_packed(seed, 0, R, C, p)
    d_in = torch.from_numpy(w.view(np.int64)).cuda()
    want = gol.step_packed(d_in, R, C, G)
    if in_place:
        got = d_in.clone()
        gol.step_packed_noalloc(got, R, C, G, got)
    else:
        got = torch.empty_like(d_in)
        got.fill_(-1)
        gol.step_packed_noalloc(d_in, R, C, G, got)
    torch.cuda.synchronize()
    return want.cpu().numpy().view(np.uint64), got.cpu().numpy().view(np.uint64)


def test_noalloc_equals_step_packed_calls_in_a_row():
    torch = pytest.importorskip("torch")
    import paper_1209_4408_amd as gol
    # the 16384^2 board of the benchmark fills half the array; then smaller,
    # ragged boards (odd widths, several passes and remainder passes)
    cases = [(1209, 16384, 16384, 30, 0.3), (4408, 2048, 4000, 37, 0.5),
             (7, 300, 1000, 13, 0.4), (11, 45, 70, 29, 0.5)]
    for seed, R, C, G, p in cases:
        print(f"noalloc case seed={seed} {R}x{C} G={G}", flush=True)
        want, got = _pair(gol, torch, seed, R, C, G, p)
        assert np.array_equal(want, got), (seed, R, C, G)


def test_noalloc_in_place_odd_pass_count_and_oracle():
    torch = pytest.importorskip("torch")
    import oracle
    import paper_1209_4408_amd as gol
    # 25 generations = one pass of 1 + two of 12: an odd pass count in place
    # starts from a copy in the fixed array
    for seed, R, C, G in ((5, 1000, 2112, 25), (6, 130, 200, 25)):
        print(f"noalloc in place seed={seed} {R}x{C} G={G}", flush=True)
        want, got = _pair(gol, torch, seed, R, C, G, 0.45, in_place=True)
        assert np.array_equal(want, got), (seed, R, C, G)
    w = seeded_inputs.board_packed(6, 0, 130, 200, 0.45)
    ref = oracle.pack(oracle.life(oracle.unpack(w, 200), 25))
    assert np.array_equal(got, ref)


def test_noalloc_rejects_boards_above_the_array():
    import paper_1209_4408_amd as gol
    L = gol.lib()
    # 16384 rows of 513 words: 8 KiB over the 64 MiB array; rejected before
    # any pointer is used
    rc = L.gol_step_packed_noalloc(None, 16384, 513 * 64, 1, None, None)
    assert rc == gol.GOL_EINVAL
    assert b"at most" in L.gol_last_error()
    assert gol.NOALLOC_MAX_BYTES == 64 << 20
    # the largest board it takes: exactly the array
    rc = L.gol_step_packed_noalloc(None, 16384, 512 * 64, 1, None, None)
    assert rc == gol.GOL_EINVAL and b"null" in L.gol_last_error()
