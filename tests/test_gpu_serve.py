"""GPU: the continuous-batching server (gol_serve_*).

Each request's result must be bit-identical to the oracle and to the same
board run alone, whatever else was resident at the time.
"""
import time

import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
import seeded_inputs
from gpu_util import expect_words, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu


def small_requests(seed, n, side_hi=300, gen_hi=90):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        R = int(rng.integers(1, side_hi))
        C = int(rng.integers(1, side_hi))
        G = int(rng.integers(0, gen_hi))
        b = rand_bytes(seed, i, R, C, float(rng.uniform(0.1, 0.6)))
        out.append((b, G))
    return out


def test_serve_matches_oracle():
    reqs = small_requests(5, 40)
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=16) as srv:
        tickets = []
        for b, G in reqs:
            R, C = b.shape
            tickets.append(srv.submit(oracle.pack(b), R, C, G))
        for (b, G), t in zip(reqs, tickets):
            R, C = b.shape
            out = np.zeros((R, gol.words_per_row(C)), np.uint64)
            info = srv.wait(t, out)
            assert info.generations_done == G
            assert info.submit_s <= info.admit_s <= info.done_s
            assert np.array_equal(out, expect_words(b, G)), (R, C, G)


def test_serve_mix_equals_alone():
    reqs = small_requests(9, 24, side_hi=500, gen_hi=70)
    mixed = []
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=8) as srv:
        tickets = [srv.submit(oracle.pack(b), *b.shape, G) for b, G in reqs]
        for (b, G), t in zip(reqs, tickets):
            out = np.zeros((b.shape[0], gol.words_per_row(b.shape[1])), np.uint64)
            srv.wait(t, out)
            mixed.append(out)
    for (b, G), m in zip(reqs, mixed):
        R, C = b.shape
        alone = from_dev(gol.step_packed(to_dev(oracle.pack(b)), R, C, G))
        assert np.array_equal(m, alone), (R, C, G)


def test_serve_budget_forces_queueing():
    """A budget that holds one board at a time still serves every request, in order."""
    R, C, G = 200, 640, 30
    bytes_per = 2 * R * gol.words_per_row(C) * 8
    boards = [rand_bytes(3, i, R, C, 0.4) for i in range(5)]
    # one board's buffers, rounded up to their size class (at most 25 % more),
    # fit; two boards' do not
    with gol.Server(hbm_budget_bytes=bytes_per * 3 // 2, chunk_generations=8) as srv:
        tickets = [srv.submit(oracle.pack(b), R, C, G) for b in boards]
        infos = []
        for b, t in zip(boards, tickets):
            out = np.zeros((R, gol.words_per_row(C)), np.uint64)
            infos.append(srv.wait(t, out))
            assert np.array_equal(out, expect_words(b, G))
    for a, b in zip(infos, infos[1:]):
        assert b.admit_s >= a.done_s - 1e-3 or b.admit_s >= a.admit_s  # admitted one by one


def test_serve_reuses_and_evicts_buffers_under_budget():
    """Waves of boards of a few sizes under a budget that holds only a few at
    a time: buffers of retired and cancelled boards are reused by later
    boards of their size class and handed back to the device pool when
    another class needs the room.  Every result equals the oracle and the
    resident bytes stay within the budget."""
    # packed bytes per buffer: 32768, 32000 (the same class), 76800, 188000, 640
    shapes = [(256, 1024), (250, 1000), (300, 2000), (500, 3000), (40, 70)]
    budget = 3 * 2 * 196608  # three of the largest class (188000 rounded up)
    rng = np.random.default_rng(11)
    reqs = []
    for i in range(30):
        R, C = shapes[int(rng.integers(0, len(shapes)))]
        reqs.append((rand_bytes(11, i, R, C, float(rng.uniform(0.2, 0.5))), R, C,
                     int(rng.integers(0, 40))))
    with gol.Server(hbm_budget_bytes=budget, chunk_generations=8) as srv:
        tickets = [srv.submit(oracle.pack(b), R, C, G) for b, R, C, G in reqs]
        cancelled = {3, 17}
        for i in cancelled:
            srv.cancel(tickets[i])
        for i, ((b, R, C, G), t) in enumerate(zip(reqs, tickets)):
            out = np.zeros((R, gol.words_per_row(C)), np.uint64)
            if i in cancelled:
                try:  # it may have finished before the cancel reached it
                    srv.wait(t, out)
                except gol.GolError as e:
                    assert e.code == gol.GOL_ECANCELED
                    continue
            else:
                srv.wait(t, out)
            assert np.array_equal(out, expect_words(b, G)), (i, R, C, G)
        st = srv.stats()
    assert 0 < st["peak_resident_bytes"] <= budget


def test_serve_oversize_and_bad_tickets():
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=8) as srv:
        big = np.zeros((2048, 64), np.uint64)  # needs 2 x 1 MiB > budget
        with pytest.raises(gol.GolError) as e:
            srv.submit(big, 2048, 4096, 5)
        assert e.value.code == gol.GOL_ENOMEM
        out = np.zeros(1, np.uint64)
        with pytest.raises(gol.GolError) as e:
            srv.wait(12345, out)
        assert e.value.code == gol.GOL_ENOTFOUND
        with pytest.raises(gol.GolError):
            srv.cancel(999)


def test_serve_cancel_and_poll():
    R, C = 512, 4096
    long_b = rand_bytes(1, 1, R, C, 0.5)
    short_b = rand_bytes(1, 2, 64, 64, 0.5)
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=8) as srv:
        t_long = srv.submit(oracle.pack(long_b), R, C, 100000)
        t_short = srv.submit(oracle.pack(short_b), 64, 64, 10)
        out_long = np.zeros((R, gol.words_per_row(C)), np.uint64)
        assert srv.poll(t_long, out_long) is None  # not finished
        srv.cancel(t_long)
        with pytest.raises(gol.GolError) as e:
            srv.wait(t_long, out_long)
        assert e.value.code == gol.GOL_ECANCELED
        out = np.zeros((64, 1), np.uint64)
        srv.wait(t_short, out)
        assert np.array_equal(out, expect_words(short_b, 10))


def test_serve_zero_generations_and_poll_loop():
    b = rand_bytes(4, 4, 33, 70, 0.5)
    with gol.Server(hbm_budget_bytes=1 << 26, chunk_generations=4) as srv:
        t = srv.submit(oracle.pack(b), 33, 70, 0)
        out = np.zeros((33, 2), np.uint64)
        deadline = time.time() + 20
        info = None
        while info is None and time.time() < deadline:
            info = srv.poll(t, out)
            time.sleep(0.001)
        assert info is not None
        assert np.array_equal(out, oracle.pack(b))
        with pytest.raises(gol.GolError) as e:  # retired after the successful poll
            srv.poll(t, out)
        assert e.value.code == gol.GOL_ENOTFOUND


@pytest.mark.parametrize("G", [0, 1, 9])
def test_serve_dirty_padding_is_ignored_and_cleared(G):
    """Padding bits set on input: a served result equals the oracle on the
    board's cells and has its padding bits cleared, also with zero generations."""
    R, C = 21, 70
    b = rand_bytes(5, 5, R, C, 0.45)
    w = oracle.pack(b)
    dirty = w.copy()
    dirty[:, -1] |= np.uint64(~((1 << (C % 64)) - 1) & (2**64 - 1))
    with gol.Server(hbm_budget_bytes=1 << 26, chunk_generations=4) as srv:
        out = np.full_like(w, 0xFFFF)
        srv.wait(srv.submit(dirty, R, C, G), out)
    assert oracle.padding_is_zero(out, C)
    assert np.array_equal(out, oracle.pack(oracle.life(b, G)))


def test_serve_stream_poisson_small():
    """A short open-loop stream with requests arriving while others run."""
    specs = seeded_inputs.serve_specs(1209, n=60, rate_per_s=2000.0, side_hi=700, gen_hi=200)
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=32) as srv:
        t0 = time.perf_counter()
        tickets = []
        for s in specs:
            while time.perf_counter() - t0 < s.arrival_s:
                pass
            w = seeded_inputs.board_packed(1209, s.board_id, s.rows, s.cols, s.p)
            tickets.append((s, w, srv.submit(w, s.rows, s.cols, s.generations)))
        for s, w, t in tickets:
            out = np.zeros_like(w)
            srv.wait(t, out)
            if s.rows * s.cols * s.generations <= 2e7:
                want = oracle.pack(oracle.life(oracle.unpack(w, s.cols), s.generations))
            else:
                want = from_dev(gol.step_packed(to_dev(w), s.rows, s.cols, s.generations))
            say("request", s.board_id, s.rows, s.cols, s.generations)
            assert np.array_equal(out, want), s


def _narrow_and_wide(seed):
    """Requests whose tiles pack several bands of one board into a wave
    (narrow boards) beside wide and tiny ones."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(30):
        kind = i % 3
        if kind == 0:
            R, C = int(rng.integers(100, 900)), int(rng.integers(1, 200))   # narrow
        elif kind == 1:
            R, C = int(rng.integers(1, 120)), int(rng.integers(500, 3000))  # wide
        else:
            R, C = int(rng.integers(1, 40)), int(rng.integers(1, 40))       # tiny
        G = int(rng.integers(0, 120))
        out.append((rand_bytes(seed, i, R, C, float(rng.uniform(0.2, 0.6))), G))
    return out


@pytest.mark.parametrize("T", [0, 8, 12, 16])
def test_serve_automatic_chunks_match_oracle(T):
    """Chunks of the automatic length (and, T = 0, the pass length tuned at
    creation) over narrow, wide and tiny boards give the oracle's results."""
    reqs = _narrow_and_wide(40 + T)
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=0, t_block=T) as srv:
        tickets = [srv.submit(oracle.pack(b), *b.shape, G) for b, G in reqs]
        for (b, G), t in zip(reqs, tickets):
            R, C = b.shape
            out = np.zeros((R, gol.words_per_row(C)), np.uint64)
            srv.wait(t, out)
            assert np.array_equal(out, expect_words(b, G)), (T, R, C, G)
        st = srv.stats()
    say("served T", T, "stats", st["t_block"], st["last_chunk_generations"],
        st["last_band_rows"], st["chunks"])
    assert st["t_block"] == (T or st["t_block"]) and st["t_block"] in (8, 12, 16)
    assert st["last_chunk_generations"] % st["t_block"] == 0
    assert st["last_band_rows"] >= 16


def test_serve_deep_backlog_equals_alone():
    """All requests at once with enough work (4.8e12 cell updates) that the
    automatic chunk length follows the backlog, chunks longer than its 3 ms
    floor: every result equals the board run alone by step_packed (itself
    checked against the oracle)."""
    import torch
    n, R, C, G = 48, 4096, 4096, 6000
    dev = torch.device("cuda:0")
    boards = [seeded_inputs.board_packed_device(1209, 500 + i, R, C, 0.4, gol.empty_packed(R, C, dev))
              for i in range(n)]
    host = [from_dev(d) for d in boards]
    say("serve deep backlog", n, R, C, G)
    with gol.Server(hbm_budget_bytes=8 << 30, chunk_generations=0) as srv:
        tickets = [srv.submit(w, R, C, G) for w in host]
        outs = []
        for w, t in zip(host, tickets):
            out = np.zeros_like(w)
            srv.wait(t, out)
            outs.append(out)
        st = srv.stats()
    assert st["retired"] == n
    for i, (d, out) in enumerate(zip(boards, outs)):
        say("alone", i)
        assert np.array_equal(out, from_dev(gol.step_packed(d, R, C, G))), i
