"""CPU: the serving scheduler's policy, run over the host executor.

The host executor keeps boards in host memory and replays each chunk's
schedule level by level and tile by tile as the device would, standing in for
a pass of t generations by adding t to every 32-bit word of the tile, so a
request's result is its input plus its generation count in every 32-bit word
only if every pass read the buffer the previous pass wrote, every word was
covered once per pass, and the result copy read the last one.  What these tests
pin: results land in the right buffers across chunks, the HBM budget is never
exceeded, admission is first-come first-served, chunks are as long as the
configuration says, and cancellation, failures, polling and bad arguments
behave as gol.h documents.  The Life rule itself is covered by the GPU tests.
"""
import time

import numpy as np
import pytest

import paper_1209_4408_amd as gol

GOL_ENOMEM, GOL_EINVAL, GOL_EDEVICE, GOL_ENOTFOUND, GOL_ECANCELED = -2, -1, -3, -5, -6


def padding_mask(cols):
    """Bits of a row's last word that are cells (the rest is padding)."""
    r = cols % 64
    return np.uint64(2**64 - 1) if r == 0 else np.uint64((1 << r) - 1)


def normalised(w, cols):
    """The board with its padding bits cleared, as the server keeps it."""
    n = w.copy()
    n[:, -1] &= padding_mask(cols)
    return n


def board(seed, rows, cols, dirty=False):
    """Random words; padding bits clear unless dirty (the server clears them)."""
    rng = np.random.default_rng(seed)
    w = rng.integers(0, 2**64, size=(rows, gol.words_per_row(cols)), dtype=np.uint64)
    w.flat[0] = np.uint64(2**64 - 3)  # the stand-in's addition must wrap
    return w if dirty else normalised(w, cols)


def expect(w, g):
    """The stand-in's result: g added to every 32-bit word (numpy wraps)."""
    return (w.view(np.uint32) + np.uint32(g & 0xFFFFFFFF)).view(np.uint64)


def bytes_of(rows, cols):
    return rows * gol.words_per_row(cols) * 8


def wait_stats(srv, pred, timeout=5.0):
    t0 = time.time()
    while time.time() - t0 < timeout:
        st = srv.stats()
        if pred(st):
            return st
        time.sleep(0.002)
    return srv.stats()


@pytest.mark.parametrize("chunk", [1, 3, 16, 256])
def test_results_follow_the_buffers_across_chunks(chunk):
    rng = np.random.default_rng(chunk)
    reqs = []
    for i in range(60):
        R, C = int(rng.integers(1, 200)), int(rng.integers(1, 300))
        G = int(rng.integers(0, 70))
        reqs.append((board(i, R, C), R, C, G))
    with gol.Server(hbm_budget_bytes=1 << 24, chunk_generations=chunk,
                    host_executor=True) as srv:
        tickets = [srv.submit(w, R, C, G) for w, R, C, G in reqs]
        for (w, R, C, G), t in zip(reqs, tickets):
            out = np.zeros_like(w)
            info = srv.wait(t, out)
            assert np.array_equal(out, expect(w, G)), (R, C, G)
            assert info.generations_done == G
            assert info.submit_s <= info.admit_s <= info.done_s
        st = wait_stats(srv, lambda s: s["resident_bytes"] == 0)
        assert st["admitted"] == st["retired"] == len(reqs)
        assert st["resident_bytes"] == 0
        assert st["cell_updates"] == sum(R * C * G for _, R, C, G in reqs)


@pytest.mark.parametrize("T", [1, 4, 8, 12, 16])
def test_every_t_block_gives_the_requested_generations(T):
    reqs = [(board(k, 17 + k, 65 * k + 1), 17 + k, 65 * k + 1, g)
            for k, g in enumerate([1, 7, 8, 9, 31, 32, 33, 100])]
    with gol.Server(hbm_budget_bytes=1 << 24, chunk_generations=40, t_block=T,
                    host_executor=True) as srv:
        tickets = [srv.submit(w, R, C, G) for w, R, C, G in reqs]
        for (w, R, C, G), t in zip(reqs, tickets):
            out = np.zeros_like(w)
            srv.wait(t, out)
            assert np.array_equal(out, expect(w, G)), (T, G)


def test_chunk_count_of_a_lone_request():
    R, C, G, chunk = 50, 100, 100, 16
    w = board(1, R, C)
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=chunk,
                    host_executor=True) as srv:
        out = np.zeros_like(w)
        srv.wait(srv.submit(w, R, C, G), out)
        st = srv.stats()
    assert np.array_equal(out, expect(w, G))
    assert st["chunks"] == -(-G // chunk)
    assert st["max_resident"] == 1
    assert st["launches"] >= st["chunks"]


@pytest.mark.parametrize("T", [8, 16])
def test_automatic_chunk_length_without_a_measured_rate(T):
    """chunk_generations 0: until a chunk's device time is known (never, on
    the host executor) each chunk runs 15 whole passes; results still land
    in the right buffers, and the server reports the length and pass count."""
    R, C, G = 9, 130, 1000
    w = board(21, R, C)
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=0, t_block=T,
                    host_executor=True) as srv:
        out = np.zeros_like(w)
        srv.wait(srv.submit(w, R, C, G), out)
        st = srv.stats()
    assert np.array_equal(out, expect(w, G))
    assert st["t_block"] == T
    assert st["last_chunk_generations"] == 15 * T
    assert st["chunks"] == -(-G // (15 * T))


@pytest.mark.parametrize("T", [4, 8, 12, 16])
@pytest.mark.parametrize("chunk", [0, 7, 16, 40])
def test_mixed_requests_short_passes_and_groups(T, chunk):
    """Chunks whose boards need different pass counts (short passes first in
    the early group, last in the late one, masked levels) over boards narrow
    enough to share waves: every 32-bit word advances by its request's
    generation count."""
    rng = np.random.default_rng(T * 100 + chunk)
    reqs = []
    for i in range(40):
        R, C = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        reqs.append((board(1000 + i, R, C), R, C, int(rng.integers(0, 90))))
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=chunk, t_block=T,
                    host_executor=True) as srv:
        tickets = [srv.submit(w, R, C, G) for w, R, C, G in reqs]
        for (w, R, C, G), t in zip(reqs, tickets):
            out = np.zeros_like(w)
            srv.wait(t, out)
            assert np.array_equal(out, expect(w, G)), (R, C, G)


def test_budget_is_never_exceeded():
    R, C = 64, 640  # 5120 bytes per buffer
    per = 2 * bytes_of(R, C)
    budget = 3 * per + per // 2  # room for three boards
    reqs = [(board(i, R, C), 5 + (i * 7) % 40) for i in range(40)]
    with gol.Server(hbm_budget_bytes=budget, chunk_generations=4,
                    host_executor=True) as srv:
        tickets = [srv.submit(w, R, C, G) for w, G in reqs]
        for (w, G), t in zip(reqs, tickets):
            out = np.zeros_like(w)
            srv.wait(t, out)
            assert np.array_equal(out, expect(w, G))
        st = srv.stats()
        peak = srv.host_peak_bytes()
    assert st["peak_resident_bytes"] <= budget
    assert peak <= budget
    assert st["max_resident"] <= 3
    assert peak == st["peak_resident_bytes"] == 3 * per  # the scheduler fills the budget


def test_resident_cap():
    R, C = 8, 64
    reqs = [(board(i, R, C), 20) for i in range(30)]
    with gol.Server(hbm_budget_bytes=1 << 30, chunk_generations=2, max_resident=4,
                    host_executor=True) as srv:
        tickets = [srv.submit(w, R, C, G) for w, G in reqs]
        for (w, G), t in zip(reqs, tickets):
            out = np.zeros_like(w)
            srv.wait(t, out)
            assert np.array_equal(out, expect(w, G))
        assert srv.stats()["max_resident"] <= 4


def test_admission_is_first_come_first_served():
    """With room for one board at a time, boards are admitted in submission
    order, and a large board at the head is not overtaken by smaller ones."""
    sizes = [(40, 640), (4, 64), (40, 640), (2, 64), (4, 64), (40, 640)]
    budget = 2 * bytes_of(40, 640)
    reqs = [(board(i, R, C), R, C, 6) for i, (R, C) in enumerate(sizes)]
    with gol.Server(hbm_budget_bytes=budget, chunk_generations=2,
                    host_executor=True) as srv:
        tickets = [srv.submit(w, R, C, G) for w, R, C, G in reqs]
        infos = []
        for (w, R, C, G), t in zip(reqs, tickets):
            out = np.zeros_like(w)
            infos.append(srv.wait(t, out))
            assert np.array_equal(out, expect(w, G))
    admits = [i.admit_s for i in infos]
    assert admits == sorted(admits)  # a small board admitted past a big one breaks this


def test_oversize_request_is_refused():
    with gol.Server(hbm_budget_bytes=2 * bytes_of(64, 64) - 1, chunk_generations=4,
                    host_executor=True) as srv:
        with pytest.raises(gol.GolError) as e:
            srv.submit(board(0, 64, 64), 64, 64, 3)
        assert e.value.code == GOL_ENOMEM
        w = board(1, 32, 64)  # half the size fits
        out = np.zeros_like(w)
        srv.wait(srv.submit(w, 32, 64, 3), out)
        assert np.array_equal(out, expect(w, 3))


def test_zero_generation_request_returns_its_input():
    w = board(3, 9, 130)
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=4,
                    host_executor=True) as srv:
        out = np.zeros_like(w)
        srv.wait(srv.submit(w, 9, 130, 0), out)
        assert srv.stats()["chunks"] == 0
    assert np.array_equal(out, w)


@pytest.mark.parametrize("cols", [1, 63, 64, 65, 130, 200])
@pytest.mark.parametrize("G", [0, 5])
def test_input_padding_bits_are_cleared(cols, G):
    """Padding bits (columns >= cols) are ignored on input: the server keeps the
    board with them cleared, so a zero-generation request returns the
    normalised input and chunks start from it (the stand-in then adds G)."""
    R = 7
    w = board(11, R, cols, dirty=True)
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=3,
                    host_executor=True) as srv:
        out = np.zeros_like(w)
        srv.wait(srv.submit(w, R, cols, G), out)
    assert np.array_equal(out, expect(normalised(w, cols), G))
    if G == 0:
        assert np.array_equal(out, normalised(w, cols))


def test_cancel_resident_and_queued():
    R, C = 16, 64
    per = 2 * bytes_of(R, C)
    with gol.Server(hbm_budget_bytes=per, chunk_generations=1,
                    host_executor=True) as srv:
        long_t = srv.submit(board(0, R, C), R, C, 10**9)   # resident, runs "forever"
        queued_t = srv.submit(board(1, R, C), R, C, 5)    # waits for the budget
        wait_stats(srv, lambda s: s["chunks"] >= 3)
        out = np.zeros((R, 1), np.uint64)
        assert srv.poll(long_t, out) is None               # not finished: EAGAIN
        srv.cancel(queued_t)
        srv.cancel(long_t)
        for t in (queued_t, long_t):
            with pytest.raises(gol.GolError) as e:
                srv.wait(t, out)
            assert e.value.code == GOL_ECANCELED
            with pytest.raises(gol.GolError) as e:         # the ticket is gone
                srv.poll(t, out)
            assert e.value.code == GOL_ENOTFOUND
        # the budget is free again: a new request is admitted and finishes
        w = board(2, R, C)
        srv.wait(srv.submit(w, R, C, 7), out)
        assert np.array_equal(out, expect(w, 7))
        st = wait_stats(srv, lambda s: s["resident_bytes"] == 0)
        assert st["resident_bytes"] == 0
        assert st["peak_resident_bytes"] == per


def test_poll_unknown_and_retired_tickets():
    w = board(4, 5, 64)
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=4,
                    host_executor=True) as srv:
        out = np.zeros_like(w)
        with pytest.raises(gol.GolError) as e:
            srv.poll(12345, out)
        assert e.value.code == GOL_ENOTFOUND
        t = srv.submit(w, 5, 64, 9)
        info = None
        t0 = time.time()
        while info is None and time.time() - t0 < 5:
            info = srv.poll(t, out)
        assert info is not None and info.generations_done == 9
        assert np.array_equal(out, expect(w, 9))
        with pytest.raises(gol.GolError) as e:
            srv.poll(t, out)
        assert e.value.code == GOL_ENOTFOUND
        with pytest.raises(gol.GolError) as e:
            srv.cancel(t)
        assert e.value.code == GOL_ENOTFOUND


def test_device_failure_fails_unfinished_requests():
    R, C = 8, 64
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=2, fail_at_chunk=3,
                    host_executor=True) as srv:
        done_t = srv.submit(board(0, R, C), R, C, 2)      # finishes in chunk 1
        w_done = board(0, R, C)
        out = np.zeros((R, 1), np.uint64)
        srv.wait(done_t, out)
        assert np.array_equal(out, expect(w_done, 2))
        # chunk 3 needs a board submitted after the first finished, so the first
        # of these is accepted; later ones may meet the failed server at submit
        late = []
        for i in range(1, 4):
            try:
                late.append(srv.submit(board(i, R, C), R, C, 50))
            except gol.GolError as e:
                assert e.code == GOL_EDEVICE and late
        for t in late:
            with pytest.raises(gol.GolError) as e:
                srv.wait(t, out)
            assert e.value.code == GOL_EDEVICE
            assert "injected" in str(e.value)
        with pytest.raises(gol.GolError) as e:          # the server stays failed
            srv.submit(board(9, R, C), R, C, 1)
        assert e.value.code == GOL_EDEVICE


@pytest.mark.parametrize("kw", [dict(chunk_generations=-1), dict(hbm_budget_bytes=0),
                                dict(t_block=3), dict(t_block=32)])
def test_bad_configuration(kw):
    args = dict(hbm_budget_bytes=1 << 20, chunk_generations=4, host_executor=True)
    args.update(kw)
    with pytest.raises(gol.GolError) as e:
        gol.Server(**args)
    assert e.value.code == GOL_EINVAL


@pytest.mark.parametrize("rows,cols,gens", [(0, 5, 1), (5, 0, 1), (3, 3, -1)])
def test_submit_rejects_bad_sizes(rows, cols, gens):
    with gol.Server(hbm_budget_bytes=1 << 20, chunk_generations=4,
                    host_executor=True) as srv:
        buf = np.zeros(max(1, rows * gol.words_per_row(max(cols, 1))), np.uint64)
        t = __import__("ctypes").c_uint64()
        rc = gol.lib().gol_serve_submit(srv._h, buf.ctypes.data, rows, cols, gens,
                                        __import__("ctypes").byref(t))
        assert rc == GOL_EINVAL


def test_many_threads_submitting():
    """Submitters on several threads: every result is right."""
    import threading
    R, C = 12, 200
    errors = []
    with gol.Server(hbm_budget_bytes=8 * 2 * bytes_of(R, C), chunk_generations=3,
                    host_executor=True) as srv:
        def worker(k):
            try:
                for j in range(25):
                    w = board(1000 * k + j, R, C)
                    g = (k * 13 + j) % 17
                    out = np.zeros_like(w)
                    srv.wait(srv.submit(w, R, C, g), out)
                    if not np.array_equal(out, expect(w, g)):
                        errors.append((k, j))
            except Exception as ex:  # noqa: BLE001 - reported below
                errors.append(repr(ex))
        ths = [threading.Thread(target=worker, args=(k,)) for k in range(6)]
        for th in ths:
            th.start()
        for th in ths:
            th.join()
        assert srv.host_peak_bytes() <= 8 * 2 * bytes_of(R, C)
    assert not errors, errors


def test_submissions_from_threads_while_the_scheduler_is_busy():
    """Submissions go through the inbox while the scheduler runs chunks: every
    ticket is distinct, can be waited on at once from another thread, and its
    result is right; the time counters are non-negative and the host
    executor reports no device time between chunks."""
    import threading
    with gol.Server(hbm_budget_bytes=1 << 26, chunk_generations=8, host_executor=True) as srv:
        boards = {}
        lock = threading.Lock()
        errors = []

        def client(k):
            try:
                for i in range(25):
                    R, C, G = 5 + (i % 7), 40 + 13 * k, (i * 5) % 37
                    w = board(100 * k + i, R, C)
                    t = srv.submit(w, R, C, G)
                    out = np.zeros_like(w)
                    srv.wait(t, out)
                    assert np.array_equal(out, expect(w, G)), (k, i)
                    with lock:
                        assert t not in boards
                        boards[t] = (R, C, G)
            except Exception as e:  # surfaced below
                errors.append(e)

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert not errors, errors
        assert len(boards) == 100
        st = srv.stats()
    for k in ("admit_host_s", "retire_host_s", "plan_host_s", "starved_s", "chunk_gap_s"):
        assert st[k] >= 0.0, (k, st[k])
    assert st["chunk_gap_s"] == 0.0
    assert st["admitted"] == 100 and st["retired"] == 100
