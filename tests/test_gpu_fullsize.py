"""GPU parity at the benchmark's full sizes, in the launch configuration bench.py times.

The oracle cannot run these boards whole, so it checks sampled outputs: a
k x k output window after G generations depends only on the input within
Chebyshev distance G, and the oracle computes it from that (k + 2G)-wide
wrapped input window.  Windows sit on both seams, at the corner where they
cross and inside.  Properties that hold at any size cover the rest: tiling
periodicity checks every cell of a tiled board, and the temporal-blocked and
one-generation-per-launch kernels must agree on every cell.
"""
import os

import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
import seeded_inputs
from gpu_util import from_dev, say, to_dev

pytestmark = pytest.mark.gpu

THREADS = max(1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
SEED = 1209


def tuner_candidates(R, C):
    """The launch configurations gol_tune times for an R x C board."""
    import torch
    nsimd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    D = 2 * ((C + 63) // 64)
    out = []
    for layout, lanes in ((gol.LAYOUT_BAND, 62), (gol.LAYOUT_PAIRED, 30)):
        ns = (D + lanes - 1) // lanes
        for T in (8, 12, 16):
            pds = [9] if layout == gol.LAYOUT_PAIRED else [{8: 9, 12: 9, 16: 12}[T]]
            if layout == gol.LAYOUT_BAND and T == 16:
                pds.append(9)
            hs = set()
            for k in (2, 3, 4, 6, 8, 10, 12):
                units = max(1, k * nsimd // ns)
                per = units if layout == gol.LAYOUT_BAND else 2 * units
                hs.add(max(1, -(-R // per)))
            for pd in pds:
                for h in sorted(hs):
                    if layout == gol.LAYOUT_PAIRED and (C % 32 or R * D * 4 >= 1 << 31):
                        continue
                    out.append(dict(t_block=T, band_rows=h, prefetch=pd, layout=layout))
    return out


def all_candidates_agree(d_in, R, C, G, want_dev):
    """Every configuration the autotuner can pick gives the same board
    (compared on the device)."""
    import torch
    d_out = torch.empty_like(d_in)
    for cfg in tuner_candidates(R, C):
        say(f"  candidate {cfg}")
        gol.step_packed(d_in, R, C, G, d_out, config=cfg)
        torch.cuda.synchronize()
        assert torch.equal(d_out, want_dev), cfg


def windows_ok(out_words, in_words, cols, G, spots, k):
    for r0, c0 in spots:
        got = oracle.torus_window_packed(out_words, cols, r0, c0, k, k)
        say(f"  window at ({r0}, {c0}) k={k} G={G}")
        assert oracle.light_cone_check(got, in_words, cols, r0, c0, k, k, G, threads=THREADS,
                                       packed=True), (r0, c0)


def test_16384_board_1000_generations_windows():
    """The benchmark's default workload: 16384^2, p = 0.3, 1000 generations, in the
    autotuned configuration bench.py times; every other tuner candidate agrees."""
    R = C = 16384
    G = 1000
    w = seeded_inputs.board_packed(SEED, 0, R, C, 0.3)
    d_in = to_dev(w)
    cfg = gol.tune_config(R, C)
    say(f"16384^2 x 1000 on the GPU, tuned {cfg}")
    d_out = gol.step_packed(d_in, R, C, G)
    out = from_dev(d_out)
    assert oracle.padding_is_zero(out, C)
    spots = [(R - 6, C - 6), (R - 5, 7000), (9001, C - 4), (4321, 12345)]
    windows_ok(out, w, C, G, spots, 12)
    all_candidates_agree(d_in, R, C, G, d_out)


def test_16384_board_tiled_every_cell():
    """Every cell of a 16384^2 board tiled from a 256^2 block, 1000 generations."""
    x = seeded_inputs.board_bytes(SEED, 7, 256, 256, 0.3)
    want_tile = oracle.life(x, 1000, threads=THREADS)
    w = np.tile(oracle.pack(x), (64, 64))
    say("tiled 16384^2 x 1000")
    out = from_dev(gol.step_packed(to_dev(w), 16384, 16384, 1000))
    assert np.array_equal(out, np.tile(oracle.pack(want_tile), (64, 64)))


@pytest.fixture(scope="module")
def c3_runs():
    R = C = 65536
    G = 200
    w = seeded_inputs.board_packed(SEED, 0, R, C, 0.5)
    d_in = to_dev(w)
    cfg = gol.tune_config(R, C)
    say(f"65536^2 x 200, temporal-blocked, tuned {cfg}")
    d_tb = gol.step_packed(d_in, R, C, G)
    all_candidates_agree(d_in, R, C, G, d_tb)
    tb = from_dev(d_tb)
    del d_tb
    say("65536^2 x 200, one generation per launch")
    t1 = from_dev(gol.step_packed(d_in, R, C, G, t_block=1))
    del d_in
    return w, tb, t1


def test_65536_board_temporal_blocked_equals_per_generation(c3_runs):
    w, tb, t1 = c3_runs
    assert np.array_equal(tb, t1)


def test_65536_board_windows(c3_runs):
    w, tb, _ = c3_runs
    R = C = 65536
    spots = [(R - 8, C - 8), (R - 3, 30000), (40000, C - 5), (0, 0), (12345, 54321),
             (65535, 31), (777, 65500), (33333, 33333)]
    windows_ok(tb, w, C, 200, spots, 16)


def test_65536_board_tiled_every_cell():
    x = seeded_inputs.board_bytes(SEED, 9, 512, 512, 0.5)
    want = np.tile(oracle.pack(oracle.life(x, 200, threads=THREADS)), (128, 128))
    w = np.tile(oracle.pack(x), (128, 128))
    say("tiled 65536^2 x 200")
    out = from_dev(gol.step_packed(to_dev(w), 65536, 65536, 200))
    assert np.array_equal(out, want)


def test_batched_4096_boards():
    """The 4096-board mix in one schedule (graph replay, as timed): every board
    equals its own single-board run, and sampled boards match the oracle."""
    import torch
    from bench import board_set_device
    specs = seeded_inputs.batch_specs(SEED, n=4096)
    host, d_in, d_out, ins, outs = board_set_device(specs, SEED)
    boards = [gol.BatchBoard(i, o, s.rows, s.cols, s.generations)
              for s, i, o in zip(specs, ins, outs)]
    st = torch.cuda.Stream()
    say("batched 4096 boards")
    plan = gol.Plan(boards)
    with torch.cuda.stream(st):
        plan.run(st)
        plan.run(st)  # second run replays the captured graph
    st.synchronize()
    got_all = from_dev(d_out)
    offs = np.concatenate([[0], np.cumsum([s.rows * ((s.cols + 63) // 64) for s in specs])])
    # every board alone
    alone = torch.empty_like(d_out)
    for s, i, a in zip(specs, ins, [alone[o:o2].view(s.rows, -1) for s, o, o2 in
                                    zip(specs, offs[:-1], offs[1:])]):
        gol.step_packed(i, s.rows, s.cols, s.generations, a)
    assert np.array_equal(got_all, from_dev(alone))
    # oracle: the cheapest boards whole, windows on others
    work = np.array([s.rows * s.cols * s.generations for s in specs], dtype=np.float64)
    for b in np.argsort(work)[:6]:
        s = specs[b]
        w = host[offs[b]:offs[b + 1]].reshape(s.rows, -1)
        got = got_all[offs[b]:offs[b + 1]].reshape(s.rows, -1)
        say("  whole board", s)
        want = oracle.pack(oracle.life(oracle.unpack(w, s.cols), s.generations, threads=THREADS))
        assert np.array_equal(got, want), s
    rng = np.random.default_rng(4408)
    cand = [b for b in range(len(specs)) if specs[b].generations <= 250]
    for b in rng.choice(cand, 6, replace=False):
        s = specs[b]
        w = host[offs[b]:offs[b + 1]].reshape(s.rows, -1)
        got = got_all[offs[b]:offs[b + 1]].reshape(s.rows, -1)
        spots = [(s.rows - 3, s.cols - 3), (int(rng.integers(s.rows)), int(rng.integers(s.cols)))]
        windows_ok(got, w, s.cols, s.generations, spots, 8)
    plan.close()


def test_served_stream_sampled():
    """The served stream (4096 requests, Poisson, 64 GiB budget): sampled requests
    equal their single-board runs and, where cheap, the oracle."""
    import time
    specs = seeded_inputs.serve_specs(SEED, n=4096, rate_per_s=2700.0)
    rng = np.random.default_rng(7)
    sample = set(int(x) for x in rng.choice(len(specs), 48, replace=False))
    work = np.array([s.rows * s.cols * s.generations for s in specs], dtype=np.float64)
    sample |= set(int(x) for x in np.argsort(work)[:8])
    payloads = {}
    with gol.Server(hbm_budget_bytes=64 << 30, chunk_generations=256) as srv:
        tickets = []
        t0 = time.perf_counter()
        for s in specs:
            while time.perf_counter() - t0 < s.arrival_s:
                pass
            w = seeded_inputs.board_packed(SEED, s.board_id, s.rows, s.cols, s.p)
            if s.board_id in sample:
                payloads[s.board_id] = w
            tickets.append(srv.submit(w, s.rows, s.cols, s.generations))
        say("served 4096 requests submitted")
        for s, t in zip(specs, tickets):
            out = np.empty((s.rows, gol.words_per_row(s.cols)), np.uint64)
            srv.wait(t, out)
            if s.board_id in sample:
                w = payloads[s.board_id]
                alone = from_dev(gol.step_packed(to_dev(w), s.rows, s.cols, s.generations))
                assert np.array_equal(out, alone), s
                if work[s.board_id] <= 3e8:
                    want = oracle.pack(oracle.life(oracle.unpack(w, s.cols), s.generations,
                                                   threads=THREADS))
                    assert np.array_equal(out, want), s
