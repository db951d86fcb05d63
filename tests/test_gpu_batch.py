"""GPU: many boards in one schedule, and plans replayed from a HIP graph."""
import numpy as np
import pytest

import oracle
import paper_1209_4408_amd as gol
import seeded_inputs
from gpu_util import expect_words, first_diff, from_dev, rand_bytes, say, to_dev

pytestmark = pytest.mark.gpu


def mixed_specs(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        R = int(rng.integers(1, 200))
        C = int(rng.choice([int(rng.integers(1, 70)), int(rng.integers(70, 2500))]))
        G = int(rng.integers(0, 40))
        out.append((R, C, G))
    return out


@pytest.mark.parametrize("T", [1, 2, 4, 8, 12, 16])
def test_batch_matches_oracle(T):
    specs = mixed_specs(T, 60)
    boards, ins, outs, want = [], [], [], []
    for i, (R, C, G) in enumerate(specs):
        b = rand_bytes(4408, i, R, C, 0.4)
        d_in = to_dev(oracle.pack(b))
        d_out = gol.empty_packed(R, C)
        boards.append(gol.BatchBoard(d_in, d_out, R, C, G))
        want.append(expect_words(b, G))
    say("batch T", T, "n", len(boards))
    p = gol.Plan(boards, t_block=T)
    p.run()
    for i, bb in enumerate(boards):
        got = from_dev(bb.d_out)
        assert np.array_equal(got, want[i]), (i, specs[i], first_diff(got, want[i], specs[i][1]))
    p.close()


def test_batch_run_one_shot_and_inplace():
    specs = mixed_specs(99, 30)
    boards, want = [], []
    for i, (R, C, G) in enumerate(specs):
        b = rand_bytes(7, i, R, C, 0.5)
        d = to_dev(oracle.pack(b))
        boards.append(gol.BatchBoard(d, d, R, C, G))  # in place
        want.append(expect_words(b, G))
    gol.batch_run(boards)
    for i, bb in enumerate(boards):
        assert np.array_equal(from_dev(bb.d_out), want[i]), (i, specs[i])


def test_batch_ignores_input_padding_bits():
    """Bits at columns >= cols are not part of the board, whatever they hold."""
    rng = np.random.default_rng(5)
    boards, want = [], []
    for i, C in enumerate([1, 3, 17, 31, 33, 40, 63, 65, 70, 100, 333, 2047]):
        R = int(rng.integers(1, 90))
        G = int(rng.integers(1, 40))
        b = rand_bytes(8, i, R, C, 0.5)
        w = oracle.pack(b)
        if C % 64:
            w[:, -1] |= ~np.uint64((1 << (C % 64)) - 1)  # every padding bit set
        d = to_dev(w)
        o = gol.empty_packed(R, C)
        boards.append(gol.BatchBoard(d, o, R, C, G))
        want.append((expect_words(b, G), (R, C, G)))
    say("batch dirty padding", len(boards))
    gol.batch_run(boards)
    for bb, (wt, spec) in zip(boards, want):
        assert np.array_equal(from_dev(bb.d_out), wt), spec


def test_plan_graph_replays():
    """Replaying the captured plan from the same input gives the same result
    every time, with the program's own work in between."""
    import torch
    specs = [(100, 300, 17), (64, 64, 8), (5, 2000, 3), (130, 77, 25)]
    boards, want = [], []
    for i, (R, C, G) in enumerate(specs):
        b = rand_bytes(3, i, R, C, 0.4)
        boards.append(gol.BatchBoard(to_dev(oracle.pack(b)), gol.empty_packed(R, C), R, C, G))
        want.append(expect_words(b, G))
    s = torch.cuda.Stream()
    p = gol.Plan(boards)
    for rep in range(4):
        with torch.cuda.stream(s):
            for bb in boards:
                bb.d_out.zero_()
            p.run(s)
        s.synchronize()
        junk = torch.randn(1000, device="cuda").sum().item()  # other eager work
        assert np.isfinite(junk)
        for i, bb in enumerate(boards):
            assert np.array_equal(from_dev(bb.d_out), want[i]), (rep, i)
    p.close()


def test_mix_equals_alone():
    """Each board gives the same result in a mix as when run alone."""
    specs = seeded_inputs.batch_specs(1209, n=48, side_hi=600, gen_hi=60)
    mix, alone = [], []
    for s in specs:
        w = seeded_inputs.board_packed(1209, s.board_id, s.rows, s.cols, s.p)
        d_in = to_dev(w)
        mix.append(gol.BatchBoard(d_in, gol.empty_packed(s.rows, s.cols), s.rows, s.cols,
                                  s.generations))
        alone.append(gol.step_packed(d_in, s.rows, s.cols, s.generations))
    gol.batch_run(mix)
    for s, m, a in zip(specs, mix, alone):
        assert np.array_equal(from_dev(m.d_out), from_dev(a)), s


def _tall_mixed(seed, n):
    """Mixed boards, some tall enough to span several bands of every height."""
    rng = np.random.default_rng(seed)
    out = mixed_specs(seed, n)
    for _ in range(6):
        out.append((int(rng.integers(130, 420)), int(rng.integers(30, 2100)),
                    int(rng.integers(1, 40))))
    return out


def _run_plan_and_check(specs, seed, **kw):
    boards, want = [], []
    for i, (R, C, G) in enumerate(specs):
        b = rand_bytes(seed, i, R, C, 0.4)
        boards.append(gol.BatchBoard(to_dev(oracle.pack(b)), gol.empty_packed(R, C), R, C, G))
        want.append(expect_words(b, G))
    p = gol.Plan(boards, **kw)
    cfg = p.config()
    p.run()
    for i, bb in enumerate(boards):
        got = from_dev(bb.d_out)
        assert np.array_equal(got, want[i]), (kw, i, specs[i],
                                              first_diff(got, want[i], specs[i][1]))
    p.close()
    return cfg


@pytest.mark.parametrize("band", [48, 64, 96, 128])
@pytest.mark.parametrize("T", [8, 12, 16])
def test_plan_every_tuner_candidate_matches_oracle(T, band):
    """Every (t_block, band_rows) the plan tuner can pick gives the oracle's boards."""
    specs = _tall_mixed(31 + T + band, 36)
    say("plan candidate", T, band)
    cfg = _run_plan_and_check(specs, 12, t_block=T, band_rows=band)
    assert cfg == {"t_block": T, "band_rows": band}


def test_plan_tuned_choice_matches_oracle():
    """With both fields 0 the plan times the candidates and keeps one of them."""
    specs = _tall_mixed(77, 40)
    cfg = _run_plan_and_check(specs, 13)
    say("tuned plan", cfg)
    assert cfg["t_block"] in (8, 12, 16) and cfg["band_rows"] in (48, 64, 96, 128)
    cfg = _run_plan_and_check(specs, 14, t_block=4)  # band tuned only
    assert cfg["t_block"] == 4 and cfg["band_rows"] in (48, 64, 96, 128)


@pytest.mark.parametrize("T", [8, 12, 16])
def test_queue_form_matches_oracle(T):
    """The persistent work-queue form (one launch, per-board pass counters)
    gives the oracle's boards, in place and with zero generations too, and
    no wave gave up waiting."""
    specs = _tall_mixed(90 + T, 40) + [(64, 64, 0), (3, 2000, 45), (200, 40, 70)]
    boards, want = [], []
    for i, (R, C, G) in enumerate(specs):
        b = rand_bytes(5, i, R, C, 0.4)
        d = to_dev(oracle.pack(b))
        o = d if i % 5 == 0 else gol.empty_packed(R, C)  # every fifth in place
        boards.append(gol.BatchBoard(d, o, R, C, G))
        want.append(expect_words(b, G))
    say("queue form T", T, len(boards))
    p = gol.Plan(boards, t_block=T, band_rows=64, queue=True)
    assert p.config()["layout"] == "queue"
    p.run()
    assert not p.queue_gave_up()
    for i, bb in enumerate(boards):
        got = from_dev(bb.d_out)
        assert np.array_equal(got, want[i]), (T, i, specs[i],
                                              first_diff(got, want[i], specs[i][1]))
    p.close()
