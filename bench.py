"""Benchmark of the Life step library on one MI355X.

Default run (no --workload): every configuration of the metric in one process,
one JSON line.  Its headline `value` is the HBM-scale single board: a 65536 x
65536 toroidal board, bit-packed, i.i.d. Bernoulli(0.5) cells from seed 1209,
advanced 200 generations by gol_step_packed in temporal-blocked passes, with
the one-generation-per-launch kernel timed beside it.  Blocks of the same line
carry the other configurations, each with its own timed region, roofline and
CPU oracle baseline:
  c2  16384 x 16384, Bernoulli(0.3), 1000 generations (plain single board);
  c4  4096 boards of uneven sizes and generation counts in one batched
      schedule, against the plain path (one gol_step_packed per board);
  c5  4096 requests of uneven sizes and generation counts through the
      continuous-batching server: the same boards as one batched schedule
      (the capacity), all requests at once (saturated), and open-loop Poisson
      streams at 0.3, 0.5, 0.7 and 0.9 of that capacity (throughput, p50 /
      p99 latency; 0.7 is the block's value), against a one-request-at-a-time
      server on the 0.7 trace;
  c1  a 256 x 256 byte board, 100 generations, through the host API.
A "step" of a block is one pass of its whole workload: one board run (c3, c2),
one schedule over all 4096 boards (c4), one stream of requests (c5).

Other workloads (--workload) run one configuration alone (c1 ... c5) or a
side study: pop (population counting), bounded (dead surroundings instead of
the torus), strip (one GPU's 8192 x 65536 share of the 65536^2 board), decomp
(Table 2's largest case, with the CPU study of the three decompositions), valu
(the issue-rate probe of each VALU instruction kind the tile pass uses), copy
(copy-kernel calibration of the traffic counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X 32-bit VALU peak: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz
# = 78.6 T ops/s, the published 157.3 TFLOP/s FP32 vector figure counted as
# one op per FMA (integer and bitwise ops issue at the same lane rate).
VALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
HBM_PEAK_BYTES = 8.0e12
# Algorithmic integer ops per cell-update: the bit-sliced full-adder network
# written with two-input logic ops, 24 ops per 32-cell word and generation.
# This is the count the ALU roofline is priced at (`frac`).
OPS_PER_CELL_UPDATE = 24.0 / 32.0
# The same network as the kernels issue it with gfx950's three-input v_bitop3:
# 2 funnel shifts + 2 (horizontal 3-sum) + 4 (vertical combine) + 4 (rule)
# = 12 ops per 32 cells; reported beside `frac`.
ISSUED_OPS_PER_CELL_UPDATE = 12.0 / 32.0
# Algorithmic HBM bytes per cell-update of a one-generation pass: read + write
# one bit.
BYTES_PER_CELL_UPDATE_T1 = 2.0 / 8.0

SEED = 1209
# client threads submitting the saturated stream
SAT_SUBMITTERS = 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return max(1, int(env))
    return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _median_rate(fn, work, reps=3):
    """Median over `reps` timed calls of fn() of work / seconds."""
    rates = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        rates.append(work / (time.perf_counter() - t0))
    return float(np.median(rates)), rates


# ---------------------------------------------------------------------------
# CPU oracle baselines (bounded samples of each workload)
# ---------------------------------------------------------------------------
def cpu_baseline_board(rows, cols, p, seed, total_gens, budget_s=15.0, gens=0):
    """The oracle (plain C, row decomposition over OpenMP threads) on a bounded
    number of generations of the workload's own board: median of three timed
    samples sized to the budget, or one timing of exactly `gens` generations;
    the oracle's single-thread rate beside it."""
    import oracle
    import seeded_inputs
    threads = cpu_threads()
    b = seeded_inputs.board_bytes(seed, 0, rows, cols, p)
    t0 = time.perf_counter()
    cur = oracle.life(b, 1, threads=threads)
    one = time.perf_counter() - t0
    if gens:
        g, reps = gens, 1
    else:
        g, reps = int(max(1, min(total_gens, budget_s / 3.0 / max(one, 1e-6)))), 3
    value, rates = _median_rate(lambda: oracle.life(cur, g, threads=threads), rows * cols * g,
                                reps=reps)
    g1 = int(max(1, min(total_gens, 2.0 / max(one * threads, 1e-6))))
    single, _ = _median_rate(lambda: oracle.life(cur, g1, threads=1), rows * cols * g1, reps=1)
    timing = "median of 3 timings" if reps == 3 else "one timing"
    return {"value": value, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{g} of the run's {total_gens} generations of the {rows}x{cols} board, "
                      f"{timing}, {threads} OpenMP threads (row decomposition), "
                      f"byte-per-cell C oracle",
            "rates": rates, "single_thread_value": single,
            "single_thread_sample": f"{g1} generations, 1 thread", "cpu_model": cpu_model()}


def cpu_baseline_boards(specs, seed, budget_s=12.0, what="boards"):
    """The oracle over a sample of a mix's boards, each run for its full
    generation count: every k-th board (k chosen so the sample's work fits the
    budget at the oracle's rate on one probe board), rate = sampled
    cell-updates / oracle seconds summed over the sample."""
    import oracle
    import seeded_inputs
    threads = cpu_threads()
    work = np.array([s.rows * s.cols * s.generations for s in specs], dtype=np.float64)
    probe = specs[int(np.argsort(work)[len(specs) // 2])]
    b = seeded_inputs.board_bytes(seed, probe.board_id, probe.rows, probe.cols, probe.p)
    g = max(1, min(probe.generations, 50))
    t0 = time.perf_counter()
    oracle.life(b, g, threads=threads)
    rate = probe.rows * probe.cols * g / max(time.perf_counter() - t0, 1e-6)
    k = max(1, int(np.ceil(work.sum() / rate / budget_s)))
    sample = specs[::k]
    done, secs = 0.0, 0.0
    for s in sample:
        b = seeded_inputs.board_bytes(seed, s.board_id, s.rows, s.cols, s.p)
        t0 = time.perf_counter()
        oracle.life(b, s.generations, threads=threads)
        secs += time.perf_counter() - t0
        done += s.rows * s.cols * s.generations
        if secs > 2.5 * budget_s:
            break
    return {"value": done / secs, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"every {k}-th of the {len(specs)} {what} run whole by the oracle "
                      f"({done:.3e} of {work.sum():.3e} cell-updates, {secs:.1f} s), summed "
                      f"over boards, {threads} OpenMP threads",
            "cpu_model": cpu_model()}


# ---------------------------------------------------------------------------
# Rooflines
# ---------------------------------------------------------------------------
def alu_roofline(cell_updates_per_launch, avg_launch_s, kernel, **extra):
    """ALU roofline record of a temporal-blocked pass: algorithmic ops (24 per
    32 cells and generation) per launch / average launch duration, against the
    78.6 T ops/s VALU peak; the issued 12-op count beside it."""
    ops = OPS_PER_CELL_UPDATE * cell_updates_per_launch
    achieved = ops / avg_launch_s / 1e12
    peak = VALU_PEAK_OPS / 1e12
    issued = ISSUED_OPS_PER_CELL_UPDATE * cell_updates_per_launch / avg_launch_s / 1e12
    rec = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
           "frac": achieved / peak, "traffic": None, "kernel": kernel,
           "avg_launch_us": avg_launch_s * 1e6, "ops_per_launch": ops,
           "ops_per_cell_update": OPS_PER_CELL_UPDATE,
           "at_issued_12_ops_per_32_cells": {"achieved": issued, "frac": issued / peak}}
    rec.update(extra)
    return rec


def hbm_roofline(cell_updates_per_launch, avg_launch_s, kernel):
    by = BYTES_PER_CELL_UPDATE_T1 * cell_updates_per_launch
    achieved = by / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_BYTES / 1e9, "unit": "GB/s",
            "frac": achieved / (HBM_PEAK_BYTES / 1e9), "traffic": None, "kernel": kernel,
            "avg_launch_us": avg_launch_s * 1e6, "bytes_per_launch": by}


_MIX_CEILING = None


def measured_mix_ceiling():
    """Cell-updates/s the chip allows for the tile pass's instruction mix at the
    issue rates the VALU probe measures now: per 32 cells and generation a
    pipeline stage issues 10 full-rate ops (v_bitop3 / v_and) and 4 half-rate
    ones (2 DPP moves, 2 v_alignbit)."""
    global _MIX_CEILING
    if _MIX_CEILING is None:
        import paper_1209_4408_amd as gol
        full = gol.valu_rate(1)                         # v_bitop3_b32
        half = 0.5 * (gol.valu_rate(2) + gol.valu_rate(3))  # v_alignbit_b32, DPP move
        _MIX_CEILING = 32.0 / (10.0 / full + 4.0 / half)
    return _MIX_CEILING


def with_mix_ceiling(rec, cell_updates_per_s):
    ceiling = measured_mix_ceiling()
    rec["measured_mix_ceiling"] = {"cell_updates_per_s": ceiling,
                                   "frac": cell_updates_per_s / ceiling}
    return rec


def measured_traffic(record: str, cfg=None):
    """HBM bytes per launch from the committed counter record (rocprofv3
    FETCH_SIZE / WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when there is none for this kernel and launch configuration, or the kernel
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    if cfg is not None and rec.get("config") != cfg:
        return None
    return rec["hbm_bytes_per_launch"]


def kernel_name(cfg, cols):
    """The tile-pass kernel a launch configuration runs on a torus of `cols`
    columns (gather 1: whole dwords, 0: rows that end inside a dword)."""
    T, pd = cfg["t_block"], cfg["prefetch"]
    if cfg["layout"] == 2:
        return f"k_board_pass_half<{T}, {pd}>"
    return f"k_board_pass<{T}, {pd}, {1 if cols % 32 == 0 else 0}>"


# ---------------------------------------------------------------------------
# Timing helpers (HIP events on the stream the kernels are launched on)
# ---------------------------------------------------------------------------
def timed_region(torch, fn, steps, warmup, stream=None):
    """warmup untimed calls, then `steps` calls bracketed by synchronisations;
    returns (wall seconds, device seconds between events on the stream)."""
    st = stream or torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3


def resolve_config(gol, R, C, args, fixed):
    """Launch configuration of a single-board block: explicit, or autotuned."""
    if fixed:
        t, h, pd, lay = (int(v) for v in fixed.split(","))
        cfg = {"t_block": t, "band_rows": h, "prefetch": pd, "layout": lay}
    elif args.t_block:
        cfg = {"t_block": args.t_block, "band_rows": 0, "prefetch": 0, "layout": 1}
    elif args.no_tune:
        cfg = {"t_block": 12, "band_rows": 0, "prefetch": 0, "layout": 1}
    else:
        # one-off autotuning of the launch configuration for this size, before timing
        cfg = gol.tune_config(R, C)
        log(f"autotuned {R}x{C}: {cfg}")
    if not cfg["prefetch"]:
        cfg["prefetch"] = {16: 12, 12: 9, 8: 9}.get(cfg["t_block"], 3)
    return cfg


def single_board(args, R, C, G, p, fixed_cfg="", compare_t1=False, cpu=True, cpu_gens=0):
    """One board of R x C cells, G generations, in the autotuned configuration.

    Timed regions: (1) the whole run, `steps` times -> value; (2) the
    dominant kernel alone: runs of G - G mod t_block generations, which are
    whole t_block passes only -> its average launch duration; (3) optionally
    the one-generation-per-launch kernel on the same board."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    log(f"generating {R}x{C} board p={p} on the device")
    d_in = torch.empty(R * ((C + 63) // 64), dtype=torch.int64, device="cuda")
    seeded_inputs.board_packed_device(SEED, 0, R, C, p, d_in)
    d_out = torch.empty_like(d_in)
    torch.cuda.synchronize()
    cfg = resolve_config(gol, R, C, args, fixed_cfg)
    T = cfg["t_block"]
    run_cfg = cfg if cfg["band_rows"] else None
    tb = 0 if run_cfg else T
    log(f"timing {R}x{C}x{G}: {args.steps} steps after {args.warmup} warmup, {cfg}")
    wall, dev = timed_region(torch, lambda: gol.step_packed(d_in, R, C, G, d_out, t_block=tb,
                                                            config=run_cfg),
                             args.steps, args.warmup)
    cells = R * C
    value = cells * G * args.steps / wall
    blk = {"metric": "cell-updates/sec", "value": value, "unit": "cell-updates/s",
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "timed_s": wall, "device_s": dev, "dtype": "u32",
           "config": {"workload": f"{R}x{C} torus, bit-packed, Bernoulli({p}), {G} generations",
                      "rows": R, "cols": C, "generations": G, "p": p, "seed": SEED, **cfg,
                      "layout": {1: "band", 2: "paired", 3: "resident"}.get(cfg["layout"])}}
    if T > 1 and cfg["layout"] != 3:
        g_main = (G // T) * T
        passes = g_main // T
        _, dev_k = timed_region(torch, lambda: gol.step_packed(d_in, R, C, g_main, d_out,
                                                               t_block=tb, config=run_cfg),
                                args.steps, 1)
        avg = dev_k / (args.steps * passes)
        roof = alu_roofline(cells * T, avg, kernel_name(cfg, C),
                            launches_timed=args.steps * passes,
                            timed_as=f"runs of {g_main} generations ({passes} passes of {T})")
        roof = with_mix_ceiling(roof, cells * T / avg)
        rec = (f"traffic_{roof['kernel'].split('<')[0]}_{R}x{C}"
               f"_t{cfg['t_block']}_b{cfg['band_rows']}.json")
        roof["traffic"] = measured_traffic(rec, cfg)
        blk["roofline"] = roof
    else:
        blk["roofline"] = None
    if compare_t1:
        n1 = max(2, args.steps // 2)
        log(f"timing {R}x{C}x{G} one generation per launch: {n1} steps")
        wall1, dev1 = timed_region(torch, lambda: gol.step_packed(d_in, R, C, G, d_out,
                                                                  t_block=1), n1, 1)
        k1 = "k_step_t1" if C % 128 == 0 else f"k_board_pass<1, 3, {1 if C % 32 == 0 else 0}>"
        roof1 = hbm_roofline(cells, dev1 / (n1 * G), k1)
        roof1["traffic"] = measured_traffic(f"traffic_{k1.split('<')[0]}_{R}x{C}.json")
        blk["t1"] = {"value": cells * G * n1 / wall1, "unit": "cell-updates/s", "steps": n1,
                     "timed_s": wall1, "roofline": roof1}
        blk["speedup_vs_t1"] = value / blk["t1"]["value"]
    del d_in, d_out
    torch.cuda.empty_cache()
    if cpu and not args.no_cpu:
        log(f"cpu baseline (oracle) on {R}x{C}")
        blk["cpu_baseline"] = cpu_baseline_board(R, C, p, SEED, G, gens=cpu_gens)
    return blk


def board_set_device(specs, seed):
    """All boards of a mix in one device buffer (inputs) and one for outputs."""
    import torch
    import seeded_inputs
    sizes = [s.rows * ((s.cols + 63) // 64) for s in specs]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    host = np.empty(int(offs[-1]), dtype=np.uint64)
    for s, o, n in zip(specs, offs[:-1], sizes):
        seeded_inputs.board_packed(seed, s.board_id, s.rows, s.cols, s.p,
                                   out=host[o:o + n].reshape(s.rows, -1))
    d_in = torch.from_numpy(host.view(np.int64)).cuda()
    d_out = torch.empty_like(d_in)
    ins = [d_in[o:o + n].view(s.rows, -1) for s, o, n in zip(specs, offs[:-1], sizes)]
    outs = [d_out[o:o + n].view(s.rows, -1) for s, o, n in zip(specs, offs[:-1], sizes)]
    return host, d_in, d_out, ins, outs


def batched(args, cpu=True):
    """4096 boards of uneven sizes and generation counts: one batched schedule
    (graph replay) against the plain path, one gol_step_packed per board with
    the library's default configuration, sequential on one stream."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    specs = seeded_inputs.batch_specs(SEED, n=args.boards)
    work = float(sum(s.rows * s.cols * s.generations for s in specs))
    log(f"generating {len(specs)} boards, {work:.3e} cell-updates")
    _, d_in, d_out, ins, outs = board_set_device(specs, SEED)
    boards = [gol.BatchBoard(i, o, s.rows, s.cols, s.generations)
              for s, i, o in zip(specs, ins, outs)]
    st = torch.cuda.Stream()
    log("creating the plan (tuned unless --t-block and --band-rows)")
    plan = gol.Plan(boards, t_block=args.t_block, band_rows=args.band_rows)
    info = plan.info()
    pcfg = plan.config()
    T = pcfg["t_block"]
    log(f"timing the batched schedule: {args.steps} steps after {args.warmup} warmup")
    with torch.cuda.stream(st):
        wall, dev = timed_region(torch, lambda: plan.run(st), args.steps, args.warmup, st)
    plan.close()
    graph_out = d_out.clone()
    # the persistent work-queue form of the same schedule (same t_block and
    # band height): one launch, per-board pass counters
    log("timing the persistent work-queue form")
    qplan = gol.Plan(boards, t_block=T, band_rows=pcfg["band_rows"], queue=True)
    d_out.zero_()
    with torch.cuda.stream(st):
        wall_q, dev_q = timed_region(torch, lambda: qplan.run(st), args.steps, args.warmup, st)
    gave_up = qplan.queue_gave_up()
    qplan.close()
    queue_blk = {"value": work * args.steps / wall_q, "unit": "cell-updates/s",
                 "steps": args.steps, "timed_s": wall_q, "device_s": dev_q,
                 "gave_up": gave_up, "equals_graph": bool(torch.equal(d_out, graph_out)),
                 "what": "one persistent launch (resident waves take per-board pass items "
                         "from a queue, device-scope counters between passes), same t_block "
                         "and band height"}
    del graph_out
    value = work * args.steps / wall
    per = dev / args.steps
    roof = alu_roofline(work, per, f"k_batch_pass<{T}, *>", launches=info["levels"],
                        note="algorithmic ops of the whole schedule over its device time "
                             "(two streams overlap, so per-launch durations are not "
                             "separable); traffic is HBM bytes per schedule")
    roof["traffic"] = measured_traffic(f"traffic_k_batch_pass_{len(specs)}_boards.json",
                                       {"t_block": T, "band_rows": pcfg["band_rows"]})
    blk = {"metric": "cell-updates/sec", "value": value, "unit": "cell-updates/s",
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "timed_s": wall, "device_s": dev, "dtype": "u32",
           "config": {"workload": f"{len(specs)} boards, rows/cols log-uniform [64, 2048], "
                                  "p U(0.1, 0.6), generations U{10..1000}, one batched "
                                  "schedule", "boards": len(specs), "seed": SEED,
                      "t_block": T, "band_rows": pcfg["band_rows"],
                      "tuned": not (args.t_block and args.band_rows), "cell_updates": work},
           "roofline": roof, "plan": info, "queue_form": queue_blk}
    if not args.no_plain:
        log("plain per-board loop (library default configuration)")
        plain_steps = 1

        def plain():
            for s, i, o in zip(specs, ins, outs):
                gol.step_packed(i, s.rows, s.cols, s.generations, o, stream=st)
        with torch.cuda.stream(st):
            wall_p, _ = timed_region(torch, plain, plain_steps, 1, st)
        blk["plain"] = {"value": work * plain_steps / wall_p, "unit": "cell-updates/s",
                        "steps": plain_steps, "timed_s": wall_p,
                        "what": "one gol_step_packed per board (library default "
                                "configuration), sequential, same stream"}
        blk["speedup_vs_plain"] = value / blk["plain"]["value"]
    del d_in, d_out, ins, outs
    torch.cuda.empty_cache()
    if cpu and not args.no_cpu:
        log("cpu baseline (oracle) on a sample of the boards")
        blk["cpu_baseline"] = cpu_baseline_boards(specs, SEED, what="boards")
    return blk


def host_api(args):
    """256 x 256 byte board, 100 generations through gol_step (host memory in
    and out), plus the same board on the packed device path."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    R = C = 256
    G = 100
    b = seeded_inputs.board_bytes(SEED, 0, R, C, 0.5)
    out = np.empty_like(b)
    for _ in range(max(3, args.warmup)):
        gol.step(b, G, out=out)
    lat = []
    n = max(20, args.steps)
    for _ in range(n):
        t0 = time.perf_counter()
        gol.step(b, G, out=out)
        lat.append(time.perf_counter() - t0)
    lat = np.array(lat)
    w = seeded_inputs.board_packed(SEED, 0, R, C, 0.5)
    d_in = torch.from_numpy(w.view(np.int64)).cuda()
    d_out = torch.empty_like(d_in)
    _, dev = timed_region(torch, lambda: gol.step_packed(d_in, R, C, G, d_out), 20, 3)
    blk = {"metric": "cell-updates/sec", "value": R * C * G / float(np.median(lat)),
           "unit": "cell-updates/s", "steps": n, "timed_s": float(lat.sum()),
           "config": {"workload": "256x256 torus, uint8 cells, Bernoulli(0.5), 100 "
                                  "generations, host API (PCIe included)", "rows": R,
                      "cols": C, "generations": G, "p": 0.5, "seed": SEED},
           "roofline": None,
           "host_api_us": {"p50": float(np.median(lat) * 1e6),
                           "p99": float(np.percentile(lat, 99, method="nearest") * 1e6)},
           "device_us_per_call": dev / 20 * 1e6}
    if not args.no_cpu:
        import oracle
        threads = cpu_threads()
        single, rates = _median_rate(lambda: oracle.life(b, G, threads=1), R * C * G)
        blk["cpu_baseline"] = {"value": single, "unit": "cell-updates/s", "cores": 1,
                               "kind": "oracle", "sample": "the whole run, median of 3, one "
                               "thread (a board this small does not gain from threads)",
                               "cpu_model": cpu_model(), "threads_available": threads}
    return blk


def wait_until(t0, at):
    """Sleep, then spin, until perf_counter() - t0 >= at."""
    rem = at - (time.perf_counter() - t0)
    if rem > 0.0005:
        time.sleep(rem - 0.0003)
    while time.perf_counter() - t0 < at:
        pass


def nearest_rank(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = max(1, int(np.ceil(q / 100.0 * len(xs))))
    return xs[k - 1]


def serve_stream(gol, specs, payloads, rate, args, saturate=False):
    """One open-loop stream through a fresh continuous-batching server:
    request i is submitted at its scheduled Poisson arrival (all at once when
    saturate), a second thread waits for the results in order.  Returns the
    results, the server's completion times, its clock at the first arrival
    and its counters."""
    import threading
    results = [None] * len(specs)
    srv = gol.Server(hbm_budget_bytes=64 << 30, chunk_generations=args.chunk,
                     t_block=args.t_block)
    # warm the pools: one small request
    w = payloads[0]
    srv.wait(srv.submit(w, specs[0].rows, specs[0].cols, 1), np.zeros_like(w))
    done = [None] * len(specs)
    tickets = [None] * len(specs)
    ready = threading.Semaphore(0)

    def waiter():
        for i in range(len(specs)):
            ready.acquire()
            out = np.empty_like(payloads[i])
            info = srv.wait(tickets[i], out)
            done[i] = info.done_s
            results[i] = out

    th = threading.Thread(target=waiter)
    th.start()
    base = srv.now()
    t0 = time.perf_counter()
    if saturate:
        # four client threads submit interleaved slices of the requests at once
        # (the server's calls are thread-safe); the waiter takes results in order
        lock = threading.Lock()
        submitted = [False] * len(specs)
        nxt = [0]

        def submitter(k):
            for i in range(k, len(specs), SAT_SUBMITTERS):
                s = specs[i]
                tickets[i] = srv.submit(payloads[i], s.rows, s.cols, s.generations)
                with lock:
                    submitted[i] = True
                    while nxt[0] < len(specs) and submitted[nxt[0]]:
                        nxt[0] += 1
                        ready.release()
        subs = [threading.Thread(target=submitter, args=(k,)) for k in range(SAT_SUBMITTERS)]
        for t in subs:
            t.start()
        for t in subs:
            t.join()
    else:
        for i, s in enumerate(specs):
            wait_until(t0, s.arrival_s)
            tickets[i] = srv.submit(payloads[i], s.rows, s.cols, s.generations)
            ready.release()
    stats = {"submit_loop_s": time.perf_counter() - t0}
    th.join()
    stats.update(srv.stats())
    srv.close()
    return results, done, base, stats


def stream_block(specs, done, base, stats, rate, work, args, saturate=False):
    arr = [base + (0.0 if saturate else s.arrival_s) for s in specs]
    lat = [d - a for d, a in zip(done, arr)]
    span = max(done) - arr[0]
    blk = {"value": work / span, "unit": "cell-updates/s", "timed_s": span,
           "rate_per_s": None if saturate else rate,
           "latency_s": {"p50": nearest_rank(lat, 50), "p99": nearest_rank(lat, 99),
                         "max": max(lat)},
           "server": stats}
    if not saturate:
        blk["offered_cell_updates_per_s"] = work / (specs[-1].arrival_s - specs[0].arrival_s)
    if stats.get("device_busy_s"):
        blk["device_busy_frac"] = stats["device_busy_s"] / span
    return blk


def served(args, rate_rho=0.7, cpu=True, plain=True):
    """The served configuration: 4096 requests (sides log-uniform [32, 8192],
    p U(0.05, 0.7), generations U{1..10000}) from seed 1209.

    capacity: the same 4096 boards as one batched schedule (tuned plan),
    the throughput the served forms are measured against; saturated: every
    request submitted at once; streams: open-loop Poisson arrivals at rho x
    capacity / mean work per request for each rho in --rhos, the headline at
    rho = rate_rho; plain: a FIFO server running one request at a time
    (gol_step_packed per request) on the headline trace.  Latency =
    completion - scheduled arrival."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    specs = seeded_inputs.serve_specs(SEED, n=args.requests, rate_per_s=1.0)
    log(f"generating {len(specs)} request boards")
    payloads = [seeded_inputs.board_packed(SEED, s.board_id, s.rows, s.cols, s.p) for s in specs]
    works = [s.rows * s.cols * s.generations for s in specs]
    work = float(sum(works))
    mean_work = work / len(specs)
    # capacity: one batched schedule over the same boards
    log("batched schedule over the served mix (capacity)")
    sizes = [s.rows * ((s.cols + 63) // 64) for s in specs]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    host = np.concatenate([p.reshape(-1) for p in payloads])
    d_in = torch.from_numpy(host.view(np.int64)).cuda()
    del host
    d_out = torch.empty_like(d_in)
    boards = [gol.BatchBoard(d_in[o:o + n].view(s.rows, -1), d_out[o:o + n].view(s.rows, -1),
                             s.rows, s.cols, s.generations)
              for s, o, n in zip(specs, offs[:-1], sizes)]
    st = torch.cuda.Stream()
    plan = gol.Plan(boards, t_block=args.t_block)
    pcfg = plan.config()
    with torch.cuda.stream(st):
        wall_b, dev_b = timed_region(torch, lambda: plan.run(st), 2, 1, st)
    plan.close()
    # every request's result, for the served-equals-alone checks
    alone = [d_out[o:o + n].cpu().numpy().view(np.uint64).reshape(s.rows, -1)
             for s, o, n in zip(specs, offs[:-1], sizes)]
    del boards, d_in, d_out
    torch.cuda.empty_cache()
    capacity = work * 2 / wall_b
    blk = {"metric": "cell-updates/sec", "unit": "cell-updates/s", "steps": 1, "dtype": "u32",
           "capacity_batched": {"value": capacity, "unit": "cell-updates/s", "steps": 2,
                                "timed_s": wall_b, "plan": pcfg,
                                "what": "the 4096 request boards as one batched schedule "
                                        "(tuned plan, graph replay)"},
           "config": {"workload": f"{len(specs)} requests, Poisson at {rate_rho} x the batched "
                                  "capacity on the same boards, sides log-uniform [32, 8192], "
                                  "p U(0.05, 0.7), generations U{1..10000}, 64 GiB budget",
                      "requests": len(specs), "chunk_generations": args.chunk or "auto",
                      "t_block": args.t_block or "tuned", "hbm_budget_bytes": 64 << 30,
                      "seed": SEED, "cell_updates": work}}

    def check(results):
        return sum(0 if np.array_equal(r.reshape(a.shape), a) else 1
                   for r, a in zip(results, alone))
    rhos = sorted({float(r) for r in args.rhos.split(",") if r} | {rate_rho})
    sweep = {}
    head = None
    for rho in rhos:
        rate = rho * capacity / mean_work
        sp = seeded_inputs.serve_specs(SEED, n=args.requests, rate_per_s=rate)
        log(f"served stream at rho {rho}: {rate:.0f} requests/s")
        res, done, base, stats = serve_stream(gol, sp, payloads, rate, args)
        b = stream_block(sp, done, base, stats, rate, work, args)
        b["mismatches_vs_batched"] = check(res)
        sweep[f"{rho:g}"] = b
        if rho == rate_rho:
            head = (sp, b)
    blk["rho_sweep"] = sweep
    # after the streams, so the library's pinned staging pool is warm as in a
    # long-running server
    log("saturated server (all requests at once), one untimed burst first")
    # the untimed burst grows the pinned staging pool to what a whole burst
    # holds at once (a long-running server keeps it)
    serve_stream(gol, specs, payloads, 0.0, args, saturate=True)
    res, done, base, stats = serve_stream(gol, specs, payloads, 0.0, args, saturate=True)
    sat = stream_block(specs, done, base, stats, None, work, args, saturate=True)
    sat["mismatches_vs_batched"] = check(res)
    sat["over_capacity"] = sat["value"] / capacity
    sat["submitters"] = SAT_SUBMITTERS
    if stats.get("device_busy_s"):
        sat["device_busy_rate"] = work / stats["device_busy_s"]
        sat["device_busy_rate_over_capacity"] = sat["device_busy_rate"] / capacity
    blk["saturated"] = sat
    sp, hb = head
    blk["value"] = hb["value"]
    blk["timed_s"] = hb["timed_s"]
    blk["latency_s"] = hb["latency_s"]
    blk["rate_per_s"] = hb["rate_per_s"]
    blk["served_equals_alone"] = all(b["mismatches_vs_batched"] == 0 for b in sweep.values()) \
        and sat["mismatches_vs_batched"] == 0
    stats = hb["server"]
    blk["roofline"] = None
    if stats.get("device_busy_s"):
        blk["roofline"] = alu_roofline(stats["cell_updates"], stats["device_busy_s"],
                                       f"k_batch_pass<{stats['t_block']}, *>",
                                       launches=stats["launches"],
                                       note="algorithmic ops of every chunk over the chunks' "
                                            "device time (first to last launch of each)")
    n_plain = min(len(sp), args.plain_requests) if plain else 0
    if n_plain > 0:
        log(f"plain one-at-a-time server on the first {n_plain} requests")
        stq = torch.cuda.current_stream()
        lat_p = []
        t0 = time.perf_counter()
        mism = 0
        for i in range(n_plain):
            s = sp[i]
            wait_until(t0, s.arrival_s)
            d_i = torch.from_numpy(payloads[i].view(np.int64)).cuda()
            d_o = gol.step_packed(d_i, s.rows, s.cols, s.generations)
            r = d_o.cpu().numpy().view(np.uint64)
            stq.synchronize()
            lat_p.append(time.perf_counter() - t0 - s.arrival_s)
            if not np.array_equal(r.reshape(alone[i].shape), alone[i]):
                mism += 1
        span_p = time.perf_counter() - t0 - sp[0].arrival_s
        work_p = float(sum(works[:n_plain]))
        blk["plain"] = {"value": work_p / span_p, "unit": "cell-updates/s", "requests": n_plain,
                        "timed_s": span_p,
                        "latency_s": {"p50": nearest_rank(lat_p, 50),
                                      "p99": nearest_rank(lat_p, 99)},
                        "mismatches_vs_batched": mism,
                        "what": "FIFO, one request at a time, gol_step_packed per request"}
        blk["speedup_vs_plain"] = blk["value"] / blk["plain"]["value"]
    if cpu and not args.no_cpu:
        log("cpu baseline (oracle) on a sample of the requests")
        blk["cpu_baseline"] = cpu_baseline_boards(specs, SEED, what="requests")
    return blk


def default_line(args):
    """Every configuration of the metric; the headline is the 65536^2 board."""
    import torch
    blocks = {}
    log("== c3: 65536^2 x 200")
    # the oracle on 20 of the 200 generations (its rate does not depend on the
    # generation count, so the sample scales linearly)
    c3 = single_board(args, 65536, 65536, 200, 0.5, args.config_c3, compare_t1=True,
                      cpu_gens=args.c3_cpu_gens)
    log("== c2: 16384^2 x 1000")
    blocks["c2"] = single_board(args, 16384, 16384, 1000, 0.3, args.config_c2)
    log("== c4: 4096 boards")
    blocks["c4"] = batched(args)
    log("== c5: served stream")
    blocks["c5"] = served(args)
    log("== c1: host API")
    blocks["c1"] = host_api(args)
    torch.cuda.synchronize()
    line = {
        "metric": "cell-updates/sec",
        "value": c3["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": c3["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {**c3["config"], "parallelism": "single GPU"},
        "roofline": c3["roofline"],
        "timed_s": c3["timed_s"],
        "t1": c3.get("t1"),
        "speedup_vs_t1": c3.get("speedup_vs_t1"),
        "blocks": blocks,
        "batched_over_plain": blocks["c4"].get("speedup_vs_plain"),
        "served_over_plain": blocks["c5"].get("speedup_vs_plain"),
    }
    if "cpu_baseline" in c3:
        line["cpu_baseline"] = c3["cpu_baseline"]
    return line


def single_line(args, blk, parallelism="single GPU"):
    """A one-configuration JSON line from a block."""
    line = {"metric": "cell-updates/sec", "value": blk["value"], "unit": "cell-updates/s",
            "n_gpus": 1, "steps": blk["steps"], "warmup": blk.get("warmup", args.warmup),
            "ms_per_step": blk["timed_s"] / blk["steps"] * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {**blk["config"], "parallelism": parallelism}}
    for k, v in blk.items():
        if k not in line and k not in ("metric", "unit"):
            line[k] = v
    return line


def copy_calibration(args):
    """A plain copy kernel of known size (generations = 0): what the FETCH_SIZE
    and WRITE_SIZE counters read for 512 MiB in and 512 MiB out (larger than
    the L2 and the Infinity Cache, so every byte comes from HBM)."""
    import torch
    import paper_1209_4408_amd as gol
    R = C = 65536
    d_in = torch.zeros((R, C // 64), dtype=torch.int64, device="cuda")
    d_out = torch.empty_like(d_in)
    gol.step_packed(d_in, R, C, 0, d_out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        gol.step_packed(d_in, R, C, 0, d_out)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / args.steps
    print(json.dumps({"copy_bytes_each_way": R * C // 8, "launches": args.steps + 1,
                      "read_plus_write_GBps": 2 * R * C / 8 / dt / 1e9}), flush=True)


def valu_workload(args):
    """The VALU issue-rate probe: lane operations per second of each
    instruction kind the tile pass issues, against the 78.6 T ops/s peak
    (256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz) the ALU rooflines use."""
    import paper_1209_4408_amd as gol
    rates = {}
    for k, name in enumerate(gol.VALU_KINDS):
        best = max(gol.valu_rate(k) for _ in range(max(1, args.steps // 2)))
        rates[name] = {"lane_ops_per_s": best, "frac_of_peak": best / VALU_PEAK_OPS}
    print(json.dumps({"valu_probe": rates, "peak_lane_ops_per_s": VALU_PEAK_OPS}), flush=True)


def population_workload(args):
    """Population (live cells, the paper's Table 1 quantity): the counting
    kernel alone on the 65536^2 board (HBM-bound: it reads the board once),
    and the 16384^2 run of 1000 generations with the population recorded at
    Table 1's iteration counts (100, 200, 500, 1000) against the same run
    without."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    R = C = 65536
    w = seeded_inputs.board_packed(SEED, 0, R, C, 0.5)
    d = torch.from_numpy(w.view(np.int64)).cuda()
    del w
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream()
    for _ in range(args.warmup + 1):
        gol.lib().gol_population(d.data_ptr(), R, C, cnt.data_ptr(), st.cuda_stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.steps):
        gol.lib().gol_population(d.data_ptr(), R, C, cnt.data_ptr(), st.cuda_stream)
    e1.record(st)
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) / 1e3 / args.steps
    bytes_ = R * C // 8
    line = {"metric": "cells counted/sec", "value": R * C / dt, "unit": "cells/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "dtype": "u64", "data": "synthetic",
            "config": {"workload": "population of a 65536x65536 bit-packed board, "
                                   "Bernoulli(0.5), seed 1209", "population": int(cnt.item())},
            "roofline": {"bound": "hbm", "achieved": bytes_ / dt / 1e9, "peak": 8000.0,
                         "unit": "GB/s", "frac": bytes_ / dt / 8e12, "traffic": None,
                         "kernel": "k_population", "bytes_per_launch": bytes_}}
    del d
    torch.cuda.empty_cache()
    # Table 1's checks on the benchmark board
    R = C = 16384
    G = 1000
    w = seeded_inputs.board_packed(SEED, 0, R, C, 0.3)
    d_in = torch.from_numpy(w.view(np.int64)).cuda()
    d_out = torch.empty_like(d_in)
    cfg = gol.tune_config(R, C)
    checks = [100, 200, 500, 1000]

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(args.steps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3 / args.steps
    t_plain = timed(lambda: gol.step_packed(d_in, R, C, G, d_out, config=cfg))
    out = {}
    t_pop = timed(lambda: out.update(c=gol.step_packed_population(d_in, R, C, G, checks,
                                                                   d_out=d_out, config=cfg)[1]))
    line["table1_checks"] = {"board": "16384x16384, p 0.3, seed 1209, 1000 generations",
                             "checks": checks, "population": out["c"].cpu().tolist(),
                             "ms_with_checks": t_pop * 1e3, "ms_without": t_plain * 1e3,
                             "overhead": t_pop / t_plain - 1.0}
    print(json.dumps(line), flush=True)


def bounded_workload(args):
    """A bounded 16384^2 board (cells beyond the edges dead), 1000 generations,
    against the same board on the torus in the same launch configuration
    (band layout, t_block 12 unless --t-block)."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    R = C = 16384
    G, p = 1000, 0.3
    w = seeded_inputs.board_packed(SEED, 0, R, C, p)
    d_in = torch.from_numpy(w.view(np.int64)).cuda()
    del w
    d_out = torch.empty_like(d_in)
    T = args.t_block or 12
    pd = {16: 12, 12: 9, 8: 9}.get(T, 3)
    cfg = {"t_block": T, "band_rows": 0, "prefetch": pd, "layout": 1}
    st = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record(st)
        for _ in range(args.steps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, a.elapsed_time(b) / 1e3
    wall, dev = timed(lambda: gol.step_packed_bounded(d_in, R, C, G, d_out, config=cfg))
    wall_t, dev_t = timed(lambda: gol.step_packed(d_in, R, C, G, d_out, config=cfg))
    avg_launch = dev / (args.steps * G) * T
    value = R * C * G * args.steps / wall
    line = {"metric": "cell-updates/sec", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic",
            "config": {"workload": "16384x16384 bounded board (cells beyond the edges dead), "
                                   "Bernoulli(0.3), 1000 generations", "rows": R, "cols": C,
                       "generations": G, "p": p, "seed": SEED, **cfg, "layout": "band",
                       "parallelism": "single GPU"},
            "roofline": alu_roofline(R * C * T, avg_launch, f"k_board_pass<{T}, {pd}, 2>"),
            "torus_same_config": {"value": R * C * G * args.steps / wall_t,
                                  "unit": "cell-updates/s"}}
    print(json.dumps(line), flush=True)


def strip_workload(args):
    """One GPU's share of the 65536^2 board under the row decomposition over 8
    GPUs: an 8192 x 65536 strip, 200 generations in passes of t (16 unless
    --t-block; a shorter last pass), each pass reading its halo rows from two
    separate buffers.  Before each pass the halo buffers are refilled by device
    copies from the strip's own edge rows -- the one-GPU ring, where the strip
    is a whole 8192 x 65536 torus; across GPUs the neighbours would send them.
    Against the whole 65536^2 board in the same configuration."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    rows, C, G, p = 8192, 65536, 200, 0.5
    t = args.t_block or 16
    pd = {16: 12, 12: 9, 8: 9}.get(t, 3)  # the library's default prefetch for t
    passes = [t] * (G // t) + ([G % t] if G % t else [])
    if any(x not in (1, 2, 4, 8, 12, 16) for x in passes):
        raise SystemExit(f"200 generations in passes of {t} leave a pass length with no kernel")
    w = seeded_inputs.board_packed(SEED, 8, rows, C, p)
    cur = torch.from_numpy(w.view(np.int64)).cuda()
    del w
    nxt = torch.empty_like(cur)
    W = cur.shape[1]
    top = torch.empty((max(passes), W), dtype=torch.int64, device="cuda")
    bot = torch.empty_like(top)
    st = torch.cuda.current_stream()

    def run():
        nonlocal cur, nxt
        for x in passes:
            top[:x].copy_(cur[rows - x:])
            bot[:x].copy_(cur[:x])
            gol.strip_pass(cur, top, bot, rows, C, x, d_out=nxt)
            cur, nxt = nxt, cur

    def kernels_only():
        for x in passes:
            gol.strip_pass(cur, top, bot, rows, C, x, d_out=nxt)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record(st)
        for _ in range(args.steps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, a.elapsed_time(b) / 1e3
    wall, _ = timed(run)
    _, dev_k = timed(kernels_only)
    # the whole board for comparison: the 65536^2 run of the same generations
    R2 = 65536
    big = torch.from_numpy(seeded_inputs.board_packed(SEED, 0, R2, C, p).view(np.int64)).cuda()
    big_out = torch.empty_like(big)
    cfg = {"t_block": t, "layout": 1}
    wall_big, _ = timed(lambda: gol.step_packed(big, R2, C, G, big_out, config=cfg))
    del big, big_out
    avg_launch = dev_k / (args.steps * len(passes))
    value = rows * C * G * args.steps / wall
    line = {"metric": "cell-updates/sec", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic",
            "config": {"workload": "8192x65536 strip of a 65536^2 torus (one of 8 row strips), "
                                   "halo rows from separate buffers, Bernoulli(0.5), "
                                   "200 generations", "rows": rows, "cols": C, "generations": G,
                       "p": p, "seed": SEED, "passes": passes, "layout": "band",
                       "parallelism": "single GPU (one GPU's share)"},
            # cell-updates per launch: the average over the passes of the run
            "roofline": alu_roofline(rows * C * G / len(passes), avg_launch,
                                     f"k_board_pass<{t}, {pd}, 5>"),
            "whole_board_same_t": {"value": R2 * C * G * args.steps / wall_big,
                                   "unit": "cell-updates/s"}}
    print(json.dumps(line), flush=True)


# Table 2: seconds on the paper's four-thread machine, 1-D decomposition
PAPER_TABLE2_S = {
    (120, 60, 500): (28.144, 18.252, 13.630, 11.214),
    (120, 60, 1000): (54.384, 34.561, 28.398, 26.567),
    (120, 60, 2000): (108.633, 85.531, 36.824, 35.971),
    (240, 120, 500): (108.674, 77.034, 49.174, 41.638),
    (240, 120, 1000): (218.939, 125.108, 94.846, 67.993),
    (240, 120, 2000): (436.149, 261.167, 156.326, 126.420),
}


def cpu_decomposition_study(p, seed):
    """The CPU-baseline leg of the decomp workload: the oracle with the row,
    column and 2-D block decompositions (Sections 2.1-2.2) at Table 2's scales,
    iteration counts and thread counts, and on a 4096^2 board where a
    generation is large enough for the split to matter more than the fork."""
    import oracle
    import seeded_inputs
    maxt = cpu_threads()
    threads = sorted({1, 2, 4, 8, maxt})
    table = []
    for (w, h, it) in PAPER_TABLE2_S:
        b = seeded_inputs.board_bytes(seed, 0, h, w, p)
        row = {"cols": w, "rows": h, "iterations": it, "paper_s": PAPER_TABLE2_S[(w, h, it)]}
        for d in ("rows", "cols", "2d"):
            row[d + "_s"] = {}
            for t in threads:
                t0 = time.perf_counter()
                oracle.life_decomp(b, it, t, d)
                row[d + "_s"][t] = time.perf_counter() - t0
        table.append(row)
    big = seeded_inputs.board_bytes(seed, 1, 4096, 4096, p)
    large = {"rows": 4096, "cols": 4096, "iterations": 20}
    for d in ("rows", "cols", "2d"):
        large[d + "_cu_per_s"] = {}
        for t in threads:
            t0 = time.perf_counter()
            oracle.life_decomp(big, 20, t, d)
            large[d + "_cu_per_s"][t] = 4096 * 4096 * 20 / (time.perf_counter() - t0)
    return table, large, maxt


def decomp_workload(args):
    """Table 2's largest case (240 x 120 cells, 2000 iterations) on the GPU,
    with the CPU decomposition study (rows, columns, 2-D) as the baseline."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    w, h, G, p = 240, 120, 2000, 0.3
    words = seeded_inputs.board_packed(SEED, 0, h, w, p)
    d_in = torch.from_numpy(words.view(np.int64)).cuda()
    d_out = torch.empty_like(d_in)
    for _ in range(args.warmup):
        gol.step_packed(d_in, h, w, G, d_out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gol.step_packed(d_in, h, w, G, d_out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    table, large, maxt = cpu_decomposition_study(p, SEED)
    last = table[-1]
    rows_s = last["rows_s"][maxt]
    line = {"metric": "cell-updates/sec", "value": w * h * G * args.steps / wall,
            "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "Table 2's largest case: 240 x 120 torus (240 columns), "
                                   "Bernoulli(0.3), 2000 iterations", "rows": h, "cols": w,
                       "generations": G, "p": p, "seed": SEED, "parallelism": "single GPU"},
            "roofline": None,
            "cpu_baseline": {"value": w * h * G / rows_s, "unit": "cell-updates/s",
                             "cores": maxt, "kind": "oracle",
                             "sample": f"the whole run, row decomposition, {maxt} OpenMP threads"},
            "cpu_decomposition_study": {"table2": table, "large": large}}
    print(json.dumps(line), flush=True)


def sweep(args):
    """Single-board tuning sweep: generations per pass x band count x prefetch.
    Band counts put the wave total just under a multiple of the SIMD count."""
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    R, C, G, p = (65536, 65536, 200, 0.5) if args.workload == "c3" else (16384, 16384, 1000, 0.3)
    w = seeded_inputs.board_packed(SEED, 0, R, C, p)
    d_in = torch.from_numpy(w.view(np.int64)).cuda()
    del w
    d_out = torch.empty_like(d_in)
    nsimd = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    D = 2 * ((C + 63) // 64)
    for layout, lanes, Ts in ((1, 62, ((8, 6), (8, 9), (12, 9), (16, 9), (16, 12))),
                              (2, 30, ((8, 9), (12, 9), (12, 12), (16, 9), (16, 12)))):
        nstrips = (D + lanes - 1) // lanes
        for T, pd in Ts:
            for k in (1, 2, 3, 4, 6, 8, 12):
                units = max(1, (k * nsimd) // nstrips)
                h = -(-R // (units if layout == 1 else 2 * units))
                if h < T:
                    continue
                cfg = {"t_block": T, "band_rows": h, "prefetch": pd, "layout": layout}
                wall, dev = timed_region(torch, lambda: gol.step_packed(d_in, R, C, G, d_out,
                                                                        config=cfg), 3, 1)
                print(json.dumps({**cfg, "k": k, "cell_updates_per_s": R * C * G * 3 / dev}),
                      flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="all",
                    choices=["all", "c1", "c2", "c3", "c4", "c5", "copy", "pop", "bounded",
                             "strip", "decomp", "valu"])
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--rhos", default="0.3,0.5,0.9",
                    help="served stream: arrival rates to sweep, as fractions of the batched "
                         "capacity on the same boards (0.7, the headline, always runs)")
    ap.add_argument("--chunk", type=int, default=0,
                    help="served stream: generations per chunk (0 = the server's automatic "
                         "length)")
    ap.add_argument("--plain-requests", type=int, default=4096)
    ap.add_argument("--boards", type=int, default=4096)
    ap.add_argument("--t-block", type=int, default=0)
    ap.add_argument("--band-rows", type=int, default=0,
                    help="batched workload: band height of the schedule (0 = tuned, with "
                         "--t-block)")
    ap.add_argument("--compare-t1", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched / served workloads: skip the one-at-a-time comparison")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (T = 12, model band)")
    ap.add_argument("--config", default="",
                    help="explicit launch configuration t_block,band_rows,prefetch,layout "
                         "(layout 1 = one band per wave, 2 = paired bands) of a single-board "
                         "workload; skips the autotuner")
    ap.add_argument("--config-c3", default="", help="--config for the default line's c3 board")
    ap.add_argument("--c3-cpu-gens", type=int, default=20,
                    help="generations of the 65536^2 board the oracle times (0 = a budget of "
                         "about 15 s)")
    ap.add_argument("--config-c2", default="", help="--config for the default line's c2 board")
    ap.add_argument("--sweep", action="store_true",
                    help="time T in {2,4,8,16} x band heights for the single-board workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding "
                                   "of the row strips is a design, not a measured path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "needs a HIP device"
    torch.cuda.set_device(0)

    if args.sweep:
        return sweep(args)
    if args.workload == "all":
        line = default_line(args)
    elif args.workload == "c2":
        line = single_line(args, single_board(args, 16384, 16384, 1000, 0.3, args.config,
                                              compare_t1=args.compare_t1))
    elif args.workload == "c3":
        line = single_line(args, single_board(args, 65536, 65536, 200, 0.5, args.config,
                                              compare_t1=True))
    elif args.workload == "c4":
        line = single_line(args, batched(args))
    elif args.workload == "c1":
        line = single_line(args, host_api(args))
    elif args.workload == "c5":
        line = single_line(args, served(args, plain=not args.no_plain))
    elif args.workload == "copy":
        copy_calibration(args)
        return
    elif args.workload == "pop":
        population_workload(args)
        return
    elif args.workload == "bounded":
        bounded_workload(args)
        return
    elif args.workload == "strip":
        strip_workload(args)
        return
    elif args.workload == "decomp":
        decomp_workload(args)
        return
    elif args.workload == "valu":
        valu_workload(args)
        return
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
