"""Benchmark of the Life step library on one MI355X.

Default workload (one "step" = the whole hot path over one input): a
16384 x 16384 toroidal board, bit-packed, i.i.d. Bernoulli(0.3) cells from seed
1209, advanced 1000 generations by gol_step_packed.  Prints one JSON line with
cell-updates/s, the roofline of the dominant kernel and the CPU oracle timed
on a bounded sample of the same workload.

Other workloads (--workload): c1 (256^2 byte board, 100 generations, host
API), c3 (65536^2, 200 generations, temporal-blocked vs one generation per
launch), c4 (4096 boards in one batched schedule vs one launch sequence per
board), c5 (Poisson request stream through the continuous-batching server vs
a one-at-a-time server).
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

# MI355X: 256 CUs x 4 SIMDs x 16 lanes, 2.4 GHz peak engine clock.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9          # 32-bit integer VALU ops/s
HBM_PEAK_BYTES = 8.0e12
# Algorithmic integer ops per cell-update of the bit-sliced step: per 32-cell
# word and generation 2 funnel shifts + 2 (horizontal 3-sum) + 4 (vertical
# combine) + 4 (rule) = 12 ops.
OPS_PER_CELL_UPDATE = 12.0 / 32.0
# Algorithmic HBM bytes per cell-update of a one-generation pass: read + write
# one bit.
BYTES_PER_CELL_UPDATE_T1 = 2.0 / 8.0

SEED = 1209


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return max(1, int(env))
    return os.cpu_count() or 1


def cpu_baseline(rows, cols, p, seed, budget_s=12.0):
    """The oracle (plain C, row decomposition over OpenMP threads) on a bounded
    number of generations of the same board; cell-updates/s."""
    import oracle
    import seeded_inputs
    threads = cpu_threads()
    b = seeded_inputs.board_bytes(seed, 0, rows, cols, p)
    t0 = time.perf_counter()
    cur = oracle.life(b, 1, threads=threads)
    one = time.perf_counter() - t0
    g = max(1, min(1000, int(budget_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.life(cur, g, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": rows * cols * g / dt, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{g} generations of the {rows}x{cols} board (of the run's 1000), "
                      f"{threads} OpenMP threads, byte-per-cell C oracle"}


def roofline_alu(cells, T, avg_launch_s):
    ops = OPS_PER_CELL_UPDATE * cells * T
    achieved = ops / avg_launch_s / 1e12
    peak = VALU_PEAK_OPS / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TOP/s",
            "frac": achieved / peak, "traffic": None,
            "kernel": f"k_board_pass<{T}>", "avg_launch_us": avg_launch_s * 1e6,
            "ops_per_launch": ops}


def roofline_hbm(cells, avg_launch_s):
    by = BYTES_PER_CELL_UPDATE_T1 * cells
    achieved = by / avg_launch_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_BYTES / 1e9, "unit": "GB/s",
            "frac": achieved / (HBM_PEAK_BYTES / 1e9), "traffic": None,
            "kernel": "k_board_pass<1>", "avg_launch_us": avg_launch_s * 1e6,
            "bytes_per_launch": by}


def time_packed(gol, torch, d_in, d_out, R, C, G, steps, warmup, T):
    for _ in range(warmup):
        gol.step_packed(d_in, R, C, G, d_out, t_block=T)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(st)
    for _ in range(steps):
        gol.step_packed(d_in, R, C, G, d_out, t_block=T)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev = e0.elapsed_time(e1) / 1e3
    return wall, dev


def single_board(args, R, C, G, p, label):
    import torch
    import paper_1209_4408_amd as gol
    import seeded_inputs
    from paper_1209_4408_amd import build as _b  # noqa: F401
    T = args.t_block or 8
    log(f"generating {R}x{C} board p={p}")
    w = seeded_inputs.board_packed(SEED, 0, R, C, p)
    d_in = torch.from_numpy(w.view(np.int64)).cuda()
    del w
    d_out = torch.empty_like(d_in)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps after {args.warmup} warmup, T={T}")
    wall, dev = time_packed(gol, torch, d_in, d_out, R, C, G, args.steps, args.warmup, T)
    cells = R * C
    value = cells * G * args.steps / wall
    launches = G // T
    avg_launch = dev / (args.steps * launches)
    res = {"value": value, "wall_s": wall, "dev_s": dev,
           "roofline": roofline_alu(cells, T, avg_launch) if T > 1 else roofline_hbm(cells,
                                                                                       avg_launch)}
    extra = {}
    if args.compare_t1:
        wall1, dev1 = time_packed(gol, torch, d_in, d_out, R, C, G, max(1, args.steps // 2), 1, 1)
        v1 = cells * G * max(1, args.steps // 2) / wall1
        extra["t1"] = {"value": v1, "unit": "cell-updates/s",
                       "roofline": roofline_hbm(cells, dev1 / (max(1, args.steps // 2) * G))}
        extra["speedup_vs_t1"] = value / v1
    return res, extra


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--t-block", type=int, default=0)
    ap.add_argument("--compare-t1", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding "
                                   "of the row strips is a design, not a measured path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "needs a HIP device"
    torch.cuda.set_device(0)

    if args.workload == "c2":
        R = C = 16384
        G, p = 1000, 0.3
        res, extra = single_board(args, R, C, G, p, "c2")
        workload = "16384x16384 torus, bit-packed, Bernoulli(0.3), 1000 generations"
    elif args.workload == "c3":
        R = C = 65536
        G, p = 200, 0.5
        args.compare_t1 = True
        res, extra = single_board(args, R, C, G, p, "c3")
        workload = "65536x65536 torus, bit-packed, Bernoulli(0.5), 200 generations"
    else:
        raise SystemExit("workload not implemented yet")
    ms = res["wall_s"] / args.steps * 1e3
    line = {
        "metric": "cell-updates/sec",
        "value": res["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": workload, "rows": R, "cols": C, "generations": G, "p": p,
                   "seed": SEED, "t_block": args.t_block or 8, "parallelism": "single GPU"},
        "roofline": res["roofline"],
    }
    line.update(extra)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(min(R, 16384), min(C, 16384), p, SEED)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
