"""ORACLE command line -- test infrastructure only, like the rest of this package.

    python -m oracle IN.npy GENERATIONS OUT.npy [--threads N] [--decomposition rows|cols|2d]
                     [--population G1,G2,...]

IN.npy holds a 2-D uint8 board (nonzero = alive; loaded without pickle).  The
board advances GENERATIONS generations on its torus with the plain C oracle
(serial, or split among N OpenMP threads by the chosen decomposition) and the
0/1 result is saved to OUT.npy.  --population prints the live-cell count after
each listed generation count (the quantity of the paper's Table 1).
"""
from __future__ import annotations

import argparse
import sys

import numpy as np

from . import life, life_decomp, population_at


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m oracle", description=__doc__.split("\n\n")[0])
    ap.add_argument("board", help="input .npy, 2-D uint8, nonzero = alive")
    ap.add_argument("generations", type=int)
    ap.add_argument("out", help="output .npy (0/1 uint8)")
    ap.add_argument("--threads", type=int, default=1)
    ap.add_argument("--decomposition", choices=["rows", "cols", "2d"], default="rows")
    ap.add_argument("--population", default="", help="comma-separated generation counts")
    a = ap.parse_args(argv)
    b = np.load(a.board, allow_pickle=False)
    if b.ndim != 2:
        print("the board must be 2-D", file=sys.stderr)
        return 2
    b = (b != 0).astype(np.uint8)
    if a.threads > 1:
        out = life_decomp(b, a.generations, a.threads, a.decomposition)
    else:
        out = life(b, a.generations)
    np.save(a.out, out)
    if a.population:
        checks = [int(x) for x in a.population.split(",")]
        for g, n in zip(checks, population_at(b, checks, threads=max(1, a.threads))):
            print(f"generation {g}: population {n}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
