"""The C oracle's domain decompositions (rows, columns, 2-D blocks of Sections
2.1-2.2) against the serial oracle and the numpy form: each splits the cells of
a generation among threads, so every split must give the same board."""
import numpy as np
import pytest

import oracle
import seeded_inputs


@pytest.mark.parametrize("decomposition", ["rows", "cols", "2d"])
@pytest.mark.parametrize("threads", [1, 2, 3, 4, 6, 8])
def test_decompositions_equal_the_serial_oracle(decomposition, threads):
    for k, (R, C) in enumerate([(1, 1), (3, 5), (7, 2), (60, 120), (120, 60), (33, 65)]):
        b = seeded_inputs.board_bytes(560, 10 * k + threads, R, C, 0.4)
        for G in (0, 1, 5):
            want = oracle.ref.life(b, G)
            got = oracle.life_decomp(b, G, threads, decomposition)
            assert np.array_equal(got, want), (decomposition, threads, R, C, G)


def test_decomposition_rejects_bad_arguments():
    b = np.zeros((4, 4), dtype=np.uint8)
    with pytest.raises(KeyError):
        oracle.life_decomp(b, 1, 2, "diagonal")
    with pytest.raises(ValueError):
        oracle.life_decomp(b, 1, 0, "rows")
    with pytest.raises(ValueError):
        oracle.life_decomp(b, -1, 2, "2d")


def test_command_line(tmp_path):
    """python -m oracle: the same board as the library call, and the population
    at the listed generations."""
    import subprocess
    import sys
    b = seeded_inputs.board_bytes(561, 0, 30, 45, 0.4)
    src, dst = tmp_path / "in.npy", tmp_path / "out.npy"
    np.save(src, b)
    r = subprocess.run([sys.executable, "-m", "oracle", str(src), "17", str(dst), "--threads", "3",
                        "--decomposition", "2d", "--population", "0,5,17"],
                       capture_output=True, text=True, check=True,
                       cwd=str(__import__("pathlib").Path(oracle.__file__).parent.parent))
    assert np.array_equal(np.load(dst), oracle.life(b, 17))
    want = oracle.population_at(b, [0, 5, 17])
    assert r.stdout.split() == [w for g, n in zip([0, 5, 17], want)
                                for w in ("generation", f"{g}:", "population", str(n))]
