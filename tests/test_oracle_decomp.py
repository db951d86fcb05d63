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
