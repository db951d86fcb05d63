"""GPU: the device form of the seeded board generator draws the same cells as
the host one (gen.c), bit for bit, padding bits included."""
import numpy as np
import pytest

import seeded_inputs
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,cols,p", [(1, 1, 0.5), (3, 65, 0.5), (100, 1000, 0.3),
                                         (257, 4097, 0.05), (64, 128, 0.0), (33, 70, 1.0),
                                         (2048, 8192, 0.5)])
def test_device_board_equals_host_board(rows, cols, p):
    import torch
    say("device board", rows, cols, p)
    want = seeded_inputs.board_packed(1209, 7, rows, cols, p)
    d = torch.empty(want.size, dtype=torch.int64, device="cuda")
    seeded_inputs.board_packed_device(1209, 7, rows, cols, p, d)
    got = d.cpu().numpy().view(np.uint64).reshape(want.shape)
    assert np.array_equal(got, want)


def test_device_board_rejects_a_wrong_buffer():
    import torch
    d = torch.empty(5, dtype=torch.int64, device="cuda")
    with pytest.raises(ValueError):
        seeded_inputs.board_packed_device(1, 0, 10, 10, 0.5, d)
