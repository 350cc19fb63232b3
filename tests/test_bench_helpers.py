"""Host-side helpers of the benchmark (no GPU): the FP32-against-FP64 error
and the byte model's invariants."""
import numpy as np

import bench


def test_fp32_error_masks_padding_and_class_flips():
    rng = np.random.default_rng(0)
    ngpc, nvar, n = 4, 3, 10
    fs64 = rng.normal(size=(ngpc, nvar, n))
    fs32 = (fs64 + 1e-6).astype(np.float32)
    ngp = np.array([4, 4, 3, 3, 2, 4, 4, 1, 4, 4])
    for c in range(n):                      # garbage past each cell's Gauss points is ignored
        fs32[ngp[c]:, :, c] = 1e9
    cls64 = np.zeros(n, np.uint8)
    cls32 = cls64.copy()
    cls32[5] = 1                            # a flipped cell is left out and counted
    fs32[:, :, 5] = 1e9
    U = np.ones((n, nvar)) * 2.0
    out = bench.fp32_error((fs64, cls64), fs32, cls32, ngp, U)
    assert out["fp32_class_flips"] == 1
    assert 1e-7 < out["fp32_state_err_vs_fp64"] < 1e-6    # about 1e-6 / 2, FP32 rounding aside


def test_workloads_are_described():
    for key, (text, tag, prec) in bench.WORKLOADS.items():
        assert prec in (32, 64) and tag and "cells" in text
