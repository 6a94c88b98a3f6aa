"""The pair kernels divide small lane-varying integers by uniform ones
(lane / chunk width, index mod block size) with a reciprocal instead of the
integer division sequence: floor(a / b) = trunc((a + 1/2) * rcp(b)) in FP32
(`small_div` in csrc/common.h).  The hardware reciprocal is within 1 ulp, so
this checks the claim over every a < 4096 and b <= 2048 (the kernels' range:
indices below twice the neighbour count) with the reciprocal rounded down,
correctly and up by one ulp."""
import numpy as np


def test_small_div_exact_over_the_kernels_range():
    a = np.arange(4096, dtype=np.int64)
    af = (a.astype(np.float32) + np.float32(0.5)).astype(np.float32)
    for b in range(1, 2049):
        inv = np.float32(1.0) / np.float32(b)
        for r in (np.nextafter(inv, np.float32(0)), inv, np.nextafter(inv, np.float32(1))):
            q = (af * np.float32(r)).astype(np.float32).astype(np.int64)  # v_cvt_u32_f32 truncates
            assert np.array_equal(q, a // b), b
