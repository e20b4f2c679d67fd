"""The general multi-step kernel numbers each level's window row by row (or
column by column) and takes the quotient r div w in FP32 as (r + 1/2) * (1/w),
truncated.  This pins that arithmetic over the range the kernel asserts at
compile time (r < 4096, w <= 80), for a correctly rounded reciprocal and for one
off by one unit in the last place either way."""
import numpy as np


def test_fp32_quotient_is_exact_over_the_kernel_range():
    r = np.arange(4096, dtype=np.int64)
    for w in range(1, 81):
        inv = np.float32(1.0) / np.float32(w)
        for inv_w in (inv, np.nextafter(inv, np.float32(0)), np.nextafter(inv, np.float32(1))):
            q = ((r.astype(np.float32) + np.float32(0.5)) * inv_w).astype(np.int64)
            assert np.array_equal(q, r // w), w


def test_fp32_quotient_fails_outside_it_without_the_half():
    # the + 1/2 is what keeps the product away from an integer: without it,
    # exact multiples of w can round just below and truncate one short
    r = np.arange(4096, dtype=np.int64)
    bad = 0
    for w in range(1, 81):
        inv = np.float32(1.0) / np.float32(w)
        q = (r.astype(np.float32) * inv).astype(np.int64)
        bad += int((q != r // w).sum())
    assert bad > 0
