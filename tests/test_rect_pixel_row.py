"""The row of the k-th pixel of a leaf rectangle (row-major, width wr) is
computed on the GPU below k = 2^22 as trunc(float(k) * rcp(float(wr))) with the
hardware reciprocal estimate (within 1 ulp), followed by one correction step
that moves the quotient by at most one.  This CPU emulation checks that the
estimate is never off by more than one for every width up to 2048 and for
sampled widths up to the largest image side, at every row boundary (the
indices just below and at each multiple of wr, where truncation is most
sensitive), with the reciprocal correctly rounded and one ulp either side."""

import numpy as np

K_LIMIT = 1 << 22


def _reciprocals(wr):
    r = np.float32(1.0) / np.float32(wr)
    return (np.nextafter(r, np.float32(0.0)), r, np.nextafter(r, np.float32(np.inf)))


def _max_row_error(wr):
    m = np.arange(0, K_LIMIT // wr + 2, dtype=np.int64)
    k = np.concatenate([m * wr - 1, m * wr, m * wr + wr // 2])
    k = k[(k >= 0) & (k < K_LIMIT)]
    exact = k // wr
    kf = k.astype(np.float32)  # exact below 2^24
    worst = 0
    for r in _reciprocals(wr):
        q = (kf * r).astype(np.float32).astype(np.int64)  # the float32 product, truncated toward zero
        worst = max(worst, int(np.abs(q - exact).max()))
    return worst


def test_row_estimate_within_one_for_small_widths():
    worst = max(_max_row_error(wr) for wr in range(1, 2049))
    assert worst <= 1


def test_row_estimate_within_one_for_sampled_large_widths():
    rng = np.random.default_rng([1809, 1334, 22])
    widths = np.unique(np.concatenate([rng.integers(2049, 32768, 300), [2049, 4095, 4096, 8191, 16384, 32767]]))
    assert max(_max_row_error(int(wr)) for wr in widths) <= 1


def test_correction_recovers_the_exact_row():
    """The kernel's single correction step gives floor(k / wr) and k mod wr."""
    rng = np.random.default_rng([1809, 1334, 23])
    for wr in (1, 3, 7, 100, 1023, 2047, 2048, 32767):
        k = rng.integers(0, K_LIMIT, 20000)
        for r in _reciprocals(wr):
            q = (k.astype(np.float32) * r).astype(np.float32).astype(np.int64)
            rem = k - q * wr
            q = np.where(rem < 0, q - 1, np.where(rem >= wr, q + 1, q))
            rem = k - q * wr
            assert np.array_equal(q, k // wr) and np.array_equal(rem, k % wr)
