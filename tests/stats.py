"""Binomial helpers shared by the statistical tests."""
import math

import numpy as np


def popcount_rows(words, shots):
    """Number of set bits per row of a record-major bit-packed array."""
    w = np.asarray(words, dtype=np.uint64)
    if w.size == 0:
        return np.zeros(w.shape[0], np.int64)
    full, rem = divmod(shots, 64)
    mask = np.full(w.shape[1], np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64)
    if rem:
        mask[full] = np.uint64((1 << rem) - 1)
    b = np.unpackbits((w & mask).view(np.uint8), axis=1)
    return b.sum(axis=1)


def within_sigma(k, n, p, nsig=5.0):
    """|k/n - p| <= nsig * sd (+1/n slack for p near 0 or 1)."""
    sd = math.sqrt(max(p * (1 - p), 1e-300) / n)
    return abs(k / n - p) <= nsig * sd + 1.0 / n


def two_sample_ok(k1, n1, k2, n2, nsig=5.0):
    """Two-sample binomial test with pooled variance."""
    p = (k1 + k2) / (n1 + n2)
    sd = math.sqrt(max(p * (1 - p), 1e-300) * (1 / n1 + 1 / n2))
    return abs(k1 / n1 - k2 / n2) <= nsig * sd + 1.0 / min(n1, n2)
