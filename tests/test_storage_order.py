"""The storage-order helper used by the GPU tests agrees with the order it
documents, written out with Python tuples (CPU)."""
import math
import struct

import numpy as np

from storage_order import band_order


def _key(t, s):
    r = 2.0 * t / s
    b = min(math.floor(r), 20) if r > 0.0 else 0
    return (b, ((1 << 63) - 1 - struct.unpack("<Q", struct.pack("<d", s))[0]) >> 6)


def test_band_order_matches_tuple_sort():
    rng = np.random.default_rng(5)
    n = 3000
    s = rng.uniform(0.03, 0.06, n)
    t = np.concatenate([rng.uniform(0.3, 0.8, n // 2), rng.exponential(1.5, n - n // 2) + 0.3])
    s[:20] = s[20:40]                      # ties in sigma: stable order
    t[5] = np.nan                          # band 0
    ref = sorted(range(n), key=lambda i: (_key(t[i], s[i]), i))
    assert np.array_equal(band_order(t, s), np.array(ref))
