"""Pins of the oracle Philox4x64-10 against numpy's independent implementation."""
import numpy as np

from oracle import philox as P


def _numpy_block(ctr, key):
    # numpy's Philox increments the 256-bit counter before producing a block,
    # so the block for counter c is the first output of state c - 1.
    c = [int(x) for x in ctr]
    i = 0
    while i < 4 and c[i] == 0:
        c[i] = (1 << 64) - 1
        i += 1
    if i < 4:
        c[i] -= 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


def test_scalar_matches_numpy():
    rng = np.random.default_rng(0)
    for _ in range(50):
        ctr = [int(v) for v in rng.integers(0, 2 ** 63, 4, dtype=np.int64)]
        ctr[0] += 1
        key = [int(v) for v in rng.integers(0, 2 ** 63, 2, dtype=np.int64)]
        assert P.philox_scalar(ctr, key) == _numpy_block(ctr, key)
    assert P.philox_scalar([0, 1, 0, 0], [7, 9]) == _numpy_block([0, 1, 0, 0], [7, 9])


def test_vectorised_matches_scalar_and_numpy():
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 64 - 1, (64, 4), dtype=np.uint64, endpoint=False)
    ctr[:, 0] |= np.uint64(1)
    key = np.array([170601423, 5], dtype=np.uint64)
    out = P.philox(ctr, key)
    for i in range(64):
        ref = P.philox_scalar([int(v) for v in ctr[i]], [int(k) for k in key])
        assert tuple(int(v) for v in out[i]) == ref
        assert ref == _numpy_block([int(v) for v in ctr[i]], [int(k) for k in key])


def test_known_answer_all_zero():
    # block for counter 0, key 0 (fixed by the definition; also numpy's
    # stream with counter 2^256 - 1 wrapped)
    x = P.philox_scalar([0, 0, 0, 0], [0, 0])
    assert x == _numpy_block([0, 0, 0, 0], [0, 0])


def test_uniform_conversion_open_interval():
    words = np.array([0, 1, 2 ** 12 - 1, 2 ** 12, 2 ** 63 + 2 ** 12 + 5, 2 ** 64 - 1], dtype=np.uint64)
    u = P.to_uniform(words)
    assert u[0] == 2.0 ** -53 and u[1] == 2.0 ** -53 and u[2] == 2.0 ** -53
    assert u[3] == 3.0 * 2.0 ** -53
    assert u[4] == 0.5 + 3.0 * 2.0 ** -53
    assert u[-1] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))
    # exact: (2k + 1) 2^-53 for every k < 2^52
    k = np.arange(2 ** 52 - 1000, 2 ** 52, dtype=np.uint64)
    assert np.all(P.to_uniform(k << np.uint64(12)) * 2.0 ** 53 == (2 * k + 1).astype(np.float64))
