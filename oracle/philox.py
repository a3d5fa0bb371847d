"""Philox4x64-10 counter-based generator (oracle test infrastructure).

Written from the published definition: J. K. Salmon, M. A. Moraes, R. O. Dror,
D. E. Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11.  One round
maps the counter (x0, x1, x2, x3) with key (k0, k1) to
    (hi(M0 x2) ^ x1 ^ k0,  lo(M0 x2)... )
in the paper's S-box form: two 64x64 -> 128-bit products of x0 and x2 by the
round multipliers, their high halves xor-ed with the other two words and the
key, then a word permutation; the key is bumped by the Weyl constants between
rounds.  Ten rounds.

Uniform doubles in (0, 1) are taken from the top 52 bits of a word:
u = ((x >> 12) + 0.5) * 2^-52 = (2k + 1) 2^-53 with k < 2^52, which every
double holds exactly, so the conversion never rounds and u is never 0 or 1.
"""
import numpy as np

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15   # golden ratio
W1 = 0xBB67AE8584CAA73B   # sqrt(3) - 1
ROUNDS = 10


def philox_scalar(ctr, key):
    """Reference on Python integers: one 4x64 block for counter ctr (4 ints)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for _ in range(ROUNDS):
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK64, (p0 >> 64) ^ x3 ^ k1, p0 & MASK64)
        k0 = (k0 + W0) & MASK64
        k1 = (k1 + W1) & MASK64
    return x0, x1, x2, x3


_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """64x64 -> (hi, lo) on uint64 arrays via 32-bit halves."""
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, a * b


def philox(ctr, key):
    """Vectorised blocks: ctr is (n, 4) uint64, key is (2,) or (n, 2); returns (n, 4)."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(key[..., 0], x0.shape).copy()
    k1 = np.broadcast_to(key[..., 1], x0.shape).copy()
    m0, m1, w0, w1 = np.uint64(M0), np.uint64(M1), np.uint64(W0), np.uint64(W1)
    with np.errstate(over="ignore"):
        for _ in range(ROUNDS):
            h0, l0 = _mulhilo(m0, x0)
            h1, l1 = _mulhilo(m1, x2)
            x0, x1, x2, x3 = h1 ^ x1 ^ k0, l1, h0 ^ x3 ^ k1, l0
            k0 = k0 + w0
            k1 = k1 + w1
    return np.stack([x0, x1, x2, x3], axis=-1)


def to_uniform(x):
    """(0, 1) doubles from uint64 words: ((x >> 12) + 0.5) * 2^-52 (exact)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)
