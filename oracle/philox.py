"""Philox4x64-10 (oracle; test infrastructure only).

Written from the generator's published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a
2-word key, ten rounds of two 64x64->128-bit multiplies with the multipliers
0xD2E7470EE14C6C93 and 0xCA5A826395121157, the high halves XOR-ed with the
other two counter words and the key, the words permuted, and the key bumped by
the Weyl constants 0x9E3779B97F4A7C15 and 0xBB67AE8584CAA73B between rounds.
Pure Python integers, so every step is exact.
"""

_MASK = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B


def _mulhilo(a, b):
    p = a * b
    return (p >> 64) & _MASK, p & _MASK


def philox4x64_10(counter, key):
    """Encrypt one 4x64 counter block under a 2x64 key; returns 4 ints."""
    x0, x1, x2, x3 = (int(v) & _MASK for v in counter)
    k0, k1 = (int(v) & _MASK for v in key)
    for _ in range(10):
        hi0, lo0 = _mulhilo(_M0, x0)
        hi1, lo1 = _mulhilo(_M1, x2)
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + _W0) & _MASK
        k1 = (k1 + _W1) & _MASK
    return [x0, x1, x2, x3]
