"""Random draws the eigensolver makes itself (refill of dependent columns).

Philox4x32-10 (Salmon et al., SC 2011), written out here for the oracle alone:
ten rounds of two 32x32->64 multiplies with constants 0xD2511F53 and
0xCD9E8D57 and a Weyl key schedule 0x9E3779B9 / 0xBB67AE85.

Refill draw for row i of column j at expansion step s, solver seed K:
counter (i mod 2^32, i >> 32, s, 0x52460000 + j), key (K mod 2^32, K >> 32);
word 0 is mapped to (w >> 8) * 2^-23 - 1, uniform in [-1, 1) and exact in FP32.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Vectorised over the counter words (numpy uint32-valued arrays)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        n0 = (p1 >> np.uint64(32)) ^ c1 ^ np.uint64(k0)
        n1 = p1 & _MASK
        n2 = (p0 >> np.uint64(32)) ^ c3 ^ np.uint64(k1)
        n3 = p0 & _MASK
        c0, c1, c2, c3 = n0, n1, n2, n3
    return c0, c1, c2, c3


def refill_column(n: int, j: int, step: int, seed: int) -> np.ndarray:
    i = np.arange(n, dtype=np.uint64)
    w0, _, _, _ = philox4x32_10(i & _MASK, i >> np.uint64(32),
                                np.full(n, step, dtype=np.uint64),
                                np.full(n, 0x52460000 + j, dtype=np.uint64),
                                seed & 0xFFFFFFFF, seed >> 32)
    return (w0 >> np.uint64(8)).astype(np.float64) * 2.0 ** -23 - 1.0
