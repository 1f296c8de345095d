"""Philox4x32-10 and the Box-Muller start block, written out in numpy from
their published definitions (test helper for the library's tm_random_block).

Philox4x32-10: Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11.  A round maps the counter (c0, c1, c2, c3) with key
(k0, k1) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key gains the Weyl increments
(0x9E3779B9, 0xBB67AE85) before every round after the first.
"""

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32-valued array; key: (k0, k1).  Returns (..., 4) uint64."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0, k1 = int(key[0]), int(key[1])
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
    return np.stack(c, axis=-1)


def random_block(n, m, seed):
    """Entry (r, j) of the n x m standard normal block: member e % 2 of the
    Box-Muller pair of counter (e / 2, 0, 0, 0), e = r m + j."""
    e = np.arange(n * m, dtype=np.uint64)
    k = e >> np.uint64(1)
    ctr = np.zeros((n * m, 4), dtype=np.uint64)
    ctr[:, 0] = k & _MASK
    ctr[:, 1] = k >> np.uint64(32)
    out = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    a = ((out[:, 1] << np.uint64(32)) | out[:, 0]) >> np.uint64(11)
    b = ((out[:, 3] << np.uint64(32)) | out[:, 2]) >> np.uint64(11)
    u1 = (a + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    v = np.where((e & np.uint64(1)) == 1, rad * np.sin(th), rad * np.cos(th))
    return v.reshape(n, m)
