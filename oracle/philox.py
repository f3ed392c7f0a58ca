"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11) and Box-Muller normals, written from the published
definition; vectorised numpy over uint64 lanes holding 32-bit values.

One round maps counter (c0, c1, c2, c3) and key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57; between rounds the key is bumped by
the Weyl constants (0x9E3779B9, 0xBB67AE85).  Ten rounds.

Gaussian test matrix: entry e (row-major index into m x ell) uses the pair
index p = e // 2 as the 64-bit counter low half (c0 = p mod 2^32,
c1 = p >> 32), the draw counter as the high half (c2, c3), and the 64-bit
seed as the key.  The four outputs give two 53-bit uniforms
u(a, b) = ((a * 2^32 + b) >> 11) * 2^-53 + 2^-54 in (0, 1), and
Box-Muller gives sqrt(-2 ln u1) cos(2 pi u2) for even e and
sqrt(-2 ln u1) sin(2 pi u2) for odd e.

Test infrastructure (see the package docstring).
"""

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    c = [v.copy() for v in c]
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    for r in range(10):
        if r > 0:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = c[0] * np.uint64(M0)
        p1 = c[2] * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [v.astype(np.uint32) for v in c]


def _u53(a, b):
    v = (a.astype(np.uint64) << np.uint64(32)) | b.astype(np.uint64)
    return (v >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 + 2.0 ** -54


def gaussian_matrix(m, ell, seed, counter):
    """m x ell FP64 standard normals from Philox4x32-10 keyed by (seed, counter)."""
    e = np.arange(m * ell, dtype=np.uint64)
    p = e >> np.uint64(1)
    o = philox4x32_10(p & np.uint64(MASK), p >> np.uint64(32),
                      counter & MASK, (counter >> 32) & MASK,
                      seed & MASK, (seed >> 32) & MASK)
    u1 = _u53(o[0], o[1])
    u2 = _u53(o[2], o[3])
    r = np.sqrt(-2.0 * np.log(u1))
    odd = (e & np.uint64(1)).astype(bool)
    g = np.where(odd, r * np.sin(2.0 * np.pi * u2), r * np.cos(2.0 * np.pi * u2))
    return g.reshape(m, ell)
