"""The beam's standard normals drawn from a seed, written from the generators' published
definitions.  TEST INFRASTRUCTURE ONLY: the tests and the smoke check import it, to check the
library's own on-device draws (pic_beam with normals = NULL).

Generator: Philox4x32-10 (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011, section 4): a 128-bit counter and a 64-bit key; each of the
ten rounds multiplies counter words 0 and 2 by fixed 32-bit multipliers, and the new counter is
(hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); between rounds the key advances
by two Weyl constants.  Normals: the Box-Muller transform (G. E. P. Box, M. E. Muller, Ann. Math.
Statist. 29, 1958) of pairs of uniforms U = (w + 1/2) 2^-32.  Which counter, word and row is which
is the library's own convention (include/pic.h, pic_beam): particle p takes the counters
(p mod 2^32, p div 2^32, j, 0), j = 0, 1, under the key (seed mod 2^32, seed div 2^32); words
(w0, w1), (w2, w3), (w4, w5) give rows (0, 1), (2, 3), (4, 5).
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
LO = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ctr (4 arrays or scalars of 32-bit words) under key (k0, k1):
    the four output words as uint64 arrays holding 32-bit values."""
    c = [np.asarray(v, dtype=np.uint64) & LO for v in ctr]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & 0xFFFFFFFF, (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> S32) ^ c[1] ^ np.uint64(k0), p1 & LO, (p0 >> S32) ^ c[3] ^ np.uint64(k1), p0 & LO]
    return c


def box_muller(wa, wb):
    """Two standard normals from two 32-bit words each (arrays)."""
    ua = (wa.astype(np.float64) + 0.5) * 2.0 ** -32
    ub = (wb.astype(np.float64) + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(ua))
    return rad * np.cos(2.0 * np.pi * ub), rad * np.sin(2.0 * np.pi * ub)


def beam_normals_from_seed(n: int, seed: int) -> np.ndarray:
    """(6, n) float64 standard normals of a beam of n macroparticles drawn from seed."""
    p = np.arange(int(n), dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    key = (seed & 0xFFFFFFFF, seed >> 32)
    w = []
    for j in (0, 1):
        w += philox4x32_10((p & LO, p >> S32, np.full_like(p, j), np.zeros_like(p)), key)
    out = np.empty((6, int(n)))
    for r in range(3):
        out[2 * r], out[2 * r + 1] = box_muller(w[2 * r], w[2 * r + 1])
    return out
