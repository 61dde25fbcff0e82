"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC 2011) and the Gaussian
sketch drawn from it.  Test infrastructure only.

philox4x32_10(c0, c1, c2, c3, k0, k1): ten rounds of
    (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by the Weyl
constants (0x9E3779B9, 0xBB67AE85) between rounds; elementwise over numpy
uint32 arrays.

Sketch entry (t, j), t < T, j < k (the on-device generator of the STR build
draws the same numbers): counter (t, j, 0, 0), key (seed mod 2^32,
seed >> 32); u1 = (out0 + 1/2) 2^-32, u2 = out1 2^-32;
S[t, j] = sqrt(-2 ln u1) cos(2 pi u2) / sqrt(k), rounded to float32.
Pinned by the generator's published known-answer vectors.
"""
import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3)]
    k = [np.asarray(v, dtype=np.uint64) & _MASK for v in (k0, k1)]
    for rnd in range(10):
        if rnd > 0:
            k = [(k[0] + _W0) & _MASK, (k[1] + _W1) & _MASK]
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k[0], p1 & _MASK, (p0 >> np.uint64(32)) ^ c[3] ^ k[1], p0 & _MASK]
    return [v.astype(np.uint32) for v in c]


def gaussian_sketch_philox(T, k, seed):
    """S (T x k), entries N(0, 1/k), returned as a C-contiguous (k, T)
    float32 array (row j is sketch column j, i.e. S column-major)."""
    t = np.arange(T, dtype=np.uint64)[None, :]
    j = np.arange(k, dtype=np.uint64)[:, None]
    zero = np.zeros((1, 1), dtype=np.uint64)
    seed = int(seed)
    o = philox4x32_10(np.broadcast_to(t, (k, T)), np.broadcast_to(j, (k, T)), zero, zero,
                      seed & 0xFFFFFFFF, seed >> 32)
    u1 = (o[0].astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = o[1].astype(np.float64) * 2.0 ** -32
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(6.283185307179586 * u2)
    return (z / np.sqrt(float(k))).astype(np.float32)
