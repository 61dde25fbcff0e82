"""Pins of oracle/philox.py: the known-answer vectors published with the
Philox4x32-10 generator, and the moments of the Gaussian sketch."""
import numpy as np

from oracle.philox import gaussian_sketch_philox, philox4x32_10

KAT = [  # counter (4 words), key (2 words) -> output (4 words)
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


def test_known_answer_vectors():
    for c, k, want in KAT:
        got = philox4x32_10(*[np.array([v]) for v in c], *[np.array([v]) for v in k])
        assert tuple(int(v[0]) for v in got) == want


def test_vectorised_matches_scalar():
    c0 = np.array([0, 1, 2, 0xffffffff], dtype=np.uint64)
    out = philox4x32_10(c0, c0 * 3, c0 ^ 0x55, 0 * c0, 7, 9)
    for i in range(4):
        one = philox4x32_10(np.array([c0[i]]), np.array([c0[i] * 3]), np.array([c0[i] ^ 0x55]), np.array([0]), 7, 9)
        assert [int(v[i]) for v in out] == [int(v[0]) for v in one]


def test_gaussian_sketch_moments():
    """E[S S^T] = I (T x T) for N(0, 1/k) entries: column norms of S^T near
    1, mean near 0, and different seeds give different sketches."""
    T, k = 300, 4000
    S = gaussian_sketch_philox(T, k, 3).astype(np.float64)   # (k, T)
    assert S.shape == (k, T)
    G = S.T @ S                                                # T x T, ~ I
    assert np.abs(np.diag(G) - 1).max() < 0.12
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 0.1
    assert abs(S.mean()) * np.sqrt(k) < 0.01
    z = S.ravel() * np.sqrt(k)
    assert abs(z.std() - 1) < 0.01 and abs(np.mean(z ** 4) - 3) < 0.05
    assert not np.array_equal(gaussian_sketch_philox(20, 10, 3), gaussian_sketch_philox(20, 10, 4))
