"""Pins for the oracle's Gaussian test matrix (Alg. 2/3 "Sample Gaussian Matrix").

The generator itself is pinned to the known-answer vectors published with Philox4x32-10
(Salmon, Moraes, Dror, Shaw, SC'11; tests/golden/philox4x32_10_kat.json); what the method
needs from it -- i.i.d. N(0,1) entries reproducible from (seed, stream, inversion index) --
is pinned statistically and structurally below."""
import json
import os

import numpy as np
from scipy import stats

import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.json")


def _kat_cases():
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


def test_philox_known_answer_vectors():
    cases = _kat_cases()
    assert len(cases) == 3
    for c in cases:
        ctr = np.array([int(x, 16) for x in c["ctr"]], dtype=np.uint64)
        key = tuple(int(x, 16) for x in c["key"])
        out = O.philox4x32_10(ctr, key)
        assert [int(v) for v in out] == [int(x, 16) for x in c["out"]], c


def test_philox_known_answer_through_omega_counter_layout():
    # Row 0, column group 0, stream 0, inversion 0 under seed 0 is the all-zero counter and
    # key: the first four words of Omega's draw are the first known-answer vector.
    c = _kat_cases()[0]
    w = O.philox_words_for(1, 4, seed=0, stream_id=0, inversion_index=0)
    assert [int(v) for v in w[0, 0]] == [int(x, 16) for x in c["out"]]
    # seed -> key: (seed mod 2^32, seed >> 32); stream/inversion -> counter words 2 and 3
    c3 = _kat_cases()[2]
    ctr = [int(x, 16) for x in c3["ctr"]]
    key = [int(x, 16) for x in c3["key"]]
    seed = key[0] | (key[1] << 32)
    w = O.philox_words_at([ctr[0]], [ctr[1]], seed, ctr[2], ctr[3])
    assert [int(v) for v in w[0, 0]] == [int(x, 16) for x in c3["out"]]
    # the row/group form agrees with the full-matrix form on a block of rows and groups
    np.testing.assert_array_equal(O.philox_words_at(np.arange(5, 9), np.arange(2, 4), 77, 3, 1),
                                  O.philox_words_for(9, 16, 77, 3, 1)[5:9, 2:4])


def test_uniform_grid_and_range():
    w = np.array([0, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = O.uniforms_from_words(w)
    np.testing.assert_array_equal(u, [0.5 * 2 ** -23, 0.5 * 2 ** -23, 1.5 * 2 ** -23,
                                      1 - 0.5 * 2 ** -23, 0.5 + 0.5 * 2 ** -23])
    assert np.all(u > 0) and np.all(u < 1)
    # every value is exactly representable in fp32
    np.testing.assert_array_equal(u.astype(np.float32).astype(np.float64), u)


def test_reproducible_and_counter_separation():
    a = O.gaussian_test_matrix(64, 10, seed=7, stream_id=3, inversion_index=2)
    b = O.gaussian_test_matrix(64, 10, seed=7, stream_id=3, inversion_index=2)
    np.testing.assert_array_equal(a, b)
    # A prefix of rows/cols does not depend on the matrix size (padding invariance).
    c = O.gaussian_test_matrix(100, 13, seed=7, stream_id=3, inversion_index=2)
    np.testing.assert_array_equal(a, c[:64, :10])
    big = O.gaussian_test_matrix(512, 16, seed=7, stream_id=3, inversion_index=2)
    for other in [dict(seed=8, stream_id=3, inversion_index=2),
                  dict(seed=7, stream_id=4, inversion_index=2),
                  dict(seed=7, stream_id=3, inversion_index=3),
                  dict(seed=7 + (1 << 32), stream_id=3, inversion_index=2)]:
        o = O.gaussian_test_matrix(512, 16, **other)
        # 8192 pairs: sample correlation std ~ 0.011
        assert np.abs(np.corrcoef(big.ravel(), o.ravel())[0, 1]) < 0.06


def test_word_uniformity_and_avalanche():
    w = O.philox_words_for(4096, 64, 1234, 0, 0).ravel()
    # top byte chi-square over 256 bins
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    # low byte as well
    counts = np.bincount((w & 0xFF).astype(np.int64), minlength=256)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4
    # flipping one counter bit flips about half of the 128 output bits
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(2000, 4), dtype=np.uint64).astype(np.uint32)
    base = O.philox4x32_10(ctr, (0x1234, 0x5678))
    flips = []
    for word in range(4):
        for bit in [0, 13, 31]:
            c2 = ctr.copy(); c2[:, word] ^= np.uint32(1 << bit)
            out = O.philox4x32_10(c2, (0x1234, 0x5678))
            x = (base ^ out).view(np.uint8)
            flips.append(np.unpackbits(x).reshape(len(ctr), -1).sum(axis=1).mean())
    assert all(abs(f - 64) < 1.5 for f in flips), flips


def test_gaussian_moments_ks_and_independence():
    z = O.gaussian_test_matrix(250000, 4, seed=42, stream_id=1, inversion_index=0)
    x = z.ravel()
    assert abs(x.mean()) < 5e-3
    assert abs(x.var() - 1) < 5e-3
    assert abs(np.mean(x ** 4) - 3) < 3e-2
    assert stats.kstest(x, "norm").pvalue > 1e-3
    # the 4 columns of one Philox call (two Box-Muller pairs) are uncorrelated
    cc = np.corrcoef(z.T)
    assert np.abs(cc - np.eye(4)).max() < 1e-2
    # cos/sin partners are uncorrelated in squares too (Box-Muller independence)
    assert abs(np.corrcoef(z[:, 0] ** 2, z[:, 1] ** 2)[0, 1]) < 1e-2
