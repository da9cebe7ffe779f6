"""The host rendering of the RSVD test-matrix generator (Philox4x32-10 + Box-Muller), pinned by
the generator's published known-answer vectors and by properties of its definition: the
vectorized rounds equal a plain integer rendering, the map
is a permutation of counters, one flipped counter bit changes about half of the output bits,
streams and seeds give unrelated sequences, and the normals have the moments of N(0, 1)."""
import numpy as np

from conftest import read_golden
from oracle import philox


def test_vectorized_rounds_equal_the_plain_rendering():
    rng = np.random.default_rng(0)
    ctrs = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64)
    keys = rng.integers(0, 2**32, size=(64, 2), dtype=np.uint64)
    for c, k in zip(ctrs, keys):
        v = philox.philox4x32_10(*(np.array([x]) for x in c), int(k[0]), int(k[1]))
        assert tuple(int(w[0]) for w in v) == philox.philox_scalar([int(x) for x in c], [int(x) for x in k])


def test_distinct_counters_give_distinct_outputs_and_avalanche():
    n = 1 << 14
    p = np.arange(n, dtype=np.uint64)
    z = np.zeros(n, dtype=np.uint64)
    out = np.stack(philox.philox4x32_10(p, z, z, z, 7, 9), axis=1)
    assert len({tuple(r) for r in out.tolist()}) == n            # a permutation of counters
    # flipping one bit of the counter flips about half of the 128 output bits
    rng = np.random.default_rng(1)
    flips = []
    for _ in range(400):
        c = [int(x) for x in rng.integers(0, 2**32, size=4)]
        a = philox.philox_scalar(c, [3, 5])
        c[rng.integers(0, 4)] ^= 1 << int(rng.integers(0, 32))
        b = philox.philox_scalar(c, [3, 5])
        flips.append(sum(bin(x ^ y).count("1") for x, y in zip(a, b)))
    assert abs(np.mean(flips) - 64) < 2.0


def test_gaussian_moments_streams_and_prefixes():
    x = philox.gaussian(400001, seed=12345)
    n = x.size
    assert abs(x.mean()) < 5 / np.sqrt(n)
    assert abs(x.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(np.mean(x ** 4) - 3) < 0.05                        # kurtosis of a normal
    assert np.isfinite(x).all()
    # a prefix of a longer draw is the shorter draw (values depend on the index only)
    assert np.array_equal(philox.gaussian(1001, seed=12345), x[:1001])
    # other streams and seeds are unrelated
    for y in (philox.gaussian(20000, seed=12345, stream=1), philox.gaussian(20000, seed=12346)):
        assert abs(np.corrcoef(x[:20000], y)[0, 1]) < 0.05


def test_published_known_answers():
    # the generator's published known-answer vectors (tests/golden/philox4x32_10_kat.txt), for
    # the plain and the vectorized rendering
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for row in rows:
        w = [int(x, 16) for x in row]
        ctr, key, want = w[0:4], w[4:6], w[6:10]
        assert list(philox.philox_scalar(ctr, key)) == want
        v = philox.philox4x32_10(*(np.array([x], dtype=np.uint64) for x in ctr), key[0], key[1])
        assert [int(x[0]) for x in v] == want
