"""Generators: reproducible by seed, exact nnz, distinct coordinates, skew."""
import numpy as np

from paper_2510_16930_amd import synth


def test_uniform_reproducible_and_distinct():
    a = synth.coo_uniform((200, 200, 200), 20000, seed=11)
    b = synth.coo_uniform((200, 200, 200), 20000, seed=11)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    key = np.ravel_multi_index(tuple(a[0].astype(np.int64)), (200, 200, 200))
    assert np.unique(key).size == 20000
    assert a[0].dtype == np.int32 and a[0].min() >= 0 and a[0].max() < 200


def test_zipf_exact_nnz_and_skew():
    dims = (20000, 10000, 400)
    idx, vals = synth.coo_zipf(dims, 100000, alpha=1.2, seed=2)
    key = np.ravel_multi_index(tuple(idx.astype(np.int64)), dims)
    assert idx.shape == (3, 100000) and np.unique(key).size == 100000
    for n, d in enumerate(dims):
        assert idx[n].max() < d
        counts = np.bincount(idx[n], minlength=d)
        assert counts.max() > 20 * counts[counts > 0].mean()   # heavy head
    assert np.all(vals > 0)                                   # lognormal


def test_table3_shapes_fixture():
    # the real-data shapes that the Zipf stand-ins copy (Table 3)
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "table3_shapes.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert [r[0] for r in rows] == ["Last", "Delicious", "Facebook", "MovieLens", "10M-MovieLens"]
    for r in rows:
        dims = tuple(int(x) for x in r[1].split(","))
        assert len(dims) == 3 and int(r[2]) < np.prod(dims, dtype=np.float64)
