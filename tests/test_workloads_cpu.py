"""CPU checks of the seeded input recipes that are not pinned elsewhere: the
Bernoulli index rows behind the paper's benchmark shapes (Sec. 4.1)."""
import numpy as np

import workloads as W


def test_bernoulli_index_rows_are_valid_and_have_the_stated_density():
    rng = np.random.default_rng(7)
    n, count, p = 300, 3000, 0.05
    rows = W.bernoulli_index_rows(rng, count, n, p, chunk=700)  # several ragged chunks
    assert rows.count == count and rows.ptr[0] == 0 and np.all(np.diff(rows.ptr) >= 0)
    for r in range(count):
        q = rows.row(r)
        assert np.all((q >= 0) & (q < n)) and np.all(np.diff(q) > 0)  # distinct, ascending
    dense = W.rows_to_dense(rows, n)
    assert dense.sum() == rows.idx.size
    # mean weight n p = 15 with standard error sqrt(n p (1 - p) / count) ~ 0.07
    assert abs(np.diff(rows.ptr).mean() - n * p) < 0.5
    # every qubit is equally likely: column frequencies near p
    assert np.abs(dense.mean(axis=0) - p).max() < 0.03


def test_paper_shape_recipe():
    w = W.paper_shape(100, 500, l=200, s=50)
    assert (w.n, w.m, w.l, w.s) == (100, 500, 200, 50)
    assert abs(np.diff(w.gates.ptr).mean() - 3.0) < 0.4  # Bernoulli(3/n) bits: weight 3
    assert abs(np.diff(w.ops.ptr).mean() - 3.0) < 0.5
    assert np.all(np.abs(w.theta) <= np.pi)
    assert w.samples.shape == (50, 100)
    # seeded: the same call gives the same rows
    w2 = W.paper_shape(100, 500, l=200, s=50)
    assert np.array_equal(w.gates.idx, w2.gates.idx) and np.array_equal(w.theta, w2.theta)
