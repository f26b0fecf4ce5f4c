"""Pins of the oracle's independent estimates (a separate sample set per
observable, the l x s x n option of Sec. 2.3): reduction to the shared-sample
estimator, exactness under full enumeration, the gradient by central
differences, and the property the option exists for, uncorrelated estimates."""
import numpy as np

import oracle
import workloads as W


def _problem(seed, n=7, m=25, l=6, s=40):
    w = W.small_random(seed, n, m, l, s)
    ops01 = W.rows_to_dense(w.ops, n)
    z = W.uniform_bits(np.random.default_rng(seed + 1), l * s, n).reshape(l, s, n)
    return w, ops01, z


def test_one_shared_set_reduces_to_the_batched_estimator():
    w, ops01, _ = _problem(1)
    z = np.broadcast_to(w.samples, (w.l,) + w.samples.shape).copy()
    m1, s1, p1 = oracle.expval_indep(w.n, w.gates, w.theta, ops01, z, phases=True)
    m0, s0, p0 = oracle.expval(w.n, w.gates, w.theta, ops01, w.samples, phases=True)
    assert np.array_equal(m1, m0) and np.array_equal(s1, s0) and np.array_equal(p1, p0)
    u = np.random.default_rng(2).normal(size=w.l)
    assert np.array_equal(oracle.expval_indep_grad(w.n, w.gates, w.theta, ops01, z, u),
                          oracle.expval_grad(w.n, w.gates, w.theta, ops01, w.samples, u))


def test_each_observable_uses_its_own_set():
    w, ops01, z = _problem(3)
    mean, se = oracle.expval_indep(w.n, w.gates, w.theta, ops01, z)
    for k in range(w.l):
        mk, sk = oracle.expval(w.n, w.gates, w.theta, ops01[k:k + 1], z[k])
        assert mean[k] == mk[0] and se[k] == sk[0]


def test_full_enumeration_per_observable_equals_state_vector():
    # every observable gets all 2^n bit strings, each in its own order
    n = 6
    w = W.small_random(5, n, 15, 8, 1)
    ops01 = W.rows_to_dense(w.ops, n)
    allz = W.all_bitstrings(n)
    rng = np.random.default_rng(6)
    z = np.stack([allz[rng.permutation(allz.shape[0])] for _ in range(w.l)])
    mean, _ = oracle.expval_indep(n, w.gates, w.theta, ops01, z)
    exact = oracle.statevector_expval(n, w.gates, w.theta, ops01)
    assert np.abs(mean - exact).max() < 1e-12


def test_indep_gradient_equals_central_differences():
    w, ops01, z = _problem(7)
    u = np.random.default_rng(8).normal(size=w.l)
    g = oracle.expval_indep_grad(w.n, w.gates, w.theta, ops01, z, u)
    eps = 1e-6
    for j in range(w.m):
        e = np.zeros(w.m)
        e[j] = eps
        fp = u @ oracle.expval_indep(w.n, w.gates, w.theta + e, ops01, z)[0]
        fm = u @ oracle.expval_indep(w.n, w.gates, w.theta - e, ops01, z)[0]
        assert abs((fp - fm) / (2 * eps) - g[j]) < 1e-8


def test_estimates_of_one_observable_twice_are_uncorrelated():
    # two copies of one observable: with shared samples the two estimates are
    # identical (correlation 1); with independent sets their correlation over
    # many draws is near 0
    n = 8
    w = W.small_random(9, n, 30, 1, 1, theta_scale=1.0)
    ops01 = np.repeat(W.rows_to_dense(w.ops, n), 2, axis=0)
    rng = np.random.default_rng(10)
    pairs = []
    for _ in range(300):
        z = W.uniform_bits(rng, 2 * 16, n).reshape(2, 16, n)
        mean, _ = oracle.expval_indep(n, w.gates, w.theta, ops01, z)
        shared, _ = oracle.expval(n, w.gates, w.theta, ops01, z[0])
        assert shared[0] == shared[1]
        pairs.append(mean)
    r = np.corrcoef(np.array(pairs).T)[0, 1]
    assert abs(r) < 0.2  # 300 draws: the standard error of r is about 0.06
