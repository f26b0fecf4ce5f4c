"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test compares the oracle's Monte Carlo estimator, gradient or MMD^2 with
a result computed another way: closed forms from the proof of Prop. 3, a
state-vector simulation (Def. 2 and the gate action of Sec. 2.5), brute force
over pairs, library matrix products, or statistics the paper states.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_ops(w):
    return W.rows_to_dense(w.ops, w.n)


def test_single_anticommuting_gate_gives_cos_2theta():
    # One gate X_g and an observable with odd overlap: <Z_a> = cos(2 theta)
    # (eq. expval_bitflip with |J| = 1); every sample gives the same phase up
    # to sign, so the estimator is exact and its standard error is zero.
    for n, gate, op in [(1, [0], [0]), (3, [0, 2], [2]), (5, [1, 2, 4], [0, 1, 3])]:
        th = 0.37 * n
        gates = W.rows_from_lists([gate])
        ops = W.rows_to_dense(W.rows_from_lists([op]), n)
        z = W.uniform_bits(np.random.default_rng(n), 257, n)
        mean, se = oracle.expval(n, gates, np.array([th]), ops, z)
        assert abs(mean[0] - math.cos(2 * th)) < 1e-13
        assert se[0] < 1e-7
        sv = oracle.statevector_expval(n, gates, np.array([th]), ops)
        assert abs(sv[0] - math.cos(2 * th)) < 1e-14


def test_one_qubit_statevector_textbook():
    # exp(i t X)|0> = cos t |0> + i sin t |1>: probabilities cos^2 t, sin^2 t.
    for t in (0.1, -1.3, 2.9):
        p = oracle.statevector_probs(1, W.rows_from_lists([[0]]), np.array([t]))
        assert np.allclose(p, [math.cos(t) ** 2, math.sin(t) ** 2], atol=1e-15)


def test_identity_observable_is_one():
    w = W.small_random(3, 7, 20, 4, 300)
    ops = np.zeros((1, w.n), dtype=np.uint8)
    mean, se = oracle.expval(w.n, w.gates, w.theta, ops, w.samples)
    assert mean[0] == 1.0 and se[0] == 0.0
    assert abs(oracle.statevector_expval(w.n, w.gates, w.theta, ops)[0] - 1.0) < 1e-12


def _golden_theta():
    with open(os.path.join(GOLDEN, "interference_3q.txt")) as f:
        for line in f:
            if line.startswith("theta"):
                return np.array([float(x) for x in line.split()[1:]])
    raise AssertionError("no theta line")


def test_golden_interference_closed_forms():
    th = _golden_theta()
    gates = W.rows_from_lists([[0], [1], [0, 2], [1, 2]])
    obs = [[0, 1], [0], [2], [0, 2], []]
    ops = W.rows_to_dense(W.rows_from_lists(obs), 3)
    c = np.cos(2 * th)
    s = np.sin(2 * th)
    expect = np.array([c.prod() + s.prod(), c[0] * c[2], c[2] * c[3], c[0] * c[3], 1.0])
    z = W.all_bitstrings(3)
    mean, _ = oracle.expval(3, gates, th, ops, z)
    assert np.abs(mean - expect).max() < 1e-14
    assert np.abs(oracle.statevector_expval(3, gates, th, ops) - expect).max() < 1e-14
    assert np.abs(oracle.subset_expval(3, gates, th, ops) - expect).max() < 1e-14
    # the bitflip (decohered) circuit drops the interference term of case A only
    bf = oracle.bitflip_expval(3, gates, th, ops)
    assert abs(bf[0] - c.prod()) < 1e-15
    assert np.abs(bf[1:] - expect[1:]).max() < 1e-15


@pytest.mark.parametrize("seed,n,m,l", [(11, 4, 9, 10), (12, 6, 16, 12), (13, 8, 24, 16),
                                        (14, 10, 40, 20)])
def test_full_enumeration_equals_statevector(seed, n, m, l):
    # With z ranging over all 2^n strings the sample mean is the exact
    # expectation of eq. op_expval, which must equal <0|U^dag Z_a U|0>.
    w = W.small_random(seed, n, m, l, 0, enumerate_samples=True)
    ops = dense_ops(w)
    mean, _ = oracle.expval(n, w.gates, w.theta, ops, w.samples)
    sv = oracle.statevector_expval(n, w.gates, w.theta, ops)
    assert np.abs(mean - sv).max() < 1e-12


@pytest.mark.parametrize("seed,n,m,l", [(21, 5, 10, 12), (22, 7, 14, 12)])
def test_subset_expansion_equals_statevector(seed, n, m, l):
    w = W.small_random(seed, n, m, l, 0)
    ops = dense_ops(w)
    sub = oracle.subset_expval(n, w.gates, w.theta, ops)
    sv = oracle.statevector_expval(n, w.gates, w.theta, ops)
    assert np.abs(sub - sv).max() < 1e-12


def test_product_form_for_weight_one_observables_at_large_n():
    # In an all-one-and-two-qubit circuit the gates anticommuting with Z_q are
    # [q] and [q, r] for r != q; their supports are GF(2)-independent, so
    # Omega is empty and <Z_q> = prod cos(2 theta_j) exactly, at any n. Full
    # enumeration at n = 9 pins the estimator to it.
    n = 9
    gates = W.local_gates(n)
    th = np.random.default_rng(5).normal(0, 0.4, size=gates.count)
    ops = np.eye(n, dtype=np.uint8)
    mean, _ = oracle.expval(n, gates, th, ops, W.all_bitstrings(n))
    bf = oracle.bitflip_expval(n, gates, th, ops)
    assert np.abs(mean - bf).max() < 1e-13


def test_batch_matrix_form_equals_per_term_phases():
    # Prop. 2: E = C Theta B^T with B = (-1)^{Z G^T}, C = 1 - (-1)^{A G^T},
    # here built from dense integer matrix products (numpy) and compared with
    # the oracle's index-list phases.
    w = W.small_random(31, 12, 30, 9, 40)
    ops = dense_ops(w)
    G = W.rows_to_dense(w.gates, w.n).astype(np.int64)
    B = 1 - 2 * ((w.samples.astype(np.int64) @ G.T) % 2)
    C = 1 - (1 - 2 * ((ops.astype(np.int64) @ G.T) % 2))
    E = C @ np.diag(w.theta) @ B.T
    mean, se, ph = oracle.expval(w.n, w.gates, w.theta, ops, w.samples, phases=True)
    assert np.abs(ph - E).max() < 1e-12
    assert np.abs(mean - np.cos(E).mean(axis=1)).max() < 1e-14


def test_parity_brute_force_and_gf2_linearity():
    rng = np.random.default_rng(41)
    n = 70
    rows = W.uniform_bits(rng, 33, n)
    gates = W.random_weight_rows(rng, 50, n, 1, 9)
    P = oracle.parity(n, rows, gates)
    G = W.rows_to_dense(gates, n).astype(np.int64)
    assert np.array_equal(P, ((rows.astype(np.int64) @ G.T) % 2).astype(np.uint8))
    # parity(x, g xor h) = parity(x, g) xor parity(x, h)
    gx = (G[:25] ^ G[25:]).astype(np.uint8)
    P2 = oracle.parity(n, rows, W.dense_to_rows(gx))
    assert np.array_equal(P2, P[:, :25] ^ P[:, 25:])


def test_theta_shift_by_pi_is_invariant():
    # exp(i (theta + pi) X) = -exp(i theta X): a global phase.
    w = W.small_random(51, 9, 30, 12, 200)
    ops = dense_ops(w)
    m0, s0 = oracle.expval(w.n, w.gates, w.theta, ops, w.samples)
    sh = w.theta + np.pi * np.random.default_rng(1).integers(-3, 4, size=w.m)
    m1, s1 = oracle.expval(w.n, w.gates, sh, ops, w.samples)
    assert np.abs(m0 - m1).max() < 1e-12 and np.abs(s0 - s1).max() < 1e-12


def test_grad_matches_central_differences():
    w = W.small_random(61, 8, 18, 7, 150)
    ops = dense_ops(w)
    u = np.random.default_rng(2).normal(size=w.l)
    g = oracle.expval_grad(w.n, w.gates, w.theta, ops, w.samples, u)
    eps = 1e-3
    fd = np.zeros(w.m)
    for j in range(w.m):
        tp = w.theta.copy(); tp[j] += eps
        tm = w.theta.copy(); tm[j] -= eps
        fd[j] = (u @ oracle.expval(w.n, w.gates, tp, ops, w.samples)[0]
                 - u @ oracle.expval(w.n, w.gates, tm, ops, w.samples)[0]) / (2 * eps)
    assert np.abs(g - fd).max() < 1e-5 * max(1.0, np.abs(g).max())


def test_grad_with_enumeration_equals_parameter_shift():
    # With all 2^n samples the estimator is exact; <Z_a> depends on theta_j
    # through cos(2 theta_j) and sin(2 theta_j), so the shift rule
    # d<Z>/dtheta_j = <Z>(theta_j + pi/4) - <Z>(theta_j - pi/4) is exact.
    w = W.small_random(71, 6, 14, 9, 0, enumerate_samples=True)
    ops = dense_ops(w)
    u = np.random.default_rng(3).normal(size=w.l)
    g = oracle.expval_grad(w.n, w.gates, w.theta, ops, w.samples, u)
    ps = np.zeros(w.m)
    for j in range(w.m):
        tp = w.theta.copy(); tp[j] += np.pi / 4
        tm = w.theta.copy(); tm[j] -= np.pi / 4
        ps[j] = u @ (oracle.statevector_expval(w.n, w.gates, tp, ops)
                     - oracle.statevector_expval(w.n, w.gates, tm, ops))
    assert np.abs(g - ps).max() < 1e-12


def _all_ops_weighted(n, sigma):
    a = W.all_bitstrings(n)
    p = W.sigma_bit_probability(sigma)
    wgt = np.prod(np.where(a == 1, p, 1 - p), axis=1)
    return a, wgt


@pytest.mark.parametrize("sigma", [0.7, 1.0, 2.5])
def test_mmd_plugin_equals_gaussian_kernel_form(sigma):
    # Gaussian kernel k(x, y) = exp(-|x - y|^2 / (2 sigma^2)) on bitstrings.
    # MMD^2 = sum_{x,y} d(x) d(y) k(x, y) with d = p - q must equal
    # E_{a ~ P_sigma}[(<Z_a>_p - <Z_a>_q)^2] (eq. mmd_estimate). Here every a
    # is enumerated with weight P_sigma(a) and z runs over all bitstrings, so
    # the plug-in estimator is the exact value.
    n = 5
    w = W.small_random(81, n, 12, 1, 0, enumerate_samples=True, with_data=37)
    ops, wgt = _all_ops_weighted(n, sigma)
    loss, _ = oracle.mmd_loss_grad(n, w.gates, w.theta, ops, wgt, w.samples, w.data,
                                   unbiased=False, grad=False)
    q = oracle.statevector_probs(n, w.gates, w.theta)
    idx = (w.data.astype(np.int64) << np.arange(n)).sum(axis=1)
    p = np.bincount(idx, minlength=1 << n) / w.data.shape[0]
    d = p - q
    X = W.all_bitstrings(n).astype(np.int64)
    ham = np.abs(X[:, None, :] - X[None, :, :]).sum(axis=2)
    K = np.exp(-ham / (2 * sigma ** 2))
    assert abs(loss - d @ K @ d) < 1e-14


def test_mmd_unbiased_terms_equal_pair_sums():
    # U-statistics: P2 = sum_{n != n'} v_n v_n' / (N (N-1)) and
    # Q2 = sum_{i != i'} c_i c_i' / (s (s-1)), here by brute-force double loops.
    n = 6
    w = W.small_random(91, n, 15, 3, 23, with_data=11)
    ops = dense_ops(w)
    wgt = np.array([0.5, 0.3, 0.2])
    loss, _, ph, qh = oracle.mmd_loss_grad(n, w.gates, w.theta, ops, wgt, w.samples, w.data,
                                           unbiased=True, grad=False, diagnostics=True)
    _, _, E = oracle.expval(n, w.gates, w.theta, ops, w.samples, phases=True)
    expect = 0.0
    for k in range(3):
        v = 1 - 2 * ((w.data.astype(np.int64) @ ops[k].astype(np.int64)) % 2)
        c = np.cos(E[k])
        P2 = sum(v[a] * v[b] for a in range(len(v)) for b in range(len(v)) if a != b)
        P2 /= len(v) * (len(v) - 1)
        Q2 = sum(c[a] * c[b] for a in range(len(c)) for b in range(len(c)) if a != b)
        Q2 /= len(c) * (len(c) - 1)
        expect += wgt[k] * (P2 - 2 * v.mean() * c.mean() + Q2)
        assert abs(ph[k] - v.mean()) < 1e-15 and abs(qh[k] - c.mean()) < 1e-15
    assert abs(loss - expect) < 1e-13


@pytest.mark.parametrize("unbiased", [False, True])
def test_mmd_grad_matches_central_differences(unbiased):
    n = 7
    w = W.small_random(101, n, 16, 6, 60, with_data=20)
    ops = dense_ops(w)
    wgt = np.full(w.l, 1.0 / w.l)
    _, g = oracle.mmd_loss_grad(n, w.gates, w.theta, ops, wgt, w.samples, w.data,
                                unbiased=unbiased)
    eps = 1e-3
    fd = np.zeros(w.m)
    for j in range(w.m):
        tp = w.theta.copy(); tp[j] += eps
        tm = w.theta.copy(); tm[j] -= eps
        lp, _ = oracle.mmd_loss_grad(n, w.gates, tp, ops, wgt, w.samples, w.data, unbiased, False)
        lm, _ = oracle.mmd_loss_grad(n, w.gates, tm, ops, wgt, w.samples, w.data, unbiased, False)
        fd[j] = (lp - lm) / (2 * eps)
    assert np.abs(g - fd).max() < 1e-6 * max(1.0, np.abs(g).max())


def test_estimator_is_unbiased_over_seeds():
    # Prop. 1: E_z[mean] = <Z_a>. 40 independent sample sets of s = 64; the
    # average over sets must sit within 5 standard errors of the exact value.
    n = 8
    w = W.small_random(111, n, 20, 10, 0)
    ops = dense_ops(w)
    exact = oracle.statevector_expval(n, w.gates, w.theta, ops)
    rng = np.random.default_rng(7)
    est = np.array([oracle.expval(n, w.gates, w.theta, ops, W.uniform_bits(rng, 64, n))[0]
                    for _ in range(40)])
    se = est.std(axis=0, ddof=1) / math.sqrt(est.shape[0])
    assert np.all(np.abs(est.mean(axis=0) - exact) <= 5 * se + 1e-12)


def test_mmd_unbiased_estimator_over_seeds():
    # The U-statistic form is unbiased for the exact MMD^2 restricted to the
    # drawn operators; the plug-in form is biased upwards by Var terms.
    n = 6
    w = W.small_random(121, n, 12, 4, 0, enumerate_samples=True, with_data=30)
    ops = dense_ops(w)
    wgt = np.full(w.l, 0.25)
    q = oracle.statevector_expval(n, w.gates, w.theta, ops)
    p = 1 - 2 * ((w.data.astype(np.int64) @ ops.T.astype(np.int64)) % 2)
    pbar = p.mean(axis=0)
    rng = np.random.default_rng(9)
    vals = []
    for _ in range(60):
        z = W.uniform_bits(rng, 40, n)
        vals.append(oracle.mmd_loss_grad(n, w.gates, w.theta, ops, wgt, z, w.data, True,
                                         False)[0])
    vals = np.array(vals)
    # target: E over z of the unbiased form = sum_k w_k [P2_k - 2 pbar_k q_k + q_k^2]
    N = w.data.shape[0]
    P2 = ((p.sum(axis=0) ** 2) - N) / (N * (N - 1))
    target = float(np.sum(wgt * (P2 - 2 * pbar * q + q * q)))
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean() - target) <= 5 * se


def test_standard_error_at_ten_thousand_samples_is_0p007():
    # Sec. 4.1: with n_samples = 10000 the additive precision is about 0.007.
    # For large phases cos(E) is close to uniform on the circle, Var = 1/2,
    # so stderr = sqrt(1/2) / 100 = 0.00707.
    n = 40
    w = W.small_random(131, n, 400, 6, 10000, gate_w=(1, 3), op_w=(3, 6))
    ops = dense_ops(w)
    mean, se = oracle.expval(n, w.gates, w.theta, ops, w.samples)
    assert np.all(np.abs(se - 0.00707) < 0.0004), se
    # and it is the population standard deviation of cos(E) over sqrt(s)
    _, _, E = oracle.expval(n, w.gates, w.theta, ops[:2], w.samples[:500], phases=True)
    m2, se2 = oracle.expval(n, w.gates, w.theta, ops[:2], w.samples[:500])
    c = np.cos(E)
    assert np.allclose(se2, np.sqrt(((c - c.mean(axis=1, keepdims=True)) ** 2).mean(axis=1) / 500),
                       atol=1e-15)


def test_bitflip_grad_matches_central_differences():
    w = W.small_random(141, 9, 25, 8, 0)
    ops = dense_ops(w)
    u = np.random.default_rng(4).normal(size=w.l)
    g = oracle.bitflip_grad(w.n, w.gates, w.theta, ops, u)
    eps = 1e-4
    fd = np.zeros(w.m)
    for j in range(w.m):
        tp = w.theta.copy(); tp[j] += eps
        tm = w.theta.copy(); tm[j] -= eps
        fd[j] = u @ (oracle.bitflip_expval(w.n, w.gates, tp, ops)
                     - oracle.bitflip_expval(w.n, w.gates, tm, ops)) / (2 * eps)
    assert np.abs(g - fd).max() < 1e-7


def test_threads_do_not_change_results():
    w = W.small_random(151, 20, 60, 17, 300)
    ops = dense_ops(w)
    a = oracle.expval(w.n, w.gates, w.theta, ops, w.samples, threads=1)
    b = oracle.expval(w.n, w.gates, w.theta, ops, w.samples, threads=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
