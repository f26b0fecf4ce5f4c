"""Pins of the oracle's training-loop pieces: the Philox4x64-10 streams
against numpy's own Philox bit generator, the bit samplers built on them,
parameter sharing (gates as tuples of generators, Sec. 3.1.1) against central
differences of the loss, and the optimizer update against closed forms and
torch.optim."""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads as W


def numpy_stream(seed, step, tag, count):
    # numpy's Philox increments its 256-bit counter before each block, so a
    # start one below (0, step, tag, 0) yields blocks 0, 1, 2, ... of it
    start = ((int(tag) << 128) | (int(step) << 64)) - 1
    bg = np.random.Philox(counter=start % (1 << 256),
                          key=np.array([seed[0], seed[1]], dtype=np.uint64))
    return bg.random_raw(4 * ((count + 3) // 4))[:count]


@pytest.mark.parametrize("ctr,key", [([0, 0, 0, 0], [0, 0]),
                                     ([5, 7, 3, 0], [123456789, 987654321]),
                                     ([2**64 - 1, 2**63, 17, 2**40], [2**64 - 1, 1])])
def test_philox_block_equals_numpy(ctr, key):
    # numpy steps its 256-bit counter before each block: start one below
    start = (sum(int(x) << (64 * i) for i, x in enumerate(ctr)) - 1) % (1 << 256)
    bg = np.random.Philox(counter=start, key=np.array(key, dtype=np.uint64))
    assert np.array_equal(oracle.philox4x64(ctr, key), bg.random_raw(4))


@pytest.mark.parametrize("rows,n", [(1, 1), (3, 63), (5, 64), (7, 65), (11, 300)])
@pytest.mark.parametrize("step,tag", [(0, 0), (3, 0), (2, 1)])
def test_uniform_bits_are_the_stream_words(rows, n, step, tag):
    seed = (0xDEADBEEF, 42)
    Wd = (n + 63) // 64
    raw = numpy_stream(seed, step, tag, rows * Wd).reshape(rows, Wd)
    want = np.zeros((rows, n), dtype=np.uint8)
    for q in range(n):
        want[:, q] = (raw[:, q // 64] >> np.uint64(q % 64)) & np.uint64(1)
    assert np.array_equal(oracle.sample_uniform(rows, n, seed, step, tag), want)


def test_bernoulli_bits_compare_stream_words_with_threshold():
    seed, step, tag, n = (9, 10), 4, 1, 37
    rows, probs = [5, 3, 4], [0.3, 0.0, 0.49]
    raw = numpy_stream(seed, step, tag, sum(rows) * n).reshape(sum(rows), n)
    thr = np.concatenate([[oracle.bit_threshold(p)] * r for r, p in zip(rows, probs)])
    want = (raw < thr[:, None].astype(np.uint64)).astype(np.uint8)
    got = oracle.sample_bernoulli(n, rows, probs, seed, step, tag)
    assert np.array_equal(got, want)
    assert got[5:8].sum() == 0  # p = 0 never sets a bit


def test_bit_threshold_exact_and_range():
    assert oracle.bit_threshold(0.5) == 2**63
    assert oracle.bit_threshold(0.25) == 2**62
    assert oracle.bit_threshold(0.0) == 0
    assert oracle.bit_threshold(math.ldexp(1.0, -64)) == 1
    for bad in (1.0, -0.1, float("nan")):
        with pytest.raises(ValueError):
            oracle.bit_threshold(bad)


def test_sampler_statistics():
    # uniform bits have mean 1/2 and consecutive steps / tags are different
    # streams; Bernoulli frequencies match P_sigma's bit probability
    z0 = oracle.sample_uniform(400, 300, (1, 2), 0, 0).astype(float)
    z1 = oracle.sample_uniform(400, 300, (1, 2), 1, 0).astype(float)
    zt = oracle.sample_uniform(400, 300, (1, 2), 0, 1).astype(float)
    for z in (z0, z1, zt):
        assert abs(z.mean() - 0.5) < 5 * 0.5 / math.sqrt(z.size)
    assert 0.45 < (z0 != z1).mean() < 0.55 and 0.45 < (z0 != zt).mean() < 0.55
    for sg in (1.0, 5.0):
        p = W.sigma_bit_probability(sg)
        o = oracle.sample_bernoulli(300, [2000], [p], (3, 4), 0, 1).astype(float)
        assert abs(o.mean() - p) < 5 * math.sqrt(p * (1 - p) / o.size)


def shared_problem(seed=7):
    # the paper's 3-qubit example of shared parameters, gates
    # ([0, 2], [0, 1, 2]) and ([0],), extended by a fixed gate and a few more
    n = 5
    gates = W.rows_from_lists([[0, 2], [0, 1, 2], [0], [1, 3], [2, 4], [3], [0, 4]])
    param_index = np.array([0, 0, 1, -1, 2, 2, 2], dtype=np.int32)
    fixed = np.array([0, 0, 0, 0.31, 0, 0, 0], dtype=np.float64)
    rng = np.random.default_rng(seed)
    ops = oracle.sample_bernoulli(n, [6, 6], [0.3, 0.1], (5, 6), 0, 1)
    z = W.all_bitstrings(n)
    data = (rng.random((40, n)) < 0.3).astype(np.uint8)
    return n, gates, param_index, fixed, ops, z, data


def test_shared_parameter_gradient_equals_central_differences():
    n, gates, idx, fixed, ops, z, data = shared_problem()
    w = oracle.op_weights([6, 6])
    params = np.array([0.4, -1.1, 0.7])

    def loss(p):
        th = oracle.gate_theta(idx, p, fixed)
        return oracle.mmd_loss_grad(n, gates, th, ops, w, z, data, grad=False)[0]

    th = oracle.gate_theta(idx, params, fixed)
    assert th[3] == 0.31 and th[0] == th[1] == 0.4 and th[4] == th[5] == th[6] == 0.7
    _, gt = oracle.mmd_loss_grad(n, gates, th, ops, w, z, data)
    g = oracle.param_grad(idx, 3, gt)
    eps = 1e-6
    for p in range(3):
        e = np.zeros(3)
        e[p] = eps
        fd = (loss(params + e) - loss(params - e)) / (2 * eps)
        assert abs(fd - g[p]) < 1e-8 * max(1.0, abs(fd))


def test_shared_parameter_statevector():
    # exp(i t (X_a + X_b)) = exp(i t X_a) exp(i t X_b) for commuting X-type
    # generators: full enumeration of z with a shared angle equals the state
    # vector of the circuit whose two generators carry that same angle
    n, gates, idx, fixed, ops, z, _ = shared_problem()
    th = oracle.gate_theta(idx, np.array([0.4, -1.1, 0.7]), fixed)
    mean, _ = oracle.expval(n, gates, th, ops, z)
    assert np.abs(mean - oracle.statevector_expval(n, gates, th, ops)).max() < 1e-13


def test_op_weights_sum_per_group():
    w = oracle.op_weights([3, 5, 2])
    assert abs(w[:3].sum() - 1 / 3) < 1e-16 and abs(w[3:8].sum() - 1 / 3) < 1e-16
    assert abs(w.sum() - 1.0) < 1e-15


def test_gradient_descent_update_closed_form():
    p0 = np.array([1.0, -2.0, 0.5])
    g = np.array([0.1, 0.2, -0.3])
    p1, m1, m2 = oracle.optimizer_update(oracle.OPT_GD, p0, g, np.zeros(3), np.zeros(3), 0, 0.5)
    assert np.array_equal(p1, p0 - 0.5 * g) and not m1.any() and not m2.any()


def test_adam_first_step_closed_form():
    # t = 1: mhat = g and vhat = g^2, so the step is lr g / (|g| + eps)
    g = np.array([1e-3, -2.0, 0.0, 5e-9])
    p1, _, _ = oracle.optimizer_update(oracle.OPT_ADAM, np.zeros(4), g, np.zeros(4),
                                       np.zeros(4), 0, 0.01)
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)


@pytest.mark.parametrize("opt", [oracle.OPT_GD, oracle.OPT_ADAM])
def test_optimizer_trajectory_equals_torch(opt):
    rng = np.random.default_rng(0)
    P, lr, b1, b2, eps = 17, 0.03, 0.85, 0.99, 1e-7
    p = rng.normal(size=P)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    topt = (torch.optim.SGD([tp], lr=lr) if opt == oracle.OPT_GD else
            torch.optim.Adam([tp], lr=lr, betas=(b1, b2), eps=eps))
    m1, m2 = np.zeros(P), np.zeros(P)
    for t in range(6):
        g = rng.normal(size=P) * 10.0 ** rng.integers(-4, 2, size=P)
        p, m1, m2 = oracle.optimizer_update(opt, p, g, m1, m2, t, lr, b1, b2, eps)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        topt.step()
        assert np.allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15), t


def test_train_step_uses_fresh_streams_per_step():
    n, gates, idx, fixed, _, _, data = shared_problem()
    args = dict(group_rows=[4, 4], group_prob=[0.3, 0.1], s=64, data01=data, seed=(1, 2),
                opt=oracle.OPT_GD, m1=np.zeros(3), m2=np.zeros(3), lr=0.1)
    r0 = oracle.train_step(n, gates, idx, fixed, np.array([0.1, 0.2, 0.3]), step=0, **args)
    r1 = oracle.train_step(n, gates, idx, fixed, r0["params"], step=1, **args)
    assert not np.array_equal(r0["samples"], r1["samples"])
    assert np.array_equal(r0["params"], np.array([0.1, 0.2, 0.3]) - 0.1 * r0["grad"])
    assert r1["loss"] >= -1.0  # the unbiased estimator may dip below 0, never far
