"""GPU vs oracle on the edge cases of the method: the smallest sizes (one
qubit, gate, observable or sample), generators of weight 0 and heavier than
the 8-entry support lists, and the 1000-qubit workload at full size on
sampled observables (means and gradient), in every precision."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2501_04776_amd import api
from tests.gpu_util import TOL, DevWorkload, check_grad

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "split_bf16", "split3_bf16", "split_bf16_fp8", "sparse_fp32"]


def _fwd_grad(w, prec, u):
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    mean, se, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)
    g = api.iqp_expval_grad(circ, dw.ops, dw.samples, torch.from_numpy(u).cuda(), ph, prec)
    g2 = api.iqp_expval_grad(circ, dw.ops, dw.samples, torch.from_numpy(u).cuda(), None, prec)
    torch.cuda.synchronize()
    return dw, mean.cpu().numpy(), se.cpu().numpy(), g.cpu().numpy(), g2.cpu().numpy()


def _check(w, prec, u):
    dw, mean, se, g, g2 = _fwd_grad(w, prec, u)
    om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01, w.samples)
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01, w.samples, u)
    assert np.abs(mean - om).max() < TOL[prec], np.abs(mean - om).max()
    assert np.abs(se - ose).max() < TOL[prec]
    check_grad(prec, g, w, dw.ops01, u, og, "saved phases")
    check_grad(prec, g2, w, dw.ops01, u, og, "recomputed phases")
    return mean, se


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (1, 3, 2, 5), (7, 1, 4, 9), (9, 12, 1, 64),
                                   (9, 12, 5, 1), (64, 1, 1, 1025), (65, 129, 1, 2)])
def test_smallest_sizes(prec, shape):
    n, m, l, s = shape
    w = W.small_random(700 + sum(shape), n, m, l, s, theta_scale=np.pi)
    u = np.random.default_rng(7).normal(size=l)
    mean, se = _check(w, prec, u)
    if s == 1:
        assert np.all(se == 0.0)  # one sample: the population deviation is 0


@pytest.mark.parametrize("prec", PRECS)
def test_zero_weight_and_heavy_generators(prec):
    # generators of weight 0 (no effect), weight 9..20 (past the support
    # lists: the parity step walks their bit rows), mixed with light ones;
    # observables of weight 0 and of full weight
    n = 130
    rng = np.random.default_rng(11)
    lists = [[]] * 3 + [sorted(rng.choice(n, size=int(k), replace=False).tolist())
                        for k in rng.integers(9, 21, size=40)]
    lists += [sorted(rng.choice(n, size=int(k), replace=False).tolist())
              for k in rng.integers(1, 4, size=300)]
    order = rng.permutation(len(lists))
    gates = W.rows_from_lists([lists[i] for i in order])
    theta = rng.uniform(-np.pi, np.pi, size=gates.count)
    ops = W.rows_from_lists([[], list(range(n))] +
                            [sorted(rng.choice(n, size=int(k), replace=False).tolist())
                             for k in rng.integers(1, 6, size=60)])
    z = W.uniform_bits(rng, 700, n)
    w = W.Workload("heavy", n, gates, theta, ops, z)
    u = rng.normal(size=ops.count)
    mean, se = _check(w, prec, u)
    assert mean[0] == 1.0 and se[0] == 0.0


@pytest.mark.parametrize("prec", PRECS)
def test_n300_full_size_sampled(prec):
    # the 300-qubit workload (all 45150 one- and two-qubit generators,
    # theta ~ N(0, 0.1^2), 1000 weight-2 observables, 10^4 samples) at full
    # size in the launch configuration the benchmark times; the oracle
    # recomputes 12 sampled observables and the gradient of a loss on those
    w = W.local_n300()
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    pick = np.random.default_rng(2).choice(w.l, size=12, replace=False)
    u = np.zeros(w.l)
    u[pick] = np.random.default_rng(3).normal(size=pick.size)
    mean, se, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)
    g = api.iqp_expval_grad(circ, dw.ops, dw.samples, torch.from_numpy(u).cuda(), ph, prec)
    torch.cuda.synchronize()
    om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01[pick], w.samples)
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01[pick], w.samples, u[pick])
    d = np.abs(mean.cpu().numpy()[pick] - om)
    assert d.max() < TOL[prec]
    assert np.abs(se.cpu().numpy()[pick] - ose).max() < TOL[prec]
    err, rep = check_grad(prec, g.cpu().numpy(), w, dw.ops01[pick], u[pick], og)
    print("n=300 %s: max|d mean| %.3g, max|d grad| %.3g (representation %.3g)" %
          (prec, d.max(), err, rep))


@pytest.mark.parametrize("prec", PRECS)
def test_n1000_full_size_sampled(prec):
    # the 1000-qubit workload (10^5 generators of weight 1..3, theta in
    # (-pi, pi), 10^4 observables of weight 1..10, 10^4 samples) at full
    # size; the oracle recomputes 12 sampled observables and the gradient of
    # a loss on those
    w = W.random_n1000()
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    pick = np.random.default_rng(0).choice(w.l, size=12, replace=False)
    u = np.zeros(w.l)
    u[pick] = np.random.default_rng(1).normal(size=pick.size)
    mean, se, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)
    g = api.iqp_expval_grad(circ, dw.ops, dw.samples, torch.from_numpy(u).cuda(), ph, prec)
    torch.cuda.synchronize()
    om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01[pick], w.samples)
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01[pick], w.samples, u[pick])
    d = np.abs(mean.cpu().numpy()[pick] - om)
    print("n=1000 %s: max|d mean| %.3g" % (prec, d.max()))
    assert d.max() < TOL[prec]
    assert np.abs(se.cpu().numpy()[pick] - ose).max() < TOL[prec]
    err, rep = check_grad(prec, g.cpu().numpy(), w, dw.ops01[pick], u[pick], og)
    print("n=1000 %s: max|d grad| %.3g (representation %.3g)" % (prec, err, rep))


def test_calls_on_two_streams_do_not_share_scratch():
    # two different problems queued alternately on two streams: each stream
    # has its own cached workspace, so both results equal their single-stream
    # values
    ws = [W.small_random(900 + i, 80, 2000, 300, 2000) for i in range(2)]
    dws = [DevWorkload(w) for w in ws]
    circs = [api.Circuit(w.n, d.gens, d.theta) for w, d in zip(ws, dws)]
    want = []
    for c, d in zip(circs, dws):
        want.append(api.iqp_expval(c, d.ops, d.samples, "split_bf16")[0].clone())
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = [[], []]
    for rep in range(4):
        for i in range(2):
            with torch.cuda.stream(streams[i]):
                got[i].append(api.iqp_expval(circs[i], dws[i].ops, dws[i].samples,
                                             "split_bf16")[0])
    torch.cuda.synchronize()
    for i in range(2):
        for g in got[i]:
            assert torch.equal(g, want[i])


@pytest.mark.parametrize("prec", PRECS)
def test_pi_shifted_angles_give_the_same_estimates(prec):
    # exp(i(theta + k pi) X) = (-1)^k exp(i theta X) is a global phase, so every
    # mean and every gradient is unchanged; the angles are reduced to
    # [-pi/2, pi/2] in FP64 before anything is rounded to FP32 or BF16, so
    # shifts by up to 10^4 pi (which cost ~1e-12 of FP64 precision in theta
    # itself) leave the results within the estimate tolerance of the oracle
    w = W.small_random(4242, 80, 700, 90, 1500, theta_scale=np.pi)
    u = np.random.default_rng(6).normal(size=w.l)
    k = np.random.default_rng(5).integers(-10 ** 4, 10 ** 4, size=w.m)
    shifted = W.Workload(w.name, w.n, w.gates, w.theta + k * np.pi, w.ops, w.samples, seed=w.seed)
    dw, m0, s0, g0, _ = _fwd_grad(w, prec, u)
    _, m1, s1, g1, _ = _fwd_grad(shifted, prec, u)
    om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01, w.samples)
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01, w.samples, u)
    T = TOL[prec]
    assert np.abs(m1 - om).max() < T and np.abs(s1 - ose).max() < T
    assert np.abs(m1 - m0).max() < T
    check_grad(prec, g1, w, dw.ops01, u, og, "shifted")
    check_grad(prec, g0, w, dw.ops01, u, og, "unshifted")

def long_rows_workload(seed, s):
    """Rows of C longer than one list fill of the table-lookup sparse
    kernels (1024 generators): 1024 generators hold qubit 0, 1025 qubit 1
    (and not 0), 2000 neither, so Z_0 anticommutes with exactly 1024, Z_1
    with 1025, Z_0 Z_1 with 2049; a weight-30 string with about half of
    them; the empty string with none."""
    n = 64
    rng = np.random.default_rng(seed)

    def extra(lo):
        return sorted(rng.choice(np.arange(lo, n), size=int(rng.integers(0, 3)),
                                 replace=False).tolist())
    lists = [[0] + extra(2) for _ in range(1024)] + [[1] + extra(2) for _ in range(1025)]
    lists += [extra(2) or [2 + int(rng.integers(0, n - 2))] for _ in range(2000)]
    order = rng.permutation(len(lists))
    gates = W.rows_from_lists([lists[i] for i in order])
    theta = rng.uniform(-np.pi, np.pi, size=gates.count)
    ops = W.rows_from_lists([[0], [1], [0, 1], [],
                             sorted(rng.choice(n, size=30, replace=False).tolist()),
                             [5], [0, 7, 9]])
    z = W.uniform_bits(rng, s, n)
    return W.Workload("long_rows", n, gates, theta, ops, z)


@pytest.mark.parametrize("s", [1500, 64])
def test_sparse_rows_longer_than_one_list(s):
    # several list fills per block, a fill of exactly 1024 entries and one of
    # 1025 (a full fill followed by a single entry), and an empty row
    w = long_rows_workload(31 + s, s)
    ops01 = W.rows_to_dense(w.ops, w.n)
    C = oracle.parity(w.n, ops01, w.gates)
    assert list(C.sum(axis=1)[:4]) == [1024, 1025, 2049, 0]
    u = np.random.default_rng(5).normal(size=w.ops.count)
    mean, se = _check(w, "sparse_fp32", u)
    assert mean[3] == 1.0 and se[3] == 0.0

def test_sparse_grid_smaller_than_the_units(monkeypatch):
    # a grid capped below the (observable, chunk) units takes them in strides
    # (the path of launches past the block limit); results equal the one-
    # block-per-unit launch bitwise (the forward per unit, the gradient's
    # fixed-point sums in any order)
    w = W.small_random(4242, 90, 3000, 9, 3000, theta_scale=np.pi)
    u = np.random.default_rng(9).normal(size=9)
    base = _fwd_grad(w, "sparse_fp32", u)
    monkeypatch.setenv("IQP_SPARSE_GRID_CAP", "5")
    capped = _fwd_grad(w, "sparse_fp32", u)
    for x, y in zip(base[1:], capped[1:]):
        assert np.array_equal(x, y)
