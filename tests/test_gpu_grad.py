"""GPU vs oracle: the hand-written backward (gradient of a loss of the
estimates), the MMD^2 chain and its gradient, central differences and the
torch.autograd wrappers."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2501_04776_amd import IQPExpval, IQPMMDLoss, api
from tests.gpu_util import TOL, DevWorkload, check_grad

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "split_bf16", "split3_bf16", "split_bf16_fp8", "sparse_fp32"]


def _grad(dw, u, prec, saved):
    circ = api.Circuit(dw.n, dw.gens, dw.theta)
    ph = None
    if saved:
        _, _, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)
    g = api.iqp_expval_grad(circ, dw.ops, dw.samples, torch.from_numpy(u).cuda(), ph, prec)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def _gtol(prec, g):
    return TOL[prec] * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("saved", [True, False])
@pytest.mark.parametrize("shape", [(10, 55, 100, 1000), (70, 1000, 300, 700),
                                   (130, 2100, 129, 1025)])
def test_grad_matches_oracle(prec, saved, shape):
    n, m, l, s = shape
    w = W.small_random(3 * sum(shape), n, m, l, s)
    dw = DevWorkload(w)
    u = np.random.default_rng(1).normal(size=l)
    g = _grad(dw, u, prec, saved)
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01, w.samples, u)
    err, rep = check_grad(prec, g, w, dw.ops01, u, og)
    print("grad %s %s saved=%s: max|d| = %.3g (|g|max %.3g, representation %.3g)" %
          (shape, prec, saved, err, np.abs(og).max(), rep))


@pytest.mark.parametrize("tile", [None, "2x4", "2x2"])
def test_fp16_fp8_weights_match_their_emulation(tile, monkeypatch):
    """split_bf16_fp8 against the host model of its own operands (theta in
    two BF16 limbs, weights as FP16 + FP8 limbs per row, tests/precision_model):
    the gap is the kernels' FP32 phase and accumulation rounding only, a small
    fraction of what the FP8 limb itself contributes (the model without it),
    so a mispaired or dropped FP8 product fails. Every backward wave tile of
    the form; the observable weights span 10 decades, so the row exponents
    differ."""
    from tests import precision_model as PM
    if tile:
        monkeypatch.setenv("IQP_BWD_TILE", tile)
    w = W.small_random(8080, 64, 3000, 300, 513)
    dw = DevWorkload(w)
    rng = np.random.default_rng(4)
    u = rng.normal(size=w.l) * 10.0 ** rng.uniform(-5, 5, w.l)
    g = _grad(dw, u, "split_bf16_fp8", True)
    emu = PM.grad_emulated(w.n, w.gates, w.theta, dw.ops01, w.samples, u, "split_bf16_fp8")
    # the same without the FP8 limb
    th = PM.theta_represented("split_bf16_fp8", w.theta)
    _, _, ph = oracle.expval(w.n, w.gates, th, dw.ops01, w.samples, phases=True)
    S = (u[:, None] / w.s) * np.sin(ph)
    e = PM.fp16_row_exponent(np.abs(u) / w.s)[:, None]
    S16 = np.ldexp(np.ldexp(S.astype(np.float32).astype(np.float64), e).astype(np.float16)
                   .astype(np.float64), -e)
    C = oracle.parity(w.n, dw.ops01, w.gates).astype(np.float64)
    B = 1.0 - 2.0 * oracle.parity(w.n, w.samples, w.gates).astype(np.float64)
    no_lo = -2.0 * (C * (S16 @ B)).sum(axis=0)
    gap, lo = np.abs(g - emu).max(), np.abs(no_lo - emu).max()
    print("fp16+fp8 tile %s: |gpu - model| %.3g, FP8 limb's share %.3g" % (tile, gap, lo))
    assert gap < 0.1 * lo, (gap, lo)


@pytest.mark.parametrize("prec", PRECS)
def test_grad_matches_central_differences_on_gpu(prec):
    # the n = 10 all-local circuit; finite differences of the GPU forward, eps = 1e-3
    w = W.local_n10(enumerate_samples=False)
    dw = DevWorkload(w)
    u = np.random.default_rng(2).normal(size=w.l)
    g = _grad(dw, u, "fp32", True)
    eps = 1e-3
    circ_theta = w.theta.copy()
    fd = np.zeros(w.m)
    for j in range(w.m):
        vals = []
        for sgn in (1, -1):
            t = circ_theta.copy()
            t[j] += sgn * eps
            c = api.Circuit(w.n, dw.gens, torch.from_numpy(t).cuda())
            mean, _, _ = api.iqp_expval(c, dw.ops, dw.samples, "fp32")
            vals.append(float(u @ mean.cpu().numpy()))
        fd[j] = (vals[0] - vals[1]) / (2 * eps)
    gp = _grad(dw, u, prec, True)
    # FP32 phases carry ~1e-7 relative rounding, amplified by 1/(2 eps) in the FD
    assert np.abs(g - fd).max() < 2e-3 * max(1.0, np.abs(g).max())
    assert np.abs(gp - g).max() < _gtol(prec, g)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("unbiased", [True, False])
def test_mmd_loss_and_grad_match_oracle(prec, unbiased):
    n = 60
    w = W.small_random(77, n, 700, 190, 600, with_data=150)
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    loss, g = api.iqp_mmd_loss_grad(circ, dw.ops, dw.op_weight, dw.samples, dw.data, unbiased,
                                    True, prec)
    loss_only, none = api.iqp_mmd_loss_grad(circ, dw.ops, dw.op_weight, dw.samples, dw.data,
                                            unbiased, False, prec)
    torch.cuda.synchronize()
    assert none is None
    ol, og = oracle.mmd_loss_grad(w.n, w.gates, w.theta, dw.ops01, w.op_weight, w.samples, w.data,
                                  unbiased)
    print("mmd %s unbiased=%s: loss %.6g vs %.6g, grad max|d| %.3g" %
          (prec, unbiased, loss.item(), ol, np.abs(g.cpu().numpy() - og).max()))
    assert abs(loss.item() - ol) < TOL[prec]
    assert loss.item() == loss_only.item()
    assert np.abs(g.cpu().numpy() - og).max() < _gtol(prec, og)


def test_mmd_n300_shape_sampled():
    # the differentiation workload's circuit (n = 300, 45150 gates), data
    # (2000 Bernoulli(0.3) strings) and operator distribution (3 bandwidths),
    # with 200 observables per bandwidth and s = 1000 so that the oracle's
    # full loss and gradient stay within seconds
    w = W.mmd_n300(ops_per_sigma=200, s=1000)
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    for prec in PRECS:
        loss, g = api.iqp_mmd_loss_grad(circ, dw.ops, dw.op_weight, dw.samples, dw.data, True,
                                        True, prec)
        torch.cuda.synchronize()
        if prec == "fp32":
            ol, og = oracle.mmd_loss_grad(w.n, w.gates, w.theta, dw.ops01, w.op_weight,
                                          w.samples, w.data, True)
        print("mmd n=300 (200/sigma, s=1000) %s: loss %.8g vs %.8g, grad max|d| %.3g of %.3g" %
              (prec, loss.item(), ol, np.abs(g.cpu().numpy() - og).max(), np.abs(og).max()))
        assert abs(loss.item() - ol) < TOL[prec]
        assert np.abs(g.cpu().numpy() - og).max() < _gtol(prec, og)


_MMD_FULL = {}


def _mmd_full_size_case(unbiased):
    """The differentiation workload at full size in all but the number of
    operators: its circuit (n = 300, 45150 gates), all 10^4 samples and all
    2000 training strings, with 24 operators sampled from each bandwidth's
    2000 (weights 1/72 each). The oracle's loss and gradient over them are
    computed once per estimator form."""
    if unbiased not in _MMD_FULL:
        w = W.mmd_n300()
        per = w.l // 3
        rng = np.random.default_rng(12)
        pick = np.concatenate([g * per + rng.choice(per, size=24, replace=False)
                               for g in range(3)])
        ops01 = W.rows_to_dense(w.ops, w.n)[pick]
        wts = np.full(pick.size, 1.0 / pick.size)
        ol, og = oracle.mmd_loss_grad(w.n, w.gates, w.theta, ops01, wts, w.samples, w.data,
                                      unbiased)
        _MMD_FULL[unbiased] = (w, pick, wts, ol, og)
    return _MMD_FULL[unbiased]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("unbiased", [True, False])
def test_mmd_full_size_sampled_operators(prec, unbiased):
    w, pick, wts, ol, og = _mmd_full_size_case(unbiased)
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    ops = dw.ops[torch.from_numpy(pick).cuda()].contiguous()
    loss, g = api.iqp_mmd_loss_grad(circ, ops, torch.from_numpy(wts).cuda(), dw.samples,
                                    dw.data, unbiased, True, prec)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    print("mmd full size, 3 x 24 operators, %s unbiased=%s: loss %.10g vs %.10g, "
          "grad max|d| %.3g of %.3g" % (prec, unbiased, loss.item(), ol, np.abs(g - og).max(),
                                        np.abs(og).max()))
    assert abs(loss.item() - ol) < TOL[prec] * max(abs(ol), 1e-2)
    # the gradient is far below 1 here (weights 1/72), so its bar is relative
    assert np.abs(g - og).max() < TOL[prec] * np.abs(og).max()


def test_mmd_full_size_central_differences():
    """The differentiation workload at full size (n = 300, 45150 gates, 3 x
    2000 operators, s = 10^4, N = 2000, U-statistic): the analytic gradient
    of every form against central differences of the FP32 loss at the 16
    gates with the largest gradient. The differences' own error, per gate:
    their truncation, estimated from the differences at eps and 2 eps (its
    leading term, eps^2 / 6 times the third derivative, grows 4x, so
    D(2 eps) - D(eps) is about 3x it), plus the loss's rounding over eps
    (its scale taken as the distance between the FP32 loss and the one with
    theta in three limbs); twice that, plus 1e-3 of the largest gradient
    for the forms' own rounding, is the bar. The gradients here are ~1e-5
    (operator weights 1/6000), so the bar is relative to them, and it stays
    a small fraction of them."""
    w = W.mmd_n300()
    dw = DevWorkload(w)
    theta = dw.theta.clone()

    def loss_at(th, prec):
        c = api.Circuit(w.n, dw.gens, th)
        lv, _ = api.iqp_mmd_loss_grad(c, dw.ops, dw.op_weight, dw.samples, dw.data, True, False,
                                      prec)
        torch.cuda.synchronize()
        return lv.item()

    circ = api.Circuit(w.n, dw.gens, theta)
    grads = {}
    for prec in PRECS:
        _, g = api.iqp_mmd_loss_grad(circ, dw.ops, dw.op_weight, dw.samples, dw.data, True, True,
                                     prec)
        torch.cuda.synchronize()
        grads[prec] = g.cpu().numpy()
    noise = abs(loss_at(theta, "fp32") - loss_at(theta, "split3_bf16"))
    eps = 1e-3
    pick = np.argsort(-np.abs(grads["fp32"]))[:16]

    def central(j, e):
        v = []
        for sgn in (1.0, -1.0):
            th = theta.clone()
            th[int(j)] += sgn * e
            v.append(loss_at(th, "fp32"))
        return (v[0] - v[1]) / (2 * e)

    fd = np.array([central(j, eps) for j in pick])
    fd2 = np.array([central(j, 2 * eps) for j in pick])
    bar = 2.0 * (np.abs(fd2 - fd) / 3.0 + noise / eps)
    for prec in PRECS:
        gp = grads[prec][pick]
        d = np.abs(gp - fd)
        lim = bar + 1e-3 * np.abs(grads[prec]).max()
        print("mmd full size, %s: max|g - fd| %.3g, max bar %.3g, |g| %.3g..%.3g" %
              (prec, d.max(), lim.max(), np.abs(fd).min(), np.abs(fd).max()))
        assert np.all(d < lim), (prec, d, lim)
    # the bar is a small fraction of the gradients it checks
    assert (bar + 1e-3 * np.abs(grads["fp32"]).max()).max() < 0.1 * np.abs(fd).min()


@pytest.mark.parametrize("prec", PRECS)
def test_autograd_expval_end_to_end(prec):
    w = W.small_random(88, 40, 300, 50, 400)
    dw = DevWorkload(w)
    theta = dw.theta.clone().requires_grad_(True)
    mean, se = IQPExpval.apply(theta, dw.gens, dw.ops, dw.samples, w.n, prec)
    u = torch.linspace(-1, 1, w.l, dtype=torch.float64, device="cuda")
    loss = (mean * u).sum() + (mean ** 2).sum()
    loss.backward()
    ug = (u + 2 * mean.detach()).cpu().numpy()
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01, w.samples, ug)
    assert np.abs(theta.grad.cpu().numpy() - og).max() < _gtol(prec, og)
    with pytest.raises(RuntimeError):
        theta2 = dw.theta.clone().requires_grad_(True)
        m2, s2 = IQPExpval.apply(theta2, dw.gens, dw.ops, dw.samples, w.n, prec)
        s2.sum().backward()


@pytest.mark.parametrize("prec", PRECS)
def test_autograd_mmd_end_to_end(prec):
    w = W.small_random(99, 30, 200, 60, 300, with_data=80)
    dw = DevWorkload(w)
    theta = dw.theta.clone().requires_grad_(True)
    loss = IQPMMDLoss.apply(theta, dw.gens, dw.ops, dw.op_weight, dw.samples, dw.data, w.n, True,
                            prec)
    (3.0 * loss).backward()
    ol, og = oracle.mmd_loss_grad(w.n, w.gates, w.theta, dw.ops01, w.op_weight, w.samples, w.data,
                                  True)
    assert abs(loss.item() - ol) < TOL[prec]
    assert np.abs(theta.grad.cpu().numpy() - 3.0 * og).max() < _gtol(prec, 3.0 * og)


def test_grad_deterministic_repeat():
    w = W.small_random(111, 150, 2500, 300, 800)
    dw = DevWorkload(w)
    u = np.random.default_rng(5).normal(size=w.l)
    for prec in PRECS:
        a = _grad(dw, u, prec, False)
        b = _grad(dw, u, prec, False)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", PRECS)
def test_grad_every_sample_split_matches_oracle(prec, monkeypatch):
    # the backward contraction split over sample words (12 words here): one
    # split, uneven splits, and one word per split give the same gradient
    w = W.small_random(77, 70, 1500, 200, 700)
    dw = DevWorkload(w)
    u = np.random.default_rng(4).normal(size=w.l)
    og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01, w.samples, u)
    got = {}
    for ks in (1, 2, 5, 12):
        monkeypatch.setenv("IQP_BWD_SPLITS", str(ks))
        got[ks] = _grad(dw, u, prec, True)
        assert np.abs(got[ks] - og).max() < _gtol(prec, og), ks
    monkeypatch.delenv("IQP_BWD_SPLITS")
    for ks in (2, 5, 12):
        assert np.abs(got[ks] - got[1]).max() < 1e-6 * max(1.0, np.abs(og).max())


@pytest.mark.parametrize("prec", PRECS)
def test_mmd_full_size_consistency(prec):
    # the MMD workload at full size (3 x 2000 operators, 10^4 samples, 2000
    # training strings). The loss sums over every operator, so instead of
    # sampled outputs it is checked against properties that hold at any
    # size: (1) both estimator forms equal their formula rebuilt from
    # iqp_expval's means and standard errors and the oracle's exact data
    # terms; (2) the plug-in form's gradient equals iqp_expval_grad with
    # u_k = 2 w_k (q_k - p_k).
    w = W.mmd_n300()
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    N, s = w.data.shape[0], w.s
    odd = oracle.parity(w.n, w.data, w.ops).sum(axis=0).astype(np.float64)
    p = (N - 2.0 * odd) / N
    mean, se, _ = api.iqp_expval(circ, dw.ops, dw.samples, prec)
    torch.cuda.synchronize()
    q, se = mean.cpu().numpy(), se.cpu().numpy()
    sum_c = s * q
    sum_c2 = s * (s * se * se + q * q)
    wts = w.op_weight
    want = {False: float(np.sum(wts * (p - q) ** 2)),
            True: float(np.sum(wts * (((N * p) ** 2 - N) / (N * (N - 1)) - 2.0 * p * q +
                                      (sum_c ** 2 - sum_c2) / (s * (s - 1)))))}
    for unbiased in (False, True):
        loss, g = api.iqp_mmd_loss_grad(circ, dw.ops, dw.op_weight, dw.samples, dw.data,
                                        unbiased, True, prec)
        torch.cuda.synchronize()
        print("mmd full %s unbiased=%s: loss %.10g vs %.10g" % (prec, unbiased, loss.item(),
                                                               want[unbiased]))
        assert abs(loss.item() - want[unbiased]) < 1e-10 * max(1.0, abs(want[unbiased]))
        if not unbiased:
            u = torch.from_numpy(2.0 * wts * (q - p)).cuda()
            gref = api.iqp_expval_grad(circ, dw.ops, dw.samples, u, None, prec)
            torch.cuda.synchronize()
            a, b = g.cpu().numpy(), gref.cpu().numpy()
            assert np.abs(a - b).max() <= 1e-9 * max(1e-30, np.abs(b).max())
