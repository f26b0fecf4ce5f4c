"""CPU: the precision forms' operand rounding, emulated through the oracle.

Pins the host model of tests/precision_model.py (BF16 rounding against
torch's conversion, the emulated gradient without rounding against the
oracle's own gradient), then ties each form's gradient tolerance to its
arithmetic on the shape where two BF16 limbs of theta are not enough:
n = 64, m = 5000, l = 900, s = 513 (weight-1..4 generators, theta uniform on
[-pi, pi], every observable weighted). The bar is the survey's
tol * max(1, |g|_inf) with tol 1e-5 (FP32) and 1e-4 (split BF16)."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests import precision_model as PM

TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "split3_bf16": 1e-4, "split_bf16_fp8": 1e-4}


def test_bf16_rne_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.140625, -2.0 ** -130]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(PM.bf16_rne(x32), ref)


def test_e4m3_rounding_matches_torch_conversion():
    """The FP8 limb's rounding against torch's float8_e4m3fn conversion
    (round to nearest even), over normal, subnormal and tie values."""
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.normal(size=50000) * 10.0 ** rng.integers(-4, 3, 50000),
                        rng.uniform(-2.0 ** -6, 2.0 ** -6, 5000),
                        (np.arange(-64, 65) + 0.5) * 2.0 ** -9,   # subnormal ties
                        [0.0, -0.0, 448.0, -448.0, 17.0, 18.0, 19.0, 2.0 ** -9, 2.0 ** -10]])
    x = x[np.abs(x) <= 448.0].astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(PM.e4m3_rne(x.astype(np.float64)), ref)


def test_fp16_fp8_weights_keep_15_bits():
    """Row exponent and the two limbs: bound 2^e in [2^14, 2^15), FP16 limb
    within FP16's range, rest within 8 (half an FP16 ulp at 2^15) and the
    represented weight within 2^-15 of the row bound's scale plus the FP8
    rounding of the rest (2^-4 relative, 2^-10 absolute below 2^-6)."""
    rng = np.random.default_rng(8)
    bound = 10.0 ** rng.uniform(-12, 6, 300)
    e = PM.fp16_row_exponent(bound)
    sc = np.ldexp(bound, e)
    assert np.all((sc >= 2.0 ** 14) & (sc < 2.0 ** 15))
    S = (rng.uniform(-1, 1, (300, 500)) * bound[:, None]) ** 1
    S[:, :50] *= 10.0 ** rng.uniform(-9, 0, (300, 50))      # small weights too
    x = np.ldexp(S.astype(np.float32).astype(np.float64), e[:, None])
    hi = x.astype(np.float16).astype(np.float64)
    rest = x - hi
    assert np.all(np.abs(rest) <= 8.0)
    rep = PM.weights_represented("split_bf16_fp8", S, bound)
    err = np.abs(np.ldexp(rep, e[:, None]) - x)
    assert np.all(err <= np.maximum(2.0 ** -4 * np.abs(rest), 2.0 ** -10) + 1e-300)
    assert np.all(err <= 2.0 ** -15 * np.abs(x) + 2.0 ** -10)
    assert PM.fp16_row_exponent(np.array([0.0]))[0] == 0
    assert PM.fp16_row_exponent(np.array([np.inf]))[0] == 0


def test_limbs_shrink_the_residual():
    t = PM.two_theta_reduced(np.random.default_rng(1).uniform(-40, 40, 5000))
    assert np.all(np.abs(t) <= np.pi + 1e-12)
    # each limb keeps 8 significant bits of what is left: half an ulp of the
    # binade of |t| is 2^-8 |t| at most, and so on
    for k, bound in ((1, 2.0 ** -8), (2, 2.0 ** -16), (3, 2.0 ** -24)):
        r = np.abs(PM.bf16_limbs(t, k) - t)
        assert np.all(r <= bound * np.abs(t) + 1e-300), (k, (r / np.abs(t)).max())
    # split3's third limb: E4M3 (4 significant bits) of the rest after two
    # BF16 limbs, within its range (|rest| 2^20 <= 2^-16 pi 2^20 < 448), so
    # 2^-4 of the rest (<= 2^-20 |t|) plus the subnormal step's half, 2^-30
    r = np.abs(2.0 * PM.theta_represented("split3_bf16", t / 2.0) - t)
    assert np.all(r <= 2.0 ** -20 * np.abs(t) + 2.0 ** -30), (r / np.abs(t)).max()
    assert np.abs(t - PM.bf16_limbs(t, 2)).max() * 2.0 ** PM.LO8_EXP < 448.0


@pytest.fixture(scope="module")
def hard_case():
    w = W.small_random(6569, 64, 5000, 900, 513)
    ops01 = W.rows_to_dense(w.ops, w.n)
    u = np.random.default_rng(9).normal(size=w.l)
    og = oracle.expval_grad(w.n, w.gates, w.theta, ops01, w.samples, u)
    return w, ops01, u, og


def test_emulation_without_rounding_is_the_oracle(hard_case):
    w, ops01, u, og = hard_case
    g = PM.grad_emulated(w.n, w.gates, w.theta, ops01, w.samples, u)
    assert np.abs(g - og).max() < 1e-12 * max(1.0, np.abs(og).max())


def test_each_form_against_its_bar(hard_case):
    w, ops01, u, og = hard_case
    errs = {}
    for prec in ("fp32", "split_bf16", "split3_bf16", "split_bf16_fp8"):
        g = PM.grad_emulated(w.n, w.gates, w.theta, ops01, w.samples, u, prec)
        errs[prec] = np.abs(g - og).max() / (TOL[prec] * max(1.0, np.abs(og).max()))
    print("emulated gradient error / bar:", errs)
    # FP32 operands and the three-limb form meet their bars with a wide margin
    assert errs["fp32"] < 0.3
    assert errs["split3_bf16"] < 0.3
    # two BF16 limbs of theta (16 significant bits) do not, by their own
    # arithmetic: the residual of every gate repeats in all samples' phases
    assert 0.8 < errs["split_bf16"] < 1.6
    # the FP16 + FP8 weights leave that as it is
    assert abs(errs["split_bf16_fp8"] - errs["split_bf16"]) < 0.1


def test_two_limb_theta_is_the_dominant_term(hard_case):
    """The split-BF16 miss comes from theta, not from the backward weights:
    exact weights with two-limb theta give the same error, two-limb weights
    with exact theta a small fraction of it."""
    w, ops01, u, og = hard_case
    bar = 1e-4 * max(1.0, np.abs(og).max())
    th2 = PM.theta_represented("split_bf16", w.theta)
    g_theta = PM.grad_emulated(w.n, w.gates, th2, ops01, w.samples, u)
    _, _, ph = oracle.expval(w.n, w.gates, w.theta, ops01, w.samples, phases=True)
    S = PM.weights_represented("split_bf16", (u[:, None] / w.s) * np.sin(ph), np.abs(u) / w.s)
    C = oracle.parity(w.n, ops01, w.gates).astype(np.float64)
    B = 1.0 - 2.0 * oracle.parity(w.n, w.samples, w.gates).astype(np.float64)
    g_s = -2.0 * (C * (S @ B)).sum(axis=0)
    e_theta = np.abs(g_theta - og).max() / bar
    e_s = np.abs(g_s - og).max() / bar
    assert e_theta > 0.8 and e_s < 0.1, (e_theta, e_s)
    # FP16 + FP8 weights (15 significant bits per weight) also stay a small
    # fraction of the bar, within twice the error of two BF16 limbs
    S8 = PM.weights_represented("split_bf16_fp8", (u[:, None] / w.s) * np.sin(ph),
                                np.abs(u) / w.s)
    e_s8 = np.abs(-2.0 * (C * (S8 @ B)).sum(axis=0) - og).max() / bar
    assert e_s8 < 0.1 and e_s8 < 2.0 * e_s + 0.01, (e_s8, e_s)


def test_means_of_every_form_within_tolerance(hard_case):
    w, ops01, _, _ = hard_case
    m0, _ = oracle.expval(w.n, w.gates, w.theta, ops01, w.samples)
    for prec in ("fp32", "split_bf16", "split3_bf16", "split_bf16_fp8"):
        th = PM.theta_represented(prec, w.theta)
        m, _ = oracle.expval(w.n, w.gates, th, ops01, w.samples)
        assert np.abs(m - m0).max() < 0.25 * TOL[prec], prec
