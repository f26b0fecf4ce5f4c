"""GPU vs oracle: parity bits (bit-exact), forward estimates and phases, for
both precisions, through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2501_04776_amd import api, packing
from tests.gpu_util import TOL, DevWorkload, dev_rows_from_dense, dev_rows_from_index, wrap

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "split_bf16", "split3_bf16", "split_bf16_fp8", "sparse_fp32"]


def _unpack_tiled(out, R, C):
    """TILED32 words -> bits [R][C]: word ((r/32)*Cw + c/64)*32 + r%32, bit c%64."""
    Cw = (C + 63) // 64
    words = out.cpu().numpy().view(np.uint64).reshape(-1)
    r = np.arange(R)[:, None]
    c = np.arange(C)[None, :]
    idx = ((r // 32) * Cw + c // 64) * 32 + r % 32
    return ((words[idx] >> (c % 64).astype(np.uint64)) & np.uint64(1)).astype(np.uint8)


def _unpack_tiled_t(out, R, C):
    """TILED32_T words -> bits [R][C]: word ((c/32)*Rw + r/64)*32 + c%32, bit r%64."""
    Rw = (R + 63) // 64
    words = out.cpu().numpy().view(np.uint64).reshape(-1)
    r = np.arange(R)[:, None]
    c = np.arange(C)[None, :]
    idx = ((c // 32) * Rw + r // 64) * 32 + c % 32
    return ((words[idx] >> (r % 64).astype(np.uint64)) & np.uint64(1)).astype(np.uint8)


@pytest.mark.parametrize("n", [1, 10, 63, 64, 65, 300, 1000, 2000])
@pytest.mark.parametrize("layout", [api.ROW_MAJOR, api.TILED32, api.TILED32_T])
def test_parity_bit_exact(n, layout):
    rng = np.random.default_rng(1000 + n)
    R, C = 77, 130  # ragged in both directions
    rows = W.uniform_bits(rng, R, n)
    rows[5] = 0  # weight-0 row
    cols = W.random_weight_rows(rng, C, n, 1, min(n, 9))
    if n >= 300:
        # dense columns too: the bit-sliced cost grows with their weight
        dense = W.dense_to_rows(W.uniform_bits(rng, 20, n))
        cols = W.rows_from_lists([list(cols.row(i)) for i in range(C - 20)] +
                                 [list(dense.row(i)) for i in range(20)])
        cols.idx = cols.idx.astype(np.int32)
    out = api.iqp_parity(dev_rows_from_dense(rows), dev_rows_from_index(cols, n), n, layout)
    torch.cuda.synchronize()
    expect = oracle.parity(n, rows, cols)
    if layout == api.ROW_MAJOR:
        got = packing.unpack(out.cpu().numpy().view(np.uint64), C)
        # bits past the last column are zero
        words = out.cpu().numpy().view(np.uint64)
        if C % 64:
            assert np.all((words[:, -1] >> np.uint64(C % 64)) == 0)
    elif layout == api.TILED32:
        got = _unpack_tiled(out, R, C)
        pad = _unpack_tiled(out, (R + 31) // 32 * 32, C)[R:]
        assert not pad.any()
    else:
        got = _unpack_tiled_t(out, R, C)
        full = _unpack_tiled_t(out, (R + 63) // 64 * 64, (C + 63) // 64 * 64)
        assert not full[R:].any() and not full[:, C:].any()
    assert np.array_equal(got, expect)


def test_parity_gf2_linearity_and_both_layouts_agree():
    n = 300
    rng = np.random.default_rng(7)
    z = dev_rows_from_dense(W.uniform_bits(rng, 96, n))
    g = W.uniform_bits(rng, 128, n)
    h = W.uniform_bits(rng, 128, n)
    pg = api.iqp_parity(z, dev_rows_from_dense(g), n)
    ph = api.iqp_parity(z, dev_rows_from_dense(h), n)
    pgh = api.iqp_parity(z, dev_rows_from_dense(g ^ h), n)
    assert torch.equal(pgh, pg ^ ph)
    t = api.iqp_parity(z, dev_rows_from_dense(g), n, api.TILED32)
    torch.cuda.synchronize()
    assert np.array_equal(_unpack_tiled(t, 96, 128),
                          packing.unpack(pg.cpu().numpy().view(np.uint64), 128))


def _run(dw, prec, phase=False):
    circ = api.Circuit(dw.n, dw.gens, dw.theta)
    mean, se, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=phase)
    torch.cuda.synchronize()
    return mean.cpu().numpy(), se.cpu().numpy(), (ph.cpu().numpy() if phase else None)


@pytest.mark.parametrize("prec", PRECS)
def test_n10_enumeration_matches_statevector(prec):
    w = W.local_n10(enumerate_samples=True)
    dw = DevWorkload(w)
    mean, se, _ = _run(dw, prec)
    exact = oracle.statevector_expval(w.n, w.gates, w.theta, dw.ops01)
    om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01, w.samples)
    assert np.abs(om - exact).max() < 1e-12
    err = np.abs(mean - exact)
    print("n=10 enumeration %s: max|d mean| = %.3g" % (prec, err.max()))
    assert err.max() < TOL[prec]
    assert np.abs(se - ose).max() < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_n10_random_samples_match_oracle(prec):
    w = W.local_n10(enumerate_samples=False)
    dw = DevWorkload(w)
    mean, se, ph = _run(dw, prec, phase=True)
    om, ose, oph = oracle.expval(w.n, w.gates, w.theta, dw.ops01, w.samples, phases=True)
    assert np.abs(mean - om).max() < TOL[prec]
    assert np.abs(se - ose).max() < TOL[prec]
    assert np.abs(wrap(ph - oph)).max() < 100 * TOL[prec]
    assert np.all(np.abs(ph) <= np.pi + 1e-6)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(5, 190, 37, 333), (70, 1000, 300, 700), (130, 2100, 129, 1025),
                                   (2000, 700, 64, 257)])
def test_random_ragged_shapes_match_oracle(prec, shape):
    # several tiles and a ragged tail in every extent; W from 1 to 32 words
    n, m, l, s = shape
    w = W.small_random(sum(shape), n, m, l, s)
    dw = DevWorkload(w)
    mean, se, ph = _run(dw, prec, phase=True)
    om, ose, oph = oracle.expval(w.n, w.gates, w.theta, dw.ops01, w.samples, phases=True)
    d = np.abs(mean - om)
    print("shape %s %s: max|d mean| = %.3g, max|d stderr| = %.3g, max|d phase| = %.3g" %
          (shape, prec, d.max(), np.abs(se - ose).max(), np.abs(wrap(ph - oph)).max()))
    assert d.max() < TOL[prec]
    assert np.abs(se - ose).max() < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_identity_observable_and_single_gate(prec):
    n = 100
    gates = W.rows_from_lists([[3, 7]] + [[q] for q in range(10, 40)])
    theta = np.concatenate([[0.61], np.linspace(-1, 1, 30)])
    ops = W.rows_from_lists([[], [3], [7, 50], [60]])
    z = W.uniform_bits(np.random.default_rng(3), 500, n)
    w = W.Workload("id", n, gates, theta, ops, z)
    dw = DevWorkload(w)
    mean, se, _ = _run(dw, prec)
    assert mean[0] == 1.0 and se[0] == 0.0
    # one anticommuting gate: cos(2 theta) for every sample
    assert abs(mean[1] - np.cos(2 * 0.61)) < TOL[prec] and se[1] < TOL[prec]
    assert abs(mean[2] - np.cos(2 * 0.61)) < TOL[prec]
    assert mean[3] == 1.0


@pytest.mark.parametrize("prec", PRECS)
def test_theta_shift_by_pi_invariance(prec):
    w = W.small_random(5, 90, 500, 100, 300)
    dw = DevWorkload(w)
    m0, s0, _ = _run(dw, prec)
    dw.theta = torch.from_numpy(w.theta + np.pi * np.random.default_rng(2).integers(-4, 5, w.m)).cuda()
    m1, s1, _ = _run(dw, prec)
    assert np.abs(m0 - m1).max() < TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic_repeat(prec):
    w = W.small_random(9, 200, 3000, 260, 900)
    dw = DevWorkload(w)
    a = _run(dw, prec, phase=True)
    b = _run(dw, prec, phase=True)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", PRECS)
def test_n300_full_size_sampled_observables(prec):
    # the n = 300, 45150-gate, 1000 x 10000 workload at full size; the oracle
    # recomputes 24 sampled observables one by one on the same samples
    w = W.local_n300()
    dw = DevWorkload(w)
    mean, se, _ = _run(dw, prec)
    pick = np.random.default_rng(0).choice(w.l, size=24, replace=False)
    om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01[pick], w.samples)
    d = np.abs(mean[pick] - om)
    print("n=300 %s: max|d mean| = %.3g  max|d stderr| = %.3g" % (prec, d.max(),
                                                                  np.abs(se[pick] - ose).max()))
    assert d.max() < TOL[prec]
    assert np.abs(se[pick] - ose).max() < TOL[prec]
    # the weight-2 observables of this all-local circuit have an exact value
    # only through the full expansion; weight-1 ones are a product form
    ops1 = np.eye(w.n, dtype=np.uint8)[:16]
    w1 = W.Workload("w1", w.n, w.gates, w.theta, W.dense_to_rows(ops1), w.samples)
    dw1 = DevWorkload(w1)
    m1, s1, _ = _run(dw1, prec)
    exact = oracle.bitflip_expval(w.n, w.gates, w.theta, ops1)
    assert np.all(np.abs(m1 - exact) <= 5 * s1 + TOL[prec])
