"""GPU vs oracle for the batched form: many problems of uneven size in one
pass per direction (persistent contractions over a work queue, a captured
graph replayed), every tile configuration, the autotuner, and the 64-circuit
workload at full size on sampled observables."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from paper_2501_04776_amd import api
from tests.gpu_util import TOL, DevWorkload, check_grad, wrap

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "split_bf16", "split3_bf16", "split_bf16_fp8"]

# (n, m, l, s): tiny to several tiles, ragged in every extent, W = 1 .. 32
SHAPES = [(5, 40, 3, 70), (70, 1000, 300, 700), (130, 2100, 129, 1025), (2000, 700, 64, 257),
          (64, 5000, 900, 513), (300, 300, 1, 4096)]


def _workloads(seed=0, shapes=SHAPES):
    return [W.small_random(seed + 17 * i + sum(sh), *sh) for i, sh in enumerate(shapes)]


def _plan(dws, prec, graph=True):
    probs = [(api.Circuit(d.n, d.gens, d.theta), d.ops, d.samples) for d in dws]
    return api.BatchPlan(probs, prec, graph=graph)


def _check_forward(plan, ws, dws, prec, phases=True):
    torch.cuda.synchronize()
    for i, (w, d) in enumerate(zip(ws, dws)):
        om, ose, oph = oracle.expval(w.n, w.gates, w.theta, d.ops01, w.samples, phases=True)
        mean = plan.means[i].cpu().numpy()
        se = plan.stderrs[i].cpu().numpy()
        assert np.abs(mean - om).max() < TOL[prec], (i, np.abs(mean - om).max())
        assert np.abs(se - ose).max() < TOL[prec], i
        if phases:
            ph = plan.phases[i].cpu().numpy()
            assert np.abs(wrap(ph - oph)).max() < 100 * TOL[prec], i


def _check_backward(plan, ws, dws, us, prec):
    torch.cuda.synchronize()
    for i, (w, d) in enumerate(zip(ws, dws)):
        check_grad(prec, plan.grads[i].cpu().numpy(), w, d.ops01, us[i], where="problem %d" % i)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("graph", [True, False])
def test_batch_forward_and_backward_match_oracle(prec, graph):
    ws = _workloads()
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, prec, graph)
    plan.expval()
    _check_forward(plan, ws, dws, prec)
    us = [np.random.default_rng(5 + i).normal(size=w.l) for i, w in enumerate(ws)]
    plan.expval_grad([torch.from_numpy(u).cuda() for u in us])
    _check_backward(plan, ws, dws, us, prec)
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
def test_every_tile_configuration_matches_oracle(prec):
    ws = _workloads(seed=3, shapes=SHAPES[:4])
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, prec, graph=True)
    us = [np.random.default_rng(9 + i).normal(size=w.l) for i, w in enumerate(ws)]
    for fwd_tile in [(4, 4), (2, 4), (2, 2)]:
        for split in [0, 1, 2]:
            for bwd_tile in [(2, 2), (2, 4)]:
                plan.set_config(fwd_tile, split, bwd_tile)
                plan.expval()
                _check_forward(plan, ws, dws, prec)
                plan.expval_grad([torch.from_numpy(u).cuda() for u in us])
                _check_backward(plan, ws, dws, us, prec)
    plan.close()


def test_batch_equals_single_problem_calls():
    # one problem per batch entry, same tiles: only the forward's gate-word
    # split (chosen per pass) can differ, so results agree to FP32 rounding
    prec = "split_bf16"
    ws = _workloads(seed=11, shapes=SHAPES[:3])
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, prec)
    plan.expval()
    us = [np.random.default_rng(2 + i).normal(size=w.l) for i, w in enumerate(ws)]
    plan.expval_grad([torch.from_numpy(u).cuda() for u in us])
    torch.cuda.synchronize()
    for i, d in enumerate(dws):
        circ = api.Circuit(d.n, d.gens, d.theta)
        mean, se, ph = api.iqp_expval(circ, d.ops, d.samples, prec, phase_save=True)
        g = api.iqp_expval_grad(circ, d.ops, d.samples, torch.from_numpy(us[i]).cuda(), ph, prec)
        torch.cuda.synchronize()
        assert np.abs(mean.cpu().numpy() - plan.means[i].cpu().numpy()).max() < 1e-6
        assert np.abs(g.cpu().numpy() - plan.grads[i].cpu().numpy()).max() < \
            1e-5 * max(1.0, np.abs(g.cpu().numpy()).max())
    plan.close()


def test_graph_replays_match_plain_launches():
    # the captured graph, replayed several times with eager work and
    # synchronisations in between, gives the plain launches' results bitwise
    prec = "split_bf16"
    ws = _workloads(seed=21, shapes=SHAPES[:4])
    dws = [DevWorkload(w) for w in ws]
    ref = _plan(dws, prec, graph=False)
    ref.expval()
    us = [torch.from_numpy(np.random.default_rng(i).normal(size=w.l)).cuda()
          for i, w in enumerate(ws)]
    ref.expval_grad(us)
    torch.cuda.synchronize()
    want_m = [m.clone() for m in ref.means]
    want_g = [g.clone() for g in ref.grads]
    plan = _plan(dws, prec, graph=True)
    for rep in range(4):
        for m in plan.means + plan.grads:
            m.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        plan.expval()
        torch.cuda.synchronize()
        plan.expval_grad(us)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for a, b in zip(plan.means, want_m):
            assert torch.equal(a, b), rep
        for a, b in zip(plan.grads, want_g):
            assert torch.equal(a, b), rep
    # parameters updated in place are picked up by the next replay
    for d in dws:
        d.theta.add_(0.25)
    plan.expval()
    ref.expval()
    torch.cuda.synchronize()
    for a, b in zip(plan.means, ref.means):
        assert torch.equal(a, b)
    ref.close()
    plan.close()


def test_deterministic_repeat_with_work_queue():
    # work units are taken in whatever order the workgroups arrive; each unit
    # is computed by one workgroup in a fixed order, so results are bitwise
    # identical from call to call
    ws = _workloads(seed=31)
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, "split_bf16")
    us = [torch.from_numpy(np.random.default_rng(i).normal(size=w.l)).cuda()
          for i, w in enumerate(ws)]
    outs = []
    for _ in range(3):
        plan.expval()
        plan.expval_grad(us)
        torch.cuda.synchronize()
        outs.append([t.clone() for t in plan.means + plan.stderrs + plan.grads])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)
    plan.close()


@pytest.mark.parametrize("prec", ["split_bf16", "split_bf16_fp8"])
def test_tuner_picks_a_configuration_and_records_it(prec):
    # (the 128 x 64 backward tile exists for the FP16 + FP8 weights only)
    bwd_tiles = [(2, 2), (2, 4)] + ([(4, 2)] if prec == "split_bf16_fp8" else [])
    ws = _workloads(seed=41, shapes=SHAPES[1:5])
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, prec)
    assert not plan.config()["tuned"]
    us = [np.random.default_rng(i).normal(size=w.l) for i, w in enumerate(ws)]
    plan.expval()  # phases for the backward timings
    cfg = plan.tune([torch.from_numpy(u).cuda() for u in us])
    assert cfg["tuned"] and cfg["fwd_tile"] in [(4, 4), (2, 4), (2, 2)]
    assert cfg["bwd_tile"] in bwd_tiles and cfg["fwd_split"] in [0, 1, 2]
    plan.expval()
    _check_forward(plan, ws, dws, prec)
    plan.expval_grad([torch.from_numpy(u).cuda() for u in us])
    _check_backward(plan, ws, dws, us, prec)
    # a new plan over the same shapes starts from the recorded configuration
    plan2 = _plan(dws, prec)
    assert plan2.config() == cfg
    plan.close()
    plan2.close()


def test_batch_rejects_shape_mismatch_and_missing_phases():
    ws = _workloads(seed=51, shapes=SHAPES[:2])
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, "split_bf16")
    plan.ops[0] = plan.ops[0][:-1]  # a different l than planned
    with pytest.raises(api.L.IqpError):
        plan.expval()
    plan.close()
    probs = [(api.Circuit(d.n, d.gens, d.theta), d.ops, d.samples) for d in dws]
    nophase = api.BatchPlan(probs, "split_bf16", save_phases=False)
    nophase.expval()
    with pytest.raises(ValueError):
        nophase.expval_grad([torch.zeros(w.l, dtype=torch.float64, device="cuda") for w in ws])
    nophase.close()


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["split_bf16", "split3_bf16", "split_bf16_fp8"])
def test_batched_workload_full_size_sampled(prec):
    # the 64-circuit workload (n in 50..2000, m in 1e3..2e5, l in 100..5000,
    # s = 4096) at full size; the oracle recomputes 3 sampled observables of
    # 8 sampled circuits one by one, and their gradient for a dL/dmean that
    # is non-zero only on those observables
    ws = [W.batch64_circuit(i) for i in range(64)]
    dws = [DevWorkload(w) for w in ws]
    plan = _plan(dws, prec)
    plan.expval()
    rng = np.random.default_rng(0)
    pick_c = rng.choice(64, size=8, replace=False)
    us_full = []
    picks = {}
    for i, w in enumerate(ws):
        u = np.zeros(w.l)
        if i in pick_c:
            k = rng.choice(w.l, size=3, replace=False)
            u[k] = rng.normal(size=3)
            picks[i] = k
        us_full.append(torch.from_numpy(u).cuda())
    plan.expval_grad(us_full)
    torch.cuda.synchronize()
    for i, k in picks.items():
        w, d = ws[i], dws[i]
        om, ose = oracle.expval(w.n, w.gates, w.theta, d.ops01[k], w.samples)
        mean = plan.means[i].cpu().numpy()[k]
        se = plan.stderrs[i].cpu().numpy()[k]
        print("circuit %d (n=%d m=%d l=%d): max|d mean| = %.3g" % (i, w.n, w.m, w.l,
                                                                 np.abs(mean - om).max()))
        assert np.abs(mean - om).max() < TOL[prec]
        assert np.abs(se - ose).max() < TOL[prec]
        uk = us_full[i].cpu().numpy()[k]
        err, rep = check_grad(prec, plan.grads[i].cpu().numpy(), w, d.ops01[k], uk,
                              where="circuit %d" % i)
        print("circuit %d: max|d grad| = %.3g (representation %.3g)" % (i, err, rep))
    for i in range(64):
        if i not in picks:
            assert not plan.grads[i].abs().max().item()  # dL/dmean = 0 gives dtheta = 0
    plan.close()
