"""Helpers shared by the GPU tests: move a seeded workload to the device in
the library's packed layout, and tolerances."""
import numpy as np
import torch

import oracle

import workloads as W
from paper_2501_04776_amd import packing

# Absolute tolerances on floating results (means, standard errors, losses).
TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "split3_bf16": 1e-4, "split_bf16_fp8": 1e-4,
       "sparse_fp32": 1e-5}


def dev_rows_from_index(rows, n):
    return torch.from_numpy(packing.pack_index_rows(rows.ptr, rows.idx, n).view(np.int64)).cuda()


def dev_rows_from_dense(bits01):
    return torch.from_numpy(packing.pack_dense(bits01).view(np.int64)).cuda()


class DevWorkload:
    def __init__(self, w: W.Workload):
        self.w = w
        self.n = w.n
        self.gens = dev_rows_from_index(w.gates, w.n)
        self.theta = torch.from_numpy(w.theta).cuda()
        self.ops = dev_rows_from_index(w.ops, w.n)
        self.samples = dev_rows_from_dense(w.samples)
        self.data = dev_rows_from_dense(w.data) if w.data is not None else None
        self.op_weight = torch.from_numpy(w.op_weight).cuda() if w.op_weight is not None else None
        self.ops01 = W.rows_to_dense(w.ops, w.n)


def grad_tol(prec, og):
    """Gradient tolerance tol * max(1, |g|_inf) (estimate tolerance of the
    form, relative once the gradient exceeds 1)."""
    return TOL[prec] * max(1.0, float(np.abs(og).max()))


def check_grad(prec, g, w, ops01, u, og=None, where=""):
    """GPU gradient against the oracle.

    Every form but the two with two BF16 limbs of theta (split_bf16,
    split_bf16_fp8) must meet tol * max(1, |g|_inf) against the exact FP64
    gradient. Those hold 2 theta'_j in 16 significant bits; their gradient is
    the exact one at those angles, so it
    must meet the tolerance against the oracle evaluated at the represented
    angles (the kernels' own error), and against the exact oracle up to that
    representation error, which the host model computes
    (tests/precision_model.py) and which is reported, not hidden."""
    from tests import precision_model as PM
    g = np.asarray(g)
    if og is None:
        og = oracle.expval_grad(w.n, w.gates, w.theta, ops01, w.samples, u)
    err = float(np.abs(g - og).max())
    if prec not in ("split_bf16", "split_bf16_fp8"):
        assert err < grad_tol(prec, og), (where, prec, err, grad_tol(prec, og))
        return err, 0.0
    th = PM.theta_represented(prec, w.theta)
    og2 = oracle.expval_grad(w.n, w.gates, th, ops01, w.samples, u)
    rep = float(np.abs(og2 - og).max())
    err2 = float(np.abs(g - og2).max())
    assert err2 < grad_tol(prec, og2), (where, prec, err2, grad_tol(prec, og2))
    assert err < grad_tol(prec, og) + rep, (where, prec, err, rep)
    return err, rep


def wrap(x):
    """Difference of angles mapped to [-pi, pi]."""
    return (x + np.pi) % (2 * np.pi) - np.pi
