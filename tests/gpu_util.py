"""Helpers shared by the GPU tests: move a seeded workload to the device in
the library's packed layout, and tolerances."""
import numpy as np
import torch

import workloads as W
from paper_2501_04776_amd import packing

# Absolute tolerances on floating results (means, standard errors, losses).
TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "sparse_fp32": 1e-5}


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


def grad_bar(prec, w, ops01, u):
    """Per-gate tolerance of dL/dtheta_j = sum_k u_k d_kj, where each
    d_kj = -(2/s) sum_i sin(E_ki) (-1)^{b_ij} c_kj is an average of terms in
    [-2, 2] and so carries twice the estimate tolerance; the independent
    rounding errors of the observables with c_kj = 1 add in quadrature."""
    import oracle
    c = oracle.parity(w.n, ops01, w.gates).astype(np.float64)  # [l][m]
    return TOL[prec] * np.maximum(1.0, 2.0 * np.sqrt((np.asarray(u) ** 2) @ c))


def wrap(x):
    """Difference of angles mapped to [-pi, pi]."""
    return (x + np.pi) % (2 * np.pi) - np.pi
