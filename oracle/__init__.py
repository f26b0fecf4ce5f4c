"""FP64 CPU oracle for the IQP Monte Carlo estimator — TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. It wraps ``iqp_oracle.c``
(plain C, FP64, qubit index lists, threads over observables) through ctypes
and shares no code with the HIP path.

Inputs follow ``workloads``: generators and observables as index-list rows,
samples and training data as dense 0/1 uint8 matrices.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iqp_oracle.c")
# IQP_ORACLE_LIBRARY names another build of iqp_oracle.c (the sanitizer build
# of the tests)
_LIB = os.environ.get("IQP_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, i32, dp, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p
        u64 = ctypes.c_uint64
        sigs = {
            "orc_num_threads": ([], i32),
            "orc_parity": ([i64, i64, vp, i64, vp, vp, vp], i32),
            "orc_expval": ([i64, i64, vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, i32], i32),
            "orc_expval_grad": ([i64, i64, vp, vp, vp, i64, vp, i64, vp, vp, vp, i32], i32),
            "orc_mmd_loss_grad": ([i64, i64, vp, vp, vp, i64, vp, vp, i64, vp, i64, vp, i32,
                                   vp, vp, vp, vp, i32], i32),
            "orc_statevector_probs": ([i64, i64, vp, vp, vp, vp], i32),
            "orc_statevector_expval": ([i64, i64, vp, vp, vp, i64, vp, vp], i32),
            "orc_subset_expval": ([i64, i64, vp, vp, vp, i64, vp, vp], i32),
            "orc_bitflip_expval": ([i64, i64, vp, vp, vp, i64, vp, vp], i32),
            "orc_bitflip_grad": ([i64, i64, vp, vp, vp, i64, vp, vp, vp], i32),
            "orc_expval_indep": ([i64, i64, vp, vp, vp, i64, vp, i64, vp, vp, vp, vp, i32],
                                 i32),
            "orc_expval_indep_grad": ([i64, i64, vp, vp, vp, i64, vp, i64, vp, vp, vp, i32], i32),
            "orc_philox4x64": ([vp, vp, vp], None),
            "orc_sample_uniform": ([i64, i64, u64, u64, u64, u64, vp], i32),
            "orc_sample_bernoulli": ([i64, i64, vp, u64, u64, u64, u64, vp], i32),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(st, what):
    if st != 0:
        raise RuntimeError("oracle %s failed with status %d" % (what, st))


def _gates(gates):
    return _c(gates.ptr, np.int64), _c(gates.idx, np.int32)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def parity(n, rows01, gates):
    """out[r, j] = |g_j ∩ rows_r| mod 2 as uint8."""
    rows01 = _c(rows01, np.uint8)
    gp, gi = _gates(gates)
    out = np.zeros((rows01.shape[0], gates.count), dtype=np.uint8)
    _check(lib().orc_parity(n, rows01.shape[0], _p(rows01), gates.count, _p(gp), _p(gi),
                            _p(out)), "parity")
    return out


def expval(n, gates, theta, ops01, samples01, phases=False, threads=0):
    """(mean[l], stderr[l]) of eq. expvalsample; optionally the raw phases E[l][s]."""
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    samples01 = _c(samples01, np.uint8)
    l, s = ops01.shape[0], samples01.shape[0]
    mean = np.zeros(l)
    se = np.zeros(l)
    ph = np.zeros((l, s)) if phases else None
    _check(lib().orc_expval(n, gates.count, _p(gp), _p(gi), _p(theta), l, _p(ops01), s,
                            _p(samples01), _p(mean), _p(se), _p(ph), threads), "expval")
    return (mean, se, ph) if phases else (mean, se)


def expval_grad(n, gates, theta, ops01, samples01, grad_mean, threads=0):
    """dL/dtheta for u = dL/dmean."""
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    samples01 = _c(samples01, np.uint8)
    u = _c(grad_mean, np.float64)
    g = np.zeros(gates.count)
    _check(lib().orc_expval_grad(n, gates.count, _p(gp), _p(gi), _p(theta), ops01.shape[0],
                                 _p(ops01), samples01.shape[0], _p(samples01), _p(u), _p(g),
                                 threads), "expval_grad")
    return g


def expval_indep(n, gates, theta, ops01, samples01, phases=False, threads=0):
    """Independent estimates: samples01 is [l][s][n], observable k averaging
    over its own samples01[k] (the l x s x n option of Sec. 2.3)."""
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    samples01 = _c(samples01, np.uint8)
    l, s = ops01.shape[0], samples01.shape[1]
    if samples01.shape[0] != l or samples01.shape[2] != n:
        raise ValueError("samples01 must be [l][s][n]")
    mean = np.zeros(l)
    se = np.zeros(l)
    ph = np.zeros((l, s)) if phases else None
    _check(lib().orc_expval_indep(n, gates.count, _p(gp), _p(gi), _p(theta), l, _p(ops01), s,
                                  _p(samples01), _p(mean), _p(se), _p(ph), threads),
           "expval_indep")
    return (mean, se, ph) if phases else (mean, se)


def expval_indep_grad(n, gates, theta, ops01, samples01, grad_mean, threads=0):
    """dL/dtheta of the independent estimates for u = dL/dmean."""
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    samples01 = _c(samples01, np.uint8)
    u = _c(grad_mean, np.float64)
    g = np.zeros(gates.count)
    _check(lib().orc_expval_indep_grad(n, gates.count, _p(gp), _p(gi), _p(theta),
                                       ops01.shape[0], _p(ops01), samples01.shape[1],
                                       _p(samples01), _p(u), _p(g), threads),
           "expval_indep_grad")
    return g


def mmd_loss_grad(n, gates, theta, ops01, op_weight, samples01, data01, unbiased=True,
                  grad=True, threads=0, diagnostics=False):
    """(loss, grad or None[, phat, qhat]) of the MMD^2 estimator."""
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    w = _c(op_weight, np.float64)
    samples01 = _c(samples01, np.uint8)
    data01 = _c(data01, np.uint8)
    l = ops01.shape[0]
    loss = np.zeros(1)
    g = np.zeros(gates.count) if grad else None
    ph = np.zeros(l) if diagnostics else None
    qh = np.zeros(l) if diagnostics else None
    _check(lib().orc_mmd_loss_grad(n, gates.count, _p(gp), _p(gi), _p(theta), l, _p(ops01),
                                   _p(w), samples01.shape[0], _p(samples01), data01.shape[0],
                                   _p(data01), int(bool(unbiased)), _p(loss), _p(g), _p(ph),
                                   _p(qh), threads), "mmd_loss_grad")
    if diagnostics:
        return float(loss[0]), g, ph, qh
    return float(loss[0]), g


def statevector_probs(n, gates, theta):
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    probs = np.zeros(1 << n)
    _check(lib().orc_statevector_probs(n, gates.count, _p(gp), _p(gi), _p(theta), _p(probs)),
           "statevector_probs")
    return probs


def statevector_expval(n, gates, theta, ops01):
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    out = np.zeros(ops01.shape[0])
    _check(lib().orc_statevector_expval(n, gates.count, _p(gp), _p(gi), _p(theta),
                                        ops01.shape[0], _p(ops01), _p(out)),
           "statevector_expval")
    return out


def subset_expval(n, gates, theta, ops01):
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    out = np.zeros(ops01.shape[0])
    _check(lib().orc_subset_expval(n, gates.count, _p(gp), _p(gi), _p(theta), ops01.shape[0],
                                   _p(ops01), _p(out)), "subset_expval")
    return out


def bitflip_expval(n, gates, theta, ops01):
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    out = np.zeros(ops01.shape[0])
    _check(lib().orc_bitflip_expval(n, gates.count, _p(gp), _p(gi), _p(theta), ops01.shape[0],
                                    _p(ops01), _p(out)), "bitflip_expval")
    return out


def bitflip_grad(n, gates, theta, ops01, grad_out):
    gp, gi = _gates(gates)
    theta = _c(theta, np.float64)
    ops01 = _c(ops01, np.uint8)
    u = _c(grad_out, np.float64)
    g = np.zeros(gates.count)
    _check(lib().orc_bitflip_grad(n, gates.count, _p(gp), _p(gi), _p(theta), ops01.shape[0],
                                  _p(ops01), _p(u), _p(g)), "bitflip_grad")
    return g


# ---------------------------------------------------------------------------
# The training loop (Sec. 3.3 with the MMD^2 loss of Sec. 3.3.1): random
# numbers, operators drawn from P_sigma, parameter sharing and fixed gates
# (gates as tuples of generators, Sec. 3.1.1), and the optimizer update.

def philox4x64(ctr, key):
    """Philox4x64-10 of counter ctr[4] under key key[2] (Salmon et al. 2011)."""
    c = _c(np.asarray(ctr, dtype=np.uint64), np.uint64)
    k = _c(np.asarray(key, dtype=np.uint64), np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_p(c), _p(k), _p(out))
    return out


def sample_uniform(rows, n, seed, step, tag):
    """uint8 [rows][n] uniform bits: qubit q of row r is bit q % 64 of output
    r * ceil(n/64) + q / 64 of stream (seed, step, tag)."""
    out = np.zeros((rows, n), dtype=np.uint8)
    _check(lib().orc_sample_uniform(rows, n, int(seed[0]), int(seed[1]), int(step), int(tag),
                                    _p(out)), "sample_uniform")
    return out


def bit_threshold(p):
    """floor(p * 2^64) for a bit probability 0 <= p < 1 (exact: scaling by a
    power of two and truncation)."""
    if not (0.0 <= p < 1.0):
        raise ValueError("bit probability must lie in [0, 1)")
    return int(math.ldexp(float(p), 64))


def sample_bernoulli(n, group_rows, group_prob, seed, step, tag):
    """uint8 [sum(group_rows)][n]: qubit q of row r is 1 when output r * n + q
    of stream (seed, step, tag) is below the threshold of r's group."""
    thr = np.concatenate([np.full(int(r), bit_threshold(p), dtype=np.uint64)
                          for r, p in zip(group_rows, group_prob)])
    out = np.zeros((thr.size, n), dtype=np.uint8)
    _check(lib().orc_sample_bernoulli(thr.size, n, _p(thr), int(seed[0]), int(seed[1]),
                                      int(step), int(tag), _p(out)), "sample_bernoulli")
    return out


def gate_theta(param_index, params, fixed_theta):
    """theta_j = params[param_index[j]], or fixed_theta[j] where the index is
    -1 (a fixed gate): one parameter shared by all generators of a gate."""
    idx = np.asarray(param_index)
    theta = np.zeros(idx.size)
    for j in range(idx.size):
        theta[j] = params[idx[j]] if idx[j] >= 0 else fixed_theta[j]
    return theta


def param_grad(param_index, n_params, grad_theta):
    """dL/dparam_p = sum of dL/dtheta_j over the generators j of parameter p
    (chain rule through theta_j = params[param_index[j]])."""
    g = np.zeros(n_params)
    for j, p in enumerate(np.asarray(param_index)):
        if p >= 0:
            g[p] += grad_theta[j]
    return g


OPT_GD, OPT_ADAM = 0, 1


def optimizer_update(opt, params, grad, m1, m2, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One update; t is the number of earlier updates. Gradient descent:
    params - lr grad. Adam (Kingma and Ba 2015, Algorithm 1) with step count
    t + 1: biased moments, their bias corrections, params - lr mhat /
    (sqrt(vhat) + eps). Returns (params, m1, m2) as new arrays."""
    params = np.array(params, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    m1 = np.array(m1, dtype=np.float64)
    m2 = np.array(m2, dtype=np.float64)
    if opt == OPT_GD:
        return params - lr * grad, m1, m2
    k = t + 1
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** k)
    vhat = m2 / (1.0 - beta2 ** k)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def op_weights(group_rows):
    """Each bandwidth group's weights sum to 1 / (number of groups)."""
    G = len(group_rows)
    return np.concatenate([np.full(int(r), 1.0 / (G * int(r))) for r in group_rows])


TAG_SAMPLES, TAG_OPS = 0, 1


def train_step(n, gates, param_index, fixed_theta, params, group_rows, group_prob, s, data01,
               seed, step, opt, m1, m2, lr, beta1=0.9, beta2=0.999, eps=1e-8, unbiased=True):
    """One training step at step count `step`: fresh samples and operators
    from the two streams, the MMD^2 loss and gradient at the current
    parameters, then the optimizer update. Returns a dict with loss, grad
    (per parameter), params, m1, m2, samples, ops."""
    z = sample_uniform(s, n, seed, step, TAG_SAMPLES)
    ops = sample_bernoulli(n, group_rows, group_prob, seed, step, TAG_OPS)
    theta = gate_theta(param_index, params, fixed_theta)
    loss, gt = mmd_loss_grad(n, gates, theta, ops, op_weights(group_rows), z, data01,
                             unbiased=unbiased)
    gp = param_grad(param_index, len(params), gt)
    new, m1, m2 = optimizer_update(opt, params, gp, m1, m2, step, lr, beta1, beta2, eps)
    return {"loss": loss, "grad": gp, "params": new, "m1": m1, "m2": m2, "samples": z,
            "ops": ops}
