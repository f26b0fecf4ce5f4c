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
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "iqp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
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
