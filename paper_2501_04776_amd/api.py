"""Thin Python binding of the C-ABI: argument marshalling only.

Bit rows (generators, observables, samples, data) are torch int64 tensors on
the GPU holding the uint64 words of ``packing``; theta and weights are
float64. Every call runs on torch's current stream and returns without
synchronising. The workspace is a cached device buffer per device.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import torch

from . import _lib as L

FP32 = L.IQP_FP32
SPLIT_BF16 = L.IQP_SPLIT_BF16
ROW_MAJOR = L.IQP_BITS_ROW_MAJOR
TILED32 = L.IQP_BITS_TILED32
TILED32_T = L.IQP_BITS_TILED32_T

_PRECISIONS = {"fp32": FP32, "split_bf16": SPLIT_BF16, FP32: FP32, SPLIT_BF16: SPLIT_BF16}


def precision_id(p) -> int:
    try:
        return _PRECISIONS[p]
    except KeyError:
        raise ValueError("precision must be 'fp32' or 'split_bf16'") from None


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _rows(t: torch.Tensor, name: str, W: int) -> torch.Tensor:
    if not t.is_cuda or t.dtype != torch.int64 or t.dim() != 2 or t.shape[1] != W:
        raise ValueError("%s must be a CUDA int64 tensor of shape [rows, %d]" % (name, W))
    return t.contiguous()


def _vec(t: torch.Tensor, name: str, size: int, dtype=torch.float64) -> torch.Tensor:
    if not t.is_cuda or t.dtype != dtype or t.numel() != size:
        raise ValueError("%s must be a CUDA %s tensor with %d elements" % (name, dtype, size))
    return t.contiguous()


class _Workspace:
    def __init__(self):
        self.buf = {}

    def get(self, device: torch.device, nbytes: int) -> Tuple[torch.Tensor, int]:
        key = device.index
        cur = self.buf.get(key)
        if cur is None or cur.numel() < nbytes:
            # drop the old buffer before allocating the larger one; work still
            # queued on it is ordered on the stream by torch's allocator
            self.buf.pop(key, None)
            cur = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self.buf[key] = cur
        return cur, cur.numel()


workspace = _Workspace()


class Circuit:
    """Generators (bit rows) and parameters of a parameterized IQP circuit."""

    def __init__(self, n_qubits: int, gens: torch.Tensor, theta: torch.Tensor):
        self.n = int(n_qubits)
        self.W = (self.n + 63) // 64
        self.gens = _rows(gens, "gens", self.W)
        self.m = self.gens.shape[0]
        self.theta = _vec(theta, "theta", self.m)
        self.device = self.gens.device

    def struct(self) -> L.IqpCircuit:
        return L.IqpCircuit(self.n, self.W, self.m, self.gens.data_ptr(), self.theta.data_ptr())


def workspace_bytes(call: int, n: int, m: int, l: int, s: int, N: int = 0,
                    precision=SPLIT_BF16) -> int:
    c = L.IqpCircuit(n, (n + 63) // 64, m, None, None)
    return int(L.lib().iqp_workspace_bytes(call, ctypes.byref(c), l, s, N,
                                           precision_id(precision)))


def iqp_parity(rows: torch.Tensor, cols: torch.Tensor, n_qubits: int,
               layout: int = ROW_MAJOR) -> torch.Tensor:
    """Bits (r, c) = popcount(rows[r] & cols[c]) mod 2 in one of the layouts
    of include/iqp.h (cost grows with the weight of the cols rows)."""
    W = (n_qubits + 63) // 64
    rows = _rows(rows, "rows", W)
    cols = _rows(cols, "cols", W)
    R, C = rows.shape[0], cols.shape[0]
    if layout == TILED32_T:
        shape = ((C + 63) // 64 * 64, (R + 63) // 64)
    else:
        shape = ((R + 31) // 32 * 32 if layout == TILED32 else R, (C + 63) // 64)
    out = torch.empty(shape, dtype=torch.int64, device=rows.device)
    need = int(L.lib().iqp_parity_workspace_bytes(R, W, layout))
    ws, nb = workspace.get(rows.device, need)
    L.check(L.lib().iqp_parity(R, _ptr(rows), C, _ptr(cols), W, layout, _ptr(out), _ptr(ws), nb,
                               _stream(rows)), "iqp_parity")
    return out


def iqp_expval(circ: Circuit, ops: torch.Tensor, samples: torch.Tensor,
               precision=SPLIT_BF16, stderr: bool = True, phase_save: bool = False):
    """(mean[l], stderr[l] or None, phase[l][s] or None)."""
    p = precision_id(precision)
    ops = _rows(ops, "ops", circ.W)
    samples = _rows(samples, "samples", circ.W)
    l, s = ops.shape[0], samples.shape[0]
    dev = circ.device
    mean = torch.empty(l, dtype=torch.float64, device=dev)
    se = torch.empty(l, dtype=torch.float64, device=dev) if stderr else None
    ph = torch.empty((l, s), dtype=torch.float32, device=dev) if phase_save else None
    need = workspace_bytes(L.IQP_CALL_EXPVAL, circ.n, circ.m, l, s, 0, p)
    ws, nb = workspace.get(dev, need)
    c = circ.struct()
    L.check(L.lib().iqp_expval(ctypes.byref(c), l, _ptr(ops), s, _ptr(samples), p, _ptr(mean),
                               _ptr(se), _ptr(ph), _ptr(ws), nb, _stream(ops)), "iqp_expval")
    return mean, se, ph


def iqp_expval_grad(circ: Circuit, ops: torch.Tensor, samples: torch.Tensor,
                    grad_mean: torch.Tensor, phase_save: Optional[torch.Tensor] = None,
                    precision=SPLIT_BF16) -> torch.Tensor:
    """dL/dtheta [m] for u = dL/dmean."""
    p = precision_id(precision)
    ops = _rows(ops, "ops", circ.W)
    samples = _rows(samples, "samples", circ.W)
    l, s = ops.shape[0], samples.shape[0]
    u = _vec(grad_mean, "grad_mean", l)
    if phase_save is not None:
        phase_save = _vec(phase_save, "phase_save", l * s, torch.float32)
    g = torch.empty(circ.m, dtype=torch.float64, device=circ.device)
    call = L.IQP_CALL_EXPVAL_GRAD if phase_save is not None else L.IQP_CALL_EXPVAL_GRAD_RECOMPUTE
    need = workspace_bytes(call, circ.n, circ.m, l, s, 0, p)
    ws, nb = workspace.get(circ.device, need)
    c = circ.struct()
    L.check(L.lib().iqp_expval_grad(ctypes.byref(c), l, _ptr(ops), s, _ptr(samples), p,
                                    _ptr(u), _ptr(phase_save), _ptr(g), _ptr(ws), nb,
                                    _stream(ops)), "iqp_expval_grad")
    return g


def iqp_mmd_loss_grad(circ: Circuit, ops: torch.Tensor, op_weight: torch.Tensor,
                      samples: torch.Tensor, data: torch.Tensor, unbiased: bool = True,
                      grad: bool = True, precision=SPLIT_BF16):
    """(loss[1], grad_theta[m] or None)."""
    p = precision_id(precision)
    ops = _rows(ops, "ops", circ.W)
    samples = _rows(samples, "samples", circ.W)
    data = _rows(data, "data", circ.W)
    l, s, N = ops.shape[0], samples.shape[0], data.shape[0]
    w = _vec(op_weight, "op_weight", l)
    loss = torch.empty(1, dtype=torch.float64, device=circ.device)
    g = torch.empty(circ.m, dtype=torch.float64, device=circ.device) if grad else None
    call = L.IQP_CALL_MMD_GRAD if grad else L.IQP_CALL_MMD
    need = workspace_bytes(call, circ.n, circ.m, l, s, N, p)
    ws, nb = workspace.get(circ.device, need)
    c = circ.struct()
    L.check(L.lib().iqp_mmd_loss_grad(ctypes.byref(c), l, _ptr(ops), _ptr(w), s, _ptr(samples),
                                      N, _ptr(data), int(bool(unbiased)), p, _ptr(loss), _ptr(g),
                                      _ptr(ws), nb, _stream(ops)), "iqp_mmd_loss_grad")
    return loss, g


# --- per-kernel timing (measurement only) ----------------------------------
def profile_enable(on: bool = True) -> None:
    L.check(L.lib().iqp_profile_enable(int(on)), "iqp_profile_enable")


def profile_reset() -> None:
    L.check(L.lib().iqp_profile_reset(), "iqp_profile_reset")


def profile_query(name: str) -> Tuple[float, int]:
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    L.check(L.lib().iqp_profile_query(name.encode(), ctypes.byref(ms), ctypes.byref(n)),
            "iqp_profile_query")
    return ms.value, n.value
