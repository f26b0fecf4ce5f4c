"""Thin Python binding of the C-ABI: argument marshalling only.

Bit rows (generators, observables, samples, data) are torch int64 tensors on
the GPU holding the uint64 words of ``packing``; theta and weights are
float64. Every call runs on torch's current stream and returns without
synchronising. The workspace is a cached device buffer per device and
stream.
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

SPARSE_FP32 = L.IQP_SPARSE_FP32
SPLIT3_BF16 = L.IQP_SPLIT3_BF16
SPLIT_BF16_FP8 = L.IQP_SPLIT_BF16_FP8

_PRECISIONS = {"fp32": FP32, "split_bf16": SPLIT_BF16, "sparse_fp32": SPARSE_FP32,
               "split3_bf16": SPLIT3_BF16, "split_bf16_fp8": SPLIT_BF16_FP8, FP32: FP32,
               SPLIT_BF16: SPLIT_BF16, SPARSE_FP32: SPARSE_FP32, SPLIT3_BF16: SPLIT3_BF16,
               SPLIT_BF16_FP8: SPLIT_BF16_FP8}


def precision_id(p) -> int:
    try:
        return _PRECISIONS[p]
    except KeyError:
        raise ValueError("precision must be 'fp32', 'split_bf16', 'split3_bf16', "
                         "'split_bf16_fp8' or 'sparse_fp32'") from None


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
    """One cached workspace per (device, stream): calls queued on one stream
    reuse it in order; calls on different streams get different buffers, so
    they never share scratch memory."""

    def __init__(self):
        self.buf = {}

    def get(self, device: torch.device, nbytes: int) -> Tuple[torch.Tensor, int]:
        key = (device.index, torch.cuda.current_stream(device).cuda_stream)
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
    need = int(L.lib().iqp_parity_workspace_bytes(R, C, W, layout))
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


def iqp_expval_noalloc(circ: Circuit, ops: torch.Tensor, samples: torch.Tensor,
                       precision=SPLIT_BF16, stderr: bool = True, phase_save: bool = False):
    """iqp_expval with the library's static device workspace (no workspace
    allocation; outputs are allocated here as for iqp_expval)."""
    p = precision_id(precision)
    ops = _rows(ops, "ops", circ.W)
    samples = _rows(samples, "samples", circ.W)
    l, s = ops.shape[0], samples.shape[0]
    dev = circ.device
    mean = torch.empty(l, dtype=torch.float64, device=dev)
    se = torch.empty(l, dtype=torch.float64, device=dev) if stderr else None
    ph = torch.empty((l, s), dtype=torch.float32, device=dev) if phase_save else None
    c = circ.struct()
    L.check(L.lib().iqp_expval_noalloc(ctypes.byref(c), l, _ptr(ops), s, _ptr(samples), p,
                                       _ptr(mean), _ptr(se), _ptr(ph), _stream(ops)),
            "iqp_expval_noalloc")
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


def _indep_samples(samples: torch.Tensor, l: int, W: int) -> torch.Tensor:
    if not samples.is_cuda or samples.dtype != torch.int64 or samples.dim() != 3 or \
            samples.shape[0] != l or samples.shape[2] != W:
        raise ValueError("samples must be a CUDA int64 tensor of shape [%d, s, %d]" % (l, W))
    return samples.contiguous()


def iqp_expval_indep(circ: Circuit, ops: torch.Tensor, samples: torch.Tensor,
                     stderr: bool = True, phase_save: bool = False):
    """Independent estimates: samples [l][s][W], observable k averaging over
    samples[k]. Returns (mean[l], stderr[l] or None, phase[l][s] or None)."""
    ops = _rows(ops, "ops", circ.W)
    l = ops.shape[0]
    samples = _indep_samples(samples, l, circ.W)
    s = samples.shape[1]
    dev = circ.device
    mean = torch.empty(l, dtype=torch.float64, device=dev)
    se = torch.empty(l, dtype=torch.float64, device=dev) if stderr else None
    ph = torch.empty((l, s), dtype=torch.float32, device=dev) if phase_save else None
    need = workspace_bytes(L.IQP_CALL_INDEP, circ.n, circ.m, l, s)
    ws, nb = workspace.get(dev, need)
    c = circ.struct()
    L.check(L.lib().iqp_expval_indep(ctypes.byref(c), l, _ptr(ops), s, _ptr(samples),
                                     _ptr(mean), _ptr(se), _ptr(ph), _ptr(ws), nb, _stream(ops)),
            "iqp_expval_indep")
    return mean, se, ph


def iqp_expval_indep_grad(circ: Circuit, ops: torch.Tensor, samples: torch.Tensor,
                          grad_mean: torch.Tensor,
                          phase_save: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/dtheta [m] of the independent estimates for u = dL/dmean."""
    ops = _rows(ops, "ops", circ.W)
    l = ops.shape[0]
    samples = _indep_samples(samples, l, circ.W)
    s = samples.shape[1]
    u = _vec(grad_mean, "grad_mean", l)
    if phase_save is not None:
        phase_save = _vec(phase_save, "phase_save", l * s, torch.float32)
    g = torch.empty(circ.m, dtype=torch.float64, device=circ.device)
    call = L.IQP_CALL_INDEP_GRAD if phase_save is not None else L.IQP_CALL_INDEP_GRAD_RECOMPUTE
    need = workspace_bytes(call, circ.n, circ.m, l, s)
    ws, nb = workspace.get(circ.device, need)
    c = circ.struct()
    L.check(L.lib().iqp_expval_indep_grad(ctypes.byref(c), l, _ptr(ops), s, _ptr(samples),
                                          _ptr(u), _ptr(phase_save), _ptr(g), _ptr(ws), nb,
                                          _stream(ops)), "iqp_expval_indep_grad")
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


# --- stochastic bitflip circuits (exact product form) ------------------------
def iqp_bitflip_expval(circ: Circuit, ops: torch.Tensor) -> torch.Tensor:
    """Exact <Z_a> [l] of the bitflip version of the circuit."""
    ops = _rows(ops, "ops", circ.W)
    l = ops.shape[0]
    mean = torch.empty(l, dtype=torch.float64, device=circ.device)
    need = workspace_bytes(L.IQP_CALL_BITFLIP, circ.n, circ.m, l, 1)
    ws, nb = workspace.get(circ.device, need)
    c = circ.struct()
    L.check(L.lib().iqp_bitflip_expval(ctypes.byref(c), l, _ptr(ops), _ptr(mean), _ptr(ws), nb,
                                       _stream(ops)), "iqp_bitflip_expval")
    return mean


def iqp_bitflip_expval_grad(circ: Circuit, ops: torch.Tensor,
                            grad_mean: torch.Tensor) -> torch.Tensor:
    """dL/dtheta [m] of the bitflip expectation values for u = dL/d<Z>."""
    ops = _rows(ops, "ops", circ.W)
    l = ops.shape[0]
    u = _vec(grad_mean, "grad_mean", l)
    g = torch.empty(circ.m, dtype=torch.float64, device=circ.device)
    need = workspace_bytes(L.IQP_CALL_BITFLIP_GRAD, circ.n, circ.m, l, 1)
    ws, nb = workspace.get(circ.device, need)
    c = circ.struct()
    L.check(L.lib().iqp_bitflip_expval_grad(ctypes.byref(c), l, _ptr(ops), _ptr(u), _ptr(g),
                                            _ptr(ws), nb, _stream(ops)),
            "iqp_bitflip_expval_grad")
    return g


# --- batched form -------------------------------------------------------------
class BatchPlan:
    """Many problems (circuit, observables, samples) of uneven size run as one
    pass per direction (iqp_batch_* of include/iqp.h). The plan owns its
    workspace (the captured graphs are bound to it) and the output buffers:
    ``means``, ``stderrs``, ``phases`` (forward) and ``grads`` (backward),
    one tensor per problem, overwritten by each pass. Calls run on torch's
    current stream and return without synchronising. Circuit parameters may
    be updated in place between calls."""

    def __init__(self, problems, precision=SPLIT_BF16, graph: bool = True,
                 save_phases: bool = True):
        if not problems:
            raise ValueError("a batch needs at least one problem")
        self.p = precision_id(precision)
        self.circuits, self.ops, self.samples = [], [], []
        for circ, ops, samples in problems:
            if not isinstance(circ, Circuit):
                raise ValueError("each problem is (Circuit, ops, samples)")
            self.circuits.append(circ)
            self.ops.append(_rows(ops, "ops", circ.W))
            self.samples.append(_rows(samples, "samples", circ.W))
        self.device = self.circuits[0].device
        if any(c.device != self.device for c in self.circuits):
            raise ValueError("all problems must be on one device")
        self.n = len(problems)
        dev = self.device
        self.means = [torch.empty(o.shape[0], dtype=torch.float64, device=dev) for o in self.ops]
        self.stderrs = [torch.empty(o.shape[0], dtype=torch.float64, device=dev) for o in self.ops]
        self.phases = ([torch.empty((o.shape[0], z.shape[0]), dtype=torch.float32, device=dev)
                        for o, z in zip(self.ops, self.samples)] if save_phases else None)
        self.grads = [torch.empty(c.m, dtype=torch.float64, device=dev) for c in self.circuits]
        self._grad_means = [None] * self.n
        self._handle = ctypes.c_void_p()
        flags = 0 if graph else L.IQP_BATCH_NO_GRAPH
        L.check(L.lib().iqp_batch_plan_create(self.n, self._table(), self.p, flags,
                                              ctypes.byref(self._handle)),
                "iqp_batch_plan_create")
        self.ws_bytes = int(L.lib().iqp_batch_workspace_bytes(self._handle))
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)

    def _table(self):
        arr = (L.IqpProblem * self.n)()
        for i, c in enumerate(self.circuits):
            q = arr[i]
            q.circuit = c.struct()
            q.n_ops, q.ops = self.ops[i].shape[0], self.ops[i].data_ptr()
            q.n_samples, q.samples = self.samples[i].shape[0], self.samples[i].data_ptr()
            q.mean, q.stderr_ = self.means[i].data_ptr(), self.stderrs[i].data_ptr()
            q.phase_save = self.phases[i].data_ptr() if self.phases is not None else None
            u = self._grad_means[i]
            q.grad_mean = u.data_ptr() if u is not None else None
            q.grad_theta = self.grads[i].data_ptr()
        return arr

    def _set_grad_means(self, grad_means):
        if self.phases is None:
            raise ValueError("the backward pass needs a plan with save_phases=True")
        if len(grad_means) != self.n:
            raise ValueError("one grad_mean per problem")
        self._grad_means = [_vec(u, "grad_mean", o.shape[0]) for u, o in zip(grad_means, self.ops)]

    def expval(self):
        """Forward pass: (means, stderrs), lists of [l] tensors."""
        L.check(L.lib().iqp_batch_expval(self._handle, self._table(), _ptr(self.ws), self.ws_bytes,
                                         _stream(self.ws)), "iqp_batch_expval")
        return self.means, self.stderrs

    def expval_grad(self, grad_means):
        """Backward pass from dL/dmean per problem (after ``expval`` with the
        same parameters): list of dL/dtheta [m] tensors."""
        self._set_grad_means(grad_means)
        L.check(L.lib().iqp_batch_expval_grad(self._handle, self._table(), _ptr(self.ws),
                                              self.ws_bytes, _stream(self.ws)),
                "iqp_batch_expval_grad")
        return self.grads

    def tune(self, grad_means=None) -> dict:
        """Autotune the forward (and the backward when grad_means is given)
        on these problems; synchronises. Returns the chosen configuration."""
        passes = 1
        if grad_means is not None:
            self._set_grad_means(grad_means)
            passes = 3
        L.check(L.lib().iqp_batch_tune(self._handle, self._table(), passes, _ptr(self.ws),
                                       self.ws_bytes, _stream(self.ws)), "iqp_batch_tune")
        return self.config()

    def config(self) -> dict:
        c = (ctypes.c_int32 * 6)()
        L.check(L.lib().iqp_batch_get_config(self._handle, c), "iqp_batch_get_config")
        return {"fwd_tile": (c[0], c[1]), "fwd_split": c[2], "bwd_tile": (c[3], c[4]),
                "tuned": bool(c[5])}

    def set_config(self, fwd_tile=(4, 4), fwd_split=1, bwd_tile=(2, 2)) -> None:
        c = (ctypes.c_int32 * 5)(fwd_tile[0], fwd_tile[1], fwd_split, bwd_tile[0], bwd_tile[1])
        L.check(L.lib().iqp_batch_set_config(self._handle, c), "iqp_batch_set_config")

    def close(self) -> None:
        if self._handle:
            torch.cuda.synchronize(self.device)
            L.lib().iqp_batch_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- training on the device ---------------------------------------------------
OPT_GD = L.IQP_OPT_GD
OPT_ADAM = L.IQP_OPT_ADAM
TAG_SAMPLES, TAG_OPS = 0, 1
_OPTIMIZERS = {"gd": OPT_GD, "adam": OPT_ADAM, OPT_GD: OPT_GD, OPT_ADAM: OPT_ADAM}


def _seed(seed):
    s0, s1 = (int(seed[0]), int(seed[1]))
    if not (0 <= s0 < 2**64 and 0 <= s1 < 2**64):
        raise ValueError("seed words must lie in [0, 2^64)")
    return s0, s1


def _step_tensor(step: torch.Tensor) -> torch.Tensor:
    if not step.is_cuda or step.dtype != torch.int64 or step.numel() != 1:
        raise ValueError("step must be a CUDA int64 tensor with one element")
    return step


def sample_uniform(rows: int, n_qubits: int, seed, step: torch.Tensor, tag: int = TAG_SAMPLES,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Uniform bit strings [rows][W] from the Philox stream (seed, *step, tag)."""
    step = _step_tensor(step)
    W = (int(n_qubits) + 63) // 64
    if out is None:
        out = torch.empty((rows, W), dtype=torch.int64, device=step.device)
    out = _rows(out, "out", W)
    s0, s1 = _seed(seed)
    L.check(L.lib().iqp_sample_uniform(rows, n_qubits, s0, s1, _ptr(step), int(tag), _ptr(out),
                                       _stream(step)), "iqp_sample_uniform")
    return out


def sample_bernoulli(n_qubits: int, group_rows, group_prob, seed, step: torch.Tensor,
                     tag: int = TAG_OPS, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Bernoulli bit rows [sum(group_rows)][W]: the bits of group g are set
    with probability group_prob[g] (Philox stream (seed, *step, tag))."""
    step = _step_tensor(step)
    rows = (ctypes.c_int64 * len(group_rows))(*[int(r) for r in group_rows])
    probs = (ctypes.c_double * len(group_prob))(*[float(p) for p in group_prob])
    if len(group_rows) != len(group_prob):
        raise ValueError("one probability per group")
    W = (int(n_qubits) + 63) // 64
    if out is None:
        out = torch.empty((sum(int(r) for r in group_rows), W), dtype=torch.int64,
                          device=step.device)
    out = _rows(out, "out", W)
    s0, s1 = _seed(seed)
    L.check(L.lib().iqp_sample_bernoulli(n_qubits, len(group_rows), rows, probs, s0, s1,
                                         _ptr(step), int(tag), _ptr(out), _stream(step)),
            "iqp_sample_bernoulli")
    return out


def gather_theta(param_index: torch.Tensor, params: torch.Tensor,
                 fixed_theta: Optional[torch.Tensor] = None,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """theta[j] = params[param_index[j]], or fixed_theta[j] where the index is -1."""
    m = param_index.numel()
    idx = _vec(param_index, "param_index", m, torch.int32)
    if out is None:
        out = torch.empty(m, dtype=torch.float64, device=idx.device)
    fixed = _vec(fixed_theta, "fixed_theta", m) if fixed_theta is not None else None
    L.check(L.lib().iqp_gather_theta(m, _ptr(idx), _ptr(params.contiguous()), _ptr(fixed),
                                     _ptr(out), _stream(idx)), "iqp_gather_theta")
    return out


def param_tables(param_index, n_params: int, device) -> Tuple[torch.Tensor, torch.Tensor]:
    """(offsets [P+1] int64, gates int32) of each parameter's gates, in gate
    order, from a host index array (host-side bookkeeping only)."""
    import numpy as np
    idx = np.asarray(param_index, dtype=np.int64)
    order = np.argsort(np.where(idx >= 0, idx, n_params), kind="stable")
    counts = np.bincount(idx[idx >= 0], minlength=n_params)
    offs = np.zeros(n_params + 1, dtype=np.int64)
    np.cumsum(counts, out=offs[1:])
    gates = order[:int(offs[-1])].astype(np.int32)
    return (torch.from_numpy(offs).to(device),
            torch.from_numpy(gates if gates.size else np.zeros(1, np.int32)).to(device))


def reduce_grad(offsets: torch.Tensor, gates: torch.Tensor, grad_theta: torch.Tensor,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/dparam_p = sum of dL/dtheta_j over the gates of p."""
    P = offsets.numel() - 1
    offs = _vec(offsets, "offsets", P + 1, torch.int64)
    if out is None:
        out = torch.empty(P, dtype=torch.float64, device=offs.device)
    L.check(L.lib().iqp_reduce_grad(P, _ptr(offs), _ptr(gates.contiguous()),
                                    _ptr(grad_theta.contiguous()), _ptr(out), _stream(offs)),
            "iqp_reduce_grad")
    return out


def optimizer_update(optimizer, params: torch.Tensor, grad: torch.Tensor,
                     m1: Optional[torch.Tensor], m2: Optional[torch.Tensor], step: torch.Tensor,
                     lr: float, beta1: float = 0.9, beta2: float = 0.999,
                     eps: float = 1e-8) -> None:
    """One update of params in place ('gd' or 'adam'), then step += 1."""
    P = params.numel()
    if not params.is_contiguous():
        raise ValueError("params must be contiguous (updated in place)")
    opt = _OPTIMIZERS[optimizer]
    L.check(L.lib().iqp_optimizer_update(opt, P, _ptr(params), _ptr(_vec(grad, "grad", P)),
                                         _ptr(m1), _ptr(m2), _ptr(_step_tensor(step)), lr, beta1,
                                         beta2, eps, _stream(params)), "iqp_optimizer_update")


class Trainer:
    """MMD^2 training on the device (iqp_train_* of include/iqp.h): every
    step draws fresh samples and operators (operator group g has
    ``group_ops[g]`` rows with bit probability ``group_prob[g]``, e.g. one
    group per Gaussian-kernel bandwidth), evaluates the loss and its gradient
    at the current parameters and updates them in place. ``param_index`` (host,
    one entry per generator) maps generators to parameters (shared
    parameters), -1 marking fixed gates whose angles are ``fixed_theta``.
    ``group_precision`` (one precision per group, or None for ``precision``
    everywhere, or "auto" to let the plan pick the sparse form for groups
    whose expected density of C is low) computes each group's loss and
    gradient by a call of its own, e.g. the sparse form for groups of
    low-weight operators. The trainer owns its workspace (optimizer moments
    and step count live there)."""

    def __init__(self, n_qubits: int, gens: torch.Tensor, param_index, n_params: int,
                 data: torch.Tensor, group_ops, group_prob, n_samples: int,
                 fixed_theta: Optional[torch.Tensor] = None, unbiased: bool = True,
                 precision=SPLIT_BF16, optimizer="adam", lr: float = 1e-3, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, seed=(0, 0), graph: bool = True,
                 step: int = 0, group_precision=None):
        import numpy as np
        self.n = int(n_qubits)
        self.W = (self.n + 63) // 64
        self.gens = _rows(gens, "gens", self.W)
        self.m = self.gens.shape[0]
        self.P = int(n_params)
        self.device = self.gens.device
        self.data = _rows(data, "data", self.W)
        idx = np.ascontiguousarray(param_index, dtype=np.int32)
        if idx.size != self.m:
            raise ValueError("param_index needs one entry per generator")
        self.fixed = _vec(fixed_theta, "fixed_theta", self.m) if fixed_theta is not None else None
        self.group_ops = np.ascontiguousarray(group_ops, dtype=np.int64)
        self.group_prob = np.ascontiguousarray(group_prob, dtype=np.float64)
        self.l = int(self.group_ops.sum())
        self.s = int(n_samples)
        s0, s1 = _seed(seed)
        d = L.IqpTrainDesc()
        d.n_qubits, d.n_words, d.n_gates, d.gens = self.n, self.W, self.m, self.gens.data_ptr()
        d.n_params = self.P
        d.param_index = idx.ctypes.data
        d.fixed_theta = self.fixed.data_ptr() if self.fixed is not None else None
        d.n_groups = self.group_ops.size
        d.group_ops = self.group_ops.ctypes.data
        d.group_prob = self.group_prob.ctypes.data
        d.n_samples, d.n_data, d.data = self.s, self.data.shape[0], self.data.data_ptr()
        d.unbiased, d.precision = int(bool(unbiased)), precision_id(precision)
        d.optimizer = _OPTIMIZERS[optimizer]
        d.lr, d.beta1, d.beta2, d.eps = lr, beta1, beta2, eps
        d.seed0, d.seed1 = s0, s1
        self.group_prec = None
        auto = isinstance(group_precision, str) and group_precision == "auto"
        if group_precision is not None and not auto:
            if len(group_precision) != self.group_ops.size:
                raise ValueError("group_precision needs one entry per group")
            self.group_prec = np.array([precision_id(p) for p in group_precision], dtype=np.int32)
            d.group_precision = self.group_prec.ctypes.data
        self._handle = ctypes.c_void_p()
        flags = (0 if graph else L.IQP_TRAIN_NO_GRAPH) | (L.IQP_TRAIN_AUTO_PRECISION if auto else 0)
        L.check(L.lib().iqp_train_plan_create(ctypes.byref(d), flags, ctypes.byref(self._handle)),
                "iqp_train_plan_create")
        self.ws_bytes = int(L.lib().iqp_train_workspace_bytes(self._handle))
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        self.grad = torch.zeros(self.P, dtype=torch.float64, device=self.device)
        self._loss = {}
        self.reset(step)

    def group_precisions(self):
        """The precision name each operator group runs in."""
        import numpy as np
        out = np.zeros(self.group_ops.size, dtype=np.int32)
        L.check(L.lib().iqp_train_group_precision(self._handle, out.ctypes.data),
                "iqp_train_group_precision")
        names = {v: k for k, v in _PRECISIONS.items() if isinstance(k, str)}
        return [names[int(p)] for p in out]

    def reset(self, step: int = 0) -> None:
        """Zero the optimizer moments and set the step count."""
        L.check(L.lib().iqp_train_init(self._handle, int(step), _ptr(self.ws), self.ws_bytes,
                                       _stream(self.ws)), "iqp_train_init")

    def step(self, params: torch.Tensor, n_steps: int = 1) -> torch.Tensor:
        """n_steps updates of params (in place); returns the loss of each step
        (a device tensor, overwritten by the next call with the same n_steps)
        and leaves the last step's parameter gradient in ``self.grad``."""
        if not params.is_contiguous() or params.numel() != self.P or \
                params.dtype != torch.float64 or not params.is_cuda:
            raise ValueError("params must be a contiguous CUDA float64 tensor of %d" % self.P)
        loss = self._loss.get(n_steps)
        if loss is None:
            loss = self._loss[n_steps] = torch.zeros(n_steps, dtype=torch.float64,
                                                     device=self.device)
        L.check(L.lib().iqp_train_step(self._handle, int(n_steps), _ptr(params), _ptr(loss),
                                       _ptr(self.grad), _ptr(self.ws), self.ws_bytes,
                                       _stream(params)), "iqp_train_step")
        return loss

    def buffers(self):
        """(samples [s][W], ops [l][W], step [1]) views of the workspace: the
        last step's draws and the step count."""
        z, a, t = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        L.check(L.lib().iqp_train_buffers(self._handle, _ptr(self.ws), ctypes.byref(z),
                                          ctypes.byref(a), ctypes.byref(t)), "iqp_train_buffers")
        base = self.ws.data_ptr()
        flat = self.ws.view(torch.int64)

        def view(ptr, count):
            off = (ptr - base) // 8
            return flat[off:off + count]
        return (view(z.value, self.s * self.W).view(self.s, self.W),
                view(a.value, self.l * self.W).view(self.l, self.W), view(t.value, 1))

    def close(self) -> None:
        if self._handle:
            torch.cuda.synchronize(self.device)
            L.lib().iqp_train_plan_destroy(self._handle)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
