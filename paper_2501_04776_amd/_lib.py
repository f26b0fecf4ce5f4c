"""ctypes loader for libiqp.so (the C-ABI of include/iqp.h).

The library must have been built in-tree (``python -m
paper_2501_04776_amd.build`` or ``__graft_entry__.build()``). There is no
fallback: if it is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# IQP_LIBRARY_PATH names another build of the same sources (the sanitizer
# build of the tests); it must embed the same source hash
LIB_PATH = os.environ.get("IQP_LIBRARY_PATH") or os.path.join(_HERE, "libiqp.so")

IQP_OK = 0
IQP_ERR_INVALID_ARG = -1
IQP_ERR_WORKSPACE = -2
IQP_ERR_HIP = -3
IQP_ERR_UNSUPPORTED = -4

IQP_FP32 = 0
IQP_SPLIT_BF16 = 1
IQP_SPARSE_FP32 = 2
IQP_SPLIT3_BF16 = 3
IQP_SPLIT_BF16_FP8 = 4

IQP_CALL_EXPVAL = 0
IQP_CALL_EXPVAL_GRAD = 1
IQP_CALL_EXPVAL_GRAD_RECOMPUTE = 2
IQP_CALL_MMD = 3
IQP_CALL_MMD_GRAD = 4
IQP_CALL_BITFLIP = 5
IQP_CALL_BITFLIP_GRAD = 6
IQP_CALL_INDEP = 7
IQP_CALL_INDEP_GRAD = 8
IQP_CALL_INDEP_GRAD_RECOMPUTE = 9

IQP_BITS_ROW_MAJOR = 0
IQP_BITS_TILED32 = 1
IQP_BITS_TILED32_T = 2

# every symbol include/iqp.h declares
EXPORTED = ("iqp_workspace_bytes", "iqp_parity_workspace_bytes", "iqp_parity", "iqp_expval",
            "iqp_expval_noalloc",
            "iqp_expval_grad", "iqp_expval_indep", "iqp_expval_indep_grad",
            "iqp_mmd_loss_grad", "iqp_bitflip_expval",
            "iqp_bitflip_expval_grad", "iqp_batch_plan_create",
            "iqp_batch_plan_destroy", "iqp_batch_workspace_bytes", "iqp_batch_expval",
            "iqp_batch_expval_grad", "iqp_batch_tune", "iqp_batch_get_config",
            "iqp_batch_set_config", "iqp_sample_uniform", "iqp_sample_bernoulli",
            "iqp_gather_theta", "iqp_reduce_grad", "iqp_optimizer_update",
            "iqp_train_plan_create", "iqp_train_plan_destroy", "iqp_train_workspace_bytes",
            "iqp_train_init", "iqp_train_step", "iqp_train_buffers", "iqp_train_group_precision",
            "iqp_source_sha256", "iqp_strerror", "iqp_last_error", "iqp_profile_enable",
            "iqp_profile_query", "iqp_profile_reset")

IQP_BATCH_NO_GRAPH = 1
IQP_TRAIN_NO_GRAPH = 1
IQP_TRAIN_AUTO_PRECISION = 2
IQP_OPT_GD = 0
IQP_OPT_ADAM = 1


class IqpCircuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_words", ctypes.c_int32),
                ("n_gates", ctypes.c_int64), ("gens", ctypes.c_void_p),
                ("theta", ctypes.c_void_p)]


class IqpProblem(ctypes.Structure):
    _fields_ = [("circuit", IqpCircuit), ("n_ops", ctypes.c_int64), ("ops", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64), ("samples", ctypes.c_void_p),
                ("mean", ctypes.c_void_p), ("stderr_", ctypes.c_void_p),
                ("phase_save", ctypes.c_void_p), ("grad_mean", ctypes.c_void_p),
                ("grad_theta", ctypes.c_void_p)]


class IqpTrainDesc(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_words", ctypes.c_int32),
                ("n_gates", ctypes.c_int64), ("gens", ctypes.c_void_p),
                ("n_params", ctypes.c_int64), ("param_index", ctypes.c_void_p),
                ("fixed_theta", ctypes.c_void_p), ("n_groups", ctypes.c_int32),
                ("group_ops", ctypes.c_void_p), ("group_prob", ctypes.c_void_p),
                ("n_samples", ctypes.c_int64), ("n_data", ctypes.c_int64),
                ("data", ctypes.c_void_p), ("unbiased", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("optimizer", ctypes.c_int32),
                ("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("seed0", ctypes.c_uint64), ("seed1", ctypes.c_uint64),
                ("group_precision", ctypes.c_void_p)]


class IqpError(RuntimeError):
    def __init__(self, status, what, detail):
        super().__init__("%s failed: %s (%d)%s" % (what, strerror(status), status,
                                                   (": " + detail) if detail else ""))
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libiqp.so is not built at %s; run `python -m "
                           "paper_2501_04776_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    # refuse a binary built from other sources than the ones beside it
    from .build import source_sha256
    L.iqp_source_sha256.argtypes = []
    L.iqp_source_sha256.restype = ctypes.c_char_p
    built, here = L.iqp_source_sha256().decode(), source_sha256()
    if built != here:
        raise RuntimeError("libiqp.so at %s was built from other sources (built %s, sources %s); "
                           "rebuild with `python -m paper_2501_04776_amd.build`" %
                           (LIB_PATH, built[:16], here[:16]))
    i32, i64, vp, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    cp = ctypes.POINTER(IqpCircuit)
    L.iqp_workspace_bytes.argtypes = [i32, cp, i64, i64, i64, i32]
    L.iqp_workspace_bytes.restype = sz
    L.iqp_parity_workspace_bytes.argtypes = [i64, i64, ctypes.c_int32, i32]
    L.iqp_parity_workspace_bytes.restype = sz
    L.iqp_parity.argtypes = [i64, vp, i64, vp, ctypes.c_int32, i32, vp, vp, sz, vp]
    L.iqp_parity.restype = i32
    L.iqp_expval.argtypes = [cp, i64, vp, i64, vp, i32, vp, vp, vp, vp, sz, vp]
    L.iqp_expval.restype = i32
    L.iqp_expval_noalloc.argtypes = [cp, i64, vp, i64, vp, i32, vp, vp, vp, vp]
    L.iqp_expval_noalloc.restype = i32
    L.iqp_expval_grad.argtypes = [cp, i64, vp, i64, vp, i32, vp, vp, vp, vp, sz, vp]
    L.iqp_expval_grad.restype = i32
    L.iqp_expval_indep.argtypes = [cp, i64, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    L.iqp_expval_indep.restype = i32
    L.iqp_expval_indep_grad.argtypes = [cp, i64, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    L.iqp_expval_indep_grad.restype = i32
    L.iqp_mmd_loss_grad.argtypes = [cp, i64, vp, vp, i64, vp, i64, vp, i32, i32, vp, vp, vp,
                                    sz, vp]
    L.iqp_mmd_loss_grad.restype = i32
    L.iqp_bitflip_expval.argtypes = [cp, i64, vp, vp, vp, sz, vp]
    L.iqp_bitflip_expval.restype = i32
    L.iqp_bitflip_expval_grad.argtypes = [cp, i64, vp, vp, vp, vp, sz, vp]
    L.iqp_bitflip_expval_grad.restype = i32
    pp = ctypes.POINTER(IqpProblem)
    L.iqp_batch_plan_create.argtypes = [ctypes.c_int32, pp, i32, i32, ctypes.POINTER(vp)]
    L.iqp_batch_plan_create.restype = i32
    L.iqp_batch_plan_destroy.argtypes = [vp]
    L.iqp_batch_plan_destroy.restype = i32
    L.iqp_batch_workspace_bytes.argtypes = [vp]
    L.iqp_batch_workspace_bytes.restype = sz
    L.iqp_batch_expval.argtypes = [vp, pp, vp, sz, vp]
    L.iqp_batch_expval.restype = i32
    L.iqp_batch_expval_grad.argtypes = [vp, pp, vp, sz, vp]
    L.iqp_batch_expval_grad.restype = i32
    L.iqp_batch_tune.argtypes = [vp, pp, i32, vp, sz, vp]
    L.iqp_batch_tune.restype = i32
    L.iqp_batch_get_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.iqp_batch_get_config.restype = i32
    L.iqp_batch_set_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.iqp_batch_set_config.restype = i32
    u64, dbl = ctypes.c_uint64, ctypes.c_double
    L.iqp_sample_uniform.argtypes = [i64, ctypes.c_int32, u64, u64, vp, u64, vp, vp]
    L.iqp_sample_uniform.restype = i32
    L.iqp_sample_bernoulli.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, u64, u64, vp, u64,
                                       vp, vp]
    L.iqp_sample_bernoulli.restype = i32
    L.iqp_gather_theta.argtypes = [i64, vp, vp, vp, vp, vp]
    L.iqp_gather_theta.restype = i32
    L.iqp_reduce_grad.argtypes = [i64, vp, vp, vp, vp, vp]
    L.iqp_reduce_grad.restype = i32
    L.iqp_optimizer_update.argtypes = [i32, i64, vp, vp, vp, vp, vp, dbl, dbl, dbl, dbl, vp]
    L.iqp_optimizer_update.restype = i32
    L.iqp_train_plan_create.argtypes = [ctypes.POINTER(IqpTrainDesc), i32, ctypes.POINTER(vp)]
    L.iqp_train_plan_create.restype = i32
    L.iqp_train_plan_destroy.argtypes = [vp]
    L.iqp_train_plan_destroy.restype = i32
    L.iqp_train_workspace_bytes.argtypes = [vp]
    L.iqp_train_workspace_bytes.restype = sz
    L.iqp_train_init.argtypes = [vp, i64, vp, sz, vp]
    L.iqp_train_init.restype = i32
    L.iqp_train_step.argtypes = [vp, ctypes.c_int32, vp, vp, vp, vp, sz, vp]
    L.iqp_train_step.restype = i32
    L.iqp_train_buffers.argtypes = [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(vp)]
    L.iqp_train_buffers.restype = i32
    L.iqp_train_group_precision.argtypes = [vp, vp]
    L.iqp_train_group_precision.restype = i32
    L.iqp_strerror.argtypes = [i32]
    L.iqp_strerror.restype = ctypes.c_char_p
    L.iqp_last_error.argtypes = []
    L.iqp_last_error.restype = ctypes.c_char_p
    L.iqp_profile_enable.argtypes = [i32]
    L.iqp_profile_enable.restype = i32
    L.iqp_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64)]
    L.iqp_profile_query.restype = i32
    L.iqp_profile_reset.argtypes = []
    L.iqp_profile_reset.restype = i32
    _lib = L
    return L


def strerror(status: int) -> str:
    return lib().iqp_strerror(status).decode()


def last_error() -> str:
    return lib().iqp_last_error().decode()


def check(status: int, what: str) -> None:
    if status != IQP_OK:
        raise IqpError(status, what, last_error())
