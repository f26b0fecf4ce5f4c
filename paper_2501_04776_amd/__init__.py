"""MI355X-native Monte Carlo estimator of Pauli-Z expectation values of
parameterized IQP circuits, its gradient and an MMD^2 loss (arXiv 2501.04776).

The compute path is the gfx950 HIP library libiqp.so behind the C-ABI of
include/iqp.h; this package only marshals arguments to it.
"""
from . import packing
from ._lib import IqpError
from .api import (FP32, OPT_ADAM, OPT_GD, ROW_MAJOR, SPARSE_FP32, SPLIT_BF16, TILED32,
                  TILED32_T, BatchPlan, Circuit, Trainer, gather_theta, optimizer_update,
                  param_tables, reduce_grad, sample_bernoulli, sample_uniform,
                  iqp_bitflip_expval, iqp_bitflip_expval_grad, iqp_expval, iqp_expval_grad,
                  iqp_expval_indep, iqp_expval_indep_grad,
                  iqp_mmd_loss_grad, iqp_parity, profile_enable, profile_query, profile_reset,
                  workspace_bytes)
from .autograd import IQPBitflipExpval, IQPExpval, IQPMMDLoss

__all__ = ["packing", "IqpError", "FP32", "SPLIT_BF16", "SPARSE_FP32", "ROW_MAJOR", "TILED32",
           "TILED32_T", "BatchPlan", "Circuit", "Trainer", "OPT_GD", "OPT_ADAM", "gather_theta",
           "optimizer_update", "param_tables", "reduce_grad", "sample_bernoulli",
           "sample_uniform", "iqp_bitflip_expval", "iqp_bitflip_expval_grad", "iqp_expval",
           "iqp_expval_grad", "iqp_expval_indep", "iqp_expval_indep_grad", "iqp_mmd_loss_grad",
           "iqp_parity", "profile_enable", "profile_query", "profile_reset", "workspace_bytes",
           "IQPBitflipExpval", "IQPExpval", "IQPMMDLoss"]
