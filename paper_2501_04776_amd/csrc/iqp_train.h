// Internal interface between the training runtime (iqp_train.cpp) and its
// kernels (iqp_train_kernels.hip). Not installed; the public ABI is
// include/iqp.h.
#pragma once

#include "iqp.h"
#include "iqp_internal.h"

namespace iqp {

// Bernoulli row groups per launch (one per kernel bandwidth).
constexpr int kMaxGroups = 16;

struct SampleUniformArgs {
    int64_t rows, W;
    uint64_t tail_mask;  // bits of the last word of a row that hold qubits
    uint64_t seed0, seed1, tag;
    const int64_t *step;
    uint64_t *out;
};

struct SampleBernoulliArgs {
    int64_t rows, W;
    int n, n_groups;
    int64_t row_end[kMaxGroups];     // exclusive end row of each group
    uint64_t threshold[kMaxGroups];  // floor(p * 2^64) of each group
    uint64_t seed0, seed1, tag;
    const int64_t *step;
    uint64_t *out;
};

struct OptimizerArgs {
    int opt;
    int64_t P;
    double *params;
    const double *grad;
    double *m1, *m2;
    int64_t *step;
    double lr, beta1, beta2, eps;
};

hipError_t launch_sample_uniform(hipStream_t st, const SampleUniformArgs &a);
hipError_t launch_sample_bernoulli(hipStream_t st, const SampleBernoulliArgs &a);
hipError_t launch_gather_theta(hipStream_t st, int64_t m, const int32_t *index,
                               const double *params, const double *fixed, double *theta);
hipError_t launch_reduce_grad(hipStream_t st, int64_t P, const int64_t *offsets,
                              const int32_t *gates, const double *grad_theta,
                              double *grad_params);
// the update, then step += 1
hipError_t launch_sum_groups(hipStream_t st, int32_t n_groups, int64_t m,
                             const double *loss_parts, const double *grad_parts, double *loss,
                             double *grad_theta);
hipError_t launch_optimizer(hipStream_t st, const OptimizerArgs &a);
hipError_t launch_fill_f64(hipStream_t st, double *x, int64_t count, double v);
hipError_t launch_set_step(hipStream_t st, int64_t *step, int64_t v);

}  // namespace iqp
