// gfx950 kernels of the on-device training step (the optimisation loop of
// Sec. 3.3 with the MMD^2 loss of Sec. 3.3.1): counter-based random bits for
// the samples z and the operators a ~ P_sigma, the parameter-sharing gather
// and its gradient, and the optimizer update. All of them are small next to
// the loss and its gradient; they exist so that a whole step stays on the
// device, in one graph.
#include "iqp_train.h"

#include <math.h>

namespace iqp {

// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds, each
// multiplying counter words 0 and 2 by two odd constants into 128-bit
// products and mixing the halves with words 1, 3 and the key; the key is
// bumped by two Weyl constants between rounds.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kWeyl1 = 0xBB67AE8584CAA73Bull;

struct Block4 {
    uint64_t v0, v1, v2, v3;
};

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                uint64_t c3, uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t lo0 = kPhiloxM0 * c0, hi0 = __umul64hi(kPhiloxM0, c0);
        const uint64_t lo1 = kPhiloxM1 * c2, hi1 = __umul64hi(kPhiloxM1, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Block4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint64_t word_of(const Block4 &b, int e) {
    return e == 0 ? b.v0 : e == 1 ? b.v1 : e == 2 ? b.v2 : b.v3;
}

// One thread per Philox block: outputs 4b .. 4b + 3 are words of the
// row-major [rows][W] result, the last word of each row masked to n bits.
__global__ void __launch_bounds__(256) sample_uniform_kernel(SampleUniformArgs a) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t words = a.rows * a.W;
    if (4 * b >= words) return;
    const uint64_t t = (uint64_t)*a.step;
    const Block4 r = philox4x64_10((uint64_t)b, t, a.tag, 0, a.seed0, a.seed1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t o = 4 * b + e;
        if (o < words) {
            uint64_t v = word_of(r, e);
            if (o % a.W == a.W - 1) v &= a.tail_mask;
            a.out[o] = v;
        }
    }
}

// One thread per output word (row r, word w): qubits q of that word use
// outputs r n + q; each Philox block gives four of them.
__global__ void __launch_bounds__(256) sample_bernoulli_kernel(SampleBernoulliArgs a) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= a.rows * a.W) return;
    const int64_t r = idx / a.W;
    const int w = (int)(idx - r * a.W);
    int g = 0;
    while (g + 1 < a.n_groups && r >= a.row_end[g]) ++g;
    const uint64_t thr = a.threshold[g];
    const uint64_t t = (uint64_t)*a.step;
    const int q0 = 64 * w, q1 = min(a.n, q0 + 64);
    uint64_t bits = 0;
    int64_t cur = -1;
    Block4 blk{0, 0, 0, 0};
    for (int q = q0; q < q1; ++q) {
        const int64_t o = r * a.n + q;
        if ((o >> 2) != cur) {
            cur = o >> 2;
            blk = philox4x64_10((uint64_t)cur, t, a.tag, 0, a.seed0, a.seed1);
        }
        bits |= (uint64_t)(word_of(blk, (int)(o & 3)) < thr) << (q - q0);
    }
    a.out[idx] = bits;
}

__global__ void __launch_bounds__(256) gather_theta_kernel(int64_t m, const int32_t *index,
                                                           const double *params,
                                                           const double *fixed, double *theta) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    const int32_t p = index[j];
    theta[j] = p >= 0 ? params[p] : fixed[j];
}

__global__ void __launch_bounds__(256) reduce_grad_kernel(int64_t P, const int64_t *offsets,
                                                          const int32_t *gates,
                                                          const double *grad_theta,
                                                          double *grad_params) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    double acc = 0.0;
    for (int64_t t = offsets[p]; t < offsets[p + 1]; ++t) acc += grad_theta[gates[t]];
    grad_params[p] = acc;
}

// The loss and gradient of the operator groups, summed in group order: one
// thread per gate; thread 0 also sums the losses.
__global__ void __launch_bounds__(256) sum_groups_kernel(int32_t n_groups, int64_t m,
                                                         const double *loss_parts,
                                                         const double *grad_parts, double *loss,
                                                         double *grad_theta) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j == 0) {
        double l = 0.0;
        for (int g = 0; g < n_groups; ++g) l += loss_parts[g];
        *loss = l;
    }
    if (j >= m) return;
    double acc = 0.0;
    for (int g = 0; g < n_groups; ++g) acc += grad_parts[(int64_t)g * m + j];
    grad_theta[j] = acc;
}

// Gradient descent or Adam (Kingma and Ba 2015, Algorithm 1) at step count
// t + 1, t = *step, one thread per parameter. The step count is advanced by
// a separate launch, after every thread has read it.
__global__ void __launch_bounds__(256) optimizer_kernel(OptimizerArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.P) return;
    const double g = a.grad[p];
    if (a.opt == IQP_OPT_GD) {
        a.params[p] = a.params[p] - a.lr * g;
        return;
    }
    const double k = (double)(*a.step + 1);
    const double m1 = a.beta1 * a.m1[p] + (1.0 - a.beta1) * g;
    const double m2 = a.beta2 * a.m2[p] + (1.0 - a.beta2) * (g * g);
    a.m1[p] = m1;
    a.m2[p] = m2;
    const double mhat = m1 / (1.0 - pow(a.beta1, k));
    const double vhat = m2 / (1.0 - pow(a.beta2, k));
    a.params[p] = a.params[p] - (a.lr * mhat) / (sqrt(vhat) + a.eps);
}

__global__ void advance_step_kernel(int64_t *step) {
    if (threadIdx.x == 0) step[0] = step[0] + 1;
}

// Fills: zeroes doubles and sets the step count (used when a workspace is
// prepared, and capturable, unlike a memset node).
__global__ void __launch_bounds__(256) fill_f64_kernel(double *x, int64_t count, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = v;
}

__global__ void set_step_kernel(int64_t *step, int64_t v) {
    if (threadIdx.x == 0) step[0] = v;
}

static unsigned grid_of(int64_t count) { return (unsigned)ceil_div(count, (int64_t)256); }

hipError_t launch_sample_uniform(hipStream_t st, const SampleUniformArgs &a) {
    const int64_t blocks = ceil_div(a.rows * a.W, (int64_t)4);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(sample_uniform_kernel, dim3(grid_of(blocks)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sample_bernoulli(hipStream_t st, const SampleBernoulliArgs &a) {
    if (a.rows * a.W == 0) return hipSuccess;
    hipLaunchKernelGGL(sample_bernoulli_kernel, dim3(grid_of(a.rows * a.W)), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

hipError_t launch_gather_theta(hipStream_t st, int64_t m, const int32_t *index,
                               const double *params, const double *fixed, double *theta) {
    hipLaunchKernelGGL(gather_theta_kernel, dim3(grid_of(m)), dim3(256), 0, st, m, index, params,
                       fixed, theta);
    return hipGetLastError();
}

hipError_t launch_reduce_grad(hipStream_t st, int64_t P, const int64_t *offsets,
                              const int32_t *gates, const double *grad_theta,
                              double *grad_params) {
    hipLaunchKernelGGL(reduce_grad_kernel, dim3(grid_of(P)), dim3(256), 0, st, P, offsets, gates,
                       grad_theta, grad_params);
    return hipGetLastError();
}

hipError_t launch_sum_groups(hipStream_t st, int32_t n_groups, int64_t m,
                             const double *loss_parts, const double *grad_parts, double *loss,
                             double *grad_theta) {
    hipLaunchKernelGGL(sum_groups_kernel, dim3(grid_of(m)), dim3(256), 0, st, n_groups, m,
                       loss_parts, grad_parts, loss, grad_theta);
    return hipGetLastError();
}

hipError_t launch_optimizer(hipStream_t st, const OptimizerArgs &a) {
    hipLaunchKernelGGL(optimizer_kernel, dim3(grid_of(a.P)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, st, a.step);
    return hipGetLastError();
}

hipError_t launch_fill_f64(hipStream_t st, double *x, int64_t count, double v) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_of(count)), dim3(256), 0, st, x, count, v);
    return hipGetLastError();
}

hipError_t launch_set_step(hipStream_t st, int64_t *step, int64_t v) {
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, st, step, v);
    return hipGetLastError();
}

}  // namespace iqp
