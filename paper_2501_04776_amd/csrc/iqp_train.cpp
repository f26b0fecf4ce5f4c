// Host runtime of the on-device training step: validation, the workspace
// layout of a training plan, and the graph that chains one step (sampling,
// parameter gather, MMD^2 loss and gradient, gradient reduction, optimizer
// update) on the device.
#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

#include "iqp_plan.h"
#include "iqp_train.h"

using namespace iqp;

namespace {

constexpr int32_t kMaxQubits = 1 << 20;
// Expected density of C below which a group runs in the sparse form: the
// sparse form's time grows with the non-zeros of C, the dense forms' does
// not, and on MI355X they cross at about 7-9 % (the sparse form 1.23x the
// dense time at 8 % and 11 %); 6 % leaves margin on the dense side. The MMD
// workload's groups sit at ~30 %, ~2 % and ~0.2 %.
constexpr double kSparseDensity = 0.06;

int check_seed_step(const int64_t *step, const uint64_t *out, int64_t rows) {
    if (!step) return fail(IQP_ERR_INVALID_ARG, "step is NULL");
    if (!out && rows > 0) return fail(IQP_ERR_INVALID_ARG, "out is NULL");
    return IQP_OK;
}

int check_groups(int32_t n_groups, const int64_t *group_rows, const double *group_prob,
                 int64_t *rows) {
    if (n_groups < 1 || n_groups > kMaxGroups)
        return fail(IQP_ERR_INVALID_ARG, "n_groups out of range [1, 16]");
    if (!group_rows || !group_prob)
        return fail(IQP_ERR_INVALID_ARG, "group_rows or group_prob is NULL");
    int64_t total = 0;
    for (int g = 0; g < n_groups; ++g) {
        if (group_rows[g] < 0 || group_rows[g] > kMaxRows)
            return fail(IQP_ERR_INVALID_ARG, "group_rows out of range [0, 2^24]");
        if (!(group_prob[g] >= 0.0 && group_prob[g] < 1.0))
            return fail(IQP_ERR_INVALID_ARG, "group_prob must lie in [0, 1)");
        total += group_rows[g];
    }
    if (total > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "more than 2^24 rows in all");
    *rows = total;
    return IQP_OK;
}

SampleUniformArgs uniform_args(int64_t rows, int32_t n, uint64_t seed0, uint64_t seed1,
                               const int64_t *step, uint64_t tag, uint64_t *out) {
    const int tail = n % 64;
    return SampleUniformArgs{rows,  ceil_div(n, 64), tail ? (1ull << tail) - 1 : ~0ull,
                             seed0, seed1,           tag,
                             step,  out};
}

SampleBernoulliArgs bernoulli_args(int32_t n, int32_t n_groups, const int64_t *group_rows,
                                   const double *group_prob, uint64_t seed0, uint64_t seed1,
                                   const int64_t *step, uint64_t tag, uint64_t *out) {
    SampleBernoulliArgs a{};
    a.W = ceil_div(n, 64);
    a.n = n;
    a.n_groups = n_groups;
    int64_t end = 0;
    for (int g = 0; g < n_groups; ++g) {
        end += group_rows[g];
        a.row_end[g] = end;
        // p * 2^64 is exact (a power-of-two scale) and below 2^64 for p < 1
        a.threshold[g] = (uint64_t)ldexp(group_prob[g], 64);
    }
    a.rows = end;
    a.seed0 = seed0;
    a.seed1 = seed1;
    a.tag = tag;
    a.step = step;
    a.out = out;
    return a;
}

int check_optimizer(int opt, double lr, double beta1, double beta2, double eps) {
    if (opt != IQP_OPT_GD && opt != IQP_OPT_ADAM)
        return fail(IQP_ERR_INVALID_ARG, "optimizer must be IQP_OPT_GD or IQP_OPT_ADAM");
    if (!(lr > 0.0) || !isfinite(lr)) return fail(IQP_ERR_INVALID_ARG, "lr must be > 0, finite");
    if (opt == IQP_OPT_ADAM) {
        if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
            return fail(IQP_ERR_INVALID_ARG, "beta1 and beta2 must lie in [0, 1)");
        if (!(eps >= 0.0) || !isfinite(eps))
            return fail(IQP_ERR_INVALID_ARG, "eps must be >= 0, finite");
    }
    return IQP_OK;
}

}  // namespace

struct iqp_train_plan {
    iqp_train_desc d{};
    int flags = 0;
    std::vector<int64_t> group_ops;
    std::vector<double> group_prob;
    // loss calls: consecutive groups of one precision share a call (their
    // operators and weights are contiguous); empty: one call in `precision`
    struct LossCall {
        int64_t first_op = 0, n_ops = 0;
        int32_t precision = 0;
    };
    std::vector<LossCall> calls;
    std::vector<int32_t> group_prec;  // the precision of each group
    int64_t l = 0, s = 0, W = 0, m = 0, P = 0;
    bool has_fixed = false;
    // workspace layout
    size_t o_z = 0, o_ops = 0, o_theta = 0, o_gtheta = 0, o_gpar = 0, o_m1 = 0, o_m2 = 0;
    size_t o_step = 0, o_tab = 0, tab_bytes = 0, o_mmd = 0, mmd_bytes = 0, total = 0;
    size_t o_lparts = 0, o_gparts = 0;  // per-group losses and gradients
    // offsets inside the table region (operator weights, parameter index,
    // gates of each parameter): the same bytes as the pinned staging copy
    size_t t_w = 0, t_index = 0, t_offs = 0, t_gates = 0;
    void *staging = nullptr;
    hipStream_t cap = nullptr;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        void *ws = nullptr;
        double *params = nullptr, *loss = nullptr, *grad = nullptr;
        int32_t n_steps = 0;
    } graph;
};

namespace {

template <typename T>
T *ws_at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

void destroy(iqp_train_plan *tp) {
    if (!tp) return;
    if (tp->graph.exec) (void)hipGraphExecDestroy(tp->graph.exec);
    if (tp->cap) (void)hipStreamDestroy(tp->cap);
    if (tp->staging) (void)hipHostFree(tp->staging);
    delete tp;
}

int check_ws(const iqp_train_plan *tp, void *ws, size_t ws_bytes) {
    if (!tp) return fail(IQP_ERR_INVALID_ARG, "plan is NULL");
    if (ws_bytes < tp->total)
        return fail(IQP_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) +
                                           " bytes, need " + std::to_string(tp->total));
    if (!ws) return fail(IQP_ERR_INVALID_ARG, "ws is NULL");
    return IQP_OK;
}

// One training step on stream `st`; loss_i receives its loss.
int enqueue_step(const iqp_train_plan *tp, void *ws, double *params, double *loss_i,
                 double *grad_out, hipStream_t st) {
    const iqp_train_desc &d = tp->d;
    int64_t *step = ws_at<int64_t>(ws, tp->o_step);
    uint64_t *z = ws_at<uint64_t>(ws, tp->o_z);
    uint64_t *ops = ws_at<uint64_t>(ws, tp->o_ops);
    double *theta = ws_at<double>(ws, tp->o_theta);
    double *gtheta = ws_at<double>(ws, tp->o_gtheta);
    double *gpar = grad_out ? grad_out : ws_at<double>(ws, tp->o_gpar);
    char *tab = ws_at<char>(ws, tp->o_tab);
    IQP_TRY(launch_sample_uniform(st, uniform_args(tp->s, d.n_qubits, d.seed0, d.seed1, step, 0,
                                                   z)),
            "sample_uniform");
    IQP_TRY(launch_sample_bernoulli(st, bernoulli_args(d.n_qubits, d.n_groups,
                                                       tp->group_ops.data(),
                                                       tp->group_prob.data(), d.seed0, d.seed1,
                                                       step, 1, ops)),
            "sample_bernoulli");
    IQP_TRY(launch_gather_theta(st, tp->m, reinterpret_cast<const int32_t *>(tab + tp->t_index),
                                params, d.fixed_theta, theta),
            "gather_theta");
    const iqp_circuit c{d.n_qubits, d.n_words, d.n_gates, d.gens, theta};
    const double *w = reinterpret_cast<const double *>(tab + tp->t_w);
    if (tp->calls.empty()) {
        const int rc = iqp_mmd_loss_grad(&c, tp->l, ops, w, tp->s, z, d.n_data, d.data,
                                         d.unbiased, d.precision, loss_i, gtheta,
                                         ws_at<char>(ws, tp->o_mmd), tp->mmd_bytes, st);
        if (rc) return rc;
    } else {
        // one call per run of groups in one precision, each into its own
        // loss and gradient slot, then summed in call order
        double *lparts = ws_at<double>(ws, tp->o_lparts);
        double *gparts = ws_at<double>(ws, tp->o_gparts);
        const int nc = (int)tp->calls.size();
        for (int i = 0; i < nc; ++i) {
            const auto &cl = tp->calls[i];
            const int rc = iqp_mmd_loss_grad(&c, cl.n_ops, ops + cl.first_op * tp->W,
                                             w + cl.first_op, tp->s, z, d.n_data, d.data,
                                             d.unbiased, cl.precision, lparts + i,
                                             gparts + i * tp->m, ws_at<char>(ws, tp->o_mmd),
                                             tp->mmd_bytes, st);
            if (rc) return rc;
        }
        IQP_TRY(launch_sum_groups(st, nc, tp->m, lparts, gparts, loss_i, gtheta), "sum_groups");
    }
    IQP_TRY(launch_reduce_grad(st, tp->P, reinterpret_cast<const int64_t *>(tab + tp->t_offs),
                               reinterpret_cast<const int32_t *>(tab + tp->t_gates), gtheta, gpar),
            "reduce_grad");
    IQP_TRY(launch_optimizer(st, OptimizerArgs{d.optimizer, tp->P, params, gpar,
                                               ws_at<double>(ws, tp->o_m1),
                                               ws_at<double>(ws, tp->o_m2), step, d.lr, d.beta1,
                                               d.beta2, d.eps}),
            "optimizer");
    return IQP_OK;
}

int step_graph(iqp_train_plan *tp, int32_t n_steps, double *params, double *loss, double *grad,
               void *ws, hipGraphExec_t *out) {
    auto &g = tp->graph;
    if (g.exec && g.ws == ws && g.params == params && g.loss == loss && g.grad == grad &&
        g.n_steps == n_steps) {
        *out = g.exec;
        return IQP_OK;
    }
    if (g.exec) {
        IQP_TRY(hipGraphExecDestroy(g.exec), "hipGraphExecDestroy");
        g.exec = nullptr;
    }
    IQP_TRY(hipStreamBeginCapture(tp->cap, hipStreamCaptureModeThreadLocal),
            "hipStreamBeginCapture");
    int st = IQP_OK;
    for (int32_t i = 0; i < n_steps && st == IQP_OK; ++i)
        st = enqueue_step(tp, ws, params, loss + i, grad, tp->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(tp->cap, &graph);
    if (st) {
        if (e == hipSuccess && graph) hipGraphDestroy(graph);
        return st;
    }
    IQP_TRY(e, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        g.exec = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
    }
    g.ws = ws;
    g.params = params;
    g.loss = loss;
    g.grad = grad;
    g.n_steps = n_steps;
    *out = g.exec;
    return IQP_OK;
}

}  // namespace

extern "C" {

int iqp_sample_uniform(int64_t rows, int32_t n_qubits, uint64_t seed0, uint64_t seed1,
                       const int64_t *step, uint64_t tag, uint64_t *out, void *stream) {
    clear_error();
    if (rows < 0 || rows > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "rows out of range [0, 2^24]");
    if (n_qubits < 1 || n_qubits > kMaxQubits)
        return fail(IQP_ERR_INVALID_ARG, "n_qubits out of range [1, 2^20]");
    int st = check_seed_step(step, out, rows);
    if (st || (st = check_device())) return st;
    IQP_TRY(launch_sample_uniform(reinterpret_cast<hipStream_t>(stream),
                                  uniform_args(rows, n_qubits, seed0, seed1, step, tag, out)),
            "sample_uniform");
    return IQP_OK;
}

int iqp_sample_bernoulli(int32_t n_qubits, int32_t n_groups, const int64_t *group_rows,
                         const double *group_prob, uint64_t seed0, uint64_t seed1,
                         const int64_t *step, uint64_t tag, uint64_t *out, void *stream) {
    clear_error();
    if (n_qubits < 1 || n_qubits > kMaxQubits)
        return fail(IQP_ERR_INVALID_ARG, "n_qubits out of range [1, 2^20]");
    int64_t rows = 0;
    int st = check_groups(n_groups, group_rows, group_prob, &rows);
    if (st || (st = check_seed_step(step, out, rows)) || (st = check_device())) return st;
    IQP_TRY(launch_sample_bernoulli(reinterpret_cast<hipStream_t>(stream),
                                    bernoulli_args(n_qubits, n_groups, group_rows, group_prob,
                                                   seed0, seed1, step, tag, out)),
            "sample_bernoulli");
    return IQP_OK;
}

int iqp_gather_theta(int64_t n_gates, const int32_t *param_index, const double *params,
                     const double *fixed_theta, double *theta, void *stream) {
    clear_error();
    if (n_gates < 1 || n_gates > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_gates out of range [1, 2^24]");
    if (!param_index || !params || !theta)
        return fail(IQP_ERR_INVALID_ARG, "param_index, params or theta is NULL");
    int st = check_device();
    if (st) return st;
    IQP_TRY(launch_gather_theta(reinterpret_cast<hipStream_t>(stream), n_gates, param_index,
                                params, fixed_theta, theta),
            "gather_theta");
    return IQP_OK;
}

int iqp_reduce_grad(int64_t n_params, const int64_t *param_offsets, const int32_t *param_gates,
                    const double *grad_theta, double *grad_params, void *stream) {
    clear_error();
    if (n_params < 1 || n_params > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_params out of range [1, 2^24]");
    if (!param_offsets || !param_gates || !grad_theta || !grad_params)
        return fail(IQP_ERR_INVALID_ARG,
                    "param_offsets, param_gates, grad_theta or grad_params is NULL");
    int st = check_device();
    if (st) return st;
    IQP_TRY(launch_reduce_grad(reinterpret_cast<hipStream_t>(stream), n_params, param_offsets,
                               param_gates, grad_theta, grad_params),
            "reduce_grad");
    return IQP_OK;
}

int iqp_optimizer_update(int optimizer, int64_t n_params, double *params, const double *grad,
                         double *m1, double *m2, int64_t *step, double lr, double beta1,
                         double beta2, double eps, void *stream) {
    clear_error();
    if (n_params < 1 || n_params > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_params out of range [1, 2^24]");
    int st = check_optimizer(optimizer, lr, beta1, beta2, eps);
    if (st) return st;
    if (!params || !grad || !step)
        return fail(IQP_ERR_INVALID_ARG, "params, grad or step is NULL");
    if (optimizer == IQP_OPT_ADAM && (!m1 || !m2))
        return fail(IQP_ERR_INVALID_ARG, "Adam needs m1 and m2");
    if ((st = check_device())) return st;
    IQP_TRY(launch_optimizer(reinterpret_cast<hipStream_t>(stream),
                             OptimizerArgs{optimizer, n_params, params, grad, m1, m2, step, lr,
                                           beta1, beta2, eps}),
            "optimizer");
    return IQP_OK;
}

int iqp_train_plan_create(const iqp_train_desc *desc, int flags, iqp_train_plan **plan) {
    clear_error();
    if (!plan) return fail(IQP_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    if (!desc) return fail(IQP_ERR_INVALID_ARG, "desc is NULL");
    const iqp_train_desc &d = *desc;
    if (flags & ~(int)(IQP_TRAIN_NO_GRAPH | IQP_TRAIN_AUTO_PRECISION))
        return fail(IQP_ERR_INVALID_ARG, "unknown flags");
    if ((flags & IQP_TRAIN_AUTO_PRECISION) && d.group_precision)
        return fail(IQP_ERR_INVALID_ARG, "IQP_TRAIN_AUTO_PRECISION needs group_precision NULL");
    if (d.n_qubits < 1 || d.n_qubits > kMaxQubits)
        return fail(IQP_ERR_INVALID_ARG, "n_qubits out of range [1, 2^20]");
    if (d.n_words != (int32_t)ceil_div(d.n_qubits, 64))
        return fail(IQP_ERR_INVALID_ARG, "n_words must equal ceil(n_qubits / 64)");
    if (d.n_gates < 1 || d.n_gates > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_gates out of range [1, 2^24]");
    if (!d.gens) return fail(IQP_ERR_INVALID_ARG, "gens is NULL");
    if (d.n_params < 1 || d.n_params > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_params out of range [1, 2^24]");
    if (!d.param_index) return fail(IQP_ERR_INVALID_ARG, "param_index is NULL");
    int64_t l = 0;
    int st = check_groups(d.n_groups, d.group_ops, d.group_prob, &l);
    if (st) return st;
    for (int g = 0; g < d.n_groups; ++g)
        if (d.group_ops[g] < 1) return fail(IQP_ERR_INVALID_ARG, "group_ops must be >= 1");
    if (d.n_samples < 1 || d.n_samples > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_samples out of range [1, 2^24]");
    if (d.n_data < 1 || d.n_data > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_data out of range [1, 2^24]");
    if (!d.data) return fail(IQP_ERR_INVALID_ARG, "data is NULL");
    if (d.unbiased && (d.n_data < 2 || d.n_samples < 2))
        return fail(IQP_ERR_INVALID_ARG, "the unbiased estimator needs N >= 2 and s >= 2");
    if (!valid_precision(d.precision))
        return fail(IQP_ERR_INVALID_ARG, "precision must be IQP_FP32, IQP_SPLIT_BF16, "
                                         "IQP_SPARSE_FP32, IQP_SPLIT3_BF16 or "
                                         "IQP_SPLIT_BF16_FP8");
    if ((st = check_optimizer(d.optimizer, d.lr, d.beta1, d.beta2, d.eps))) return st;
    if (d.group_precision)
        for (int g = 0; g < d.n_groups; ++g) {
            const int32_t p = d.group_precision[g];
            if (!valid_precision(p))
                return fail(IQP_ERR_INVALID_ARG, "group_precision[" + std::to_string(g) +
                                                     "] must be IQP_FP32, IQP_SPLIT_BF16, "
                                                     "IQP_SPARSE_FP32, IQP_SPLIT3_BF16 or "
                                                     "IQP_SPLIT_BF16_FP8");
        }
    // gates of each parameter, in gate order
    std::vector<int64_t> offs(d.n_params + 1, 0);
    bool has_fixed = false;
    for (int64_t j = 0; j < d.n_gates; ++j) {
        const int32_t p = d.param_index[j];
        if (p < -1 || p >= d.n_params)
            return fail(IQP_ERR_INVALID_ARG, "param_index[" + std::to_string(j) +
                                                 "] out of range [-1, n_params)");
        if (p < 0) has_fixed = true;
        else ++offs[p + 1];
    }
    if (has_fixed && !d.fixed_theta)
        return fail(IQP_ERR_INVALID_ARG, "fixed_theta is NULL but some gates are fixed");
    for (int64_t p = 0; p < d.n_params; ++p) offs[p + 1] += offs[p];
    std::vector<int32_t> gates(std::max<int64_t>(offs[d.n_params], 1), 0);
    {
        std::vector<int64_t> fillp(offs.begin(), offs.end() - 1);
        for (int64_t j = 0; j < d.n_gates; ++j)
            if (d.param_index[j] >= 0) gates[fillp[d.param_index[j]]++] = (int32_t)j;
    }
    if ((st = check_device())) return st;

    iqp_train_plan *tp = new iqp_train_plan();
    tp->d = d;
    tp->flags = flags;
    tp->group_ops.assign(d.group_ops, d.group_ops + d.n_groups);
    tp->group_prob.assign(d.group_prob, d.group_prob + d.n_groups);
    std::vector<int32_t> prec(d.n_groups, d.precision);
    if (d.group_precision) prec.assign(d.group_precision, d.group_precision + d.n_groups);
    if (flags & IQP_TRAIN_AUTO_PRECISION) {
        // expected density of C per group from the generators' weights
        std::vector<uint64_t> g((size_t)d.n_gates * d.n_words);
        const hipError_t e = hipMemcpy(g.data(), d.gens, g.size() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            destroy(tp);
            return hip_fail(e, "copy of the generators");
        }
        // generators per weight; pad bits past n_qubits are masked off (they
        // must be zero, but they are not checked, and must not index past
        // the table)
        std::vector<int64_t> count(d.n_qubits + 1, 0);
        const int tail = d.n_qubits & 63;
        const uint64_t last_mask = tail ? ((1ull << tail) - 1) : ~0ull;
        for (int64_t j = 0; j < d.n_gates; ++j) {
            int w = 0;
            for (int32_t k = 0; k < d.n_words; ++k) {
                uint64_t x = g[j * d.n_words + k];
                if (k == d.n_words - 1) x &= last_mask;
                w += __builtin_popcountll(x);
            }
            ++count[w];
        }
        for (int gi = 0; gi < d.n_groups; ++gi) {
            const double q = 1.0 - 2.0 * tp->group_prob[gi];
            double dens = 0.0;
            for (int w = 0; w <= d.n_qubits; ++w)
                if (count[w]) dens += (double)count[w] * 0.5 * (1.0 - std::pow(q, w));
            dens /= (double)d.n_gates;
            prec[gi] = dens < kSparseDensity ? IQP_SPARSE_FP32 : d.precision;
        }
    }
    tp->group_prec = prec;
    if (d.group_precision || (flags & IQP_TRAIN_AUTO_PRECISION)) {
        int64_t off = 0;
        for (int g = 0; g < d.n_groups; ++g) {
            if (g > 0 && prec[g] == prec[g - 1])
                tp->calls.back().n_ops += tp->group_ops[g];
            else
                tp->calls.push_back({off, tp->group_ops[g], prec[g]});
            off += tp->group_ops[g];
        }
    }
    tp->d.group_ops = nullptr;  // host arrays are the plan's copies from here on
    tp->d.group_prob = nullptr;
    tp->d.param_index = nullptr;
    tp->d.group_precision = nullptr;
    tp->l = l;
    tp->s = d.n_samples;
    tp->W = d.n_words;
    tp->m = d.n_gates;
    tp->P = d.n_params;
    tp->has_fixed = has_fixed;

    size_t cur = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = cur;
        cur += (bytes + 255) & ~(size_t)255;
        return o;
    };
    tp->o_z = carve((size_t)tp->s * tp->W * 8);
    tp->o_ops = carve((size_t)tp->l * tp->W * 8);
    tp->o_theta = carve((size_t)tp->m * 8);
    tp->o_gtheta = carve((size_t)tp->m * 8);
    tp->o_gpar = carve((size_t)tp->P * 8);
    tp->o_m1 = carve((size_t)tp->P * 8);
    tp->o_m2 = carve((size_t)tp->P * 8);
    tp->o_step = carve(8);
    size_t tcur = 0;
    auto tcarve = [&](size_t bytes) {
        const size_t o = tcur;
        tcur += (bytes + 255) & ~(size_t)255;
        return o;
    };
    tp->t_w = tcarve((size_t)tp->l * 8);
    tp->t_index = tcarve((size_t)tp->m * 4);
    tp->t_offs = tcarve((size_t)(tp->P + 1) * 8);
    tp->t_gates = tcarve(gates.size() * 4);
    tp->tab_bytes = tcur;
    tp->o_tab = carve(tp->tab_bytes);
    const iqp_circuit c{d.n_qubits, d.n_words, d.n_gates, d.gens, nullptr};
    if (tp->calls.empty()) {
        tp->mmd_bytes = iqp_workspace_bytes(IQP_CALL_MMD_GRAD, &c, tp->l, tp->s, d.n_data,
                                            d.precision);
    } else {
        // the loss calls run one after another on the stream and share it
        for (const auto &cl : tp->calls) {
            const size_t b = iqp_workspace_bytes(IQP_CALL_MMD_GRAD, &c, cl.n_ops, tp->s,
                                                 d.n_data, cl.precision);
            if (b == 0) {
                tp->mmd_bytes = 0;
                break;
            }
            tp->mmd_bytes = std::max(tp->mmd_bytes, b);
        }
        tp->o_lparts = carve(tp->calls.size() * 8);
        tp->o_gparts = carve(tp->calls.size() * tp->m * 8);
    }
    if (tp->mmd_bytes == 0) {
        destroy(tp);
        return fail(IQP_ERR_INVALID_ARG, "loss workspace size query failed");
    }
    tp->o_mmd = carve(tp->mmd_bytes);
    tp->total = cur;

    if ((st = injected_fault("alloc"))) {
        destroy(tp);
        return st;
    }
    hipError_t e = hipHostMalloc(&tp->staging, tp->tab_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&tp->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy(tp);
        return hip_fail(e, "plan resources");
    }
    char *stg = static_cast<char *>(tp->staging);
    double *w = reinterpret_cast<double *>(stg + tp->t_w);
    int64_t r = 0;
    for (int g = 0; g < d.n_groups; ++g)
        for (int64_t i = 0; i < tp->group_ops[g]; ++i)
            w[r++] = 1.0 / ((double)d.n_groups * (double)tp->group_ops[g]);
    std::copy(desc->param_index, desc->param_index + d.n_gates,
              reinterpret_cast<int32_t *>(stg + tp->t_index));
    std::copy(offs.begin(), offs.end(), reinterpret_cast<int64_t *>(stg + tp->t_offs));
    std::copy(gates.begin(), gates.end(), reinterpret_cast<int32_t *>(stg + tp->t_gates));
    *plan = tp;
    return IQP_OK;
}

int iqp_train_plan_destroy(iqp_train_plan *plan) {
    destroy(plan);
    return IQP_OK;
}

size_t iqp_train_workspace_bytes(const iqp_train_plan *plan) { return plan ? plan->total : 0; }

int iqp_train_init(iqp_train_plan *plan, int64_t step, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int st = check_ws(plan, ws, ws_bytes);
    if (st) return st;
    if (step < 0) return fail(IQP_ERR_INVALID_ARG, "step must be >= 0");
    if ((st = check_device())) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    IQP_TRY(hipMemcpyAsync(ws_at<char>(ws, plan->o_tab), plan->staging, plan->tab_bytes,
                           hipMemcpyHostToDevice, s),
            "table upload");
    IQP_TRY(launch_fill_f64(s, ws_at<double>(ws, plan->o_m1), plan->P, 0.0), "zero m1");
    IQP_TRY(launch_fill_f64(s, ws_at<double>(ws, plan->o_m2), plan->P, 0.0), "zero m2");
    IQP_TRY(launch_set_step(s, ws_at<int64_t>(ws, plan->o_step), step), "set step");
    return IQP_OK;
}

int iqp_train_step(iqp_train_plan *plan, int32_t n_steps, double *params, double *loss,
                   double *grad_params, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int st = check_ws(plan, ws, ws_bytes);
    if (st) return st;
    if (n_steps < 1 || n_steps > 4096)
        return fail(IQP_ERR_INVALID_ARG, "n_steps out of range [1, 4096]");
    if (!params || !loss) return fail(IQP_ERR_INVALID_ARG, "params or loss is NULL");
    if ((st = check_device())) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((plan->flags & IQP_TRAIN_NO_GRAPH) || timing_enabled()) {
        for (int32_t i = 0; i < n_steps; ++i)
            if ((st = enqueue_step(plan, ws, params, loss + i, grad_params, s))) return st;
        return IQP_OK;
    }
    hipGraphExec_t exec = nullptr;
    if ((st = step_graph(plan, n_steps, params, loss, grad_params, ws, &exec))) return st;
    IQP_TRY(hipGraphLaunch(exec, s), "hipGraphLaunch");
    return IQP_OK;
}

int iqp_train_group_precision(const iqp_train_plan *plan, int32_t *out) {
    clear_error();
    if (!plan) return fail(IQP_ERR_INVALID_ARG, "plan is NULL");
    if (!out) return fail(IQP_ERR_INVALID_ARG, "out is NULL");
    std::copy(plan->group_prec.begin(), plan->group_prec.end(), out);
    return IQP_OK;
}

int iqp_train_buffers(const iqp_train_plan *plan, void *ws, uint64_t **samples, uint64_t **ops,
                      int64_t **step) {
    clear_error();
    if (!plan) return fail(IQP_ERR_INVALID_ARG, "plan is NULL");
    if (!ws) return fail(IQP_ERR_INVALID_ARG, "ws is NULL");
    if (samples) *samples = ws_at<uint64_t>(ws, plan->o_z);
    if (ops) *ops = ws_at<uint64_t>(ws, plan->o_ops);
    if (step) *step = ws_at<int64_t>(ws, plan->o_step);
    return IQP_OK;
}

}  // extern "C"
