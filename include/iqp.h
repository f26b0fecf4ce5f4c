/*
 * iqp.h — C-ABI of the MI355X (gfx950) Monte Carlo estimator of Pauli-Z
 * expectation values of parameterized IQP circuits (arXiv 2501.04776).
 *
 * The method (Sec. 2.1-2.2, Prop. 1-2 of the paper): an n-qubit circuit of m
 * commuting gates exp(i theta_j X_{g_j}) acting on |0>, and l observables
 * Z_{a_k}. For s bitstrings z_i the estimator of <Z_{a_k}> is
 *     mean_k = (1/s) sum_i cos(E_ki),   E = C Theta B^T            (eq. Emat)
 * with B_ij = (-1)^{z_i . g_j}, C_kj = 1 - (-1)^{a_k . g_j} in {0, 2}, and
 * Theta = diag(theta). Each call runs three GPU steps — bit-exact parity
 * matrices, the phase contraction E, and a cos / mean / standard-error
 * reduction — plus, for the gradient, the transposed contraction.
 *
 * Conventions shared by every entry point
 *   - Bit rows: a binary vector of n qubits is packed into W = ceil(n/64)
 *     little-endian uint64 words; qubit q is bit (q & 63) of word (q >> 6).
 *     Bits at positions >= n ("pad bits") must be zero; they are not checked
 *     on the device.
 *   - Pointers marked "device" must be device (or managed) memory readable
 *     from the GPU that is current when the call is made. The caller owns all
 *     memory, including the workspace; the library keeps no pointer after a
 *     call returns. Pointers marked "host" are read before the call returns.
 *   - Every call validates its arguments on the host before it enqueues any
 *     work and returns IQP_ERR_INVALID_ARG / IQP_ERR_WORKSPACE without touching
 *     the GPU. Otherwise all work is enqueued asynchronously on `stream` (a
 *     hipStream_t; NULL = the default stream) and the call returns before it
 *     completes. Results are valid once the stream has been synchronised.
 *   - HIP failures return IQP_ERR_HIP; iqp_last_error() gives the text.
 *   - Calls are deterministic: the same inputs, precision and device give
 *     bitwise-identical outputs (fixed-order reductions, no float atomics).
 *   - Non-finite theta propagates NaN into the results.
 *   - Calls that share one workspace must not overlap in time.
 */
#ifndef IQP_H
#define IQP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IQP_OK = 0,
    IQP_ERR_INVALID_ARG = -1, /* a null pointer, a size out of range, n/W mismatch */
    IQP_ERR_WORKSPACE = -2,   /* ws_bytes smaller than iqp_workspace_bytes() */
    IQP_ERR_HIP = -3,         /* a HIP runtime call failed (see iqp_last_error) */
    IQP_ERR_UNSUPPORTED = -4  /* an option the library does not implement */
} iqp_status;

/* Arithmetic of the phase contraction E = C Theta B^T.
 *   IQP_FP32:        2 theta_j in FP32, one FP32 matrix-core product per term.
 *   IQP_SPLIT_BF16:  2 theta_j = hi + lo with hi, lo BF16 (round to nearest
 *                    even), two BF16 matrix-core products per term (the +-1
 *                    and 0/1 parity operands are exact in BF16), FP32
 *                    accumulation. 2 theta_j keeps 16 significant bits: the
 *                    means meet 1e-4, but each gate's residual (up to
 *                    2^-16 |2 theta_j|) repeats in every sample's phase, so
 *                    with many anticommuting gates and many weighted
 *                    observables the gradient can exceed 1e-4 * max(1, |g|).
 *                    The backward weights S (below) are hi + lo BF16 too.
 *   IQP_SPLIT3_BF16: 2 theta_j = hi + mid + lo: hi and mid BF16 limbs, lo the
 *                    FP8 E4M3 rounding of what they leave, scaled by 2^20
 *                    (the product's scale operand takes it back); error at
 *                    most 2^-20 |2 theta_j| + 2^-30. Per term two BF16
 *                    products and one FP8 product (at twice the BF16 rate)
 *                    in the forward, FP32 accumulation.
 *                    The backward weights S_ki = dL/dcos(E_ki) sin(E_ki) are
 *                    held in 16-bit fixed point per observable,
 *                    S_ki ~ q_k (256 d1_ki + d0_ki) with signed 8-bit limbs,
 *                    q_k = bound_k / 32639 (bound_k = |a_k| + |b_k| >= |S_ki|
 *                    for dL/dcos(E_ki) = a_k + b_k cos(E_ki): the plain
 *                    gradient has b_k = 0, the U-statistic MMD^2 b_k != 0),
 *                    and contracted on the INT8
 *                    matrix cores with exact INT32 sums: two INT8 products
 *                    per term, the matrix-core time of one BF16 product. The
 *                    gradient meets 1e-4 * max(1, |g|).
 *   IQP_SPLIT_BF16_FP8: the forward of IQP_SPLIT_BF16 (2 theta_j in two
 *                    BF16 limbs); the backward weights are scaled per
 *                    observable by a power of two, S_ki 2^e_k with
 *                    2^14 <= bound_k 2^e_k < 2^15, and held as an FP16 limb
 *                    (round to nearest even) plus an FP8 E4M3 limb of what it
 *                    leaves (|rest| <= 16, 4 significant bits): 15 significant
 *                    bits per weight against 16 for two BF16 limbs, for one
 *                    FP16 and one FP8 product per term, three quarters of the
 *                    matrix-core time of two BF16 products; FP32
 *                    accumulation, 2^-e_k applied per row in the epilogue.
 *                    Its gradient error is that of IQP_SPLIT_BF16 to within
 *                    the weights' rounding.
 *   IQP_SPARSE_FP32: only the non-zero entries of C: for each observable the
 *                    sum of +-2 theta_j over the generators that anticommute
 *                    with it (FP32 on the vector units), so the work is the
 *                    number of non-zero entries of C times s instead of
 *                    l m s; faster when C is sparse (a few percent of
 *                    entries). The gradient sums per-gate contributions in
 *                    int64 fixed point, bitwise reproducible.
 * In all, theta is first reduced to [-pi/2, pi/2] by whole multiples of pi
 * (exp(i(theta + pi) X) = -exp(i theta X) is a global phase, Sec. 2.1), and
 * every phase is reduced modulo 2 pi in FP64 before its cos / sin. */
typedef enum {
    IQP_FP32 = 0,
    IQP_SPLIT_BF16 = 1,
    IQP_SPARSE_FP32 = 2,
    IQP_SPLIT3_BF16 = 3,
    IQP_SPLIT_BF16_FP8 = 4
} iqp_precision;

/* A parameterized IQP circuit (Def. 1): generators g_j as bit rows and their
 * parameters theta_j. */
typedef struct {
    int32_t n_qubits;      /* n >= 1 */
    int32_t n_words;       /* W, must equal ceil(n / 64) */
    int64_t n_gates;       /* m >= 1 */
    const uint64_t *gens;  /* device, [m][W] bit rows g_j */
    const double *theta;   /* device, [m] theta_j */
} iqp_circuit;

/* Which call a workspace is sized for. */
enum {
    IQP_CALL_EXPVAL = 0,
    IQP_CALL_EXPVAL_GRAD = 1,      /* with phase_save supplied */
    IQP_CALL_EXPVAL_GRAD_RECOMPUTE = 2, /* phase_save == NULL */
    IQP_CALL_MMD = 3,
    IQP_CALL_MMD_GRAD = 4,
    IQP_CALL_BITFLIP = 5,
    IQP_CALL_BITFLIP_GRAD = 6,
    IQP_CALL_INDEP = 7,
    IQP_CALL_INDEP_GRAD = 8,       /* with phase_save supplied */
    IQP_CALL_INDEP_GRAD_RECOMPUTE = 9 /* phase_save == NULL */
};

/* Bytes of workspace the given call needs for these sizes (N is only read for
 * the MMD calls; s and precision are not read for the bitflip calls,
 * precision not for the independent-estimate calls). Returns 0 for invalid
 * sizes. */
size_t iqp_workspace_bytes(int call, const iqp_circuit *c, int64_t l, int64_t s, int64_t N,
                           int precision);

/* Parity bit matrix (the exponents of B = (-1)^{Z G^T} and of
 * C = 1 - (-1)^{A G^T}, Sec. 2.2): bit (r, c) = popcount(row_r AND col_c) mod 2.
 * Computed bit-sliced: the rows are transposed into per-qubit bit columns and
 * the parity against col_c is the XOR of the columns in col_c's support, so
 * the cost grows with the weight of the col rows (pass the sparse operand,
 * e.g. the generators, as cols).
 *   rows      device [n_rows][W], cols device [n_cols][W]
 *   layout    IQP_BITS_ROW_MAJOR:  out[r * ceil(n_cols/64) + c/64], bit c % 64
 *             IQP_BITS_TILED32:    rows padded to a multiple of 32,
 *               out[((r / 32) * ceil(n_cols/64) + c/64) * 32 + r % 32], bit c % 64
 *               (the layout the phase-contraction kernels read)
 *             IQP_BITS_TILED32_T:  the transposed matrix, tiled32 over the
 *               columns padded to a multiple of 64:
 *               out[((c / 32) * ceil(n_rows/64) + r/64) * 32 + c % 32], bit r % 64
 *   out       device; pad rows and bits past the last row/column are written 0
 *   ws        device workspace of ws_bytes >=
 *             iqp_parity_workspace_bytes(n_rows, n_cols, W, layout)
 * n_rows >= 0, n_cols >= 0, W >= 1 (n_rows or n_cols = 0 is a no-op). Bit-exact. */
enum { IQP_BITS_ROW_MAJOR = 0, IQP_BITS_TILED32 = 1, IQP_BITS_TILED32_T = 2 };
size_t iqp_parity_workspace_bytes(int64_t n_rows, int64_t n_cols, int32_t n_words, int layout);
int iqp_parity(int64_t n_rows, const uint64_t *rows, int64_t n_cols, const uint64_t *cols,
               int32_t n_words, int layout, uint64_t *out, void *ws, size_t ws_bytes,
               void *stream);

/* Monte Carlo estimates of <Z_{a_k}> (eq. expvalsample, batched as Prop. 2).
 *   ops        device [l][W] observables a_k, l >= 1
 *   samples    device [s][W] bitstrings z_i, s >= 1 (drawn by the caller: the
 *              estimator is unbiased when they are uniform, Prop. 1)
 *   mean       device [l] (1/s) sum_i cos E_ki
 *   stderr_    device [l] or NULL: population standard deviation of
 *              cos E_ki over i, divided by sqrt(s)
 *   phase_save device [l][s] float or NULL: E_ki reduced to [-pi, pi]
 *              (row-major, k major), for iqp_expval_grad
 *   ws         device workspace of ws_bytes >= iqp_workspace_bytes(IQP_CALL_EXPVAL, ...)
 */
int iqp_expval(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
               const uint64_t *samples, int precision, double *mean, double *stderr_,
               float *phase_save, void *ws, size_t ws_bytes, void *stream);

/* iqp_expval for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same forward, with its workspace in a static device array of 64 MiB that
 * each GPU the library runs on holds until the process ends, so no ws
 * argument. Sizes whose iqp_workspace_bytes(IQP_CALL_EXPVAL, ...) exceeds
 * 64 MiB return IQP_ERR_WORKSPACE. Every call on one GPU shares that array:
 * calls that overlap in time on one GPU (other streams, other threads) race
 * and must be ordered by the caller. Outputs equal iqp_expval's bitwise.
 * Other arguments as iqp_expval. */
int iqp_expval_noalloc(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                       const uint64_t *samples, int precision, double *mean, double *stderr_,
                       float *phase_save, void *stream);

/* Gradient of a loss L(mean) through the estimator (the reverse pass of the
 * computational graph of Fig. 3, written by hand):
 *   dL/dtheta_j = -(1/s) sum_k u_k sum_i sin(E_ki) C_kj B_ij,  u_k = dL/dmean_k.
 *   grad_mean  device [l] u_k
 *   phase_save device [l][s] from iqp_expval with the same inputs and
 *              precision, or NULL to recompute the phases (parities are always
 *              recomputed, never stored)
 *   grad_theta device [m], overwritten (not accumulated)
 * Other arguments as iqp_expval. */
int iqp_expval_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                    const uint64_t *samples, int precision, const double *grad_mean,
                    const float *phase_save, double *grad_theta, void *ws, size_t ws_bytes,
                    void *stream);

/* MMD^2 between training data and the circuit through Pauli-Z expectation
 * values (eq. mmd_estimate, Sec. 3.3.1), and its gradient:
 *   p_k = (1/N) sum_n (-1)^{a_k . x_n},   q_k = mean_k (eq. expvalsample)
 *   unbiased != 0:  L = sum_k w_k [P2_k - 2 p_k q_k + Q2_k] with the
 *                   U-statistics P2_k = ((N p_k)^2 - N) / (N (N-1)),
 *                   Q2_k = ((sum_i c_ki)^2 - sum_i c_ki^2) / (s (s-1)),
 *                   c_ki = cos E_ki (needs N >= 2 and s >= 2)
 *   unbiased == 0:  L = sum_k w_k (p_k - q_k)^2
 *   ops        device [l][W], operators drawn from P_sigma by the caller
 *   op_weight  device [l] w_k (e.g. 1/(number of bandwidths * ops per bandwidth))
 *   data       device [N][W] training bitstrings x_n, N >= 1
 *   loss       device [1]
 *   grad_theta device [m] or NULL (loss only), overwritten
 * Other arguments as iqp_expval. */
int iqp_mmd_loss_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops,
                      const double *op_weight, int64_t s, const uint64_t *samples, int64_t N,
                      const uint64_t *data, int unbiased, int precision, double *loss,
                      double *grad_theta, void *ws, size_t ws_bytes, void *stream);

/* Independent estimates (the l x s x n sample tensor of Sec. 2.3): observable
 * k averages over its own s samples, so estimates of different observables
 * are uncorrelated (the shared-sample calls above correlate them). Same
 * estimator, outputs and gradient as iqp_expval / iqp_expval_grad; computed
 * in the sparse-C form (FP32 phases on the vector units, FP64 reduction), the
 * parities of each observable's anticommuting generators taken against its
 * own samples (whose bit columns are built first), at about twice the cost of
 * the shared-sample sparse form.
 *   samples    device [l][s][W]: sample i of observable k at (k s + i) W
 *   l * s <= 2^32; precision is fixed (no precision argument)
 *   ws         >= iqp_workspace_bytes(IQP_CALL_INDEP[_GRAD[_RECOMPUTE]], ...)
 *              (about the size of the samples again, for their bit columns)
 */
int iqp_expval_indep(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                     const uint64_t *samples, double *mean, double *stderr_, float *phase_save,
                     void *ws, size_t ws_bytes, void *stream);
int iqp_expval_indep_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                          const uint64_t *samples, const double *grad_mean,
                          const float *phase_save, double *grad_theta, void *ws,
                          size_t ws_bytes, void *stream);

/* Stochastic bitflip circuits (Sec. 2.5, Prop. 3): the incoherent version of
 * the circuit, where gate j flips the bits of g_j with probability
 * sin^2(theta_j). Its expectation values are exact and classical:
 *     <Z_{a_k}> = prod_{j : a_k . g_j odd} cos(2 theta_j)   (eq. expval_bitflip)
 * computed in FP64 from the C parity bits (a sum of log|cos| with a sign
 * parity and a count of zero factors per observable).
 *   ops        device [l][W], l >= 1
 *   mean       device [l] the exact expectation values
 *   grad_mean  device [l] u_k = dL/d<Z_{a_k}>
 *   grad_theta device [m] dL/dtheta_j = -2 sin(2 theta_j) sum_k u_k c_kj
 *              prod_{t in J_k, t != j} cos(2 theta_t), overwritten
 *   ws         device workspace of >= iqp_workspace_bytes(IQP_CALL_BITFLIP[_GRAD], ...)
 */
int iqp_bitflip_expval(const iqp_circuit *c, int64_t l, const uint64_t *ops, double *mean,
                       void *ws, size_t ws_bytes, void *stream);
int iqp_bitflip_expval_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops,
                            const double *grad_mean, double *grad_theta, void *ws,
                            size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent problems (circuit, observables, samples) of
 * uneven size in one pass. Each step of the estimator runs as one launch over
 * all problems; the two phase contractions run as persistent kernels that take
 * work units (tiles of every problem, longest first) from a queue, so small
 * and large circuits share the matrix cores without a tail per circuit. A pass
 * is captured once in a HIP graph and replayed. Results equal those of the
 * single-problem calls up to the order of FP32 accumulation (the gate-word
 * split of the forward may differ) and are deterministic for a fixed
 * configuration.
 *
 * One problem. Device pointers, conventions as the single-problem calls:
 *   circuit               n, W, m, gens [m][W], theta [m]
 *   n_ops / ops           l >= 1, [l][W]
 *   n_samples / samples   s >= 1, [s][W]
 *   mean, stderr_         [l] outputs of iqp_batch_expval (stderr_ may be NULL)
 *   phase_save            [l][s] float: written by iqp_batch_expval when not
 *                         NULL, read by iqp_batch_expval_grad (required there)
 *   grad_mean             [l] dL/dmean, input of iqp_batch_expval_grad
 *   grad_theta            [m] output of iqp_batch_expval_grad, overwritten
 */
typedef struct {
    iqp_circuit circuit;
    int64_t n_ops;
    const uint64_t *ops;
    int64_t n_samples;
    const uint64_t *samples;
    double *mean;
    double *stderr_;
    float *phase_save;
    const double *grad_mean;
    double *grad_theta;
} iqp_problem;

/* A plan holds the shapes of a problem list, the workspace layout, the tile
 * configuration and the captured graphs. Host object, owned by the caller
 * through create / destroy; not thread-safe. */
typedef struct iqp_batch_plan iqp_batch_plan;

/* flags of iqp_batch_plan_create */
enum {
    IQP_BATCH_NO_GRAPH = 1 /* launch the steps one by one instead of replaying a graph */
};

/* Creates a plan for n_problems >= 1 problems; only the shapes of `probs`
 * (host array) are read: n_qubits, n_words, n_gates, n_ops, n_samples. The
 * tile configuration is the one recorded for these shapes by iqp_batch_tune
 * in this process (or in the file named by the environment variable
 * IQP_TUNE_CACHE), else a default. The current device must be gfx950.
 * precision: IQP_FP32, IQP_SPLIT_BF16, IQP_SPLIT3_BF16 or IQP_SPLIT_BF16_FP8
 * (the dense forms). */
int iqp_batch_plan_create(int32_t n_problems, const iqp_problem *probs, int precision,
                          int flags, iqp_batch_plan **plan);
int iqp_batch_plan_destroy(iqp_batch_plan *plan);

/* Workspace bytes of a plan (enough for every configuration the tuner tries). */
size_t iqp_batch_workspace_bytes(const iqp_batch_plan *plan);

/* Forward pass of every problem: mean, stderr_ and (if not NULL) phase_save.
 * `probs` (host array) must have the plan's shapes; its pointers may change
 * from call to call. The pointer table is copied to the workspace on
 * `stream` before the pass; calls on one plan must be ordered on one stream. */
int iqp_batch_expval(iqp_batch_plan *plan, const iqp_problem *probs, void *ws, size_t ws_bytes,
                     void *stream);

/* Backward pass of every problem: grad_theta from grad_mean and phase_save
 * (the forward's phases with the same inputs and precision). */
int iqp_batch_expval_grad(iqp_batch_plan *plan, const iqp_problem *probs, void *ws,
                          size_t ws_bytes, void *stream);

/* Autotuner: times each candidate tile configuration of the forward (bit 0
 * of `passes`) and of the backward (bit 1; needs grad_mean and phase_save) on
 * these very problems, keeps the fastest in the plan and records it for the
 * shapes (in this process, and appended to IQP_TUNE_CACHE when set).
 * Synchronises `stream`; outputs are left unspecified. */
int iqp_batch_tune(iqp_batch_plan *plan, const iqp_problem *probs, int passes, void *ws,
                   size_t ws_bytes, void *stream);

/* Tile configuration as 6 int32: forward tile rows and columns in 32-blocks
 * (4x4, 2x4 or 2x2), forward split mode (0: no gate-word split; 1, 2: split
 * long problems so that no work unit exceeds 1/4 or 1/16 of a workgroup's
 * share), backward tile (2x2 or 2x4), and whether it came from the tuner.
 * set_config takes the first five. */
int iqp_batch_get_config(const iqp_batch_plan *plan, int32_t *cfg6);
int iqp_batch_set_config(iqp_batch_plan *plan, const int32_t *cfg5);

/* ---------------------------------------------------------------------------
 * Training on the device: the optimisation loop of Sec. 3.3 run with the MMD^2
 * loss of Sec. 3.3.1, where every step draws fresh samples z and fresh
 * operators a ~ P_sigma, evaluates the loss and its gradient at the current
 * parameters, and updates them. The pieces are separate calls; a training
 * plan chains them into one HIP graph per step.
 *
 * Random numbers: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC 2011) under the key (seed0, seed1).
 * Output o of stream `tag` at step t is word o % 4 of the block at counter
 * (o / 4, t, tag, 0). The step t is read from device memory when the kernel
 * runs, so a replayed graph draws new numbers after each update of t. The
 * same key, step and tag give the same bits on every call.
 */

/* Uniform bit strings (the samples z of eq. expvalsample, Prop. 1):
 *   out   device [rows][W], W = ceil(n_qubits / 64); word w of row r is
 *         output r * W + w, with the bits past n_qubits cleared
 *   step  device [1] int64 (read only)
 * rows >= 0 (0: nothing to do), 1 <= n_qubits <= 2^20. */
int iqp_sample_uniform(int64_t rows, int32_t n_qubits, uint64_t seed0, uint64_t seed1,
                       const int64_t *step, uint64_t tag, uint64_t *out, void *stream);

/* Independent Bernoulli bits in row groups (operators drawn from P_sigma,
 * whose bit probability is (1 - exp(-1 / (2 sigma^2))) / 2 for a Gaussian
 * kernel of bandwidth sigma, Sec. 3.3.1):
 *   group_rows  host [n_groups] rows of each group (>= 0), in row order
 *   group_prob  host [n_groups] bit probability p of each group, 0 <= p < 1
 *   out         device [sum group_rows][W]; qubit q of row r is 1 when output
 *               r * n_qubits + q is below floor(p * 2^64) of r's group
 * 1 <= n_groups <= 16. */
int iqp_sample_bernoulli(int32_t n_qubits, int32_t n_groups, const int64_t *group_rows,
                         const double *group_prob, uint64_t seed0, uint64_t seed1,
                         const int64_t *step, uint64_t tag, uint64_t *out, void *stream);

/* Parameter sharing and fixed gates (gates given as tuples of generators
 * share one parameter; initial gates keep fixed angles, Sec. 3.1.1):
 *   theta[j] = params[param_index[j]], or fixed_theta[j] when
 *   param_index[j] == -1.
 *   param_index  device [n_gates] int32, each in [-1, n_params) (not checked
 *                on the device: the training plan checks its host copy)
 *   fixed_theta  device [n_gates] or NULL when no index is -1 */
int iqp_gather_theta(int64_t n_gates, const int32_t *param_index, const double *params,
                     const double *fixed_theta, double *theta, void *stream);

/* Gradient of the parameters from that of the gates (chain rule of the
 * gather above): grad_params[p] = sum of grad_theta[j] over the gates of p,
 * added in the order listed, in FP64.
 *   param_offsets  device [n_params + 1] int64, offsets into param_gates
 *   param_gates    device int32 gate indices grouped by parameter */
int iqp_reduce_grad(int64_t n_params, const int64_t *param_offsets, const int32_t *param_gates,
                    const double *grad_theta, double *grad_params, void *stream);

/* optimizers */
enum {
    IQP_OPT_GD = 0,  /* params -= lr * grad */
    IQP_OPT_ADAM = 1 /* Adam (Kingma and Ba 2015): moments m1, m2 and bias
                        correction with step count t + 1 */
};

/* One optimizer update of n_params parameters in place, in FP64, followed by
 * step += 1 (step is device [1] int64: the number of earlier updates).
 * m1, m2 device [n_params] moments (read and written by Adam; unused and may
 * be NULL for gradient descent). lr > 0, 0 <= beta < 1, eps >= 0, finite. */
int iqp_optimizer_update(int optimizer, int64_t n_params, double *params, const double *grad,
                         double *m1, double *m2, int64_t *step, double lr, double beta1,
                         double beta2, double eps, void *stream);

/* A training plan: the circuit structure, the loss and the optimizer. */
typedef struct {
    int32_t n_qubits;
    int32_t n_words;
    int64_t n_gates;
    const uint64_t *gens;        /* device [m][W] generators */
    int64_t n_params;
    const int32_t *param_index;  /* host [m]: parameter of gate j, or -1 (fixed gate) */
    const double *fixed_theta;   /* device [m] angles of the fixed gates, or NULL */
    int32_t n_groups;            /* operator groups (one per kernel bandwidth), 1..16 */
    const int64_t *group_ops;    /* host [n_groups] operators per group per step */
    const double *group_prob;    /* host [n_groups] bit probability of each group */
    int64_t n_samples;           /* samples z per step */
    int64_t n_data;
    const uint64_t *data;        /* device [N][W] training bit strings */
    int32_t unbiased;            /* MMD^2 estimator form, as iqp_mmd_loss_grad */
    int32_t precision;           /* any iqp_precision */
    int32_t optimizer;           /* IQP_OPT_GD or IQP_OPT_ADAM */
    double lr, beta1, beta2, eps;
    uint64_t seed0, seed1;       /* Philox key; samples use tag 0, operators tag 1 */
    const int32_t *group_precision; /* host [n_groups] precision of each group, or
                                       NULL: every group takes `precision` */
} iqp_train_desc;

typedef struct iqp_train_plan iqp_train_plan;

/* flags of iqp_train_plan_create */
enum {
    IQP_TRAIN_NO_GRAPH = 1,      /* launch the steps one by one instead of replaying a graph */
    IQP_TRAIN_AUTO_PRECISION = 2 /* choose each group's precision (group_precision must be
                                    NULL): see iqp_train_plan_create */
};

/* Creates a plan; reads the host arrays of `desc` (the pointers to device
 * memory are kept and must stay valid). Each operator group's weights sum to
 * 1 / n_groups. With group_precision, the loss and gradient are one
 * iqp_mmd_loss_grad call per run of consecutive groups in one precision (MMD^2
 * and its gradient are sums over the operators, Sec. 3.3.1), summed in order:
 * for groups whose operators anticommute with few generators (the narrow
 * kernels' sparse operators) IQP_SPARSE_FP32 does a small fraction of the
 * dense work. With IQP_TRAIN_AUTO_PRECISION the plan copies the generators to
 * the host once (a synchronous copy) and runs group g in IQP_SPARSE_FP32 when
 * its expected density of C, the mean over generators j of
 * (1 - (1 - 2 p_g)^{|g_j|}) / 2 (the probability that a string with
 * Bernoulli(p_g) bits overlaps g_j in an odd number of qubits), is below
 * 6 %, and in `precision` otherwise. Host object, not thread-safe. */
int iqp_train_plan_create(const iqp_train_desc *desc, int flags, iqp_train_plan **plan);
int iqp_train_plan_destroy(iqp_train_plan *plan);
size_t iqp_train_workspace_bytes(const iqp_train_plan *plan);

/* Prepares a workspace: uploads the plan's tables (operator weights, the
 * parameter index, the gates of each parameter), zeroes the moments and sets
 * the step count to `step` (>= 0). Ordered on `stream`. */
int iqp_train_init(iqp_train_plan *plan, int64_t step, void *ws, size_t ws_bytes, void *stream);

/* n_steps >= 1 training steps. Step i draws z (s samples) and the operators
 * at the current step count t, writes loss[i] (the MMD^2 at the parameters
 * before its update), takes the gradient, updates params (device
 * [n_params], in place) and sets t = t + 1. grad_params: device [n_params]
 * gradient of the last step, or NULL. Without IQP_TRAIN_NO_GRAPH the steps
 * are one captured graph (recaptured when ws, params, loss, grad_params or
 * n_steps change) replayed on `stream`. */
int iqp_train_step(iqp_train_plan *plan, int32_t n_steps, double *params, double *loss,
                   double *grad_params, void *ws, size_t ws_bytes, void *stream);

/* The precision each operator group's loss and gradient run in (host
 * [n_groups], written). */
int iqp_train_group_precision(const iqp_train_plan *plan, int32_t *out);

/* Device pointers into a workspace: the samples [s][W] and operators
 * [l][W] of the last step, and the step count [1]. Any may be NULL. */
int iqp_train_buffers(const iqp_train_plan *plan, void *ws, uint64_t **samples,
                      uint64_t **ops, int64_t **step);

/* SHA-256 (lowercase hex) of the sources this library was built from, as
 * the in-tree build computes it over the kernel and host sources and this
 * header; "unknown" when built without it. Loaders compare it with the
 * sources beside the binary to refuse a stale build. Static string. */
const char *iqp_source_sha256(void);

/* Static text for a status code. */
const char *iqp_strerror(int status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *iqp_last_error(void);

/* Per-kernel timing, for measurement only. When enabled, every kernel launch
 * of the library is bracketed by HIP events on its stream; iqp_profile_query
 * synchronises those events and returns the total milliseconds and the
 * number of launches recorded for the kernel family `name` ("parity",
 * "theta_prep", "phase_fwd", "phase_epilogue", "finalize", "weights",
 * "phase_bwd", "grad_reduce", "mmd"). Not thread-safe; off by default. */
int iqp_profile_enable(int on);
int iqp_profile_query(const char *name, double *total_ms, int64_t *launches);
int iqp_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* IQP_H */
