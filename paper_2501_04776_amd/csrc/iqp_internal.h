// Internal interface between the host runtime (iqp_api.cpp) and the gfx950
// kernels (iqp_kernels.hip). Not installed; the public ABI is include/iqp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace iqp {

// Every extent the kernels tile over is padded to a multiple of this.
constexpr int64_t kPad = 128;
// IQP_SPLIT3_BF16: the third theta limb is E4M3(rest * 2^kLo8Exp)
constexpr int kLo8Exp = 20;

// Work slots of one MI355X at one wave per SIMD: 256 CUs x 4 SIMDs.
constexpr int64_t kWaveSlots = 1024;

// Samples per block of the epilogue reduction (fixed: part of the
// deterministic summation order).
constexpr int64_t kEpiChunk = 1024;

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Tile configuration of the two contractions (wave tile = 32*fm x 32*fn).
struct TileCfg {
    int fm = 4, fn = 4;      // forward: observables x samples
    int bfm = 2, bfn = 2;    // backward: observables x gates
    int64_t splits = 0;      // forward split over gate words; 0 = choose
    int64_t bsplits = 0;     // backward split over sample words; 0 = choose
    int64_t obgroup = 4;     // backward unit order: observable blocks per group
};

// Kernel-family ids for the optional per-kernel timing.
enum KernelFamily {
    KF_PARITY = 0, KF_THETA, KF_FWD, KF_EPI, KF_FIN, KF_WEIGHTS, KF_BWD, KF_GRAD, KF_MMD,
    KF_COUNT
};

// A launch records (family, start, stop) events when timing is on.
struct LaunchCtx {
    hipStream_t stream;
    bool timing;
};

void timed_begin(const LaunchCtx &lc, int family, hipEvent_t *ev);
void timed_end(const LaunchCtx &lc, int family, hipEvent_t ev);

// Fixed-point backward weights (IQP_SPLIT3_BF16): |S_ki| <= sigma_k maps to
// integers N with |N| <= kI8Max = 127 * 256 + 127, the largest magnitude two
// signed 8-bit limbs hold as N = 256 hi + lo with hi = floor((N + 128) / 256)
// in [-127, 127] and lo in [-128, 127]. Over at most 2^16 samples per work
// unit the INT32 sums of each limb, and 256 hi_sum + lo_sum, stay exact
// (|256 * 127 K + 128 K| < 2^31 for K <= 2^16).
constexpr double kI8Max = 32639.0;
constexpr int64_t kI8MaxSamplesPerUnit = (int64_t)1 << 16;

// Support-list capacity: the qubits of a generator of weight <= kSupCap are
// listed; heavier generators are read from their bit rows.
constexpr int kSupCap = 8;

// ---- per-step arguments -----------------------------------------------------
// Each step's kernel body takes one of these and a block (or work-unit)
// index. A single-problem launch passes the struct as the kernel argument; a
// batched launch reads one struct per problem from a device array and maps
// its flat block index to (problem, local block) through a prefix sum of the
// per-problem block counts.

// prec: IQP_FP32 (t32 split by gate parity), IQP_SPLIT_BF16 and
// IQP_SPLIT_BF16_FP8 (hi, lo), IQP_SPARSE_FP32 (t32 plain), IQP_SPLIT3_BF16
// (hi, mid, lo).
struct ThetaArgs {
    const double *theta;
    int64_t m, m_pad;
    int prec;
    uint16_t *hi, *lo, *mid;
    float *t32;
};
inline int64_t blocks_of(const ThetaArgs &a) { return ceil_div(a.m_pad, 256); }

// Bit columns of `rows`: Xt[q * ldx + rw], q < 64 W, rw < ldx (>= ceil(R/64)),
// and a zero column q = 64 W (Xt holds 64 W + 1 columns).
struct BitsliceArgs {
    const uint64_t *rows;
    int64_t R;
    int W;
    int64_t ldx;
    uint64_t *Xt;
};
inline int64_t blocks_of(const BitsliceArgs &a) { return ceil_div(a.ldx * a.W, 4); }

// Support lists of `rows` generators (m real ones, W words each; rows >= m
// are written as weight 0): sup[j * kSupCap + k] = qubit of the k-th set bit
// of generator j, -1 past its weight, and sup[j * kSupCap] = -2 for a
// generator heavier than kSupCap.
struct SupportArgs {
    const uint64_t *gens;
    int64_t m;
    int W;
    int64_t rows;
    int32_t *sup;
};
inline int64_t blocks_of(const SupportArgs &a) { return ceil_div(a.rows, 256); }

// Parity of each generator (m of them, W words each, support lists `sup`
// covering 64 Gw rows) against the rows behind Xt (Rw words of 64 rows), in
// layout 0 (row-major), 1 (tiled32) or 2 (transposed tiled32); Gw = output
// words per row in layouts 0/1, generator words in layout 2. One wave per 64
// generators x 64 row words.
struct ParityArgs {
    const uint64_t *gens;
    const int32_t *sup;
    int64_t m;
    int W;
    const uint64_t *Xt;
    int64_t Rw, ldx, R_out, Gw;
    uint64_t *out;
};
inline int64_t blocks_of(const ParityArgs &a) { return ceil_div(a.Gw * ceil_div(a.Rw, 64), 4); }

// E = C Theta B^T, tiled over observables x samples, gate words split
// `splits` ways (partials E[split][l_pad][s_pad]).
struct FwdArgs {
    const uint64_t *cbits, *bbits;
    const uint16_t *thh, *thl, *thm;  // thm: third limb (IQP_SPLIT3_BF16 only)
    const float *t32;
    int64_t m_pad, l_pad, s_pad, splits;
    float *E;
};
inline int64_t fwd_units(const FwdArgs &a, int fm, int fn) {
    return (a.l_pad / (32 * fm)) * ceil_div(a.s_pad / (32 * fn), 4) * a.splits;
}

struct EpiArgs {
    const float *E;
    int64_t splits, l, s, l_pad, s_pad;
    float *phase_out;
    double *part;
};
inline int64_t blocks_of(const EpiArgs &a) { return a.l * ceil_div(a.s, kEpiChunk); }

struct FinArgs {
    const double *part;
    int64_t l, s;
    double *mean, *stderr_, *rowsum;
};
inline int64_t blocks_of(const FinArgs &a) { return ceil_div(a.l, 256); }

// coef[2k], coef[2k+1] = alpha_k, beta_k of the backward weights. For the
// fixed-point weights (IQP_SPLIT3_BF16) also the row scale
// sq[k] = (|alpha_k| + |beta_k|) / kI8Max and a zeroed non-finite flag nf[k];
// both pointers are NULL for the other forms.
struct CoefArgs {
    const double *grad_mean;
    int64_t l, s;
    double *coef;
    double *sq;
    int32_t *nf;
};
inline int64_t blocks_of(const CoefArgs &a) { return ceil_div(a.l, 256); }

// IQP_SPLIT3_BF16: shi / slo hold the high / low signed 8-bit limbs of
// N_ki = rint(S_ki / sq[k]) (|N| <= kI8Max), and nf[k] is set to 1 where a
// weight of row k is not finite. IQP_SPLIT_BF16_FP8: shi holds the FP16 limb
// and slo (one byte per weight) the FP8 E4M3 limb of S_ki 2^e_k, and sq[k] is
// set to 2^-e_k.
struct WeightsArgs {
    const float *phase;
    const double *coef;
    int64_t l, s, l_pad, s_pad;
    int prec;
    uint16_t *shi, *slo;
    float *s32;
    int32_t *nf;
    double *sq;
};
inline int64_t blocks_of(const WeightsArgs &a) { return (a.s_pad / 64) * (a.l_pad / 64); }

// T = S B (observables x gates, K = samples, split `ksplits` ways over the
// sample words) and the gradient partials gpart[ksplits][l_pad / (32 fm)][m_pad];
// btbits / ctbits are the transposed tiled32 parities of the samples /
// observables against the generators. Every split must hold >= 1 sample word.
struct BwdArgs {
    const uint16_t *shi, *slo;
    const float *s32;
    const uint64_t *btbits, *ctbits;
    int64_t m_pad, l_pad, s_pad, ksplits;
    float *gpart;
    const double *sq;   // row scales (IQP_SPLIT3_BF16, IQP_SPLIT_BF16_FP8) and
                        // non-finite flags (IQP_SPLIT3_BF16)
    const int32_t *nf;
    int64_t obgroup;    // observable blocks per unit group (unit order only)
};
inline int64_t bwd_units(const BwdArgs &a, int fm, int fn) {
    return ceil_div(a.m_pad / (32 * fn), 4) * (a.l_pad / (32 * fm)) * a.ksplits;
}

struct GradArgs {
    const float *gpart;
    int64_t n_parts, m, m_pad;
    double *grad;
};
inline int64_t blocks_of(const GradArgs &a) { return ceil_div(a.m, 256); }

// Stochastic bitflip circuits (exact product form).
struct BitflipPrepArgs {
    const double *theta;
    int64_t m;
    double *enc;  // [m] copysign(-log|cos 2 theta|, cos 2 theta)
};
inline int64_t blocks_of(const BitflipPrepArgs &a) { return ceil_div(a.m, 256); }

struct BitflipFwdArgs {
    const uint64_t *cbits;  // tiled32 C bits, mw gate words per observable row
    const double *enc;
    int64_t l, mw;
    double *mean, *stderr_;  // stderr_ may be NULL (written 0: the value is exact)
    double *stat;            // [l][2]
};
inline int64_t blocks_of(const BitflipFwdArgs &a) { return ceil_div(a.l, 4); }

struct BitflipGradArgs {
    const uint64_t *ctbits;  // transposed tiled32 C^T bits, lw observable words per gate row
    const double *enc, *theta, *stat, *grad_mean;
    int64_t m, lw;
    double *grad;
};
inline int64_t blocks_of(const BitflipGradArgs &a) { return ceil_div(a.m, 256); }

// Where the sparse kernels read the sample parities b_ij of generator j
// (bit i % 64 of word i / 64):
//   shared samples:       btrm, B^T row-major, Rwb sample words per generator
//   independent samples:  xt, the bit columns of each observable's own
//                         samples (xt + k * xstride, column q at q * Rwb),
//                         combined over the support list sup (or the bit row
//                         of gens for a generator heavier than kSupCap)
struct SampleParity {
    const uint64_t *btrm;
    const uint64_t *xt;  // NULL for shared samples
    int64_t Rwb, xstride;
    const int32_t *sup;
    const uint64_t *gens;
    int W;
};

// Sparse-C contraction (FP32 on the vector units): the phases summed over
// each observable's anticommuting generators only.
//   crm   C row-major: Gw gate words per observable row
//   t32   2 theta' per generator (plain FP32)
struct SparseFwdArgs {
    const uint64_t *crm;
    int64_t Gw;
    const float *t32;
    SampleParity bsrc;
    int64_t l, s;
    float *phase_out;  // [l][s] or NULL
    double *part;      // [l][ceil(s / kEpiChunk)][2] as the dense epilogue writes it
};

// acc[m_pad + 1] int64 (the last slot flags a non-finite contribution) and
// *scale: the fixed-point scale of the gradient sums, from the bound
// sum_k s (|alpha_k| + |beta_k|) on every partial sum.
struct SparseBoundArgs {
    const double *coef;
    int64_t l, s, m_pad;
    long long *acc;
    double *scale;
};
inline int64_t blocks_of(const SparseBoundArgs &a) { return ceil_div(a.m_pad + 1, 256); }

struct SparseBwdArgs {
    const uint64_t *crm;
    int64_t Gw;
    SampleParity bsrc;
    int64_t l, s, m_pad;  // j < m_pad; acc[m_pad] is the non-finite flag
    const float *phase;
    const double *coef, *scale;
    long long *acc;
};

// Bit columns of l sample sets of s rows each ([l][s][W], row i of set k at
// samples + (k s + i) W): xt[k * 64 W * ldx + q * ldx + rw], bit r = qubit q
// of row 64 rw + r of set k (rows >= s read as 0), q < 64 W, rw < ldx (a
// multiple of 16; one block per set and 16 row words).
struct IndepSliceArgs {
    const uint64_t *samples;
    int64_t l, s;
    int W;
    int64_t ldx;
    uint64_t *xt;
};

struct SparseFinishArgs {
    const long long *acc;
    const double *scale;
    int64_t m, m_pad;
    double *grad;
};
inline int64_t blocks_of(const SparseFinishArgs &a) { return ceil_div(a.m, 256); }

// ---- launchers (iqp_kernels.hip, iqp_sparse_kernels.hip); each returns
// hipGetLastError() ----
hipError_t launch_theta_prep(const LaunchCtx &lc, const ThetaArgs &a);
hipError_t launch_bitslice(const LaunchCtx &lc, const BitsliceArgs &a);
hipError_t launch_support(const LaunchCtx &lc, const SupportArgs &a);
hipError_t launch_parity_bs(const LaunchCtx &lc, int layout, const ParityArgs &a);
hipError_t launch_phase_fwd(const LaunchCtx &lc, int prec, int fm, int fn, const FwdArgs &a);
hipError_t launch_epilogue(const LaunchCtx &lc, const EpiArgs &a);
hipError_t launch_finalize(const LaunchCtx &lc, const FinArgs &a);
hipError_t launch_coef_plain(const LaunchCtx &lc, const CoefArgs &a);
hipError_t launch_weights(const LaunchCtx &lc, const WeightsArgs &a);
hipError_t launch_phase_bwd(const LaunchCtx &lc, int prec, int fm, int fn, const BwdArgs &a);
hipError_t launch_grad_reduce(const LaunchCtx &lc, const GradArgs &a);
hipError_t launch_sparse_fwd(const LaunchCtx &lc, const SparseFwdArgs &a);
hipError_t launch_sparse_bound(const LaunchCtx &lc, const SparseBoundArgs &a);
hipError_t launch_sparse_bwd(const LaunchCtx &lc, const SparseBwdArgs &a);
hipError_t launch_sparse_finish(const LaunchCtx &lc, const SparseFinishArgs &a);
hipError_t launch_indep_slice(const LaunchCtx &lc, const IndepSliceArgs &a);
hipError_t launch_bitflip_prep(const LaunchCtx &lc, const BitflipPrepArgs &a);
hipError_t launch_bitflip_fwd(const LaunchCtx &lc, const BitflipFwdArgs &a);
hipError_t launch_bitflip_grad(const LaunchCtx &lc, const BitflipGradArgs &a);

// Batched launches: `args` is a device array of np argument structs of the
// step's type and `off` a device array of np + 1 prefix sums of their block
// counts (off[0] = 0, off[np] = total > 0).
enum StepKind {
    SK_THETA = 0, SK_BITSLICE, SK_PARITY0, SK_PARITY1, SK_PARITY2, SK_EPI, SK_FIN, SK_COEF,
    SK_WEIGHTS, SK_GRAD, SK_SUPPORT, SK_COUNT
};
hipError_t launch_batched(const LaunchCtx &lc, int kind, const void *args, const int64_t *off,
                          int np, int64_t total);

// Persistent contractions over a work queue: `grid` workgroups take work
// units 0 .. off[np]-1 in order from `counter` (which must read 0 at launch);
// unit u belongs to problem p with off[p] <= u < off[p+1] and is that
// problem's local unit u - off[p].
hipError_t launch_phase_fwd_persistent(const LaunchCtx &lc, int prec, int fm, int fn,
                                       const FwdArgs *args, const int64_t *off, int np,
                                       unsigned long long *counter, int grid);
hipError_t launch_phase_bwd_persistent(const LaunchCtx &lc, int prec, int fm, int fn,
                                       const BwdArgs *args, const int64_t *off, int np,
                                       unsigned long long *counter, int grid);
// Workgroups of the persistent contraction that fit on the device at once.
int persistent_grid(bool fwd, int prec, int fm, int fn);
// Zero n work-queue counters (a kernel, so it can be captured in a graph).
hipError_t launch_reset_counters(const LaunchCtx &lc, unsigned long long *c, int n);

// pstat[2k] = sum_n (-1)^{a_k . x_n}, pstat[2k+1] = that sum / N, for the
// observables ops [l][W] against the training strings data [N][W].
hipError_t launch_data_stats(const LaunchCtx &lc, const uint64_t *ops, int64_t l,
                             const uint64_t *data, int64_t N, int W, double *pstat);

hipError_t launch_mmd_loss(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int64_t N, int unbiased,
                           double *loss);

hipError_t launch_coef_mmd(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int unbiased,
                           double *coef, double *sq, int32_t *nf);

}  // namespace iqp
