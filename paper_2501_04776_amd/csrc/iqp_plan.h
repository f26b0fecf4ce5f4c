// Host-side pieces shared by the single-problem entry points (iqp_api.cpp)
// and the batched ones (iqp_batch.cpp): error reporting, the device check,
// the workspace plan of one problem and the argument structs of its steps.
#pragma once

#include <string>

#include "iqp.h"
#include "iqp_internal.h"

namespace iqp {

// Error reporting: the message goes to the thread's last-error slot.
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *where);
void clear_error();

// IQP_OK if the current device is gfx950 (and no launch fault is injected).
int check_device();

// IQP_ERR_HIP when the environment variable IQP_FAULT equals `what`
// ("launch" or "alloc"), for tests of the error paths; IQP_OK otherwise.
int injected_fault(const char *what);

LaunchCtx make_ctx(void *stream);

// iqp_expval after its argument checks: validates, lays out `ws` and
// enqueues the forward; `timing` = false keeps the per-kernel timing off for
// this call (it would create events).
int expval_call(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                const uint64_t *samples, int precision, double *mean, double *stderr_,
                float *phase_save, void *ws, size_t ws_bytes, void *stream, bool timing);

// The per-kernel timing collects (family, start, stop) events.
bool timing_enabled();

#define IQP_TRY(call, where)                              \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

// Size limits that keep every grid dimension and index in range.
constexpr int64_t kMaxRows = (int64_t)1 << 24;
// Sample rows l * s of the independent estimates.
constexpr int64_t kMaxIndepRows = (int64_t)1 << 32;

int check_circuit(const iqp_circuit *c);

// The precision forms of the single-problem calls.
inline bool valid_precision(int p) {
    return p == IQP_FP32 || p == IQP_SPLIT_BF16 || p == IQP_SPARSE_FP32 || p == IQP_SPLIT3_BF16 ||
           p == IQP_SPLIT_BF16_FP8;
}
// The dense forms (all but the sparse one).
inline bool dense_precision(int p) { return valid_precision(p) && p != IQP_SPARSE_FP32; }

// ---------------------------------------------------------------------------
// Workspace plan of one problem: padded extents and the byte offset of every
// buffer the steps use.
struct Plan {
    int prec = 0;
    int64_t n = 0, W = 0, m = 0, l = 0, s = 0, N = 0;
    int64_t m_pad = 0, l_pad = 0, s_pad = 0, mw = 0, lw = 0;
    TileCfg tc;
    int64_t nchunk = 0;
    bool fwd = false, phi = false, bwd = false, mmd = false;
    size_t o_thh = 0, o_thl = 0, o_t32 = 0, o_cbits = 0, o_bbits = 0, o_E = 0, o_part = 0;
    size_t o_rowsum = 0, o_phi = 0, o_coef = 0, o_ctbits = 0, o_shi = 0, o_slo = 0, o_s32 = 0;
    size_t o_gpart = 0, o_pstat = 0;
    size_t o_thm = 0;                     // third theta limb (IQP_SPLIT3_BF16)
    size_t o_sq = 0, o_nf = 0;            // fixed-point weights: row scales, non-finite flags
    size_t o_xz = 0, o_xa = 0;            // bit columns of samples, ops
    size_t o_btbits = 0;                  // B^T: samples against generators, transposed
    size_t o_sup = 0;                     // support lists of the generators
    size_t o_enc = 0, o_stat = 0;         // bitflip circuits: factors, per-observable sums
    size_t o_acc = 0, o_scale = 0;        // sparse gradient: int64 sums (+ flag), scale
    int64_t ldz = 0, lda = 0;
    size_t total = 0;
};

// Which parts a plan lays out.
struct PlanParts {
    bool fwd = true;   // forward buffers (theta limbs, C and B bits, E, sums)
    bool bwd = false;  // backward buffers (weights, B^T and C^T bits, partials)
    bool phi = false;  // a phase buffer of its own (backward without saved phases)
    bool mmd = false;  // data statistics
};

// Gate-word splits of the forward that fill `kWaveSlots` wave slots.
int64_t choose_splits(int64_t tiles, int64_t mw);
// Sample-word splits of the backward for `units` workgroup units, with
// `wgs_per_cu` of them resident per CU.
int64_t choose_bsplits(int64_t units, int64_t sw, int wgs_per_cu);
int bwd_wgs_per_cu(int prec, int bfm, int bfn);

// Lays out the buffers; tc.splits <= 0 picks the split count.
void make_plan(Plan &P, const PlanParts &parts, int64_t n, int64_t m, int64_t l, int64_t s,
               int64_t N, int prec, const TileCfg &tc);

template <typename T>
inline T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ---- argument structs of one problem, from its plan and workspace ---------
inline ThetaArgs theta_args(const Plan &P, const double *theta, void *ws) {
    return ThetaArgs{theta,
                     P.m,
                     P.m_pad,
                     P.prec,
                     at<uint16_t>(ws, P.o_thh),
                     at<uint16_t>(ws, P.o_thl),
                     P.prec == IQP_SPLIT3_BF16 ? at<uint16_t>(ws, P.o_thm) : nullptr,
                     at<float>(ws, P.o_t32)};
}
inline BitsliceArgs bitslice_ops_args(const Plan &P, const uint64_t *ops, void *ws) {
    return BitsliceArgs{ops, P.l, (int)P.W, P.lda, at<uint64_t>(ws, P.o_xa)};
}
inline BitsliceArgs bitslice_samples_args(const Plan &P, const uint64_t *samples, void *ws) {
    return BitsliceArgs{samples, P.s, (int)P.W, P.ldz, at<uint64_t>(ws, P.o_xz)};
}
// support lists of the generators (m_pad rows)
inline SupportArgs support_args(const Plan &P, const uint64_t *gens, void *ws) {
    return SupportArgs{gens, P.m, (int)P.W, P.m_pad, at<int32_t>(ws, P.o_sup)};
}
// C and B (tiled32) for the forward
inline ParityArgs parity_c_args(const Plan &P, const uint64_t *gens, void *ws) {
    return ParityArgs{gens,    at<int32_t>(ws, P.o_sup), P.m,   (int)P.W,
                      at<uint64_t>(ws, P.o_xa), P.l_pad / 64, P.lda, P.l_pad,
                      P.mw,    at<uint64_t>(ws, P.o_cbits)};
}
inline ParityArgs parity_b_args(const Plan &P, const uint64_t *gens, void *ws) {
    return ParityArgs{gens,    at<int32_t>(ws, P.o_sup), P.m,   (int)P.W,
                      at<uint64_t>(ws, P.o_xz), P.s_pad / 64, P.ldz, P.s_pad,
                      P.mw,    at<uint64_t>(ws, P.o_bbits)};
}
// B^T and C^T (transposed tiled32) for the backward
inline ParityArgs parity_bt_args(const Plan &P, const uint64_t *gens, void *ws) {
    return ParityArgs{gens,    at<int32_t>(ws, P.o_sup), P.m,   (int)P.W,
                      at<uint64_t>(ws, P.o_xz), P.s_pad / 64, P.ldz, 0,
                      P.mw,    at<uint64_t>(ws, P.o_btbits)};
}
inline ParityArgs parity_ct_args(const Plan &P, const uint64_t *gens, void *ws) {
    return ParityArgs{gens,    at<int32_t>(ws, P.o_sup), P.m, (int)P.W,
                      at<uint64_t>(ws, P.o_xa), P.lw,     P.lda, 0,
                      P.mw,    at<uint64_t>(ws, P.o_ctbits)};
}
inline FwdArgs fwd_args(const Plan &P, void *ws, int64_t splits) {
    return FwdArgs{at<uint64_t>(ws, P.o_cbits), at<uint64_t>(ws, P.o_bbits),
                   at<uint16_t>(ws, P.o_thh),   at<uint16_t>(ws, P.o_thl),
                   P.prec == IQP_SPLIT3_BF16 ? at<uint16_t>(ws, P.o_thm) : nullptr,
                   at<float>(ws, P.o_t32),      P.m_pad,
                   P.l_pad,                     P.s_pad,
                   splits,                      at<float>(ws, P.o_E)};
}
inline EpiArgs epi_args(const Plan &P, void *ws, int64_t splits, float *phase_out) {
    return EpiArgs{at<float>(ws, P.o_E), splits,   P.l, P.s, P.l_pad, P.s_pad,
                   phase_out,            at<double>(ws, P.o_part)};
}
inline FinArgs fin_args(const Plan &P, void *ws, double *mean, double *se, double *rowsum) {
    return FinArgs{at<double>(ws, P.o_part), P.l, P.s, mean, se, rowsum};
}
inline CoefArgs coef_args(const Plan &P, const double *grad_mean, void *ws) {
    const bool fx = P.prec == IQP_SPLIT3_BF16;
    return CoefArgs{grad_mean, P.l, P.s, at<double>(ws, P.o_coef),
                    fx ? at<double>(ws, P.o_sq) : nullptr, fx ? at<int32_t>(ws, P.o_nf) : nullptr};
}
inline WeightsArgs weights_args(const Plan &P, const float *phase, void *ws) {
    return WeightsArgs{phase,  at<double>(ws, P.o_coef), P.l, P.s, P.l_pad, P.s_pad, P.prec,
                       at<uint16_t>(ws, P.o_shi), at<uint16_t>(ws, P.o_slo),
                       at<float>(ws, P.o_s32),
                       P.prec == IQP_SPLIT3_BF16 ? at<int32_t>(ws, P.o_nf) : nullptr,
                       P.prec == IQP_SPLIT_BF16_FP8 ? at<double>(ws, P.o_sq) : nullptr};
}
inline BwdArgs bwd_args(const Plan &P, void *ws) {
    const bool fx = P.prec == IQP_SPLIT3_BF16;
    const bool rs = fx || P.prec == IQP_SPLIT_BF16_FP8;
    return BwdArgs{at<uint16_t>(ws, P.o_shi),    at<uint16_t>(ws, P.o_slo),
                   at<float>(ws, P.o_s32),       at<uint64_t>(ws, P.o_btbits),
                   at<uint64_t>(ws, P.o_ctbits), P.m_pad,
                   P.l_pad,                      P.s_pad,
                   P.tc.bsplits,                 at<float>(ws, P.o_gpart),
                   rs ? at<double>(ws, P.o_sq) : nullptr,
                   fx ? at<int32_t>(ws, P.o_nf) : nullptr,
                   P.tc.obgroup};
}
inline GradArgs grad_args(const Plan &P, void *ws, int bfm, double *grad_theta) {
    return GradArgs{at<float>(ws, P.o_gpart), P.tc.bsplits * (P.l_pad / (32 * bfm)), P.m, P.m_pad,
                    grad_theta};
}

}  // namespace iqp
