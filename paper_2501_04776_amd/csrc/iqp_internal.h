// Internal interface between the host runtime (iqp_api.cpp) and the gfx950
// kernels (iqp_kernels.hip). Not installed; the public ABI is include/iqp.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace iqp {

// Every extent the kernels tile over is padded to a multiple of this.
constexpr int64_t kPad = 128;

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

// ---- launchers (iqp_kernels.hip); each returns hipGetLastError() ----
hipError_t launch_theta_prep(const LaunchCtx &lc, const double *theta, int64_t m, int64_t m_pad,
                             int prec, uint16_t *hi, uint16_t *lo, float *t32);

// Bit columns of `rows`: Xt[q * ldx + rw], q < 64 W, rw < ldx (>= ceil(R/64)).
hipError_t launch_bitslice(const LaunchCtx &lc, const uint64_t *rows, int64_t R, int W,
                           int64_t ldx, uint64_t *Xt);

// Parity of each generator (m of them, W words each) against the rows behind
// Xt (Rw words of 64 rows), in layout 0 (row-major), 1 (tiled32) or 2
// (transposed tiled32); Gw = output words per row in layouts 0/1.
hipError_t launch_parity_bs(const LaunchCtx &lc, const uint64_t *gens, int64_t m, int W,
                            const uint64_t *Xt, int64_t Rw, int64_t ldx, int64_t R_out,
                            int64_t Gw, int layout, uint64_t *out);

hipError_t launch_phase_fwd(const LaunchCtx &lc, int prec, int fm, int fn, const uint64_t *cbits,
                            const uint64_t *bbits, const uint16_t *thh, const uint16_t *thl,
                            const float *t32, int64_t m_pad, int64_t l_pad, int64_t s_pad,
                            int64_t splits, float *E);

hipError_t launch_epilogue(const LaunchCtx &lc, const float *E, int64_t splits, int64_t l,
                           int64_t s, int64_t l_pad, int64_t s_pad, float *phase_out,
                           double *part);

hipError_t launch_finalize(const LaunchCtx &lc, const double *part, int64_t l, int64_t s,
                           double *mean, double *stderr_, double *rowsum);

hipError_t launch_coef_plain(const LaunchCtx &lc, const double *grad_mean, int64_t l, int64_t s,
                             double *coef);

hipError_t launch_weights(const LaunchCtx &lc, int prec, const float *phase, const double *coef,
                          int64_t l, int64_t s, int64_t l_pad, int64_t s_pad, uint16_t *shi,
                          uint16_t *slo, float *s32);

// T = S B (observables x gates, K = samples) and the gradient partials
// gpart[l_pad / (32 fm)][m_pad]; btbits / ctbits are the transposed tiled32
// parities of the samples / observables against the generators.
hipError_t launch_phase_bwd(const LaunchCtx &lc, int prec, int fm, int fn, const uint16_t *shi,
                            const uint16_t *slo, const float *s32, const uint64_t *btbits,
                            const uint64_t *ctbits, int64_t m_pad, int64_t l_pad, int64_t s_pad,
                            float *gpart);

hipError_t launch_grad_reduce(const LaunchCtx &lc, const float *gpart, int64_t n_parts,
                              int64_t m, int64_t m_pad, double *grad);

hipError_t launch_data_stats(const LaunchCtx &lc, const uint64_t *dbits, int64_t l, int64_t Nw,
                             int64_t N, double *pstat);

hipError_t launch_mmd_loss(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int64_t N, int unbiased,
                           double *loss);

hipError_t launch_coef_mmd(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int unbiased,
                           double *coef);

}  // namespace iqp
