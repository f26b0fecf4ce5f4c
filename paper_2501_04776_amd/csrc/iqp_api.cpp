// Host runtime of the C-ABI declared in include/iqp.h: argument validation,
// workspace planning and carving, kernel dispatch on the caller's stream, and
// the optional per-kernel timing.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <utility>
#include <vector>

#include "iqp.h"
#include "iqp_internal.h"
#include "iqp_plan.h"

namespace iqp {

static thread_local std::string g_last_error;

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

void clear_error() { g_last_error.clear(); }

int hip_fail(hipError_t e, const char *where) {
    g_last_error = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) +
                   ")";
    return IQP_ERR_HIP;
}

// ---------------------------------------------------------------------------
// per-kernel timing
struct Timing {
    bool on = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[KF_COUNT] = {};
    int64_t launches[KF_COUNT] = {};
};
static Timing g_timing;

static hipEvent_t take_event() {
    if (!g_timing.pool.empty()) {
        hipEvent_t e = g_timing.pool.back();
        g_timing.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Event failures only lose a timing sample: the launch itself is unaffected.
void timed_begin(const LaunchCtx &lc, int, hipEvent_t *ev) {
    *ev = nullptr;
    if (!lc.timing) return;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, lc.stream) == hipSuccess) *ev = e;
    else if (e) g_timing.pool.push_back(e);
}

void timed_end(const LaunchCtx &lc, int family, hipEvent_t ev) {
    if (!lc.timing || !ev) return;
    hipEvent_t e2 = take_event();
    if (e2 && hipEventRecord(e2, lc.stream) == hipSuccess) {
        g_timing.pending.push_back({family, {ev, e2}});
        return;
    }
    g_timing.pool.push_back(ev);
    if (e2) g_timing.pool.push_back(e2);
}

static hipError_t drain_timing() {
    hipError_t first = hipSuccess;
    for (auto &p : g_timing.pending) {
        hipError_t e = hipEventSynchronize(p.second.second);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.second.first, p.second.second);
        if (e == hipSuccess) {
            g_timing.total_ms[p.first] += ms;
            g_timing.launches[p.first] += 1;
        } else if (first == hipSuccess) {
            first = e;
        }
        g_timing.pool.push_back(p.second.first);
        g_timing.pool.push_back(p.second.second);
    }
    g_timing.pending.clear();
    return first;
}

static const char *kFamilyNames[KF_COUNT] = {"parity", "theta_prep", "phase_fwd",
                                             "phase_epilogue", "finalize", "weights",
                                             "phase_bwd", "grad_reduce", "mmd"};

// ---------------------------------------------------------------------------
// device check: the kernels are built for gfx950 only
// Fault injection for tests of the error paths (IQP_FAULT in the
// environment, read on every call): "launch" fails every call that would use
// the device at its device check, before any work is enqueued; "alloc" fails
// plan creation where it would allocate its host and stream resources.
int injected_fault(const char *what) {
    const char *f = getenv("IQP_FAULT");
    if (f && strcmp(f, what) == 0)
        return fail(IQP_ERR_HIP, std::string("injected fault (IQP_FAULT=") + what +
                                     "): nothing was enqueued or allocated");
    return IQP_OK;
}

int check_device() {
    if (int st = injected_fault("launch")) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    static int checked_dev = -1;
    static bool ok = false;
    if (checked_dev != dev) {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        ok = strncmp(prop.gcnArchName, "gfx950", 6) == 0;
        checked_dev = dev;
        if (!ok)
            return fail(IQP_ERR_UNSUPPORTED,
                        std::string("device arch ") + prop.gcnArchName + " is not gfx950");
    }
    return ok ? IQP_OK : fail(IQP_ERR_UNSUPPORTED, "device is not gfx950");
}

// ---------------------------------------------------------------------------
// workspace plan
// Each split adds an l x s partial E that the forward writes and the
// epilogue reads back: per 128 x 128 tile about as long as 10 gate words of
// matrix-core work, while a split raises the last round's fill by at most a
// few percent. So a split is added only for every 128 gate words (m = 10^3
// keeps one split: 0.84 -> 0.72 ms at l = s = 10^4; the 300-qubit workload
// keeps three).
int64_t choose_splits(int64_t tiles, int64_t mw) {
    int64_t best = 1;
    double best_eff = -1.0;
    for (int64_t sp = 1; sp <= 16; ++sp) {
        if (sp > 1 && mw < 128 * (sp - 1)) break;
        const int64_t units = tiles * sp;
        const double eff =
            (double)units / (double)(ceil_div(units, kWaveSlots) * kWaveSlots);
        if (eff >= 0.9) return sp;
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = sp;
        }
    }
    return best;
}

// Workgroups of the backward contraction resident per CU (register and LDS
// use of each kernel, 32 KB of LDS each): BF16 64x64 three, BF16 64x128 two,
// INT8 64x64 two, INT8 64x128 one, FP32 64x64 three, FP32 64x128 one; the
// FP16 + FP8 kernels as the BF16 ones, and their 128x64 tile two.
int bwd_wgs_per_cu(int prec, int bfm, int bfn) {
    if (prec == IQP_SPLIT_BF16 || prec == IQP_SPLIT_BF16_FP8) return bfm * bfn == 4 ? 3 : 2;
    if (prec == IQP_SPLIT3_BF16) return bfn == 2 ? 2 : 1;
    return bfn == 2 ? 3 : 1;
}

// Sample-word splits of the backward contraction, chosen like the forward's:
// the smallest count that keeps >= 95 % of the resident workgroups busy in
// the last round (on 256 CUs), with >= 8 sample words per split. The count
// is then trimmed so that no split is empty.
int64_t choose_bsplits(int64_t units, int64_t sw, int wgs_per_cu) {
    const int64_t resident = (int64_t)wgs_per_cu * 256;
    int64_t best = 1;
    double best_eff = -1.0;
    for (int64_t ks = 1; ks <= 8; ++ks) {
        if (ks > 1 && sw < 8 * ks) break;
        const int64_t u = units * ks;
        const double eff = (double)u / (double)(ceil_div(u, resident) * resident);
        if (eff >= 0.95) {
            best = ks;
            break;
        }
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = ks;
        }
    }
    return ceil_div(sw, ceil_div(sw, best));
}

static size_t carve(size_t &cur, size_t bytes) {
    const size_t o = cur;
    cur += (bytes + 255) & ~(size_t)255;
    return o;
}

// Tile overrides for measurement sweeps: IQP_FWD_TILE = "FMxFN" (4x4, 2x4,
// 2x2), IQP_BWD_TILE (2x4, 2x2; 4x2 for IQP_SPLIT_BF16_FP8), IQP_FWD_SPLITS = number of gate-word splits
// of the forward, IQP_BWD_SPLITS = number of sample-word splits of the
// backward.
static void apply_env_tiles(TileCfg &tc, int prec) {
    const char *f = getenv("IQP_FWD_TILE");
    int a = 0, b = 0;
    if (f && sscanf(f, "%dx%d", &a, &b) == 2 &&
        ((a == 4 && b == 4) || (a == 2 && b == 4) || (a == 2 && b == 2))) {
        tc.fm = a;
        tc.fn = b;
    }
    const char *g = getenv("IQP_BWD_TILE");
    if (g && sscanf(g, "%dx%d", &a, &b) == 2 &&
        ((a == 2 && b == 4) || (a == 2 && b == 2) ||
         (a == 4 && b == 2 && prec == IQP_SPLIT_BF16_FP8))) {
        tc.bfm = a;
        tc.bfn = b;
    }
    const char *sp = getenv("IQP_FWD_SPLITS");
    if (sp && atoi(sp) > 0) tc.splits = atoi(sp);
    const char *bs = getenv("IQP_BWD_SPLITS");
    if (bs && atoi(bs) > 0) tc.bsplits = atoi(bs);
    const char *og = getenv("IQP_BWD_OBGROUP");
    if (og && atoi(og) > 0) tc.obgroup = atoi(og);
}

void make_plan(Plan &P, const PlanParts &parts, int64_t n, int64_t m, int64_t l, int64_t s,
               int64_t N, int prec, const TileCfg &tc) {
    P.tc = tc;
    P.prec = prec;
    P.n = n;
    P.W = ceil_div(n, 64);
    P.m = m;
    P.l = l;
    P.s = s;
    P.N = N;
    P.m_pad = round_up(m, kPad);
    P.l_pad = round_up(l, kPad);
    // the sparse kernels read the sample parities of whole chunks
    P.s_pad = round_up(s, prec == IQP_SPARSE_FP32 ? kEpiChunk : kPad);
    P.mw = P.m_pad / 64;
    P.lw = P.l_pad / 64;
    P.nchunk = ceil_div(s, kEpiChunk);
    const int64_t tiles = (P.l_pad / (32 * P.tc.fm)) * (P.s_pad / (32 * P.tc.fn));
    if (P.tc.splits <= 0) P.tc.splits = choose_splits(tiles, P.mw);
    if (P.tc.splits > P.mw) P.tc.splits = P.mw;
    const int64_t sw = P.s_pad / 64;
    const int64_t bunits = ceil_div(P.m_pad / (32 * P.tc.bfn), 4) * (P.l_pad / (32 * P.tc.bfm));
    if (P.tc.bsplits <= 0)
        P.tc.bsplits = choose_bsplits(bunits, sw, bwd_wgs_per_cu(prec, P.tc.bfm, P.tc.bfn));
    if (prec == IQP_SPLIT3_BF16) {
        // the INT32 sums of the fixed-point weights stay exact per unit
        const int64_t min_ks = ceil_div(sw * 64, kI8MaxSamplesPerUnit);
        if (P.tc.bsplits < min_ks) P.tc.bsplits = min_ks;
    }
    if (P.tc.bsplits > sw) P.tc.bsplits = sw;
    P.tc.bsplits = ceil_div(sw, ceil_div(sw, P.tc.bsplits));
    if (prec == IQP_SPLIT3_BF16) {
        // the INT8 contraction splits whole blocks of two sample words
        const int64_t nb2 = sw / 2;
        if (P.tc.bsplits > nb2) P.tc.bsplits = nb2;
        P.tc.bsplits = ceil_div(nb2, ceil_div(nb2, P.tc.bsplits));
    }
    P.fwd = parts.fwd;
    P.bwd = parts.bwd;
    P.phi = parts.phi;
    P.mmd = parts.mmd;
    size_t cur = 0;
    // bit columns (64 W qubits, plus one zero column, x ld words of 64 rows)
    // for the bit-sliced parity
    P.ldz = round_up(P.s_pad / 64, 4);
    P.lda = round_up(P.l_pad / 64, 4);
    P.o_xz = carve(cur, (size_t)(64 * P.W + 1) * P.ldz * 8);
    P.o_xa = carve(cur, (size_t)(64 * P.W + 1) * P.lda * 8);
    P.o_sup = carve(cur, (size_t)P.m_pad * kSupCap * 4);
    if (prec == IQP_SPARSE_FP32) {
        // C row-major (observable rows) and B^T row-major (generator rows),
        // read by both passes
        P.o_cbits = carve(cur, (size_t)l * P.mw * 8);
        P.o_btbits = carve(cur, (size_t)P.m_pad * (P.s_pad / 64) * 8);
        if (P.fwd) {
            P.o_t32 = carve(cur, (size_t)P.m_pad * 4);
            P.o_part = carve(cur, (size_t)l * P.nchunk * 2 * 8);
            P.o_rowsum = carve(cur, (size_t)l * 2 * 8);
        }
        if (P.phi) P.o_phi = carve(cur, (size_t)l * s * 4);
        if (P.bwd) {
            P.o_coef = carve(cur, (size_t)l * 2 * 8);
            P.o_acc = carve(cur, (size_t)(P.m_pad + 1) * 8);  // int64 sums and a flag
            P.o_scale = carve(cur, 8);
        }
        if (P.mmd) P.o_pstat = carve(cur, (size_t)l * 2 * 8);
        P.total = cur;
        return;
    }
    if (P.fwd) {
        P.o_bbits = carve(cur, (size_t)P.s_pad * P.mw * 8);
        if (prec == IQP_SPLIT_BF16 || prec == IQP_SPLIT3_BF16 || prec == IQP_SPLIT_BF16_FP8) {
            P.o_thh = carve(cur, (size_t)P.m_pad * 2);
            P.o_thl = carve(cur, (size_t)P.m_pad * 2);
            if (prec == IQP_SPLIT3_BF16) P.o_thm = carve(cur, (size_t)P.m_pad * 2);
        } else {
            P.o_t32 = carve(cur, (size_t)P.m_pad * 4);
        }
        P.o_cbits = carve(cur, (size_t)P.l_pad * P.mw * 8);
        P.o_E = carve(cur, (size_t)P.tc.splits * P.l_pad * P.s_pad * 4);
        P.o_part = carve(cur, (size_t)l * P.nchunk * 2 * 8);
        P.o_rowsum = carve(cur, (size_t)l * 2 * 8);
    }
    if (P.phi) P.o_phi = carve(cur, (size_t)l * s * 4);
    if (P.bwd) {
        P.o_coef = carve(cur, (size_t)l * 2 * 8);
        P.o_ctbits = carve(cur, (size_t)P.m_pad * P.lw * 8);
        P.o_btbits = carve(cur, (size_t)P.m_pad * (P.s_pad / 64) * 8);
        if (prec == IQP_SPLIT_BF16) {
            P.o_shi = carve(cur, (size_t)P.s_pad * P.l_pad * 2);
            P.o_slo = carve(cur, (size_t)P.s_pad * P.l_pad * 2);
        } else if (prec == IQP_SPLIT3_BF16) {
            // signed 8-bit limbs, row scales and non-finite flags
            P.o_shi = carve(cur, (size_t)P.s_pad * P.l_pad);
            P.o_slo = carve(cur, (size_t)P.s_pad * P.l_pad);
            P.o_sq = carve(cur, (size_t)P.l_pad * 8);
            P.o_nf = carve(cur, (size_t)P.l_pad * 4);
        } else if (prec == IQP_SPLIT_BF16_FP8) {
            // FP16 limbs, FP8 limbs, row scales 2^-e_k (rows past l are never
            // read: their C^T bits are 0)
            P.o_shi = carve(cur, (size_t)P.s_pad * P.l_pad * 2);
            P.o_slo = carve(cur, (size_t)P.s_pad * P.l_pad);
            P.o_sq = carve(cur, (size_t)P.l_pad * 8);
        } else {
            P.o_s32 = carve(cur, (size_t)P.s_pad * P.l_pad * 4);
        }
        P.o_gpart = carve(cur, (size_t)P.tc.bsplits * (P.l_pad / (32 * P.tc.bfm)) * P.m_pad * 4);
    }
    if (P.mmd) {
        P.o_pstat = carve(cur, (size_t)l * 2 * 8);
    }
    P.total = cur;
}

// Plan of the bitflip-circuit calls: bit columns and support lists for the C
// parity, C (tiled32), the encoded factors and per-observable sums, and C^T
// for the gradient.
static void make_bitflip_plan(Plan &P, bool grad, int64_t n, int64_t m, int64_t l) {
    P = Plan();
    P.n = n;
    P.W = ceil_div(n, 64);
    P.m = m;
    P.l = l;
    P.m_pad = round_up(m, kPad);
    P.l_pad = round_up(l, kPad);
    P.mw = P.m_pad / 64;
    P.lw = P.l_pad / 64;
    P.lda = round_up(P.l_pad / 64, 4);
    size_t cur = 0;
    P.o_xa = carve(cur, (size_t)(64 * P.W + 1) * P.lda * 8);
    P.o_sup = carve(cur, (size_t)P.m_pad * kSupCap * 4);
    P.o_cbits = carve(cur, (size_t)P.l_pad * P.mw * 8);
    P.o_enc = carve(cur, (size_t)P.m_pad * 8);
    P.o_stat = carve(cur, (size_t)P.l_pad * 2 * 8);
    P.o_rowsum = carve(cur, (size_t)P.l_pad * 8);  // the product, when only the gradient is asked
    if (grad) P.o_ctbits = carve(cur, (size_t)P.m_pad * P.lw * 8);
    P.total = cur;
}

// Plan of the independent-estimate calls (the sparse form over one sample
// set per observable): bit columns of A, support lists, C row-major,
// 2 theta', the bit columns of every observable's sample set (ldz words per
// column), the forward's sums, and the gradient's buffers.
static void make_indep_plan(Plan &P, int call, int64_t n, int64_t m, int64_t l, int64_t s) {
    P = Plan();
    P.prec = IQP_SPARSE_FP32;
    P.n = n;
    P.W = ceil_div(n, 64);
    P.m = m;
    P.l = l;
    P.s = s;
    P.m_pad = round_up(m, kPad);
    P.l_pad = round_up(l, kPad);
    P.s_pad = round_up(s, kPad);
    P.mw = P.m_pad / 64;
    P.lw = P.l_pad / 64;
    P.nchunk = ceil_div(s, kEpiChunk);
    P.fwd = call != IQP_CALL_INDEP_GRAD;
    P.bwd = call != IQP_CALL_INDEP;
    P.phi = call == IQP_CALL_INDEP_GRAD_RECOMPUTE;
    P.lda = round_up(P.l_pad / 64, 4);
    P.ldz = round_up(ceil_div(s, 64), kEpiChunk / 64);  // whole chunks, zero past s
    size_t cur = 0;
    P.o_xa = carve(cur, (size_t)(64 * P.W + 1) * P.lda * 8);
    P.o_sup = carve(cur, (size_t)P.m_pad * kSupCap * 4);
    P.o_cbits = carve(cur, (size_t)l * P.mw * 8);
    P.o_xz = carve(cur, (size_t)l * 64 * P.W * P.ldz * 8);
    if (P.fwd) {
        P.o_t32 = carve(cur, (size_t)P.m_pad * 4);
        P.o_part = carve(cur, (size_t)l * P.nchunk * 2 * 8);
        P.o_rowsum = carve(cur, (size_t)l * 2 * 8);
    }
    if (P.phi) P.o_phi = carve(cur, (size_t)l * s * 4);
    if (P.bwd) {
        P.o_coef = carve(cur, (size_t)l * 2 * 8);
        P.o_acc = carve(cur, (size_t)(P.m_pad + 1) * 8);
        P.o_scale = carve(cur, 8);
    }
    P.total = cur;
}

// Plan of a single-problem call: its parts, the default tiles and any
// override from the environment.
static void make_call_plan(Plan &P, int call, int64_t n, int64_t m, int64_t l, int64_t s,
                           int64_t N, int prec) {
    PlanParts parts;
    parts.fwd = call != IQP_CALL_EXPVAL_GRAD;
    parts.bwd = call == IQP_CALL_EXPVAL_GRAD || call == IQP_CALL_EXPVAL_GRAD_RECOMPUTE ||
                call == IQP_CALL_MMD_GRAD;
    parts.phi = call == IQP_CALL_EXPVAL_GRAD_RECOMPUTE || call == IQP_CALL_MMD_GRAD;
    parts.mmd = call == IQP_CALL_MMD || call == IQP_CALL_MMD_GRAD;
    TileCfg tc;
    // the BF16 backward runs the 64 x 128 wave tile at two waves per SIMD:
    // half the LDS reads of the 64 x 64 tile per product (n = 300 workload:
    // 1.245 -> 1.161 ms per backward)
    if (prec == IQP_SPLIT_BF16) tc.bfn = 4;
    // the FP16 + FP8 backward runs 128 x 64: its B operands (the FP16 and the
    // FP8 +-1 expansions) serve four row blocks instead of two, half the
    // vector work per product (n = 300: 0.972 -> 0.952 ms; 64 circuits:
    // 160 -> 154 ms)
    if (prec == IQP_SPLIT_BF16_FP8) tc.bfm = 4;
    apply_env_tiles(tc, prec);
    make_plan(P, parts, n, m, l, s, N, prec, tc);
}

int check_circuit(const iqp_circuit *c) {
    if (!c) return fail(IQP_ERR_INVALID_ARG, "circuit is NULL");
    if (c->n_qubits < 1) return fail(IQP_ERR_INVALID_ARG, "n_qubits must be >= 1");
    if (c->n_words != (int32_t)ceil_div(c->n_qubits, 64))
        return fail(IQP_ERR_INVALID_ARG, "n_words must equal ceil(n_qubits / 64)");
    if (c->n_gates < 1 || c->n_gates > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_gates out of range [1, 2^24]");
    if (!c->gens) return fail(IQP_ERR_INVALID_ARG, "gens is NULL");
    if (!c->theta) return fail(IQP_ERR_INVALID_ARG, "theta is NULL");
    return IQP_OK;
}

static int check_common(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                        const uint64_t *samples, int precision) {
    int st = check_circuit(c);
    if (st) return st;
    if (l < 1 || l > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "l out of range [1, 2^24]");
    if (s < 1 || s > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "s out of range [1, 2^24]");
    if (!ops) return fail(IQP_ERR_INVALID_ARG, "ops is NULL");
    if (!samples) return fail(IQP_ERR_INVALID_ARG, "samples is NULL");
    if (!valid_precision(precision))
        return fail(IQP_ERR_INVALID_ARG, "precision must be IQP_FP32, IQP_SPLIT_BF16, "
                                         "IQP_SPARSE_FP32, IQP_SPLIT3_BF16 or "
                                         "IQP_SPLIT_BF16_FP8");
    return IQP_OK;
}

static int check_ws(const Plan &P, void *ws, size_t ws_bytes) {
    if (ws_bytes < P.total)
        return fail(IQP_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) +
                                           " bytes, need " + std::to_string(P.total));
    if (!ws) return fail(IQP_ERR_INVALID_ARG, "ws is NULL");
    return IQP_OK;
}


// The sparse kernels' sample parities: B^T row-major, shared by all observables.
static SampleParity shared_parity(const Plan &P, void *ws) {
    return SampleParity{at<uint64_t>(ws, P.o_btbits), nullptr, P.s_pad / 64, 0, nullptr, nullptr,
                        (int)P.W};
}

// Independent estimates: the bit columns of each observable's own samples.
static SampleParity indep_parity(const Plan &P, const iqp_circuit *c, void *ws) {
    return SampleParity{nullptr,     at<uint64_t>(ws, P.o_xz), P.ldz,   64 * P.W * P.ldz,
                        at<int32_t>(ws, P.o_sup), c->gens,     (int)P.W};
}

// C row-major and the per-observable sample bit columns of the independent
// estimates.
static int run_indep_parities(const Plan &P, const iqp_circuit *c, const uint64_t *ops,
                              const uint64_t *samples, void *ws, const LaunchCtx &lc) {
    IQP_TRY(launch_support(lc, support_args(P, c->gens, ws)), "support");
    IQP_TRY(launch_bitslice(lc, bitslice_ops_args(P, ops, ws)), "bitslice(A)");
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_ROW_MAJOR,
                             ParityArgs{c->gens, at<int32_t>(ws, P.o_sup), P.m, (int)P.W,
                                        at<uint64_t>(ws, P.o_xa), P.l_pad / 64, P.lda, P.l, P.mw,
                                        at<uint64_t>(ws, P.o_cbits)}),
            "parity(C, row-major)");
    IQP_TRY(launch_indep_slice(lc, IndepSliceArgs{samples, P.l, P.s, (int)P.W, P.ldz,
                                                  at<uint64_t>(ws, P.o_xz)}),
            "bitslice(per-observable Z)");
    return IQP_OK;
}

// Sparse form: the row-major C and B^T parities its kernels walk.
static int run_sparse_parities(const Plan &P, const iqp_circuit *c, const uint64_t *ops,
                               const uint64_t *samples, void *ws, const LaunchCtx &lc) {
    IQP_TRY(launch_support(lc, support_args(P, c->gens, ws)), "support");
    IQP_TRY(launch_bitslice(lc, bitslice_ops_args(P, ops, ws)), "bitslice(A)");
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_ROW_MAJOR,
                             ParityArgs{c->gens, at<int32_t>(ws, P.o_sup), P.m, (int)P.W,
                                        at<uint64_t>(ws, P.o_xa), P.l_pad / 64, P.lda, P.l, P.mw,
                                        at<uint64_t>(ws, P.o_cbits)}),
            "parity(C, row-major)");
    IQP_TRY(launch_bitslice(lc, bitslice_samples_args(P, samples, ws)), "bitslice(Z)");
    IQP_TRY(launch_parity_bs(lc, 3,
                             ParityArgs{c->gens, at<int32_t>(ws, P.o_sup), P.m, (int)P.W,
                                        at<uint64_t>(ws, P.o_xz), P.s_pad / 64, P.ldz, 0, P.mw,
                                        at<uint64_t>(ws, P.o_btbits)}),
            "parity(B^T, row-major)");
    return IQP_OK;
}

static int run_forward(const Plan &P, const iqp_circuit *c, const uint64_t *ops,
                       const uint64_t *samples, void *ws, const LaunchCtx &lc, float *phase_out,
                       double *mean, double *se, double *rowsum) {
    if (P.prec == IQP_SPARSE_FP32) {
        IQP_TRY(launch_theta_prep(lc, theta_args(P, c->theta, ws)), "theta_prep");
        int st = run_sparse_parities(P, c, ops, samples, ws, lc);
        if (st) return st;
        IQP_TRY(launch_sparse_fwd(lc, SparseFwdArgs{at<uint64_t>(ws, P.o_cbits), P.mw,
                                                    at<float>(ws, P.o_t32), shared_parity(P, ws),
                                                    P.l, P.s, phase_out,
                                                    at<double>(ws, P.o_part)}),
                "sparse_fwd");
        IQP_TRY(launch_finalize(lc, fin_args(P, ws, mean, se, rowsum)), "finalize");
        return IQP_OK;
    }
    IQP_TRY(launch_theta_prep(lc, theta_args(P, c->theta, ws)), "theta_prep");
    IQP_TRY(launch_support(lc, support_args(P, c->gens, ws)), "support");
    IQP_TRY(launch_bitslice(lc, bitslice_ops_args(P, ops, ws)), "bitslice(A)");
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_TILED32, parity_c_args(P, c->gens, ws)), "parity(C)");
    IQP_TRY(launch_bitslice(lc, bitslice_samples_args(P, samples, ws)), "bitslice(Z)");
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_TILED32, parity_b_args(P, c->gens, ws)), "parity(B)");
    IQP_TRY(launch_phase_fwd(lc, P.prec, P.tc.fm, P.tc.fn, fwd_args(P, ws, P.tc.splits)),
            "phase_fwd");
    IQP_TRY(launch_epilogue(lc, epi_args(P, ws, P.tc.splits, phase_out)), "phase_epilogue");
    IQP_TRY(launch_finalize(lc, fin_args(P, ws, mean, se, rowsum)), "finalize");
    return IQP_OK;
}

// Backward from the coefficients at o_coef and the phases `phase`. When the
// forward ran in the same call, the bit columns of A and Z are already in the
// workspace.
static int run_backward(const Plan &P, const iqp_circuit *c, const uint64_t *ops,
                        const uint64_t *samples, const float *phase, bool bitcols_ready, void *ws,
                        const LaunchCtx &lc, double *grad_theta) {
    if (P.prec == IQP_SPARSE_FP32) {
        long long *acc = at<long long>(ws, P.o_acc);
        double *scale = at<double>(ws, P.o_scale);
        IQP_TRY(launch_sparse_bound(lc, SparseBoundArgs{at<double>(ws, P.o_coef), P.l, P.s,
                                                        P.m_pad, acc, scale}),
                "sparse_bound");
        if (!bitcols_ready) {
            int st = run_sparse_parities(P, c, ops, samples, ws, lc);
            if (st) return st;
        }
        IQP_TRY(launch_sparse_bwd(lc, SparseBwdArgs{at<uint64_t>(ws, P.o_cbits), P.mw,
                                                    shared_parity(P, ws), P.l, P.s, P.m_pad,
                                                    phase, at<double>(ws, P.o_coef), scale, acc}),
                "sparse_bwd");
        IQP_TRY(launch_sparse_finish(lc, SparseFinishArgs{acc, scale, P.m, P.m_pad, grad_theta}),
                "sparse_finish");
        return IQP_OK;
    }
    IQP_TRY(launch_weights(lc, weights_args(P, phase, ws)), "weights");
    if (!bitcols_ready) {
        IQP_TRY(launch_support(lc, support_args(P, c->gens, ws)), "support");
        IQP_TRY(launch_bitslice(lc, bitslice_ops_args(P, ops, ws)), "bitslice(A)");
        IQP_TRY(launch_bitslice(lc, bitslice_samples_args(P, samples, ws)), "bitslice(Z)");
    }
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_TILED32_T, parity_bt_args(P, c->gens, ws)),
            "parity(B^T)");
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_TILED32_T, parity_ct_args(P, c->gens, ws)),
            "parity(C^T)");
    IQP_TRY(launch_phase_bwd(lc, P.prec, P.tc.bfm, P.tc.bfn, bwd_args(P, ws)), "phase_bwd");
    IQP_TRY(launch_grad_reduce(lc, grad_args(P, ws, P.tc.bfm, grad_theta)), "grad_reduce");
    return IQP_OK;
}

int expval_call(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                const uint64_t *samples, int precision, double *mean, double *stderr_,
                float *phase_save, void *ws, size_t ws_bytes, void *stream, bool timing) {
    int st = check_common(c, l, ops, s, samples, precision);
    if (st) return st;
    if (!mean) return fail(IQP_ERR_INVALID_ARG, "mean is NULL");
    Plan P;
    make_call_plan(P, IQP_CALL_EXPVAL, c->n_qubits, c->n_gates, l, s, 0, precision);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    LaunchCtx lc = make_ctx(stream);
    lc.timing = lc.timing && timing;
    return run_forward(P, c, ops, samples, ws, lc, phase_save, mean, stderr_,
                       at<double>(ws, P.o_rowsum));
}

LaunchCtx make_ctx(void *stream) {
    LaunchCtx lc;
    lc.stream = reinterpret_cast<hipStream_t>(stream);
    lc.timing = g_timing.on;
    return lc;
}

bool timing_enabled() { return g_timing.on; }

}  // namespace iqp

using namespace iqp;

#ifndef IQP_SOURCE_SHA256
#define IQP_SOURCE_SHA256 "unknown"
#endif

extern "C" {

const char *iqp_source_sha256(void) { return IQP_SOURCE_SHA256; }

size_t iqp_workspace_bytes(int call, const iqp_circuit *c, int64_t l, int64_t s, int64_t N,
                           int precision) {
    if (!c || c->n_qubits < 1 || c->n_gates < 1 || l < 1) return 0;
    if (call == IQP_CALL_BITFLIP || call == IQP_CALL_BITFLIP_GRAD) {
        Plan P;
        make_bitflip_plan(P, call == IQP_CALL_BITFLIP_GRAD, c->n_qubits, c->n_gates, l);
        return P.total;
    }
    if (s < 1) return 0;
    if (call >= IQP_CALL_INDEP && call <= IQP_CALL_INDEP_GRAD_RECOMPUTE) {
        if (l * s > kMaxIndepRows) return 0;
        Plan P;
        make_indep_plan(P, call, c->n_qubits, c->n_gates, l, s);
        return P.total;
    }
    if (call < IQP_CALL_EXPVAL || call > IQP_CALL_MMD_GRAD) return 0;
    if (!valid_precision(precision)) return 0;
    if ((call == IQP_CALL_MMD || call == IQP_CALL_MMD_GRAD) && N < 1) return 0;
    Plan P;
    make_call_plan(P, call, c->n_qubits, c->n_gates, l, s, N, precision);
    return P.total;
}

static int64_t parity_rows_out(int64_t n_rows, int layout) {
    return layout == IQP_BITS_ROW_MAJOR ? n_rows : round_up(n_rows, 32);
}

// iqp_parity workspace: bit columns of the rows, then the support lists of
// the columns (n_cols rounded up to 64).
static size_t parity_xt_bytes(int64_t n_rows, int32_t n_words, int layout) {
    const int64_t rw = ceil_div(parity_rows_out(n_rows, layout), 64);
    return ((size_t)(64 * (int64_t)n_words + 1) * round_up(rw, 4) * 8 + 255) & ~(size_t)255;
}

size_t iqp_parity_workspace_bytes(int64_t n_rows, int64_t n_cols, int32_t n_words, int layout) {
    if (n_rows < 0 || n_cols < 0 || n_words < 1) return 0;
    return parity_xt_bytes(n_rows, n_words, layout) +
           (size_t)round_up(n_cols, 64) * kSupCap * 4 + 256;
}

int iqp_parity(int64_t n_rows, const uint64_t *rows, int64_t n_cols, const uint64_t *cols,
               int32_t n_words, int layout, uint64_t *out, void *ws, size_t ws_bytes,
               void *stream) {
    g_last_error.clear();
    if (n_rows < 0 || n_rows > kMaxRows * 4) return fail(IQP_ERR_INVALID_ARG, "n_rows out of range");
    if (n_cols < 0 || n_cols > kMaxRows * 4) return fail(IQP_ERR_INVALID_ARG, "n_cols out of range");
    if (n_words < 1) return fail(IQP_ERR_INVALID_ARG, "n_words must be >= 1");
    if (layout != IQP_BITS_ROW_MAJOR && layout != IQP_BITS_TILED32 && layout != IQP_BITS_TILED32_T)
        return fail(IQP_ERR_INVALID_ARG, "unknown layout");
    if (n_rows == 0 || n_cols == 0) return IQP_OK;
    if (!rows || !cols || !out) return fail(IQP_ERR_INVALID_ARG, "NULL pointer");
    const size_t need = iqp_parity_workspace_bytes(n_rows, n_cols, n_words, layout);
    if (ws_bytes < need)
        return fail(IQP_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) +
                                           " bytes, need " + std::to_string(need));
    if (!ws) return fail(IQP_ERR_INVALID_ARG, "ws is NULL");
    int st = check_device();
    if (st) return st;
    LaunchCtx lc = make_ctx(stream);
    const int64_t R_out = parity_rows_out(n_rows, layout);
    const int64_t rw = ceil_div(R_out, 64);
    const int64_t ldx = round_up(rw, 4);
    uint64_t *xt = static_cast<uint64_t *>(ws);
    int32_t *sup = at<int32_t>(ws, parity_xt_bytes(n_rows, n_words, layout));
    const int64_t Gw = ceil_div(n_cols, 64);
    IQP_TRY(launch_bitslice(lc, BitsliceArgs{rows, n_rows, n_words, ldx, xt}), "bitslice");
    IQP_TRY(launch_support(lc, SupportArgs{cols, n_cols, n_words, Gw * 64, sup}), "support");
    if (layout == IQP_BITS_TILED32_T)
        IQP_TRY(launch_parity_bs(lc, layout,
                                 ParityArgs{cols, sup, n_cols, n_words, xt, ceil_div(n_rows, 64),
                                            ldx, 0, Gw, out}),
                "parity");
    else
        IQP_TRY(launch_parity_bs(lc, layout,
                                 ParityArgs{cols, sup, n_cols, n_words, xt, rw, ldx, R_out, Gw,
                                            out}),
                "parity");
    return IQP_OK;
}

int iqp_expval(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
               const uint64_t *samples, int precision, double *mean, double *stderr_,
               float *phase_save, void *ws, size_t ws_bytes, void *stream) {
    g_last_error.clear();
    return expval_call(c, l, ops, s, samples, precision, mean, stderr_, phase_save, ws, ws_bytes,
                       stream, true);
}

int iqp_expval_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                    const uint64_t *samples, int precision, const double *grad_mean,
                    const float *phase_save, double *grad_theta, void *ws, size_t ws_bytes,
                    void *stream) {
    g_last_error.clear();
    int st = check_common(c, l, ops, s, samples, precision);
    if (st) return st;
    if (!grad_mean) return fail(IQP_ERR_INVALID_ARG, "grad_mean is NULL");
    if (!grad_theta) return fail(IQP_ERR_INVALID_ARG, "grad_theta is NULL");
    Plan P;
    const int call = phase_save ? IQP_CALL_EXPVAL_GRAD : IQP_CALL_EXPVAL_GRAD_RECOMPUTE;
    make_call_plan(P, call, c->n_qubits, c->n_gates, l, s, 0, precision);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    LaunchCtx lc = make_ctx(stream);
    const float *phase = phase_save;
    if (!phase) {
        st = run_forward(P, c, ops, samples, ws, lc, at<float>(ws, P.o_phi), nullptr, nullptr,
                         at<double>(ws, P.o_rowsum));
        if (st) return st;
        phase = at<float>(ws, P.o_phi);
    }
    IQP_TRY(launch_coef_plain(lc, coef_args(P, grad_mean, ws)), "coef");
    return run_backward(P, c, ops, samples, phase, phase_save == nullptr, ws, lc, grad_theta);
}

// Forward of the independent estimates into the plan's buffers.
static int run_indep_forward(const Plan &P, const iqp_circuit *c, const uint64_t *ops,
                             const uint64_t *samples, void *ws, const LaunchCtx &lc,
                             float *phase_out, double *mean, double *se) {
    IQP_TRY(launch_theta_prep(lc, theta_args(P, c->theta, ws)), "theta_prep");
    int st = run_indep_parities(P, c, ops, samples, ws, lc);
    if (st) return st;
    IQP_TRY(launch_sparse_fwd(lc, SparseFwdArgs{at<uint64_t>(ws, P.o_cbits), P.mw,
                                                at<float>(ws, P.o_t32), indep_parity(P, c, ws),
                                                P.l, P.s, phase_out, at<double>(ws, P.o_part)}),
            "sparse_fwd(indep)");
    IQP_TRY(launch_finalize(lc, fin_args(P, ws, mean, se, at<double>(ws, P.o_rowsum))),
            "finalize");
    return IQP_OK;
}

static int check_indep(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                       const uint64_t *samples) {
    int st = check_common(c, l, ops, s, samples, IQP_SPARSE_FP32);
    if (st) return st;
    if (l * s > kMaxIndepRows)
        return fail(IQP_ERR_INVALID_ARG, "l * s above 2^32 sample rows");
    return IQP_OK;
}

int iqp_expval_indep(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                     const uint64_t *samples, double *mean, double *stderr_, float *phase_save,
                     void *ws, size_t ws_bytes, void *stream) {
    g_last_error.clear();
    int st = check_indep(c, l, ops, s, samples);
    if (st) return st;
    if (!mean) return fail(IQP_ERR_INVALID_ARG, "mean is NULL");
    Plan P;
    make_indep_plan(P, IQP_CALL_INDEP, c->n_qubits, c->n_gates, l, s);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    return run_indep_forward(P, c, ops, samples, ws, make_ctx(stream), phase_save, mean,
                             stderr_);
}

int iqp_expval_indep_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops, int64_t s,
                          const uint64_t *samples, const double *grad_mean,
                          const float *phase_save, double *grad_theta, void *ws,
                          size_t ws_bytes, void *stream) {
    g_last_error.clear();
    int st = check_indep(c, l, ops, s, samples);
    if (st) return st;
    if (!grad_mean) return fail(IQP_ERR_INVALID_ARG, "grad_mean is NULL");
    if (!grad_theta) return fail(IQP_ERR_INVALID_ARG, "grad_theta is NULL");
    Plan P;
    make_indep_plan(P, phase_save ? IQP_CALL_INDEP_GRAD : IQP_CALL_INDEP_GRAD_RECOMPUTE,
                    c->n_qubits, c->n_gates, l, s);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    LaunchCtx lc = make_ctx(stream);
    const float *phase = phase_save;
    if (!phase) {
        if ((st = run_indep_forward(P, c, ops, samples, ws, lc, at<float>(ws, P.o_phi), nullptr,
                                    nullptr)))
            return st;
        phase = at<float>(ws, P.o_phi);
    } else if ((st = run_indep_parities(P, c, ops, samples, ws, lc))) {
        return st;
    }
    IQP_TRY(launch_coef_plain(lc, coef_args(P, grad_mean, ws)), "coef");
    long long *acc = at<long long>(ws, P.o_acc);
    double *scale = at<double>(ws, P.o_scale);
    IQP_TRY(launch_sparse_bound(lc, SparseBoundArgs{at<double>(ws, P.o_coef), P.l, P.s, P.m_pad,
                                                    acc, scale}),
            "sparse_bound");
    IQP_TRY(launch_sparse_bwd(lc, SparseBwdArgs{at<uint64_t>(ws, P.o_cbits), P.mw,
                                                indep_parity(P, c, ws), P.l, P.s, P.m_pad, phase,
                                                at<double>(ws, P.o_coef), scale, acc}),
            "sparse_bwd(indep)");
    IQP_TRY(launch_sparse_finish(lc, SparseFinishArgs{acc, scale, P.m, P.m_pad, grad_theta}),
            "sparse_finish");
    return IQP_OK;
}

int iqp_mmd_loss_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops,
                      const double *op_weight, int64_t s, const uint64_t *samples, int64_t N,
                      const uint64_t *data, int unbiased, int precision, double *loss,
                      double *grad_theta, void *ws, size_t ws_bytes, void *stream) {
    g_last_error.clear();
    int st = check_common(c, l, ops, s, samples, precision);
    if (st) return st;
    if (!op_weight) return fail(IQP_ERR_INVALID_ARG, "op_weight is NULL");
    if (N < 1 || N > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "N out of range [1, 2^24]");
    if (!data) return fail(IQP_ERR_INVALID_ARG, "data is NULL");
    if (!loss) return fail(IQP_ERR_INVALID_ARG, "loss is NULL");
    if (unbiased && (N < 2 || s < 2))
        return fail(IQP_ERR_INVALID_ARG, "the unbiased estimator needs N >= 2 and s >= 2");
    Plan P;
    make_call_plan(P, grad_theta ? IQP_CALL_MMD_GRAD : IQP_CALL_MMD, c->n_qubits, c->n_gates, l, s, N,
              precision);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    LaunchCtx lc = make_ctx(stream);
    float *phi = grad_theta ? at<float>(ws, P.o_phi) : nullptr;
    st = run_forward(P, c, ops, samples, ws, lc, phi, nullptr, nullptr, at<double>(ws, P.o_rowsum));
    if (st) return st;
    IQP_TRY(launch_data_stats(lc, ops, l, data, N, (int)P.W, at<double>(ws, P.o_pstat)),
            "data_stats");
    IQP_TRY(launch_mmd_loss(lc, at<double>(ws, P.o_pstat), at<double>(ws, P.o_rowsum), op_weight,
                            l, s, N, unbiased, loss),
            "mmd_loss");
    if (!grad_theta) return IQP_OK;
    const CoefArgs ca = coef_args(P, nullptr, ws);
    IQP_TRY(launch_coef_mmd(lc, at<double>(ws, P.o_pstat), at<double>(ws, P.o_rowsum), op_weight,
                            l, s, unbiased, ca.coef, ca.sq, ca.nf),
            "coef_mmd");
    return run_backward(P, c, ops, samples, phi, true, ws, lc, grad_theta);
}

// Forward of a bitflip circuit into the plan's buffers (mean may be the
// workspace's own slot).
static int run_bitflip_forward(const Plan &P, const iqp_circuit *c, const uint64_t *ops,
                               void *ws, const LaunchCtx &lc, double *mean) {
    IQP_TRY(launch_bitflip_prep(lc, BitflipPrepArgs{c->theta, P.m, at<double>(ws, P.o_enc)}),
            "bitflip_prep");
    IQP_TRY(launch_support(lc, support_args(P, c->gens, ws)), "support");
    IQP_TRY(launch_bitslice(lc, BitsliceArgs{ops, P.l, (int)P.W, P.lda, at<uint64_t>(ws, P.o_xa)}),
            "bitslice(A)");
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_TILED32,
                             ParityArgs{c->gens, at<int32_t>(ws, P.o_sup), P.m, (int)P.W,
                                        at<uint64_t>(ws, P.o_xa), P.l_pad / 64, P.lda, P.l_pad,
                                        P.mw, at<uint64_t>(ws, P.o_cbits)}),
            "parity(C)");
    IQP_TRY(launch_bitflip_fwd(lc, BitflipFwdArgs{at<uint64_t>(ws, P.o_cbits),
                                                   at<double>(ws, P.o_enc), P.l, P.mw, mean,
                                                   nullptr, at<double>(ws, P.o_stat)}),
            "bitflip_fwd");
    return IQP_OK;
}

int iqp_bitflip_expval(const iqp_circuit *c, int64_t l, const uint64_t *ops, double *mean,
                       void *ws, size_t ws_bytes, void *stream) {
    g_last_error.clear();
    int st = check_circuit(c);
    if (st) return st;
    if (l < 1 || l > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "l out of range [1, 2^24]");
    if (!ops) return fail(IQP_ERR_INVALID_ARG, "ops is NULL");
    if (!mean) return fail(IQP_ERR_INVALID_ARG, "mean is NULL");
    Plan P;
    make_bitflip_plan(P, false, c->n_qubits, c->n_gates, l);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    return run_bitflip_forward(P, c, ops, ws, make_ctx(stream), mean);
}

int iqp_bitflip_expval_grad(const iqp_circuit *c, int64_t l, const uint64_t *ops,
                            const double *grad_mean, double *grad_theta, void *ws,
                            size_t ws_bytes, void *stream) {
    g_last_error.clear();
    int st = check_circuit(c);
    if (st) return st;
    if (l < 1 || l > kMaxRows) return fail(IQP_ERR_INVALID_ARG, "l out of range [1, 2^24]");
    if (!ops) return fail(IQP_ERR_INVALID_ARG, "ops is NULL");
    if (!grad_mean) return fail(IQP_ERR_INVALID_ARG, "grad_mean is NULL");
    if (!grad_theta) return fail(IQP_ERR_INVALID_ARG, "grad_theta is NULL");
    Plan P;
    make_bitflip_plan(P, true, c->n_qubits, c->n_gates, l);
    if ((st = check_ws(P, ws, ws_bytes))) return st;
    if ((st = check_device())) return st;
    LaunchCtx lc = make_ctx(stream);
    st = run_bitflip_forward(P, c, ops, ws, lc, at<double>(ws, P.o_rowsum));
    if (st) return st;
    IQP_TRY(launch_parity_bs(lc, IQP_BITS_TILED32_T,
                             ParityArgs{c->gens, at<int32_t>(ws, P.o_sup), P.m, (int)P.W,
                                        at<uint64_t>(ws, P.o_xa), P.lw, P.lda, 0, P.mw,
                                        at<uint64_t>(ws, P.o_ctbits)}),
            "parity(C^T)");
    IQP_TRY(launch_bitflip_grad(lc, BitflipGradArgs{at<uint64_t>(ws, P.o_ctbits),
                                                     at<double>(ws, P.o_enc), c->theta,
                                                     at<double>(ws, P.o_stat), grad_mean, P.m,
                                                     P.lw, grad_theta}),
            "bitflip_grad");
    return IQP_OK;
}

const char *iqp_strerror(int status) {
    switch (status) {
        case IQP_OK: return "success";
        case IQP_ERR_INVALID_ARG: return "invalid argument";
        case IQP_ERR_WORKSPACE: return "workspace too small";
        case IQP_ERR_HIP: return "HIP runtime error";
        case IQP_ERR_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

const char *iqp_last_error(void) { return g_last_error.c_str(); }

int iqp_profile_enable(int on) {
    g_timing.on = on != 0;
    return IQP_OK;
}

int iqp_profile_query(const char *name, double *total_ms, int64_t *launches) {
    if (!name || !total_ms || !launches) return fail(IQP_ERR_INVALID_ARG, "NULL pointer");
    hipError_t e = drain_timing();
    if (e != hipSuccess) return hip_fail(e, "profile drain");
    for (int f = 0; f < KF_COUNT; ++f) {
        if (strcmp(name, kFamilyNames[f]) == 0) {
            *total_ms = g_timing.total_ms[f];
            *launches = g_timing.launches[f];
            return IQP_OK;
        }
    }
    return fail(IQP_ERR_INVALID_ARG, std::string("unknown kernel family ") + name);
}

int iqp_profile_reset(void) {
    hipError_t e = drain_timing();
    for (int f = 0; f < KF_COUNT; ++f) {
        g_timing.total_ms[f] = 0.0;
        g_timing.launches[f] = 0;
    }
    return e == hipSuccess ? IQP_OK : hip_fail(e, "profile drain");
}

}  // extern "C"
