// Batched form of the estimator: a plan over many problems of uneven size
// (shapes, workspace layout, tile configuration), the per-call table of step
// arguments, graph capture and replay of each pass, and the autotuner that
// picks the tile configuration by timing the candidates on the problems.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "iqp.h"
#include "iqp_internal.h"
#include "iqp_plan.h"

namespace iqp {

struct BatchCfg {
    int fm = 4, fn = 4;    // forward wave tile (32-blocks)
    int split = 1;         // forward gate-word split mode (0, 1, 2)
    int bfm = 2, bfn = 2;  // backward wave tile
    bool tuned = false;
};

static bool same_tiles(const BatchCfg &a, const BatchCfg &b) {
    return a.fm == b.fm && a.fn == b.fn && a.split == b.split && a.bfm == b.bfm && a.bfn == b.bfn;
}

// (the 128 x 64 backward tile exists for the FP16 + FP8 form only)
static bool valid_cfg(const BatchCfg &c, int prec) {
    const bool f = (c.fm == 4 && c.fn == 4) || (c.fm == 2 && c.fn == 4) || (c.fm == 2 && c.fn == 2);
    const bool b = (c.bfm == 2 && (c.bfn == 2 || c.bfn == 4)) ||
                   (c.bfm == 4 && c.bfn == 2 && prec == IQP_SPLIT_BF16_FP8);
    return f && b && c.split >= 0 && c.split <= 2;
}

static const int kFwdTiles[3][2] = {{4, 4}, {2, 4}, {2, 2}};
static const int kBwdTiles[3][2] = {{2, 2}, {2, 4}, {4, 2}};
static int n_bwd_tiles(int prec) { return prec == IQP_SPLIT_BF16_FP8 ? 3 : 2; }
static const int kMaxSplit = 16;
static const int kMaxProblems = 1 << 16;

// Kinds beyond the batched step kinds: the persistent contractions.
enum { SK_FWD_PERSISTENT = 100, SK_BWD_PERSISTENT = 101 };

struct StepRec {
    int kind;
    size_t args_off, off_off;  // byte offsets in the table
    int jobs;
    int64_t total;  // blocks (batched) or work units (persistent)
};

// Host image of a pass's argument table; arrays 64-byte aligned.
struct Table {
    std::vector<char> buf;
    std::vector<StepRec> steps;
    size_t push(const void *p, size_t bytes) {
        const size_t o = (buf.size() + 63) & ~(size_t)63;
        buf.resize(o + bytes);
        if (bytes) memcpy(buf.data() + o, p, bytes);
        return o;
    }
    template <typename A>
    void add(int kind, const std::vector<A> &args, const std::vector<int64_t> &counts) {
        std::vector<int64_t> off(args.size() + 1, 0);
        for (size_t i = 0; i < args.size(); ++i) off[i + 1] = off[i] + counts[i];
        StepRec r;
        r.kind = kind;
        r.args_off = push(args.data(), sizeof(A) * args.size());
        r.off_off = push(off.data(), sizeof(int64_t) * off.size());
        r.jobs = (int)args.size();
        r.total = off.back();
        steps.push_back(r);
    }
};

// Gate-word splits of each problem's forward in split mode `mode`: none (0),
// or so that no work unit is longer than 1/4 (1) or 1/16 (2) of one
// workgroup's share of the pass (at least 8 gate words per split).
static std::vector<int64_t> batch_splits(const std::vector<Plan> &plans, int fm, int fn, int mode,
                                         int grid) {
    std::vector<int64_t> sp(plans.size(), 1);
    if (mode == 0 || grid < 1) return sp;
    double total = 0.0;
    for (const Plan &P : plans)
        total += (double)((P.l_pad / (32 * fm)) * ceil_div(P.s_pad / (32 * fn), 4)) * (double)P.mw;
    const double share = total / grid;
    const double maxw = std::max(8.0, share / (mode == 1 ? 4.0 : 16.0));
    for (size_t p = 0; p < plans.size(); ++p) {
        int64_t k = (int64_t)std::ceil((double)plans[p].mw / maxw);
        k = std::min<int64_t>(k, std::max<int64_t>(1, plans[p].mw / 8));
        sp[p] = std::max<int64_t>(1, std::min<int64_t>(k, kMaxSplit));
    }
    return sp;
}

// Process-wide record of tuned configurations, keyed by precision and shapes.
static std::mutex g_tune_mu;
static std::map<std::string, BatchCfg> g_tune;
static bool g_tune_loaded = false;

static std::string shape_key(int prec, const std::vector<Plan> &plans) {
    std::string k = "prec" + std::to_string(prec) + ":";
    for (const Plan &P : plans)
        k += std::to_string(P.n) + "," + std::to_string(P.m) + "," + std::to_string(P.l) + "," +
             std::to_string(P.s) + ";";
    return k;
}

// IQP_TUNE_CACHE lines: "<key> <fm> <fn> <split> <bfm> <bfn>"
static void load_tune_file_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = getenv("IQP_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    std::string line;
    int ch;
    while (true) {
        line.clear();
        while ((ch = fgetc(f)) != EOF && ch != '\n') line.push_back((char)ch);
        if (!line.empty()) {
            const size_t sp = line.find(' ');
            int prec = -1;
            if (sp != std::string::npos && sscanf(line.c_str(), "prec%d:", &prec) == 1) {
                BatchCfg c;
                if (sscanf(line.c_str() + sp + 1, "%d %d %d %d %d", &c.fm, &c.fn, &c.split, &c.bfm,
                           &c.bfn) == 5 &&
                    valid_cfg(c, prec)) {
                    c.tuned = true;
                    g_tune[line.substr(0, sp)] = c;
                }
            }
        }
        if (ch == EOF) break;
    }
    fclose(f);
}

static bool lookup_tuned(const std::string &key, BatchCfg *out) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

static void record_tuned(const std::string &key, const BatchCfg &c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_file_locked();
    g_tune[key] = c;
    const char *path = getenv("IQP_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), c.fm, c.fn, c.split, c.bfm, c.bfn);
    fclose(f);
}

}  // namespace iqp

using namespace iqp;

struct iqp_batch_plan {
    int np = 0, prec = 0, flags = 0;
    std::vector<Plan> plans;     // per problem layout, sized for every configuration
    std::vector<size_t> region;  // byte offset of each problem's buffers
    size_t table_off[2] = {0, 0}, table_bytes[2] = {0, 0};
    size_t counters_off = 0;
    size_t total = 0;
    BatchCfg cfg;
    std::string key;
    int grid_fwd[3] = {0, 0, 0}, grid_bwd[3] = {0, 0, 0};
    void *staging[2] = {nullptr, nullptr};
    size_t staging_bytes = 0;
    hipEvent_t staged[2] = {nullptr, nullptr};
    int next = 0;
    hipStream_t cap = nullptr;
    struct Graph {
        hipGraphExec_t exec = nullptr;
        void *ws = nullptr;
        BatchCfg cfg;
    } graph[2];
};

namespace iqp {

static int fwd_tile_index(const BatchCfg &c) {
    for (int i = 0; i < 3; ++i)
        if (kFwdTiles[i][0] == c.fm && kFwdTiles[i][1] == c.fn) return i;
    return -1;
}
static int bwd_tile_index(const BatchCfg &c) {
    for (int i = 0; i < 3; ++i)
        if (kBwdTiles[i][0] == c.bfm && kBwdTiles[i][1] == c.bfn) return i;
    return -1;
}

// Argument table of one pass (0 forward, 1 backward) for the plan's current
// configuration. `probs` may be NULL (sizes only).
static void build_table(const iqp_batch_plan *bp, int pass, const iqp_problem *probs, void *ws,
                        Table &tb) {
    const int np = bp->np;
    const BatchCfg &c = bp->cfg;
    auto base = [&](int p) -> void * {
        return ws ? static_cast<char *>(ws) + bp->region[p] : nullptr;
    };
    auto pr = [&](int p) -> const iqp_problem * { return probs ? &probs[p] : nullptr; };
    std::vector<BitsliceArgs> bs;
    std::vector<SupportArgs> su;
    std::vector<ParityArgs> par;
    std::vector<int64_t> bsn, sun, parn;
    for (int p = 0; p < np; ++p) {
        const Plan &P = bp->plans[p];
        const iqp_problem *q = pr(p);
        su.push_back(support_args(P, q ? q->circuit.gens : nullptr, base(p)));
        sun.push_back(blocks_of(su.back()));
        bs.push_back(bitslice_ops_args(P, q ? q->ops : nullptr, base(p)));
        bs.push_back(bitslice_samples_args(P, q ? q->samples : nullptr, base(p)));
        const uint64_t *g = q ? q->circuit.gens : nullptr;
        if (pass == 0) {
            par.push_back(parity_c_args(P, g, base(p)));
            par.push_back(parity_b_args(P, g, base(p)));
        } else {
            par.push_back(parity_bt_args(P, g, base(p)));
            par.push_back(parity_ct_args(P, g, base(p)));
        }
    }
    for (auto &a : bs) bsn.push_back(blocks_of(a));
    for (auto &a : par) parn.push_back(blocks_of(a));

    // persistent contractions take the problems with the longest work units first
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    if (pass == 0) {
        const int ti = fwd_tile_index(c);
        const std::vector<int64_t> sp =
            batch_splits(bp->plans, c.fm, c.fn, c.split, ti >= 0 ? bp->grid_fwd[ti] : 1);
        std::vector<ThetaArgs> th;
        std::vector<EpiArgs> ep;
        std::vector<FinArgs> fi;
        std::vector<int64_t> thn, epn, fin;
        for (int p = 0; p < np; ++p) {
            const Plan &P = bp->plans[p];
            const iqp_problem *q = pr(p);
            th.push_back(theta_args(P, q ? q->circuit.theta : nullptr, base(p)));
            ep.push_back(epi_args(P, base(p), sp[p], q ? q->phase_save : nullptr));
            fi.push_back(fin_args(P, base(p), q ? q->mean : nullptr, q ? q->stderr_ : nullptr,
                                  nullptr));
            thn.push_back(blocks_of(th.back()));
            epn.push_back(blocks_of(ep.back()));
            fin.push_back(blocks_of(fi.back()));
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return ceil_div(bp->plans[a].mw, sp[a]) > ceil_div(bp->plans[b].mw, sp[b]);
        });
        std::vector<FwdArgs> fw;
        std::vector<int64_t> fwn;
        for (int p : order) {
            fw.push_back(fwd_args(bp->plans[p], base(p), sp[p]));
            fwn.push_back(fwd_units(fw.back(), c.fm, c.fn));
        }
        tb.add(SK_THETA, th, thn);
        tb.add(SK_SUPPORT, su, sun);
        tb.add(SK_BITSLICE, bs, bsn);
        tb.add(SK_PARITY1, par, parn);
        tb.add(SK_FWD_PERSISTENT, fw, fwn);
        tb.add(SK_EPI, ep, epn);
        tb.add(SK_FIN, fi, fin);
    } else {
        std::vector<CoefArgs> co;
        std::vector<WeightsArgs> we;
        std::vector<GradArgs> gr;
        std::vector<int64_t> con, wen, grn;
        for (int p = 0; p < np; ++p) {
            const Plan &P = bp->plans[p];
            const iqp_problem *q = pr(p);
            co.push_back(coef_args(P, q ? q->grad_mean : nullptr, base(p)));
            we.push_back(weights_args(P, q ? q->phase_save : nullptr, base(p)));
            gr.push_back(grad_args(P, base(p), c.bfm, q ? q->grad_theta : nullptr));
            con.push_back(blocks_of(co.back()));
            wen.push_back(blocks_of(we.back()));
            grn.push_back(blocks_of(gr.back()));
        }
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return bp->plans[a].s_pad > bp->plans[b].s_pad;
        });
        std::vector<BwdArgs> bw;
        std::vector<int64_t> bwn;
        for (int p : order) {
            bw.push_back(bwd_args(bp->plans[p], base(p)));
            bwn.push_back(bwd_units(bw.back(), c.bfm, c.bfn));
        }
        tb.add(SK_COEF, co, con);
        tb.add(SK_WEIGHTS, we, wen);
        tb.add(SK_SUPPORT, su, sun);
        tb.add(SK_BITSLICE, bs, bsn);
        tb.add(SK_PARITY2, par, parn);
        tb.add(SK_BWD_PERSISTENT, bw, bwn);
        tb.add(SK_GRAD, gr, grn);
    }
}

// The kernels of one pass, in order, on lc.stream (plain launches or inside a
// graph capture). The table must already be in the workspace.
static int enqueue_pass(const iqp_batch_plan *bp, int pass, const Table &tb, void *ws,
                        const LaunchCtx &lc) {
    char *tbl = static_cast<char *>(ws) + bp->table_off[pass];
    unsigned long long *counter =
        at<unsigned long long>(ws, bp->counters_off) + (pass == 0 ? 0 : 1);
    IQP_TRY(launch_reset_counters(lc, counter, 1), "reset_counters");
    const BatchCfg &c = bp->cfg;
    for (const StepRec &r : tb.steps) {
        const void *args = tbl + r.args_off;
        const int64_t *off = reinterpret_cast<const int64_t *>(tbl + r.off_off);
        if (r.total == 0) continue;
        if (r.kind == SK_FWD_PERSISTENT) {
            const int grid = (int)std::min<int64_t>(bp->grid_fwd[fwd_tile_index(c)], r.total);
            IQP_TRY(launch_phase_fwd_persistent(lc, bp->prec, c.fm, c.fn,
                                                static_cast<const FwdArgs *>(args), off, r.jobs,
                                                counter, grid),
                    "phase_fwd (persistent)");
        } else if (r.kind == SK_BWD_PERSISTENT) {
            const int grid = (int)std::min<int64_t>(bp->grid_bwd[bwd_tile_index(c)], r.total);
            IQP_TRY(launch_phase_bwd_persistent(lc, bp->prec, c.bfm, c.bfn,
                                                static_cast<const BwdArgs *>(args), off, r.jobs,
                                                counter, grid),
                    "phase_bwd (persistent)");
        } else {
            IQP_TRY(launch_batched(lc, r.kind, args, off, r.jobs, r.total), "batched step");
        }
    }
    return IQP_OK;
}

// Copies the table to the workspace on `stream` through a pinned staging
// buffer (two, alternating; a buffer is reused only after its copy ended).
static int upload_table(iqp_batch_plan *bp, int pass, const Table &tb, void *ws,
                        hipStream_t stream) {
    if (tb.buf.size() > bp->table_bytes[pass] || tb.buf.size() > bp->staging_bytes)
        return fail(IQP_ERR_HIP, "internal: argument table larger than planned");
    const int i = bp->next;
    bp->next ^= 1;
    IQP_TRY(hipEventSynchronize(bp->staged[i]), "hipEventSynchronize(staging)");
    memcpy(bp->staging[i], tb.buf.data(), tb.buf.size());
    IQP_TRY(hipMemcpyAsync(static_cast<char *>(ws) + bp->table_off[pass], bp->staging[i],
                           tb.buf.size(), hipMemcpyHostToDevice, stream),
            "hipMemcpyAsync(table)");
    IQP_TRY(hipEventRecord(bp->staged[i], stream), "hipEventRecord(staging)");
    return IQP_OK;
}

// The graph of a pass for this workspace and configuration (captured on first
// use, recaptured when either changes).
static int pass_graph(iqp_batch_plan *bp, int pass, const Table &tb, void *ws,
                      hipGraphExec_t *out) {
    auto &g = bp->graph[pass];
    if (g.exec && g.ws == ws && same_tiles(g.cfg, bp->cfg)) {
        *out = g.exec;
        return IQP_OK;
    }
    if (g.exec) {
        IQP_TRY(hipGraphExecDestroy(g.exec), "hipGraphExecDestroy");
        g.exec = nullptr;
    }
    IQP_TRY(hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal),
            "hipStreamBeginCapture");
    LaunchCtx lc;
    lc.stream = bp->cap;
    lc.timing = false;
    const int st = enqueue_pass(bp, pass, tb, ws, lc);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(bp->cap, &graph);
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
    g.cfg = bp->cfg;
    *out = g.exec;
    return IQP_OK;
}

static int check_problem_shape(const iqp_problem &q, int i) {
    const std::string at_i = " (problem " + std::to_string(i) + ")";
    int st = check_circuit(&q.circuit);
    if (st) return fail(st, std::string(iqp_last_error()) + at_i);
    if (q.n_ops < 1 || q.n_ops > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_ops out of range [1, 2^24]" + at_i);
    if (q.n_samples < 1 || q.n_samples > kMaxRows)
        return fail(IQP_ERR_INVALID_ARG, "n_samples out of range [1, 2^24]" + at_i);
    return IQP_OK;
}

// The problems of a call: the plan's shapes and the pointers the pass reads
// and writes.
static int check_call(const iqp_batch_plan *bp, const iqp_problem *probs, int pass, void *ws,
                      size_t ws_bytes) {
    if (!bp) return fail(IQP_ERR_INVALID_ARG, "plan is NULL");
    if (!probs) return fail(IQP_ERR_INVALID_ARG, "probs is NULL");
    for (int p = 0; p < bp->np; ++p) {
        const iqp_problem &q = probs[p];
        const Plan &P = bp->plans[p];
        const std::string at_p = " (problem " + std::to_string(p) + ")";
        if (q.circuit.n_qubits != P.n || q.circuit.n_words != P.W || q.circuit.n_gates != P.m ||
            q.n_ops != P.l || q.n_samples != P.s)
            return fail(IQP_ERR_INVALID_ARG, "shape differs from the plan's" + at_p);
        if (!q.circuit.gens || !q.ops || !q.samples)
            return fail(IQP_ERR_INVALID_ARG, "gens, ops or samples is NULL" + at_p);
        if (pass == 0 && (!q.circuit.theta || !q.mean))
            return fail(IQP_ERR_INVALID_ARG, "theta or mean is NULL" + at_p);
        if (pass == 1 && (!q.grad_mean || !q.phase_save || !q.grad_theta))
            return fail(IQP_ERR_INVALID_ARG, "grad_mean, phase_save or grad_theta is NULL" + at_p);
    }
    if (ws_bytes < bp->total)
        return fail(IQP_ERR_WORKSPACE, "workspace of " + std::to_string(ws_bytes) +
                                           " bytes, need " + std::to_string(bp->total));
    if (!ws) return fail(IQP_ERR_INVALID_ARG, "ws is NULL");
    return check_device();
}

static int run_pass(iqp_batch_plan *bp, int pass, const iqp_problem *probs, void *ws,
                    void *stream, bool force_plain) {
    Table tb;
    build_table(bp, pass, probs, ws, tb);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc = upload_table(bp, pass, tb, ws, st);
    if (rc) return rc;
    if (force_plain || (bp->flags & IQP_BATCH_NO_GRAPH) || timing_enabled())
        return enqueue_pass(bp, pass, tb, ws, make_ctx(stream));
    hipGraphExec_t exec = nullptr;
    if ((rc = pass_graph(bp, pass, tb, ws, &exec))) return rc;
    IQP_TRY(hipGraphLaunch(exec, st), "hipGraphLaunch");
    return IQP_OK;
}

// Milliseconds of one pass under the plan's current configuration (best of
// two after one warm-up), launched step by step.
static int time_pass(iqp_batch_plan *bp, int pass, const iqp_problem *probs, void *ws,
                     void *stream, float *ms_out) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    IQP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        hipEventDestroy(e0);
        return hip_fail(he, "hipEventCreate");
    }
    int rc = IQP_OK;
    float best = -1.0f;
    for (int rep = 0; rep < 3 && rc == IQP_OK; ++rep) {
        if ((he = hipEventRecord(e0, st)) != hipSuccess) { rc = hip_fail(he, "hipEventRecord"); break; }
        if ((rc = run_pass(bp, pass, probs, ws, stream, true))) break;
        if ((he = hipEventRecord(e1, st)) != hipSuccess) { rc = hip_fail(he, "hipEventRecord"); break; }
        if ((he = hipEventSynchronize(e1)) != hipSuccess) { rc = hip_fail(he, "hipEventSynchronize"); break; }
        float ms = 0.0f;
        if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { rc = hip_fail(he, "hipEventElapsedTime"); break; }
        if (rep > 0 && (best < 0.0f || ms < best)) best = ms;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms_out = best;
    return rc;
}

static void destroy_plan(iqp_batch_plan *bp) {
    if (!bp) return;
    for (auto &g : bp->graph)
        if (g.exec) hipGraphExecDestroy(g.exec);
    for (int i = 0; i < 2; ++i) {
        if (bp->staged[i]) {
            hipEventSynchronize(bp->staged[i]);
            hipEventDestroy(bp->staged[i]);
        }
        if (bp->staging[i]) hipHostFree(bp->staging[i]);
    }
    if (bp->cap) hipStreamDestroy(bp->cap);
    delete bp;
}

}  // namespace iqp

extern "C" {

int iqp_batch_plan_create(int32_t n_problems, const iqp_problem *probs, int precision, int flags,
                          iqp_batch_plan **plan) {
    clear_error();
    if (!plan) return fail(IQP_ERR_INVALID_ARG, "plan is NULL");
    *plan = nullptr;
    if (n_problems < 1 || n_problems > kMaxProblems)
        return fail(IQP_ERR_INVALID_ARG, "n_problems out of range [1, 65536]");
    if (!probs) return fail(IQP_ERR_INVALID_ARG, "probs is NULL");
    if (!dense_precision(precision))
        return fail(IQP_ERR_INVALID_ARG, "precision must be IQP_FP32, IQP_SPLIT_BF16, "
                                         "IQP_SPLIT3_BF16 or IQP_SPLIT_BF16_FP8");
    if (flags & ~(int)IQP_BATCH_NO_GRAPH) return fail(IQP_ERR_INVALID_ARG, "unknown flags");
    int st;
    for (int p = 0; p < n_problems; ++p)
        if ((st = check_problem_shape(probs[p], p))) return st;
    if ((st = check_device())) return st;

    iqp_batch_plan *bp = new iqp_batch_plan();
    bp->np = n_problems;
    bp->prec = precision;
    bp->flags = flags;
    for (int i = 0; i < 3; ++i) {
        bp->grid_fwd[i] = persistent_grid(true, precision, kFwdTiles[i][0], kFwdTiles[i][1]);
        if (bp->grid_fwd[i] < 1) {
            destroy_plan(bp);
            return fail(IQP_ERR_HIP, "occupancy query of the forward contraction failed");
        }
    }
    for (int i = 0; i < n_bwd_tiles(precision); ++i) {
        bp->grid_bwd[i] = persistent_grid(false, precision, kBwdTiles[i][0], kBwdTiles[i][1]);
        if (bp->grid_bwd[i] < 1) {
            destroy_plan(bp);
            return fail(IQP_ERR_HIP, "occupancy query of the backward contraction failed");
        }
    }
    // layouts with the default tiles, then the largest split count any
    // configuration may use
    PlanParts parts;
    parts.fwd = true;
    parts.bwd = true;
    TileCfg tc0;
    tc0.splits = 1;
    tc0.bfm = 2;
    tc0.bsplits = 1;  // the work queue balances the backward
    // Grouped unit order helps launches whose workgroups stay on one XCD in
    // contiguous unit ranges; the persistent queue hands consecutive units to
    // all XCDs, where groups of 4 only add fetches (about 1.4x the bytes) and
    // cost 3 % of clock and time, so none here. Per-XCD queues did not help
    // either: chunks of 32..256 consecutive units per XCD fetched twice the
    // bytes and ran 3 % slower; unit u on XCD u % 8 with groups of 8 (each
    // XCD keeping one S strip, all eight walking the same B^T strips) cut the
    // fetches by 8 % and ran 0.7 % slower.
    tc0.obgroup = 1;
    const char *og = getenv("IQP_BWD_OBGROUP");  // unit-order override for sweeps
    if (og && atoi(og) > 0) tc0.obgroup = atoi(og);
    bp->plans.resize(n_problems);
    for (int p = 0; p < n_problems; ++p) {
        const iqp_problem &q = probs[p];
        make_plan(bp->plans[p], parts, q.circuit.n_qubits, q.circuit.n_gates, q.n_ops,
                  q.n_samples, 0, precision, tc0);
    }
    std::vector<int64_t> maxsp(n_problems, 1);
    for (int i = 0; i < 3; ++i)
        for (int mode = 1; mode <= 2; ++mode) {
            const auto sp = batch_splits(bp->plans, kFwdTiles[i][0], kFwdTiles[i][1], mode,
                                         bp->grid_fwd[i]);
            for (int p = 0; p < n_problems; ++p) maxsp[p] = std::max(maxsp[p], sp[p]);
        }
    size_t cur = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = cur;
        cur += (bytes + 255) & ~(size_t)255;
        return o;
    };
    for (int pass = 0; pass < 2; ++pass) {
        Table tb;
        build_table(bp, pass, nullptr, nullptr, tb);
        bp->table_bytes[pass] = tb.buf.size() + 64;
        bp->table_off[pass] = carve(bp->table_bytes[pass]);
    }
    bp->counters_off = carve(256);
    bp->region.resize(n_problems);
    for (int p = 0; p < n_problems; ++p) {
        const iqp_problem &q = probs[p];
        TileCfg tc = tc0;
        tc.splits = maxsp[p];
        make_plan(bp->plans[p], parts, q.circuit.n_qubits, q.circuit.n_gates, q.n_ops,
                  q.n_samples, 0, precision, tc);
        bp->region[p] = carve(bp->plans[p].total);
    }
    bp->total = cur;
    bp->key = shape_key(precision, bp->plans);
    BatchCfg c;
    // the defaults of single calls
    if (precision == IQP_SPLIT_BF16) bp->cfg.bfn = 4;
    if (precision == IQP_SPLIT_BF16_FP8) bp->cfg.bfm = 4;
    if (lookup_tuned(bp->key, &c)) bp->cfg = c;

    bp->staging_bytes = std::max(bp->table_bytes[0], bp->table_bytes[1]);
    if ((st = injected_fault("alloc"))) {
        destroy_plan(bp);
        return st;
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc(&bp->staging[i], bp->staging_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&bp->staged[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        destroy_plan(bp);
        return hip_fail(e, "plan resources");
    }
    *plan = bp;
    return IQP_OK;
}

int iqp_batch_plan_destroy(iqp_batch_plan *plan) {
    destroy_plan(plan);
    return IQP_OK;
}

size_t iqp_batch_workspace_bytes(const iqp_batch_plan *plan) { return plan ? plan->total : 0; }

int iqp_batch_expval(iqp_batch_plan *plan, const iqp_problem *probs, void *ws, size_t ws_bytes,
                     void *stream) {
    clear_error();
    int st = check_call(plan, probs, 0, ws, ws_bytes);
    if (st) return st;
    return run_pass(plan, 0, probs, ws, stream, false);
}

int iqp_batch_expval_grad(iqp_batch_plan *plan, const iqp_problem *probs, void *ws,
                          size_t ws_bytes, void *stream) {
    clear_error();
    int st = check_call(plan, probs, 1, ws, ws_bytes);
    if (st) return st;
    return run_pass(plan, 1, probs, ws, stream, false);
}

int iqp_batch_tune(iqp_batch_plan *plan, const iqp_problem *probs, int passes, void *ws,
                   size_t ws_bytes, void *stream) {
    clear_error();
    if (passes < 1 || passes > 3) return fail(IQP_ERR_INVALID_ARG, "passes must be 1, 2 or 3");
    int st;
    if ((passes & 1) && (st = check_call(plan, probs, 0, ws, ws_bytes))) return st;
    if ((passes & 2) && (st = check_call(plan, probs, 1, ws, ws_bytes))) return st;
    BatchCfg best = plan->cfg;
    if (passes & 1) {
        float best_ms = -1.0f;
        for (int i = 0; i < 3; ++i)
            for (int mode = 0; mode <= 2; ++mode) {
                plan->cfg.fm = kFwdTiles[i][0];
                plan->cfg.fn = kFwdTiles[i][1];
                plan->cfg.split = mode;
                float ms = 0.0f;
                if ((st = time_pass(plan, 0, probs, ws, stream, &ms))) {
                    plan->cfg = best;
                    return st;
                }
                if (best_ms < 0.0f || ms < best_ms) {
                    best_ms = ms;
                    best.fm = plan->cfg.fm;
                    best.fn = plan->cfg.fn;
                    best.split = mode;
                }
            }
        plan->cfg = best;
    }
    if (passes & 2) {
        float best_ms = -1.0f;
        for (int i = 0; i < n_bwd_tiles(plan->prec); ++i) {
            plan->cfg.bfm = kBwdTiles[i][0];
            plan->cfg.bfn = kBwdTiles[i][1];
            float ms = 0.0f;
            if ((st = time_pass(plan, 1, probs, ws, stream, &ms))) {
                plan->cfg = best;
                return st;
            }
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                best.bfm = plan->cfg.bfm;
                best.bfn = plan->cfg.bfn;
            }
        }
    }
    best.tuned = true;
    plan->cfg = best;
    record_tuned(plan->key, best);
    return IQP_OK;
}

int iqp_batch_get_config(const iqp_batch_plan *plan, int32_t *cfg6) {
    clear_error();
    if (!plan || !cfg6) return fail(IQP_ERR_INVALID_ARG, "NULL pointer");
    const BatchCfg &c = plan->cfg;
    cfg6[0] = c.fm;
    cfg6[1] = c.fn;
    cfg6[2] = c.split;
    cfg6[3] = c.bfm;
    cfg6[4] = c.bfn;
    cfg6[5] = c.tuned ? 1 : 0;
    return IQP_OK;
}

int iqp_batch_set_config(iqp_batch_plan *plan, const int32_t *cfg5) {
    clear_error();
    if (!plan || !cfg5) return fail(IQP_ERR_INVALID_ARG, "NULL pointer");
    BatchCfg c;
    c.fm = cfg5[0];
    c.fn = cfg5[1];
    c.split = cfg5[2];
    c.bfm = cfg5[3];
    c.bfn = cfg5[4];
    if (!valid_cfg(c, plan->prec)) return fail(IQP_ERR_INVALID_ARG, "unsupported tile configuration");
    plan->cfg = c;
    return IQP_OK;
}

}  // extern "C"
