/*
 * IQP expectation-value ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously correct FP64 CPU reference for the Monte Carlo
 * estimator of Pauli-Z expectation values of parameterized IQP circuits
 * (arXiv 2501.04776), its gradient and the MMD^2 loss built on it, plus exact
 * values used only as pins (state-vector simulation, the subset expansion of
 * Prop. 3's proof, the product form), and the random streams of the training
 * loop (Philox4x64-10 and the bit samplers built on it). Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library; the product path
 * never links or calls it, and it shares no code with the HIP path.
 *
 * Representations (independent of the HIP path's packed words):
 *   gates   : index lists in CSR form, gptr[m+1] (int64), gidx (int32 qubits)
 *   rows    : dense 0/1 bytes, row r qubit q = rows[r*n + q]
 *             (observables a_k, samples z_i, training data x_n)
 *
 * Parity unpinned: none. Every routine here is pinned by a CPU test against
 * the paper's closed forms, a state-vector simulation or brute force.
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <sched.h>
#include <stdio.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_OK 0
#define ORC_ERR_ARG -1
#define ORC_ERR_MEM -2
#define ORC_ERR_SIZE -3

/* |supp(g_j) ∩ supp(x)| for a 0/1 row x: walk g_j's index list. */
static int64_t overlap(const uint8_t *x, const int64_t *gptr, const int32_t *gidx, int64_t j)
{
    int64_t c = 0;
    for (int64_t t = gptr[j]; t < gptr[j + 1]; ++t)
        c += x[gidx[t]];
    return c;
}

/* (-1)^{g_j . x} */
static double sign_of(const uint8_t *x, const int64_t *gptr, const int32_t *gidx, int64_t j)
{
    return (overlap(x, gptr, gidx, j) & 1) ? -1.0 : 1.0;
}

/* Threads = CPUs in this process's affinity mask, capped by OMP_NUM_THREADS
 * when that is set (the host's share of cores for this job). */
int orc_num_threads(void)
{
    int n = 0;
    cpu_set_t set;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
    if (n <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        n = c > 0 ? (int)c : 1;
    }
    const char *env = getenv("OMP_NUM_THREADS");
    if (env) {
        int cap = atoi(env);
        if (cap > 0 && cap < n) n = cap;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Parity bits: out[r*m + j] = |g_j ∩ rows_r| mod 2 (the exponent of the
 * matrices B = (-1)^{Z G^T} and C = 1 - (-1)^{A G^T}, Sec. 2.2). */
int orc_parity(int64_t n, int64_t R, const uint8_t *rows, int64_t m, const int64_t *gptr,
               const int32_t *gidx, uint8_t *out)
{
    if (n < 1 || R < 0 || m < 0) return ORC_ERR_ARG;
    for (int64_t r = 0; r < R; ++r)
        for (int64_t j = 0; j < m; ++j)
            out[r * m + j] = (uint8_t)(overlap(rows + r * n, gptr, gidx, j) & 1);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Threading helper: a static split of observables over threads. */
typedef struct {
    int64_t k0, k1;
    void *ctx;
    int tid;
} range_t;

typedef void (*range_fn)(range_t *);

static int run_ranges(int64_t count, int nthreads, range_fn fn, void *ctx)
{
    if (nthreads <= 0) nthreads = orc_num_threads();
    if (nthreads > count) nthreads = count > 0 ? (int)count : 1;
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    range_t *rg = malloc(sizeof(range_t) * nthreads);
    if (!th || !rg) { free(th); free(rg); return ORC_ERR_MEM; }
    for (int t = 0; t < nthreads; ++t) {
        rg[t].k0 = count * t / nthreads;
        rg[t].k1 = count * (t + 1) / nthreads;
        rg[t].ctx = ctx;
        rg[t].tid = t;
    }
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, (void *(*)(void *))fn, &rg[t]);
    fn(&rg[0]);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    free(th);
    free(rg);
    return ORC_OK;
}

typedef struct {
    int64_t n, m, l, s;
    const int64_t *gptr;
    const int32_t *gidx;
    const double *theta;
    const uint8_t *ops, *samples;
    /* expval outputs */
    double *mean, *stderr_;
    float *phases;          /* optional [l][s]: the raw phase E_ki */
    double *phases64;       /* optional [l][s] */
    /* gradient */
    const double *grad_mean;
    double *grad_part;      /* [nthreads][m] */
    /* mmd */
    const double *op_weight;
    int64_t N;
    const uint8_t *data;
    int unbiased;
    double *loss_part;      /* [nthreads] */
    double *phat, *qhat;    /* optional [l] diagnostics */
    /* samples of observable k start at samples + k * zstride: 0 when all
     * observables share one set, s * n for independent sets (the l x s x n
     * option of Sec. 2.3) */
    int64_t zstride;
    int status;
} job_t;

/* J_k = {j : C_kj != 0}, with C_kj = 1 - (-1)^{a_k . g_j} in {0, 2}. */
static int64_t anticommuting(const job_t *jb, int64_t k, int64_t *J, double *Ckj)
{
    int64_t cnt = 0;
    const uint8_t *a = jb->ops + k * jb->n;
    for (int64_t j = 0; j < jb->m; ++j) {
        double c = 1.0 - sign_of(a, jb->gptr, jb->gidx, j);
        if (c != 0.0) {
            J[cnt] = j;
            Ckj[cnt] = c;
            ++cnt;
        }
    }
    return cnt;
}

/* Sample i of observable k. */
static const uint8_t *sample_of(const job_t *jb, int64_t k, int64_t i)
{
    return jb->samples + k * jb->zstride + i * jb->n;
}

/* E_ki = sum_j B_ij C_kj theta_j (eq. Emat), summed over j in J_k ascending:
 * the terms with C_kj = 0 vanish exactly. */
static double phase(const job_t *jb, int64_t k, int64_t i, const int64_t *J, const double *Ckj,
                    int64_t nj)
{
    const uint8_t *z = sample_of(jb, k, i);
    double e = 0.0;
    for (int64_t t = 0; t < nj; ++t) {
        int64_t j = J[t];
        e += sign_of(z, jb->gptr, jb->gidx, j) * Ckj[t] * jb->theta[j];
    }
    return e;
}

/* Sample mean of cos E_ki over the s samples (eq. expvalsample) and its
 * standard error: population standard deviation / sqrt(s). */
static void expval_range(range_t *rg)
{
    job_t *jb = rg->ctx;
    int64_t *J = malloc(sizeof(int64_t) * (jb->m + 1));
    double *C = malloc(sizeof(double) * (jb->m + 1));
    if (!J || !C) { jb->status = ORC_ERR_MEM; free(J); free(C); return; }
    for (int64_t k = rg->k0; k < rg->k1; ++k) {
        int64_t nj = anticommuting(jb, k, J, C);
        double sc = 0.0, sc2 = 0.0;
        for (int64_t i = 0; i < jb->s; ++i) {
            double e = phase(jb, k, i, J, C, nj);
            if (jb->phases) jb->phases[k * jb->s + i] = (float)e;
            if (jb->phases64) jb->phases64[k * jb->s + i] = e;
            double c = cos(e);
            sc += c;
            sc2 += c * c;
        }
        double mu = sc / (double)jb->s;
        double var = sc2 / (double)jb->s - mu * mu;
        jb->mean[k] = mu;
        if (jb->stderr_) jb->stderr_[k] = sqrt((var > 0.0 ? var : 0.0) / (double)jb->s);
    }
    free(J);
    free(C);
}

int orc_expval(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
               const double *theta, int64_t l, const uint8_t *ops, int64_t s,
               const uint8_t *samples, double *mean, double *stderr_, double *phases,
               int nthreads)
{
    if (n < 1 || m < 0 || l < 0 || s < 1 || !mean) return ORC_ERR_ARG;
    job_t jb = {0};
    jb.n = n; jb.m = m; jb.l = l; jb.s = s;
    jb.gptr = gptr; jb.gidx = gidx; jb.theta = theta;
    jb.ops = ops; jb.samples = samples;
    jb.mean = mean; jb.stderr_ = stderr_; jb.phases64 = phases;
    int st = run_ranges(l, nthreads, expval_range, &jb);
    return st ? st : jb.status;
}

/* ------------------------------------------------------------------------ */
/* Gradient of L(mean) with u_k = dL/dmean_k:
 *   dmean_k/dtheta_j = -(1/s) sum_i sin(E_ki) B_ij C_kj,
 *   dL/dtheta_j = sum_k u_k dmean_k/dtheta_j.
 * Each thread accumulates into its own row of grad_part; rows are summed in
 * thread order afterwards. */
static void grad_range(range_t *rg)
{
    job_t *jb = rg->ctx;
    int64_t *J = malloc(sizeof(int64_t) * (jb->m + 1));
    double *C = malloc(sizeof(double) * (jb->m + 1));
    double *g = jb->grad_part + (int64_t)rg->tid * jb->m;
    if (!J || !C) { jb->status = ORC_ERR_MEM; free(J); free(C); return; }
    for (int64_t k = rg->k0; k < rg->k1; ++k) {
        int64_t nj = anticommuting(jb, k, J, C);
        double u = jb->grad_mean[k];
        if (u == 0.0) continue;
        for (int64_t i = 0; i < jb->s; ++i) {
            const uint8_t *z = sample_of(jb, k, i);
            double e = phase(jb, k, i, J, C, nj);
            double w = -u * sin(e) / (double)jb->s;
            for (int64_t t = 0; t < nj; ++t)
                g[J[t]] += w * sign_of(z, jb->gptr, jb->gidx, J[t]) * C[t];
        }
    }
    free(J);
    free(C);
}

static int reduce_parts(const double *part, int nparts, int64_t m, double *out)
{
    for (int64_t j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int t = 0; t < nparts; ++t) acc += part[(int64_t)t * m + j];
        out[j] = acc;
    }
    return ORC_OK;
}

int orc_expval_grad(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                    const double *theta, int64_t l, const uint8_t *ops, int64_t s,
                    const uint8_t *samples, const double *grad_mean, double *grad_theta,
                    int nthreads)
{
    if (n < 1 || m < 0 || l < 0 || s < 1 || !grad_theta || !grad_mean) return ORC_ERR_ARG;
    if (nthreads <= 0) nthreads = orc_num_threads();
    if (nthreads > l) nthreads = l > 0 ? (int)l : 1;
    job_t jb = {0};
    jb.n = n; jb.m = m; jb.l = l; jb.s = s;
    jb.gptr = gptr; jb.gidx = gidx; jb.theta = theta;
    jb.ops = ops; jb.samples = samples; jb.grad_mean = grad_mean;
    jb.grad_part = calloc((size_t)nthreads * (size_t)(m > 0 ? m : 1), sizeof(double));
    if (!jb.grad_part) return ORC_ERR_MEM;
    int st = run_ranges(l, nthreads, grad_range, &jb);
    if (!st) st = jb.status;
    if (!st) reduce_parts(jb.grad_part, nthreads, m, grad_theta);
    free(jb.grad_part);
    return st;
}

/* Independent estimates: observable k averages over its own s samples,
 * samples[k][i][q] (the l x s x n sample tensor of Sec. 2.3), so that the
 * estimates of different observables are uncorrelated. Same estimator and
 * gradient as above otherwise. */
int orc_expval_indep(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                     const double *theta, int64_t l, const uint8_t *ops, int64_t s,
                     const uint8_t *samples, double *mean, double *stderr_, double *phases,
                     int nthreads)
{
    if (n < 1 || m < 0 || l < 0 || s < 1 || !mean) return ORC_ERR_ARG;
    job_t jb = {0};
    jb.n = n; jb.m = m; jb.l = l; jb.s = s;
    jb.gptr = gptr; jb.gidx = gidx; jb.theta = theta;
    jb.ops = ops; jb.samples = samples; jb.zstride = s * n;
    jb.mean = mean; jb.stderr_ = stderr_; jb.phases64 = phases;
    int st = run_ranges(l, nthreads, expval_range, &jb);
    return st ? st : jb.status;
}

int orc_expval_indep_grad(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                          const double *theta, int64_t l, const uint8_t *ops, int64_t s,
                          const uint8_t *samples, const double *grad_mean, double *grad_theta,
                          int nthreads)
{
    if (n < 1 || m < 0 || l < 0 || s < 1 || !grad_theta || !grad_mean) return ORC_ERR_ARG;
    if (nthreads <= 0) nthreads = orc_num_threads();
    if (nthreads > l) nthreads = l > 0 ? (int)l : 1;
    job_t jb = {0};
    jb.n = n; jb.m = m; jb.l = l; jb.s = s;
    jb.gptr = gptr; jb.gidx = gidx; jb.theta = theta;
    jb.ops = ops; jb.samples = samples; jb.zstride = s * n; jb.grad_mean = grad_mean;
    jb.grad_part = calloc((size_t)nthreads * (size_t)(m > 0 ? m : 1), sizeof(double));
    if (!jb.grad_part) return ORC_ERR_MEM;
    int st = run_ranges(l, nthreads, grad_range, &jb);
    if (!st) st = jb.status;
    if (!st) reduce_parts(jb.grad_part, nthreads, m, grad_theta);
    free(jb.grad_part);
    return st;
}

/* ------------------------------------------------------------------------ */
/* MMD^2 through Pauli-Z expectation values (eq. mmd_estimate): for each
 * observable a_k drawn from P_sigma with weight w_k,
 *   p_k = (1/N) sum_n (-1)^{a_k . x_n}       (training data, Sec. 3.3.1)
 *   q_k = (1/s) sum_i cos E_ki               (model, eq. expvalsample)
 * plug-in:   L = sum_k w_k (p_k - q_k)^2
 * unbiased:  L = sum_k w_k [P2_k - 2 p_k q_k + Q2_k] with the U-statistics
 *            P2_k = sum_{n != n'} v_n v_n' / (N(N-1)),  v_n = (-1)^{a_k . x_n}
 *            Q2_k = sum_{i != i'} c_i c_i' / (s(s-1)),  c_i = cos E_ki.
 * Gradient: dL/dc_ki times dc_ki/dtheta_j = -sin(E_ki) B_ij C_kj. */
static void mmd_range(range_t *rg)
{
    job_t *jb = rg->ctx;
    int64_t *J = malloc(sizeof(int64_t) * (jb->m + 1));
    double *C = malloc(sizeof(double) * (jb->m + 1));
    double *cs = malloc(sizeof(double) * jb->s);
    double *sn = malloc(sizeof(double) * jb->s);
    double *g = jb->grad_part ? jb->grad_part + (int64_t)rg->tid * jb->m : NULL;
    if (!J || !C || !cs || !sn) {
        jb->status = ORC_ERR_MEM;
        free(J); free(C); free(cs); free(sn);
        return;
    }
    double loss = 0.0;
    for (int64_t k = rg->k0; k < rg->k1; ++k) {
        const uint8_t *a = jb->ops + k * jb->n;
        /* data side */
        double sv = 0.0;
        for (int64_t d = 0; d < jb->N; ++d) {
            const uint8_t *x = jb->data + d * jb->n;
            int64_t ov = 0;
            for (int64_t q = 0; q < jb->n; ++q) ov += (int64_t)(a[q] & x[q]);
            sv += (ov & 1) ? -1.0 : 1.0;
        }
        double p = sv / (double)jb->N;
        /* model side */
        int64_t nj = anticommuting(jb, k, J, C);
        double sc = 0.0, sc2 = 0.0;
        for (int64_t i = 0; i < jb->s; ++i) {
            double e = phase(jb, k, i, J, C, nj);
            cs[i] = cos(e);
            sn[i] = sin(e);
            sc += cs[i];
            sc2 += cs[i] * cs[i];
        }
        double q = sc / (double)jb->s;
        double N = (double)jb->N, S = (double)jb->s;
        double term;
        if (jb->unbiased) {
            double P2 = (sv * sv - N) / (N * (N - 1.0));
            double Q2 = (sc * sc - sc2) / (S * (S - 1.0));
            term = P2 - 2.0 * p * q + Q2;
        } else {
            term = (p - q) * (p - q);
        }
        double w = jb->op_weight[k];
        loss += w * term;
        if (jb->phat) jb->phat[k] = p;
        if (jb->qhat) jb->qhat[k] = q;
        if (!g) continue;
        for (int64_t i = 0; i < jb->s; ++i) {
            double dLdc;
            if (jb->unbiased)
                dLdc = w * (-2.0 * p / S + 2.0 * (sc - cs[i]) / (S * (S - 1.0)));
            else
                dLdc = w * 2.0 * (q - p) / S;
            double f = -dLdc * sn[i];
            const uint8_t *z = sample_of(jb, k, i);
            for (int64_t t = 0; t < nj; ++t)
                g[J[t]] += f * sign_of(z, jb->gptr, jb->gidx, J[t]) * C[t];
        }
    }
    jb->loss_part[rg->tid] = loss;
    free(J); free(C); free(cs); free(sn);
}

int orc_mmd_loss_grad(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                      const double *theta, int64_t l, const uint8_t *ops,
                      const double *op_weight, int64_t s, const uint8_t *samples, int64_t N,
                      const uint8_t *data, int unbiased, double *loss, double *grad_theta,
                      double *phat, double *qhat, int nthreads)
{
    if (n < 1 || m < 0 || l < 1 || s < 1 || N < 1 || !loss || !op_weight) return ORC_ERR_ARG;
    if (unbiased && (s < 2 || N < 2)) return ORC_ERR_ARG;
    if (nthreads <= 0) nthreads = orc_num_threads();
    if (nthreads > l) nthreads = (int)l;
    job_t jb = {0};
    jb.n = n; jb.m = m; jb.l = l; jb.s = s;
    jb.gptr = gptr; jb.gidx = gidx; jb.theta = theta;
    jb.ops = ops; jb.samples = samples; jb.op_weight = op_weight;
    jb.N = N; jb.data = data; jb.unbiased = unbiased;
    jb.phat = phat; jb.qhat = qhat;
    jb.loss_part = calloc((size_t)nthreads, sizeof(double));
    if (grad_theta)
        jb.grad_part = calloc((size_t)nthreads * (size_t)(m > 0 ? m : 1), sizeof(double));
    if (!jb.loss_part || (grad_theta && !jb.grad_part)) {
        free(jb.loss_part); free(jb.grad_part);
        return ORC_ERR_MEM;
    }
    int st = run_ranges(l, nthreads, mmd_range, &jb);
    if (!st) st = jb.status;
    if (!st) {
        double acc = 0.0;
        for (int t = 0; t < nthreads; ++t) acc += jb.loss_part[t];
        *loss = acc;
        if (grad_theta) reduce_parts(jb.grad_part, nthreads, m, grad_theta);
    }
    free(jb.loss_part);
    free(jb.grad_part);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Exact values (pins only). */

/* State-vector simulation (n <= 20): start in |0>, apply each gate through
 * exp(i theta X_g)|x> = cos(theta)|x> + i sin(theta)|x xor g> (Sec. 2.5),
 * return the output probabilities |<x|U|0>|^2. Basis index bit q = qubit q. */
int orc_statevector_probs(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                          const double *theta, double *probs)
{
    if (n < 1 || n > 20 || m < 0 || !probs) return ORC_ERR_ARG;
    int64_t D = (int64_t)1 << n;
    double complex *psi = calloc((size_t)D, sizeof(double complex));
    double complex *nxt = calloc((size_t)D, sizeof(double complex));
    if (!psi || !nxt) { free(psi); free(nxt); return ORC_ERR_MEM; }
    psi[0] = 1.0;
    for (int64_t j = 0; j < m; ++j) {
        int64_t mask = 0;
        for (int64_t t = gptr[j]; t < gptr[j + 1]; ++t) mask ^= (int64_t)1 << gidx[t];
        double c = cos(theta[j]), sn = sin(theta[j]);
        for (int64_t x = 0; x < D; ++x)
            nxt[x] = c * psi[x] + I * sn * psi[x ^ mask];
        double complex *tmp = psi; psi = nxt; nxt = tmp;
    }
    for (int64_t x = 0; x < D; ++x) probs[x] = creal(psi[x] * conj(psi[x]));
    free(psi);
    free(nxt);
    return ORC_OK;
}

/* <Z_a> = sum_x q(x) (-1)^{a . x} from the output probabilities (Def. 2). */
int orc_statevector_expval(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                           const double *theta, int64_t l, const uint8_t *ops, double *out)
{
    if (n < 1 || n > 20) return ORC_ERR_ARG;
    int64_t D = (int64_t)1 << n;
    double *probs = malloc(sizeof(double) * (size_t)D);
    if (!probs) return ORC_ERR_MEM;
    int st = orc_statevector_probs(n, m, gptr, gidx, theta, probs);
    if (st) { free(probs); return st; }
    for (int64_t k = 0; k < l; ++k) {
        int64_t amask = 0;
        for (int64_t q = 0; q < n; ++q) if (ops[k * n + q]) amask |= (int64_t)1 << q;
        double acc = 0.0;
        for (int64_t x = 0; x < D; ++x)
            acc += probs[x] * ((__builtin_popcountll((unsigned long long)(x & amask)) & 1) ? -1.0 : 1.0);
        out[k] = acc;
    }
    free(probs);
    return ORC_OK;
}

/* The interference expansion of Prop. 3's proof (eq. expval_intefere):
 *   <Z_a> = Re sum_{omega subset of J_a, prod_{j in omega} X_{g_j} = I}
 *              prod_{j in J_a \ omega} cos(2 theta_j) prod_{j in omega} i sin(-2 theta_j)
 * enumerated over all 2^{|J_a|} subsets (|J_a| <= 24). omega = {} gives the
 * product term. */
int orc_subset_expval(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                      const double *theta, int64_t l, const uint8_t *ops, double *out)
{
    if (n < 1 || m < 0) return ORC_ERR_ARG;
    int64_t *J = malloc(sizeof(int64_t) * (m + 1));
    uint8_t *acc = malloc((size_t)n);
    if (!J || !acc) { free(J); free(acc); return ORC_ERR_MEM; }
    for (int64_t k = 0; k < l; ++k) {
        const uint8_t *a = ops + k * n;
        int64_t nj = 0;
        for (int64_t j = 0; j < m; ++j)
            if (overlap(a, gptr, gidx, j) & 1) J[nj++] = j;
        if (nj > 24) { free(J); free(acc); return ORC_ERR_SIZE; }
        double complex total = 0.0;
        for (int64_t w = 0; w < ((int64_t)1 << nj); ++w) {
            memset(acc, 0, (size_t)n);
            for (int64_t t = 0; t < nj; ++t)
                if ((w >> t) & 1)
                    for (int64_t u = gptr[J[t]]; u < gptr[J[t] + 1]; ++u) acc[gidx[u]] ^= 1;
            int identity = 1;
            for (int64_t q = 0; q < n; ++q) if (acc[q]) { identity = 0; break; }
            if (!identity) continue;
            double complex term = 1.0;
            for (int64_t t = 0; t < nj; ++t) {
                double th = theta[J[t]];
                if ((w >> t) & 1) term *= I * sin(-2.0 * th);
                else term *= cos(2.0 * th);
            }
            total += term;
        }
        out[k] = creal(total);
    }
    free(J);
    free(acc);
    return ORC_OK;
}

/* Stochastic bitflip circuit (eq. expval_bitflip): <Z_a> = prod_{j in J_a} cos(2 theta_j). */
int orc_bitflip_expval(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                       const double *theta, int64_t l, const uint8_t *ops, double *out)
{
    if (n < 1 || m < 0) return ORC_ERR_ARG;
    for (int64_t k = 0; k < l; ++k) {
        const uint8_t *a = ops + k * n;
        double p = 1.0;
        for (int64_t j = 0; j < m; ++j)
            if (overlap(a, gptr, gidx, j) & 1) p *= cos(2.0 * theta[j]);
        out[k] = p;
    }
    return ORC_OK;
}

/* d/dtheta_j of the bitflip expectation: -2 sin(2 theta_j) prod_{t in J_a, t != j} cos(2 theta_t),
 * contracted with u_k = dL/d<Z_{a_k}>. */
int orc_bitflip_grad(int64_t n, int64_t m, const int64_t *gptr, const int32_t *gidx,
                     const double *theta, int64_t l, const uint8_t *ops, const double *grad_out,
                     double *grad_theta)
{
    if (n < 1 || m < 0) return ORC_ERR_ARG;
    int64_t *J = malloc(sizeof(int64_t) * (m + 1));
    if (!J) return ORC_ERR_MEM;
    for (int64_t j = 0; j < m; ++j) grad_theta[j] = 0.0;
    for (int64_t k = 0; k < l; ++k) {
        const uint8_t *a = ops + k * n;
        int64_t nj = 0;
        for (int64_t j = 0; j < m; ++j)
            if (overlap(a, gptr, gidx, j) & 1) J[nj++] = j;
        for (int64_t t = 0; t < nj; ++t) {
            double p = -2.0 * sin(2.0 * theta[J[t]]);
            for (int64_t u = 0; u < nj; ++u)
                if (u != t) p *= cos(2.0 * theta[J[u]]);
            grad_theta[J[t]] += grad_out[k] * p;
        }
    }
    free(J);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Random numbers for the training loop: Philox4x64-10, the counter-based
 * generator of Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011), written from that definition. Ten rounds; each
 * round multiplies counter words 0 and 2 by two fixed odd constants into
 * 128-bit products, and the key is bumped by two Weyl constants between
 * rounds.
 */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B97F4A7C15ull;
            k1 += 0xBB67AE8584CAA73Bull;
        }
        const unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * c0;
        const unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * c2;
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Output o of stream `tag` at training step `step`: word o % 4 of
 * Philox(counter (o / 4, step, tag, 0), key (seed0, seed1)). */
static uint64_t stream_word(uint64_t seed0, uint64_t seed1, uint64_t step, uint64_t tag,
                            uint64_t o)
{
    const uint64_t ctr[4] = {o / 4, step, tag, 0};
    const uint64_t key[2] = {seed0, seed1};
    uint64_t out[4];
    orc_philox4x64(ctr, key, out);
    return out[o % 4];
}

/* Uniform bit strings (the samples z of eq. expvalsample, Prop. 1): qubit q
 * of row r is bit q % 64 of output r * ceil(n / 64) + q / 64. */
int orc_sample_uniform(int64_t rows, int64_t n, uint64_t seed0, uint64_t seed1, uint64_t step,
                       uint64_t tag, uint8_t *out01)
{
    if (rows < 0 || n < 1 || !out01) return ORC_ERR_ARG;
    const int64_t W = (n + 63) / 64;
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t q = 0; q < n; ++q) {
            const uint64_t word = stream_word(seed0, seed1, step, tag, (uint64_t)(r * W + q / 64));
            out01[r * n + q] = (uint8_t)((word >> (q % 64)) & 1u);
        }
    return ORC_OK;
}

/* Independent Bernoulli bits (operators drawn from P_sigma, Sec. 3.3.1):
 * qubit q of row r is 1 when output r * n + q is below the row's threshold
 * (floor(p * 2^64) for bit probability p). */
int orc_sample_bernoulli(int64_t rows, int64_t n, const uint64_t *row_threshold, uint64_t seed0,
                         uint64_t seed1, uint64_t step, uint64_t tag, uint8_t *out01)
{
    if (rows < 0 || n < 1 || !row_threshold || !out01) return ORC_ERR_ARG;
    for (int64_t r = 0; r < rows; ++r)
        for (int64_t q = 0; q < n; ++q) {
            const uint64_t v = stream_word(seed0, seed1, step, tag, (uint64_t)(r * n + q));
            out01[r * n + q] = (uint8_t)(v < row_threshold[r]);
        }
    return ORC_OK;
}
