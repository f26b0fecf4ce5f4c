// gfx950 kernels of the sparse-C contraction and of independent estimates.
//
// Sparse-C: E_ki = sum_{j in J_k} t_j (-1)^{b_ij}, t_j = 2 theta'_j, over the
// generators J_k that anticommute with observable k (the set bits of row k of
// C), on the vector units in FP32: the dense contraction's result with
// |J_k| / m of its work.
//
// Independent estimates (the l x s x n sample tensor of Sec. 2.3): observable
// k averages over its own s samples, so its sample parities come from the bit
// columns of its own sample set instead of one B^T shared by all observables.
// Nothing else changes, so both forms run the same bodies over a different
// source of sample-parity words.
#include "iqp_device.h"

namespace iqp {

// Buffers a launch only reads (parity words, support lists, C rows, 2 theta'),
// held in the constant address space: uniform loads through such pointers
// are scalar loads even in kernels that also write memory (the backward's
// atomics), since the compiler may assume they do not change in the launch.
#define IQP_CONST __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ const T IQP_CONST *cptr(const T *p) {
    return (const T IQP_CONST *)p;
}

// ---------------------------------------------------------------------------
// Sample-parity words: word w of generator j holds b_ij of samples 64 w ..
// 64 w + 63 (bit i % 64). A wave covers one chunk of kSpWords words of one
// observable. Two ways to read them:
//   word(j)      each lane loads the word its 16 samples lie in (lane L:
//                bits 16 (L % 4) .. 16 (L % 4) + 15 of word L / 4); the
//                forward, and the backward of independent sets
//   words(j, m)  all kSpWords words of the chunk, the same in every lane
//                (scalar loads), each used as a lane mask over the 64 samples
//                of one word (lane L: sample 64 r + L); the backward of
//                shared samples
// The sample-parity rows hold whole chunks (a multiple of kSpWords words,
// the words of samples >= s being 0), so a wave reads all its words
// unconditionally.
constexpr int kSpWords = kEpiChunk / 64;

// One B^T (row-major) for all observables.
struct SharedWords {
    const uint64_t IQP_CONST *row0;  // btrm + the wave's first sample word
    int64_t Rwb;
    const uint64_t IQP_GLOBAL *lane0;  // btrm + the lane's own word
    __device__ __forceinline__ uint64_t word(int64_t j) const { return lane0[j * Rwb]; }
    __device__ __forceinline__ void words(int64_t j, uint64_t (&m)[kSpWords]) const {
        const uint64_t IQP_CONST *row = row0 + j * Rwb;
#pragma unroll
        for (int r = 0; r < kSpWords; ++r) m[r] = row[r];
    }
};

// The bit columns of observable k's own samples: the parity of g_j is the
// XOR of the columns of its qubits (its support list; a generator heavier
// than kSupCap walks its bit row).
struct IndepWords {
    int64_t ldx;
    const int32_t IQP_CONST *sup;
    const uint64_t IQP_CONST *gens;
    int W;
    const uint64_t IQP_GLOBAL *lane0;  // xt + k * xstride + the lane's own word
    // The first four support entries come in one scalar load, so the
    // column loads of a generator of weight <= 4 issue together.
    __device__ __forceinline__ uint64_t word(int64_t j) const {
        const int32_t IQP_CONST *sj = sup + j * kSupCap;
        const int32_t q0 = sj[0], q1 = sj[1], q2 = sj[2], q3 = sj[3];
        if (q0 < 0) {
            uint64_t x = 0;
            if (q0 == -2) {
                for (int w = 0; w < W; ++w) {
                    uint64_t g = gens[j * W + w];
                    while (g) {
                        x ^= lane0[(int64_t)(w * 64 + __builtin_ctzll(g)) * ldx];
                        g &= g - 1;
                    }
                }
            }
            return x;
        }
        uint64_t x = lane0[(int64_t)q0 * ldx];
        if (q1 < 0) return x;
        x ^= lane0[(int64_t)q1 * ldx];
        if (q2 < 0) return x;
        x ^= lane0[(int64_t)q2 * ldx];
        if (q3 < 0) return x;
        x ^= lane0[(int64_t)q3 * ldx];
        for (int e = 4; e < kSupCap; ++e) {
            const int32_t q = sj[e];
            if (q < 0) break;
            x ^= lane0[(int64_t)q * ldx];
        }
        return x;
    }
};

template <bool kIndep>
struct WordsOf;
template <>
struct WordsOf<false> {
    using T = SharedWords;
    static __device__ __forceinline__ T make(const SampleParity &p, int64_t, int64_t sw0,
                                             int64_t swl) {
        return SharedWords{cptr(p.btrm) + sw0, p.Rwb, gptr(p.btrm) + swl};
    }
};
template <>
struct WordsOf<true> {
    using T = IndepWords;
    static __device__ __forceinline__ T make(const SampleParity &p, int64_t k, int64_t sw0,
                                             int64_t swl) {
        return IndepWords{p.Rwb, cptr(p.sup), cptr(p.gens), p.W, gptr(p.xt) + k * p.xstride + swl};
    }
};

// The set bits of row k of C (the generators J_k), in gate order. The row
// is scanned 64 words at a time by the wave's lanes: one coalesced load per
// 64 words and a ballot of the non-zero ones, so a zero word costs only its
// share of that load (a walk word by word on the scalar unit pays a
// dependent scalar load per word, zero or not); the non-zero words are
// then taken in order from the lanes that hold them.
struct GateWalk {
    const uint64_t IQP_GLOBAL *row;
    int64_t Gw, base, w;
    uint64_t v;   // this lane's word of the current 64-word block
    uint64_t nz;  // lanes of the current block whose word is non-zero (uniform)
    uint64_t cw;  // the current word, bits not yet taken (uniform)
    int lane;
    __device__ __forceinline__ GateWalk(const uint64_t *r, int64_t gw)
        : row(gptr(r)), Gw(gw), base(-64), w(0), v(0), nz(0), cw(0),
          lane((int)(threadIdx.x & 63)) {}
    __device__ __forceinline__ bool next(int64_t &j) {
        while (cw == 0) {
            while (nz == 0) {
                base += 64;
                if (base >= Gw) return false;
                const int64_t x = base + lane;
                v = x < Gw ? row[x] : 0ull;
                nz = __ballot(v != 0ull);
            }
            const int i = __builtin_ctzll(nz);
            nz &= nz - 1;
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, i);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), i);
            cw = ((uint64_t)hi << 32) | lo;
            w = base + i;
        }
        j = w * 64 + __builtin_ctzll(cw);
        cw &= cw - 1;
        return true;
    }
};

// x + y in the lanes whose bit of the uniform mask is set, x elsewhere: one
// add and one select on the mask held in a scalar register pair.
__device__ __forceinline__ float add_where(float x, float y, uint64_t mask) {
    const float s = x + y;
    return __builtin_amdgcn_inverse_ballot_w64(mask) ? s : x;
}

// ---------------------------------------------------------------------------
// Forward. One wave per (observable k, chunk of kEpiChunk samples); lane L
// holds 16 samples, bits 16 (L % 4) + b of the chunk's word L / 4. The row of
// C is walked with scalar loads in gate order; for each set bit j the lane
// loads its parity word and adds t_j to the samples whose bit is set (a
// signed one-bit field extract gives 0 or -1, ANDed with t_j's bits):
//   E_ki = T_k - 2 sum_{j in J_k, b_ij = 1} t_j,  T_k = sum_{j in J_k} t_j (FP64).
// The wave then reduces each phase modulo 2 pi in FP64, takes the cosine and
// writes the same per-chunk sums as the dense epilogue. (Here the per-lane
// vector load of the word keeps more loads in flight than the backward's
// scalar mask loads, which the forward's shorter loop body cannot hide.)
constexpr int kSpSamples = kEpiChunk / 64;
// generators between the folds of the forward's FP32 sums; the float
// nearest pi and a float near 1 / pi (any multiple q is exact bookkeeping)
constexpr int kSpFold = 32;
constexpr float kPiF = 3.14159274f;
constexpr float kInvPiF = 0.318309873f;

__device__ __forceinline__ float masked(float t, uint32_t f, int b) {
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)f, (unsigned)b, 1u);
    return __uint_as_float(__float_as_uint(t) & m);
}

template <bool kIndep>
__device__ __forceinline__ void sparse_fwd_body(const SparseFwdArgs &a, int64_t blk) {
    const int64_t nchunk = ceil_div(a.s, kEpiChunk);
    const int64_t unit = blk * 4 + wave_id();
    if (unit >= a.l * nchunk) return;  // uniform over the wave
    const int64_t k = unit / nchunk, ch = unit - k * nchunk;
    const int lane = threadIdx.x & 63;
    const int64_t sw0 = ch * kSpWords;
    const int sh = 16 * (lane & 3);
    const auto src = WordsOf<kIndep>::make(a.bsrc, k, sw0, sw0 + (lane >> 2));
    const uint64_t IQP_CONST *crow = cptr(a.crm) + k * a.Gw;
    const float IQP_CONST *t32 = cptr(a.t32);
    // acc[b] + kpi[b] * pi_f (pi_f the float nearest pi) is the lane's sum of
    // t_j over its sample b's generators with b_ij = 1. Every kSpFold
    // generators the whole multiples of pi_f are moved from acc to the
    // integer count kpi (exact bookkeeping: E changes by 2 pi per multiple,
    // which the FP64 reduction below removes), so acc stays within about
    // pi and its FP32 rounding does not grow with |J_k|.
    float acc[kSpSamples], kpi[kSpSamples];
#pragma unroll
    for (int b = 0; b < kSpSamples; ++b) acc[b] = kpi[b] = 0.0f;
    double T = 0.0;
    int fold = 0;
    // (the row is walked word by word on the scalar unit here: the lanes'
    // block scan of the backward costs the forward two waves per SIMD of
    // occupancy, more than it saves)
    for (int64_t w = 0; w < a.Gw; ++w) {
        uint64_t cw = crow[w];
        while (cw) {
            const int64_t j = w * 64 + __builtin_ctzll(cw);
            cw &= cw - 1;
            const float t = t32[j];
            const uint32_t f = (uint32_t)(src.word(j) >> sh);
            T += (double)t;
#pragma unroll
            for (int b = 0; b < kSpSamples; ++b) acc[b] += masked(t, f, b);
            if (++fold == kSpFold) {  // uniform over the wave
                fold = 0;
#pragma unroll
                for (int b = 0; b < kSpSamples; ++b) {
                    const float q = rintf(acc[b] * kInvPiF);
                    acc[b] = fmaf(-q, kPiF, acc[b]);
                    kpi[b] += q;
                }
            }
        }
    }
    double sc = 0.0, sc2 = 0.0;
    const int64_t i0 = ch * kEpiChunk + lane * kSpSamples;
    float IQP_GLOBAL *ph = a.phase_out ? gptr(a.phase_out) + k * a.s : nullptr;
#pragma unroll
    for (int b = 0; b < kSpSamples; ++b) {
        const int64_t i = i0 + b;
        if (i < a.s) {
            const double e = T - 2.0 * ((double)acc[b] + (double)kpi[b] * (double)kPiF);
            const double kk = rint(e * IQP_INV_TWO_PI);
            double rr = fma(-kk, IQP_TWO_PI_HI, e);
            rr = fma(-kk, IQP_TWO_PI_LO, rr);
            const float rf = (float)rr;
            const float c = cosf(rf);
            if (ph) ph[i] = rf;
            sc += (double)c;
            sc2 += (double)c * (double)c;
        }
    }
#pragma unroll
    for (int st = 32; st >= 1; st >>= 1) {
        sc += __shfl_xor(sc, st, 64);
        sc2 += __shfl_xor(sc2, st, 64);
    }
    if (lane == 0) {
        double IQP_GLOBAL *part = gptr(a.part) + (k * nchunk + ch) * 2;
        part[0] = sc;
        part[1] = sc2;
    }
}

hipError_t launch_sparse_fwd(const LaunchCtx &lc, const SparseFwdArgs &a) {
    if (a.bsrc.xt)
        return plain_launch<SparseFwdArgs, sparse_fwd_body<true>>(lc, KF_FWD, a, blocks_of(a));
    return plain_launch<SparseFwdArgs, sparse_fwd_body<false>>(lc, KF_FWD, a, blocks_of(a));
}

// ---------------------------------------------------------------------------
// Gradient: for every (k, j in J_k) the partial T_kj = sum_i S_ki (-1)^{b_ij}
// of a sample chunk is summed across the wave and added into an int64
// fixed-point accumulator of gate j. Integer addition is associative, so the
// result does not depend on the order in which the waves add, and no per-pair
// storage is needed. The scale keeps every sum below 2^62: |T_kj| <= s
// (|alpha_k| + |beta_k|) summed over k.
__device__ __forceinline__ void sparse_bound_body(const SparseBoundArgs &a, int64_t blk) {
    const int64_t j = blk * 256 + threadIdx.x;
    if (j <= a.m_pad) gptr(a.acc)[j] = 0;
    if (blk != 0) return;
    __shared__ double sh[256];
    double g = 0.0;
    for (int64_t k = threadIdx.x; k < a.l; k += 256)
        g += (double)a.s * (fabs(gptr(a.coef)[2 * k]) + fabs(gptr(a.coef)[2 * k + 1]));
    g = block_sum_256(g, sh);
    if (threadIdx.x == 0) {
        const double G = (g > 0.0 && isfinite(g)) ? g : 1.0;
        gptr(a.scale)[0] = ldexp(1.0, 61 - ilogb(G));
    }
}

hipError_t launch_sparse_bound(const LaunchCtx &lc, const SparseBoundArgs &a) {
    return plain_launch<SparseBoundArgs, sparse_bound_body>(lc, KF_WEIGHTS, a, blocks_of(a));
}

// generators per reduction batch of the backward; LDS row stride in floats
// (a multiple of 4 for 16-byte reads; 68 spreads the rows over the banks)
constexpr int kRedBatch = 16;
constexpr int kRedStride = 68;

template <bool kIndep>
__device__ __forceinline__ void sparse_bwd_body(const SparseBwdArgs &a, int64_t blk) {
    const int64_t nchunk = ceil_div(a.s, kEpiChunk);
    const int64_t unit = blk * 4 + wave_id();
    if (unit >= a.l * nchunk) return;  // uniform over the wave
    const int64_t k = unit / nchunk, ch = unit - k * nchunk;
    const int lane = threadIdx.x & 63;
    const int64_t sw0 = ch * kSpWords;
    // Lanes and samples: shared samples, lane L holds sample 64 r + L of
    // each of the chunk's 16 words r (the parity words are uniform, scalar
    // loads used as lane masks); independent sets, the forward's layout: lane
    // L holds the 16 samples of bits 16 (L % 4) .. + 15 of the chunk's word
    // L / 4 and loads its own parity word.
    const int sh = 16 * (lane & 3);
    const auto src = WordsOf<kIndep>::make(a.bsrc, k, sw0, kIndep ? sw0 + (lane >> 2) : sw0);
    GateWalk gates(a.crm + k * a.Gw, a.Gw);
    const double al = gptr(a.coef)[2 * k], be = gptr(a.coef)[2 * k + 1];
    const double scale = gptr(a.scale)[0];
    // S_ki = (alpha_k + beta_k cos E_ki) sin E_ki for the lane's samples
    float S[kSpWords];
    float Ssum = 0.0f;
#pragma unroll
    for (int r = 0; r < kSpWords; ++r) {
        const int64_t i = kIndep ? (sw0 + (lane >> 2)) * 64 + sh + r : (sw0 + r) * 64 + lane;
        float v = 0.0f;
        if (i < a.s) {
            float sn, cs;
            sincosf(gptr(a.phase)[k * a.s + i], &sn, &cs);
            v = (float)((al + be * (double)cs) * (double)sn);
        }
        S[r] = v;
        Ssum += v;
    }
    // The partials of kRedBatch generators are gathered in this wave's LDS
    // rows (row e, lane L: lane L's partial for the e-th generator of the
    // batch) and reduced together: lane L sums 16 lanes of row L % 16, two
    // shuffles add the four quarters, and lanes 0..15 add their generator's
    // total into its fixed-point accumulator. One LDS write per generator
    // instead of a full cross-lane sum and an atomic per generator.
    __shared__ __attribute__((aligned(16))) float red_all[4][kRedBatch * kRedStride];
    float *red = red_all[wave_id()];
    int nb = 0;
    int32_t jv = 0;  // lane e < nb: the generator of batch row e
    auto flush = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int e = lane & (kRedBatch - 1), q = lane >> 4;
        const float4 *row = reinterpret_cast<const float4 *>(red + e * kRedStride + 16 * q);
        const float4 v0 = row[0], v1 = row[1], v2 = row[2], v3 = row[3];
        float tot = ((v0.x + v0.y) + (v0.z + v0.w)) + ((v1.x + v1.y) + (v1.z + v1.w)) +
                    (((v2.x + v2.y) + (v2.z + v2.w)) + ((v3.x + v3.y) + (v3.z + v3.w)));
        tot += __shfl_xor(tot, 16, 64);
        tot += __shfl_xor(tot, 32, 64);
        if (lane < nb) {
            if (isfinite(tot))
                atomicAdd((unsigned long long *)&gptr(a.acc)[jv],
                          (unsigned long long)llrint((double)tot * scale));
            else
                atomicOr((unsigned long long *)&gptr(a.acc)[a.m_pad], 1ull);
        }
        // the rows are rewritten by the next batch only after every lane read
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        nb = 0;
    };
    auto add_partial = [&](int64_t j, float p) {
        red[nb * kRedStride + lane] = Ssum - 2.0f * p;
        jv = lane == nb ? (int32_t)j : jv;
        if (++nb == kRedBatch) flush();
    };
    int64_t j;
    if constexpr (!kIndep) {
        uint64_t m[kSpWords];
        // the next generator's parity words are loaded once the current ones
        // are consumed, so the load overlaps the current partial's store (the
        // independent form's support walk has no scalar registers to spare
        // for this)
        bool have = gates.next(j);
        src.words(have ? j : 0, m);
        while (have) {
            float p = 0.0f;
#pragma unroll
            for (int r = 0; r < kSpWords; ++r) p = add_where(p, S[r], m[r]);
            int64_t jn = j;
            const bool more = gates.next(jn);
            src.words(jn, m);
            add_partial(j, p);
            j = jn;
            have = more;
        }
    } else {
        // The parity word of generator j is the XOR of its support columns,
        // here per lane with vector loads: as uniform scalar words the XORs
        // ran on the scalar unit, which then bounded the kernel. Per sample a
        // one-bit field extract masks S (3 lane ops per term, as in the
        // forward).
        while (gates.next(j)) {
            const uint32_t f = (uint32_t)(src.word(j) >> sh);
            float p = 0.0f;
#pragma unroll
            for (int b = 0; b < kSpWords; ++b) p += masked(S[b], f, b);
            add_partial(j, p);
        }
    }
    if (nb > 0) flush();
}

hipError_t launch_sparse_bwd(const LaunchCtx &lc, const SparseBwdArgs &a) {
    if (a.bsrc.xt)
        return plain_launch<SparseBwdArgs, sparse_bwd_body<true>>(lc, KF_BWD, a, blocks_of(a));
    return plain_launch<SparseBwdArgs, sparse_bwd_body<false>>(lc, KF_BWD, a, blocks_of(a));
}

__device__ __forceinline__ void sparse_finish_body(const SparseFinishArgs &a, int64_t blk) {
    const int64_t j = blk * 256 + threadIdx.x;
    if (j >= a.m) return;
    const bool bad = gptr(a.acc)[a.m_pad] != 0;
    gptr(a.grad)[j] = bad ? (double)NAN : -2.0 * (double)gptr(a.acc)[j] / gptr(a.scale)[0];
}

hipError_t launch_sparse_finish(const LaunchCtx &lc, const SparseFinishArgs &a) {
    return plain_launch<SparseFinishArgs, sparse_finish_body>(lc, KF_GRAD, a, blocks_of(a));
}

// ---------------------------------------------------------------------------
// Bit columns of every observable's own sample set. A step is (set k, group g
// of 16 row words = 1024 rows, chunk c of 8 qubit words); ldx is a multiple
// of 16. Persistent blocks (two per CU: LDS and registers allow two) take
// steps b, b + grid, ...: the block reads words [8c, 8c + 8) of its 1024 rows
// with coalesced loads (8 lanes cover one row's run) into registers, moves
// them to LDS (row stride 9 words, so the column reads below hit distinct
// banks) and issues the loads of its next step, which stay in flight while
// wave v transposes words v and v + 4: for each of the 16 64-row blocks lane
// r takes row r's word from LDS and the 64 x 64 bit transpose leaves lane q
// with column 64 w + q, so lane q writes that column's 16 row words as one
// 128-byte run, a whole cache line. Every sample word is read once and every
// output line written by one lane. Rows past s read as 0.
constexpr int kSliceWords = 16;  // row words per step: 1024 rows
constexpr int kSliceChunk = 8;   // qubit words per step
constexpr int kSliceStride = kSliceChunk + 1;
constexpr int64_t kSliceBlocks = 512;

struct SliceStep {
    int64_t k, g;
    int w0, cw;
};

__device__ __forceinline__ SliceStep slice_step(const IndepSliceArgs &a, int64_t q) {
    const int64_t ngrp = a.ldx / kSliceWords;
    const int nch = (a.W + kSliceChunk - 1) / kSliceChunk;
    const int64_t u = q / nch;
    SliceStep st;
    st.w0 = (int)(q - u * nch) * kSliceChunk;
    st.cw = a.W - st.w0 < kSliceChunk ? a.W - st.w0 : kSliceChunk;
    st.k = u / ngrp;
    st.g = u - st.k * ngrp;
    return st;
}

// this thread's 32 words of a step: word j of rows r0 + 32 it (rows past s
// read row s - 1 here and are zeroed when stored to LDS, so that nothing
// waits on these loads before then)
__device__ __forceinline__ void slice_load(const IndepSliceArgs &a, const SliceStep &st, int j,
                                           int r0, uint64_t (&v)[32]) {
    if (j >= st.cw) return;
    const uint64_t IQP_GLOBAL *rows = gptr(a.samples) + st.k * a.s * a.W + st.w0 + j;
    const int64_t base = st.g * (kSliceWords * 64) + r0;
#pragma unroll
    for (int it = 0; it < 32; ++it) {
        const int64_t row = base + 32 * it;
        v[it] = rows[(row < a.s ? row : a.s - 1) * a.W];
    }
}

__device__ __forceinline__ void indep_slice_body(const IndepSliceArgs &a, int64_t blk) {
    __shared__ uint64_t stage[kSliceWords * 64 * kSliceStride];
    const int64_t total = a.l * (a.ldx / kSliceWords) * ((a.W + kSliceChunk - 1) / kSliceChunk);
    const int64_t grid = gridDim.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = tid & (kSliceChunk - 1);  // word within the chunk this thread loads
    const int r0 = tid / kSliceChunk;       // first of its rows; the rest step by 32
    uint64_t v[32];
    SliceStep st = slice_step(a, blk);
    if (blk < total) slice_load(a, st, j, r0, v);
    for (int64_t q = blk; q < total; q += grid) {
        __syncthreads();  // the previous step's LDS reads are done
        if (j < st.cw) {
            const int64_t base = st.g * (kSliceWords * 64) + r0;
#pragma unroll
            for (int it = 0; it < 32; ++it)
                stage[(r0 + 32 * it) * kSliceStride + j] = base + 32 * it < a.s ? v[it] : 0ull;
        }
        __syncthreads();
        const SliceStep cur = st;
        if (q + grid < total) {
            st = slice_step(a, q + grid);
            slice_load(a, st, j, r0, v);
        }
        uint64_t IQP_GLOBAL *set = gptr(a.xt) + cur.k * 64 * a.W * a.ldx + cur.g * kSliceWords;
        for (int jw = wave; jw < cur.cw; jw += 4) {
            uint64_t y[kSliceWords];
#pragma unroll
            for (int t = 0; t < kSliceWords; ++t)
                y[t] = transpose64(stage[(t * 64 + lane) * kSliceStride + jw], lane);
            uint64_t IQP_GLOBAL *dst = set + (int64_t)((cur.w0 + jw) * 64 + lane) * a.ldx;
#pragma unroll
            for (int t = 0; t < kSliceWords; ++t) dst[t] = y[t];
        }
    }
}

hipError_t launch_indep_slice(const LaunchCtx &lc, const IndepSliceArgs &a) {
    if (a.ldx % kSliceWords != 0 || a.s < 1) return hipErrorInvalidValue;
    const int64_t steps = a.l * (a.ldx / kSliceWords) * ((a.W + kSliceChunk - 1) / kSliceChunk);
    return plain_launch<IndepSliceArgs, indep_slice_body>(lc, KF_PARITY, a,
                                                          steps < kSliceBlocks ? steps : kSliceBlocks);
}

}  // namespace iqp
