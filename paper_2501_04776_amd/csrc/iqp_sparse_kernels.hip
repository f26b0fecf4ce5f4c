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
// 64 w + 63 (bit i % 64). In the forward a wave covers one chunk of
// kSpWords words of one observable and each lane loads, per generator, the
// word its 16 samples lie in (lane L: bits 16 (L % 4) .. 16 (L % 4) + 15 of
// word L / 4). The sample-parity rows hold whole chunks (a multiple of
// kSpWords words, the words of samples >= s being 0), so a wave reads all
// its words unconditionally.
constexpr int kSpWords = kEpiChunk / 64;

// One B^T (row-major) for all observables.
struct SharedWords {
    int64_t Rwb;
    const uint64_t IQP_GLOBAL *lane0;  // btrm + the lane's own word
    __device__ __forceinline__ uint64_t word(int64_t j) const { return lane0[j * Rwb]; }
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
        return SharedWords{p.Rwb, gptr(p.btrm) + swl};
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

// Gradient by table lookup. A block takes observable k and one chunk of
// kEpiChunk samples. Thread t computes S_ki for the four samples 4t .. 4t + 3
// of the chunk and writes their 16 signed sums
//   L_t[v] = sum_{b < 4} (-1)^{v_b} S_{k, c + 4t + b},  v = 0 .. 15,
// so that, with v_t(j) the nibble of generator j's parity bits over those
// four samples (bits 4t .. 4t + 3 of the chunk's parity words), the chunk's
// partial T_kj = sum_i S_ki (-1)^{b_ij} is the sum over t of L_t[v_t(j)]:
// 256 table reads per generator and chunk in place of 1024 masked adds. The
// generators J_k (the set bits of row k of C) are compacted into a list in
// LDS; each lane takes one generator of the list, forms its 16 parity words
// of the chunk (one 128-byte line of B^T for shared samples; for
// independent sets the XOR of the line of each support column of k's own
// samples), sums its 256 table entries and adds the total into the
// generator's fixed-point accumulator. The lanes of a wave read one table
// at a time, a 64-byte row of 16 entries in distinct banks, so the reads
// never conflict.
constexpr int kLutTables = (int)(kEpiChunk / 4);  // one per thread of the block
constexpr int kLutList = 1024;                    // generators per list fill

static_assert(kLutTables == 256, "one table per thread of a 256-thread block");

// Exclusive prefix over the block of per-thread counts c (the block's total
// in *tot); wsum holds the 4 wave totals and is reused only after the next
// barrier of the caller's loop.
__device__ __forceinline__ int block_excl_scan(int c, int *wsum, int *tot) {
    const int lane = threadIdx.x & 63, w = wave_id();
    int x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int v = wsum[i];
        before += i < w ? v : 0;
        all += v;
    }
    *tot = all;
    return before + x - c;
}


// The 16 parity words of generator j over chunk ch (lane-varying j).
template <bool kIndep>
__device__ __forceinline__ void lut_row(const SparseBwdArgs &a, int64_t k, int64_t ch, int64_t j,
                                        u32x4 (&wv)[8]);
template <>
__device__ __forceinline__ void lut_row<false>(const SparseBwdArgs &a, int64_t, int64_t ch,
                                               int64_t j, u32x4 (&wv)[8]) {
    const glb<const u32x4> src =
        (glb<const u32x4>)(gptr(a.bsrc.btrm) + j * a.bsrc.Rwb + ch * kSpWords);
#pragma unroll
    for (int q = 0; q < 8; ++q) wv[q] = src[q];
}
template <>
__device__ __forceinline__ void lut_row<true>(const SparseBwdArgs &a, int64_t k, int64_t ch,
                                              int64_t j, u32x4 (&wv)[8]) {
    const glb<const uint64_t> cols = gptr(a.bsrc.xt) + k * a.bsrc.xstride + ch * kSpWords;
    auto add_col = [&](int64_t q) {
        const glb<const u32x4> src = (glb<const u32x4>)(cols + q * a.bsrc.Rwb);
#pragma unroll
        for (int i = 0; i < 8; ++i) wv[i] ^= src[i];
    };
#pragma unroll
    for (int i = 0; i < 8; ++i) wv[i] = u32x4{0, 0, 0, 0};
    const glb<const int32_t> sj = gptr(a.bsrc.sup) + j * kSupCap;
    if (sj[0] == -2) {  // heavier than kSupCap: its bit row
        for (int w = 0; w < a.bsrc.W; ++w) {
            uint64_t g = gptr(a.bsrc.gens)[j * a.bsrc.W + w];
            while (g) {
                add_col(w * 64 + __builtin_ctzll(g));
                g &= g - 1;
            }
        }
        return;
    }
    for (int e = 0; e < kSupCap; ++e) {
        const int32_t q = sj[e];
        if (q < 0) break;
        add_col(q);
    }
}

template <bool kIndep>
__device__ __forceinline__ void sparse_bwd_lut_body(const SparseBwdArgs &a, int64_t blk) {
    // chunk-major: the blocks that run together read one 128-byte column
    // of the parity rows (fewer HBM fetches than observable-major order)
    const int64_t ch = blk / a.l, k = blk - ch * a.l;
    const int tid = threadIdx.x, lane = tid & 63;
    __shared__ __attribute__((aligned(16))) float tab[kLutTables * 16];
    __shared__ int32_t lst[kLutList];
    __shared__ int wsum[2][4];

    // the tables of this chunk
    {
        const double al = gptr(a.coef)[2 * k], be = gptr(a.coef)[2 * k + 1];
        float S[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t i = ch * kEpiChunk + 4 * tid + b;
            float v = 0.0f;
            if (i < a.s) {
                float sn, cs;
                sincosf(gptr(a.phase)[k * a.s + i], &sn, &cs);
                v = (float)((al + be * (double)cs) * (double)sn);
            }
            S[b] = v;
        }
        // x[u] over samples 0, 1 and y[u] over samples 2, 3, bit set = minus
        const float x[4] = {S[0] + S[1], S[1] - S[0], S[0] - S[1], -S[0] - S[1]};
        const float y[4] = {S[2] + S[3], S[3] - S[2], S[2] - S[3], -S[2] - S[3]};
        float4 *row = reinterpret_cast<float4 *>(tab + tid * 16);
#pragma unroll
        for (int h = 0; h < 4; ++h)
            row[h] = make_float4(x[0] + y[h], x[1] + y[h], x[2] + y[h], x[3] + y[h]);
    }

    const glb<const uint64_t> crow = gptr(a.crm) + k * a.Gw;
    const double scale = gptr(a.scale)[0];
    // each wave takes list entries wave_id() * 64 + lane, + 256, ...
    auto process = [&](int n) {
        for (int g = wave_id() * 64 + lane; g - lane < n; g += 256) {
            if (g >= n) continue;
            const int64_t j = lst[g];
            u32x4 wv[8];
            lut_row<kIndep>(a, k, ch, j, wv);
            float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const char *tb = reinterpret_cast<const char *>(tab);
#pragma unroll
            for (int r = 0; r < kSpWords; ++r) {
                // word r holds nibbles t = 16 r + e (bits 4e .. 4e + 3): byte
                // e' of x[2h] is 4 times nibble 8h + 2e', of x[2h + 1] 4 times
                // nibble 8h + 2e' + 1 (kept opaque so that each byte costs one
                // extract instead of a shift and a mask)
                uint32_t x[4];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t d = wv[r / 2][2 * (r % 2) + h];
                    x[2 * h] = (d << 2) & 0x3C3C3C3Cu;
                    x[2 * h + 1] = (d >> 2) & 0x3C3C3C3Cu;
                    asm volatile("" : "+v"(x[2 * h]), "+v"(x[2 * h + 1]));
                }
                float v[16];
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const uint32_t o = (x[e / 4 % 2 + 2 * (e / 8)] >> (8 * (e % 4))) & 0xFFu;
                    const int t = 16 * r + 8 * (e / 8) + 2 * (e % 4) + e / 4 % 2;
                    v[e] = *reinterpret_cast<const float *>(tb + t * 64 + o);
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) acc[e] += v[e] + v[e + 8];
            }
            const float tot = ((acc[0] + acc[1]) + (acc[2] + acc[3])) +
                              ((acc[4] + acc[5]) + (acc[6] + acc[7]));
            if (isfinite(tot))
                atomicAdd((unsigned long long *)&gptr(a.acc)[j],
                          (unsigned long long)llrint((double)tot * scale));
            else
                atomicOr((unsigned long long *)&gptr(a.acc)[a.m_pad], 1ull);
        }
    };

    // J_k, 256 row words at a time, into the list; a full list is processed
    // before the rest of the window is taken
    int n = 0, it = 0;
    __syncthreads();  // tables written
    for (int64_t base = 0; base < a.Gw; base += 256) {
        uint64_t v = base + tid < a.Gw ? crow[base + tid] : 0ull;
        for (;;) {
            int tot;
            const int off = block_excl_scan(__popcll(v), wsum[it & 1], &tot);
            ++it;
            const int room = kLutList - n;
            for (int pos = off; v != 0ull && pos < room; ++pos) {
                lst[n + pos] = (int32_t)((base + tid) * 64 + __builtin_ctzll(v));
                v &= v - 1;
            }
            const int take = tot < room ? tot : room;
            n += take;
            if (n == kLutList) {
                __syncthreads();
                process(n);
                __syncthreads();
                n = 0;
            }
            if (tot <= room) break;
        }
    }
    __syncthreads();
    process(n);
}

template <bool kIndep>
__global__ __launch_bounds__(256) void sparse_bwd_lut_kernel(SparseBwdArgs a) {
    sparse_bwd_lut_body<kIndep>(a, (int64_t)blockIdx.x);
}

hipError_t launch_sparse_bwd(const LaunchCtx &lc, const SparseBwdArgs &a) {
    const int64_t blocks = a.l * ceil_div(a.s, kEpiChunk);
    if (blocks <= 0) return hipSuccess;
    if (blocks > kMaxBlocks) return hipErrorInvalidConfiguration;
    hipEvent_t ev;
    timed_begin(lc, KF_BWD, &ev);
    if (a.bsrc.xt)
        hipLaunchKernelGGL(sparse_bwd_lut_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                           lc.stream, a);
    else
        hipLaunchKernelGGL(sparse_bwd_lut_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                           lc.stream, a);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_BWD, ev);
    return e;
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
