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
// source of sample-parity words. Both directions read tables: 16-entry sums
// over 4 generators (forward) or 4 samples (backward) in LDS, indexed by
// nibbles of parity bits.
#include <cstdlib>

#include "iqp_device.h"

namespace iqp {

// ---------------------------------------------------------------------------
// Sample-parity words: word w of generator j holds b_ij of samples 64 w ..
// 64 w + 63 (bit i % 64). A block covers one chunk of kSpWords words; the
// sample-parity rows hold whole chunks (a multiple of kSpWords words, the
// words of samples >= s being 0), so every load of a chunk's words is
// unconditional.
constexpr int kSpWords = kEpiChunk / 64;
// the float nearest pi and a float near 1 / pi: the forward's FP32 sums are
// folded by whole multiples q of the former (any q is exact bookkeeping)
constexpr float kPiF = 3.14159274f;
constexpr float kInvPiF = 0.318309873f;

// ---------------------------------------------------------------------------
// Gradient: for every (k, j in J_k) the partial T_kj = sum_i S_ki (-1)^{b_ij}
// of a sample chunk is added into an int64 fixed-point accumulator of gate
// j. Integer addition is associative, so the result does not depend on the
// order in which the lanes add, and no per-pair storage is needed. The scale keeps every sum below 2^62: |T_kj| <= s
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


// The set bits of a row of C (Gw words), in gate order, into the LDS list
// lst, 256 row words at a time (a block prefix sum of their popcounts places
// each word's bits); fill(n) runs on every full list (n = kLutList) and on
// the last, partial one (n may be 0), between barriers, so fill may read
// lst and the block's other shared data freely.
template <typename F>
__device__ __forceinline__ void compact_row(glb<const uint64_t> crow, int64_t Gw, int32_t *lst,
                                            int (*wsum)[4], F fill) {
    const int tid = threadIdx.x;
    int n = 0, it = 0;
    for (int64_t base = 0; base < Gw; base += 256) {
        uint64_t v = base + tid < Gw ? crow[base + tid] : 0ull;
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
            if (n == kLutList) {  // uniform over the block
                __syncthreads();
                fill(n);
                __syncthreads();
                n = 0;
            }
            if (tot <= room) break;
        }
    }
    __syncthreads();
    fill(n);
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

    __syncthreads();  // tables written
    compact_row(crow, a.Gw, lst, wsum, process);
}

// Forward by table lookup. A block takes observable k and one chunk of
// kEpiChunk samples; its waves take 4 of the chunk's 16 sample words each,
// lane L sample 64 r + L of word r. The generators J_k are compacted into
// the LDS list as in the backward, and every 4 consecutive entries get a
// 16-entry table of their angle sums,
//   G_e[v] = sum_{b < 4, v_b = 1} t_{lst[4e + b]},  t_j = 2 theta'_j (FP32),
// so that a sample's sum over the 64 entries 64g .. 64g + 63 is the sum of
// 16 table reads indexed by its parity bits for those generators, 4 at a
// time. Those bits come from a 64 x 64 bit transpose: lane L loads the
// parity word of entry 64g + L for the wave's sample word, and after the
// transpose lane L holds, for its sample, bit c = the parity of entry
// 64g + c. The nibble offsets are formed as in the backward ((x << 2) and
// (x >> 2) masked to 0x3C per byte) and a byte permute places each one
// under the group's table base (g * 1024 bytes; the table within the group
// is the LDS instruction's immediate offset). All lanes read one 16-entry
// table at a time, so the reads never conflict. Per sample,
//   E_ki = T_k - 2 sum_{j in J_k, b_ij = 1} t_j,  T_k = sum_{j in J_k} t_j (FP64),
// with the FP32 sum folded modulo the float nearest pi every 32 generators
// (the whole multiples kept in an exact count), then reduced modulo 2 pi in
// FP64 as the dense epilogue does.
template <bool kIndep>
__device__ __forceinline__ void lut_fwd_words(const SparseFwdArgs &a, int64_t k, int64_t sw,
                                              int64_t j, u32x4 (&wv)[2]);
template <>
__device__ __forceinline__ void lut_fwd_words<false>(const SparseFwdArgs &a, int64_t, int64_t sw,
                                                     int64_t j, u32x4 (&wv)[2]) {
    const glb<const u32x4> src = (glb<const u32x4>)(gptr(a.bsrc.btrm) + j * a.bsrc.Rwb + sw);
    wv[0] = src[0];
    wv[1] = src[1];
}
template <>
__device__ __forceinline__ void lut_fwd_words<true>(const SparseFwdArgs &a, int64_t k, int64_t sw,
                                                    int64_t j, u32x4 (&wv)[2]) {
    const glb<const uint64_t> cols = gptr(a.bsrc.xt) + k * a.bsrc.xstride + sw;
    auto add_col = [&](int64_t q) {
        const glb<const u32x4> src = (glb<const u32x4>)(cols + q * a.bsrc.Rwb);
        wv[0] ^= src[0];
        wv[1] ^= src[1];
    };
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
__device__ __forceinline__ void sparse_fwd_lut_body(const SparseFwdArgs &a, int64_t blk) {
    const int64_t nchunk = ceil_div(a.s, kEpiChunk);
    const int64_t ch = blk / a.l, k = blk - ch * a.l;  // chunk-major, as the backward
    const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
    __shared__ __attribute__((aligned(16))) float tab[kLutTables * 16];
    __shared__ int32_t lst[kLutList];
    __shared__ int wsum[2][4];
    __shared__ double red[3][4];
    const int64_t sw = ch * kSpWords + 4 * wave;  // the wave's first sample word
    const glb<const float> t32 = gptr(a.t32);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f}, kpi[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    double Tp = 0.0;  // this thread's share of T_k
    auto fill = [&](int n) {
        {  // table tid: entries 4 tid .. 4 tid + 3 (0 past the list)
            float t[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int e = 4 * tid + b;
                t[b] = e < n ? t32[lst[e]] : 0.0f;
                Tp += (double)t[b];
            }
            const float x[4] = {0.0f, t[0], t[1], t[0] + t[1]};
            const float y[4] = {0.0f, t[2], t[3], t[2] + t[3]};
            float4 *row = reinterpret_cast<float4 *>(tab + tid * 16);
#pragma unroll
            for (int h = 0; h < 4; ++h)
                row[h] = make_float4(x[0] + y[h], x[1] + y[h], x[2] + y[h], x[3] + y[h]);
        }
        __syncthreads();
        const char *tb = reinterpret_cast<const char *>(tab);
        for (int g = 0; 64 * g < n; ++g) {
            const int e = 64 * g + lane;
            u32x4 wv[2] = {u32x4{0, 0, 0, 0}, u32x4{0, 0, 0, 0}};
            if (e < n) lut_fwd_words<kIndep>(a, k, sw, lst[e], wv);
            const uint32_t gb = (uint32_t)g * 1024u;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint64_t xw = ((uint64_t)wv[r / 2][2 * (r % 2) + 1] << 32) |
                                    wv[r / 2][2 * (r % 2)];
                const uint64_t yb = transpose64(xw, lane);
                // m[2h] byte e': 4 * nibble 2e' of dword h, m[2h + 1]: nibble 2e' + 1
                uint32_t m[4];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t d = (uint32_t)(yb >> (32 * h));
                    m[2 * h] = (d << 2) & 0x3C3C3C3Cu;
                    m[2 * h + 1] = (d >> 2) & 0x3C3C3C3Cu;
                }
                float v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const uint32_t o = __builtin_amdgcn_perm(
                        gb, m[2 * (q / 8) + q % 2], 0x07060500u | (uint32_t)((q % 8) / 2));
                    v[q] = *reinterpret_cast<const float *>(tb + q * 64 + o);
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float p = ((v[8 * h] + v[8 * h + 1]) + (v[8 * h + 2] + v[8 * h + 3])) +
                                    ((v[8 * h + 4] + v[8 * h + 5]) + (v[8 * h + 6] + v[8 * h + 7]));
                    acc[r] += p;
                    const float qq = rintf(acc[r] * kInvPiF);
                    acc[r] = fmaf(-qq, kPiF, acc[r]);
                    kpi[r] += qq;
                }
            }
        }
    };
    compact_row(gptr(a.crm) + k * a.Gw, a.Gw, lst, wsum, fill);

    // T_k = the sum of the threads' shares (waves, then the 4 wave sums in order)
#pragma unroll
    for (int st = 32; st >= 1; st >>= 1) Tp += __shfl_xor(Tp, st, 64);
    if (lane == 0) red[0][wave] = Tp;
    __syncthreads();
    const double T = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    double sc = 0.0, sc2 = 0.0;
    float IQP_GLOBAL *ph = a.phase_out ? gptr(a.phase_out) + k * a.s : nullptr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t i = (sw + r) * 64 + lane;
        if (i < a.s) {
            const double e = T - 2.0 * ((double)acc[r] + (double)kpi[r] * (double)kPiF);
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
        red[1][wave] = sc;
        red[2][wave] = sc2;
    }
    __syncthreads();
    if (tid == 0) {
        double IQP_GLOBAL *part = gptr(a.part) + (k * nchunk + ch) * 2;
        part[0] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        part[1] = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
    }
}

// One block per (observable, chunk) unit. When the units outnumber the grid
// (at most kMaxBlocks blocks), the strided form takes them in steps of the
// grid's size, with a barrier before a block's next unit rewrites its LDS;
// it is a separate instantiation because the loop costs the body registers
// (85 and 93 instead of 77 and 76 VGPRs: a wave per SIMD).
template <bool kIndep, bool kStrided>
__global__ __launch_bounds__(256) void sparse_fwd_lut_kernel(SparseFwdArgs a, int64_t units) {
    if (!kStrided) {
        sparse_fwd_lut_body<kIndep>(a, (int64_t)blockIdx.x);
        return;
    }
    for (int64_t b = blockIdx.x; b < units; b += gridDim.x) {
        sparse_fwd_lut_body<kIndep>(a, b);
        __syncthreads();
    }
}

template <bool kIndep, bool kStrided>
__global__ __launch_bounds__(256) void sparse_bwd_lut_kernel(SparseBwdArgs a, int64_t units) {
    if (!kStrided) {
        sparse_bwd_lut_body<kIndep>(a, (int64_t)blockIdx.x);
        return;
    }
    for (int64_t b = blockIdx.x; b < units; b += gridDim.x) {
        sparse_bwd_lut_body<kIndep>(a, b);
        __syncthreads();
    }
}

// Blocks of a table-lookup launch: one per unit up to kMaxBlocks, or fewer
// when IQP_SPARSE_GRID_CAP is set, so that tests can take the strided path
// at small sizes.
static int64_t lut_grid(int64_t units) {
    const char *c = getenv("IQP_SPARSE_GRID_CAP");
    const long long v = c ? atoll(c) : 0;
    const int64_t cap = v > 0 ? (int64_t)v : (int64_t)kMaxBlocks;
    const int64_t g = units < cap ? units : cap;
    return g < kMaxBlocks ? g : kMaxBlocks;
}

hipError_t launch_sparse_fwd(const LaunchCtx &lc, const SparseFwdArgs &a) {
    const int64_t units = a.l * ceil_div(a.s, kEpiChunk);
    if (units <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)lut_grid(units);
    hipEvent_t ev;
    timed_begin(lc, KF_FWD, &ev);
    const bool strided = (int64_t)blocks < units;
    if (a.bsrc.xt && strided)
        hipLaunchKernelGGL((sparse_fwd_lut_kernel<true, true>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    else if (a.bsrc.xt)
        hipLaunchKernelGGL((sparse_fwd_lut_kernel<true, false>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    else if (strided)
        hipLaunchKernelGGL((sparse_fwd_lut_kernel<false, true>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    else
        hipLaunchKernelGGL((sparse_fwd_lut_kernel<false, false>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_FWD, ev);
    return e;
}

hipError_t launch_sparse_bwd(const LaunchCtx &lc, const SparseBwdArgs &a) {
    const int64_t units = a.l * ceil_div(a.s, kEpiChunk);
    if (units <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)lut_grid(units);
    hipEvent_t ev;
    timed_begin(lc, KF_BWD, &ev);
    const bool strided = (int64_t)blocks < units;
    if (a.bsrc.xt && strided)
        hipLaunchKernelGGL((sparse_bwd_lut_kernel<true, true>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    else if (a.bsrc.xt)
        hipLaunchKernelGGL((sparse_bwd_lut_kernel<true, false>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    else if (strided)
        hipLaunchKernelGGL((sparse_bwd_lut_kernel<false, true>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
    else
        hipLaunchKernelGGL((sparse_bwd_lut_kernel<false, false>), dim3(blocks), dim3(256), 0,
                           lc.stream, a, units);
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
