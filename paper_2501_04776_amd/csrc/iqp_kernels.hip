// gfx950 kernels of the IQP Monte Carlo expectation-value path.
//
//   theta_prep      theta -> 2 theta' (theta' = theta reduced to [-pi/2, pi/2]
//                   by whole multiples of pi), as FP32 or BF16 hi + lo
//   parity          bit-exact popcount(row AND col) mod 2 matrices (the
//                   exponents of B and C, Sec. 2.2), one wave per 64 columns
//                   x 32 rows, packed with a 64-lane ballot
//   phase_fwd       E = C Theta B^T (eq. Emat) on the matrix cores, operands
//                   expanded from parity bits in registers
//   epilogue        FP64 reduction of E modulo 2 pi, cos, per-chunk sums of
//                   cos and cos^2 (eq. expvalsample)
//   finalize        mean and standard error per observable, fixed order
//   weights         S_ki = (alpha_k + beta_k cos E_ki) sin E_ki, written in
//                   the register image of the backward matrix-core operand
//   phase_bwd       D[j][i] = sum_k c_kj S_ki on the matrix cores, epilogue
//                   sum_i (-1)^{b_ij} D[j][i] per gate
//   grad_reduce     dtheta_j = -2 sum over sample tiles, fixed order
//   data_stats, mmd_loss, coef_*: the MMD^2 chain (eq. mmd_estimate)
//
// No float atomics anywhere: every reduction runs in a fixed order, so a call
// is bitwise reproducible.
#include "iqp_internal.h"

#include <math.h>

namespace iqp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 2 pi split for a two-step Cody-Waite reduction (Cody & Waite, 1980):
// hi is the double nearest 2 pi, lo the double nearest 2 pi - hi.
#define IQP_TWO_PI_HI 6.283185307179586
#define IQP_TWO_PI_LO 2.4492935982947064e-16
#define IQP_INV_TWO_PI 0.15915494309189535
#define IQP_PI 3.141592653589793
#define IQP_INV_PI 0.3183098861837907

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
}

// Workgroups are handed to the 8 XCDs round-robin. Remap so that each XCD
// owns a contiguous range of tile indices: neighbouring tiles share operand
// strips, which then stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ uint16_t f2bf_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// theta_prep
__global__ __launch_bounds__(256) void theta_prep_kernel(const double *__restrict__ theta,
                                                         int64_t m, int64_t m_pad, int prec,
                                                         uint16_t *__restrict__ hi,
                                                         uint16_t *__restrict__ lo,
                                                         float *__restrict__ t32) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m_pad) return;
    double t = i < m ? theta[i] : 0.0;
    double tr = t - IQP_PI * rint(t * IQP_INV_PI);
    double two = 2.0 * tr;
    if (prec == 1) {
        uint16_t h = f2bf_rne((float)two);
        double rem = two - (double)bf2f(h);
        hi[i] = h;
        lo[i] = f2bf_rne((float)rem);
    } else {
        // split by gate parity: lane half h of the 32x32x2 product reads gate 2t + h
        t32[(i & 1) * (m_pad >> 1) + (i >> 1)] = (float)two;
    }
}

hipError_t launch_theta_prep(const LaunchCtx &lc, const double *theta, int64_t m, int64_t m_pad,
                             int prec, uint16_t *hi, uint16_t *lo, float *t32) {
    hipEvent_t ev;
    timed_begin(lc, KF_THETA, &ev);
    hipLaunchKernelGGL(theta_prep_kernel, dim3((unsigned)ceil_div(m_pad, 256)), dim3(256), 0,
                       lc.stream, theta, m, m_pad, prec, hi, lo, t32);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_THETA, ev);
    return e;
}

// ---------------------------------------------------------------------------
// parity: out bit (r, c) = popcount(rows[r] AND cols[c]) mod 2.
// One wave owns 64 columns (one per lane) and 32 rows. Row words are
// wave-uniform (scalar loads); the AND is XOR-folded over the W words so one
// popcount per entry remains. A ballot packs the 64 column parities of a row
// into one word, which lane (r mod 32) then stores: 32 consecutive words per
// wave for the tiled layout.
template <int LAYOUT>
__global__ __launch_bounds__(256) void parity_kernel(const uint64_t *__restrict__ rows, int64_t R,
                                                     int64_t R_out,
                                                     const uint64_t *__restrict__ cols,
                                                     int64_t C, int64_t Cw, int W,
                                                     uint64_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t unit = (int64_t)blockIdx.x * 4 + wave_id();
    const int64_t nrb = ceil_div(R_out, 32);
    if (unit >= nrb * Cw) return;
    const int64_t rb = unit / Cw, cw = unit - rb * Cw;
    const int64_t c = cw * 64 + lane;
    const bool cvalid = c < C;
    const int64_t r0 = rb * 32;
    int64_t nr64 = R - r0;
    const int nr = nr64 <= 0 ? 0 : (nr64 >= 32 ? 32 : (int)nr64);
    uint64_t acc[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[r] = 0;
    if (nr == 32) {
        for (int w = 0; w < W; ++w) {
            const uint64_t g = cvalid ? cols[c * W + w] : 0ull;
            const uint64_t *rp = rows + r0 * W + w;
#pragma unroll
            for (int r = 0; r < 32; ++r) acc[r] ^= rp[(int64_t)r * W] & g;
        }
    } else if (nr > 0) {
        for (int w = 0; w < W; ++w) {
            const uint64_t g = cvalid ? cols[c * W + w] : 0ull;
            const uint64_t *rp = rows + r0 * W + w;
#pragma unroll
            for (int r = 0; r < 32; ++r)
                if (r < nr) acc[r] ^= rp[(int64_t)r * W] & g;
        }
    }
    uint64_t mine = 0;
#pragma unroll
    for (int r = 0; r < 32; ++r) {
        const uint64_t mask = __ballot((int)(__popcll(acc[r]) & 1));
        mine = (lane == r) ? mask : mine;
    }
    if (lane < 32) {
        const int64_t rr = r0 + lane;
        if (rr < R_out) {
            if (LAYOUT == 1)
                out[(rb * Cw + cw) * 32 + lane] = mine;
            else
                out[rr * Cw + cw] = mine;
        }
    }
}

hipError_t launch_parity(const LaunchCtx &lc, const uint64_t *rows, int64_t R, int64_t R_out,
                         const uint64_t *cols, int64_t C, int64_t Cw, int W, int layout,
                         uint64_t *out) {
    const int64_t units = ceil_div(R_out, 32) * Cw;
    if (units == 0) return hipSuccess;
    hipEvent_t ev;
    timed_begin(lc, KF_PARITY, &ev);
    dim3 grid((unsigned)ceil_div(units, 4));
    if (layout == 1)
        hipLaunchKernelGGL(parity_kernel<1>, grid, dim3(256), 0, lc.stream, rows, R, R_out, cols,
                           C, Cw, W, out);
    else
        hipLaunchKernelGGL(parity_kernel<0>, grid, dim3(256), 0, lc.stream, rows, R, R_out, cols,
                           C, Cw, W, out);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_PARITY, ev);
    return e;
}

// ---------------------------------------------------------------------------
// Operand expansion from parity bits, in registers.
//
// A 32x32x16 BF16 product reads, in lane l, 8 consecutive K values
// 8*(l/32) + e, e = 0..7, packed two per dword (element 2v in the low half of
// dword v). `x` carries the lane's 8 parity bits in bits 0..7 of a 16-bit
// value (bits 8..15 are ignored). A packed 16-bit shift by (15 - 2v, 14 - 2v)
// moves bits 2v and 2v+1 to the sign positions 15 and 31 of dword v.

// B_ij = (-1)^{bit}: +1.0 = 0x3F80, -1.0 = 0xBF80.
__device__ __forceinline__ bf16x8 expand_pm1(uint32_t x16) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh = {(unsigned short)(15 - 2 * v), (unsigned short)(14 - 2 * v)};
        d[v] = (__builtin_bit_cast(uint32_t, (u16x2)(xv << sh)) & 0x80008000u) | 0x3F803F80u;
    }
    return __builtin_bit_cast(bf16x8, d);
}

// C_kj theta_j / 2 = bit ? 2 theta'_j : 0 for both limbs; the sign bit is
// spread over its half by an arithmetic shift to make the mask.
__device__ __forceinline__ void expand_masked(uint32_t x16, const u32x4 &th, const u32x4 &tl,
                                              bf16x8 &ah, bf16x8 &al) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t dh[4], dl[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh = {(unsigned short)(15 - 2 * v), (unsigned short)(14 - 2 * v)};
        const s16x2 sg = __builtin_bit_cast(s16x2, (u16x2)(xv << sh)) >> (s16x2){15, 15};
        const uint32_t msk = __builtin_bit_cast(uint32_t, sg);
        dh[v] = th[v] & msk;
        dl[v] = tl[v] & msk;
    }
    ah = __builtin_bit_cast(bf16x8, dh);
    al = __builtin_bit_cast(bf16x8, dl);
}

// c_kj in {0, 1}: 1.0 = 0x3F80.
__device__ __forceinline__ bf16x8 expand_01(uint32_t x16) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh = {(unsigned short)(15 - 2 * v), (unsigned short)(14 - 2 * v)};
        const s16x2 sg = __builtin_bit_cast(s16x2, (u16x2)(xv << sh)) >> (s16x2){15, 15};
        d[v] = __builtin_bit_cast(uint32_t, sg) & 0x3F803F80u;
    }
    return __builtin_bit_cast(bf16x8, d);
}

// The 16 accumulators of a 32x32 product in lane l hold column l % 32 and
// rows 8*(a/4) + 4*(l/32) + (a%4), a = 0..15.
__device__ __forceinline__ int acc_row(int a, int h) { return 8 * (a >> 2) + 4 * h + (a & 3); }

// ---------------------------------------------------------------------------
// phase_fwd: E[k][i] = sum_j (c_kj * 2 theta'_j) * (-1)^{b_ij}.
// Units are (split, observable block, sample block); one wave computes a
// (32 FM) x (32 FN) tile over its range of gate words. C and B parity bits
// are tiled32, so each 32-row fragment of a 64-gate word is 256 contiguous
// bytes. Within a word, K-step t (16 gates) uses byte 2t + h of the lane's
// word (h = lane / 32): the word is pre-shifted right by 8h.
template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_fwd_bf16_kernel(
    const uint64_t *__restrict__ cbits, const uint64_t *__restrict__ bbits,
    const u32x4 *__restrict__ thh, const u32x4 *__restrict__ thl, int64_t mw, int64_t n_ob,
    int64_t n_sb, int64_t units, int64_t wps, float *__restrict__ E, int64_t l_pad,
    int64_t s_pad) {
    const int lane = threadIdx.x & 63;
    const int64_t u = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave_id();
    if (u >= units) return;
    const int64_t sb = u % n_sb;
    const int64_t t0 = u / n_sb;
    const int64_t ob = t0 % n_ob;
    const int64_t split = t0 / n_ob;
    const int64_t w0 = split * wps;
    const int64_t w1 = (w0 + wps < mw) ? w0 + wps : mw;
    const int h = lane >> 5, r = lane & 31;

    const uint64_t *cp[FM];
    const uint64_t *bp[FN];
#pragma unroll
    for (int f = 0; f < FM; ++f) cp[f] = cbits + (ob * FM + f) * mw * 32 + r;
#pragma unroll
    for (int g = 0; g < FN; ++g) bp[g] = bbits + (sb * FN + g) * mw * 32 + r;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    uint64_t cwn[FM], bwn[FN];
    if (w0 < w1) {
#pragma unroll
        for (int f = 0; f < FM; ++f) cwn[f] = cp[f][w0 * 32];
#pragma unroll
        for (int g = 0; g < FN; ++g) bwn[g] = bp[g][w0 * 32];
    }
    for (int64_t w = w0; w < w1; ++w) {
        uint64_t cw[FM], bw[FN];
#pragma unroll
        for (int f = 0; f < FM; ++f) cw[f] = cwn[f] >> (8 * h);
#pragma unroll
        for (int g = 0; g < FN; ++g) bw[g] = bwn[g] >> (8 * h);
        if (w + 1 < w1) {
#pragma unroll
            for (int f = 0; f < FM; ++f) cwn[f] = cp[f][(w + 1) * 32];
#pragma unroll
            for (int g = 0; g < FN; ++g) bwn[g] = bp[g][(w + 1) * 32];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const u32x4 th = thh[8 * w + 2 * t + h];
            const u32x4 tl = thl[8 * w + 2 * t + h];
            bf16x8 bv[FN];
#pragma unroll
            for (int g = 0; g < FN; ++g) {
                const uint32_t d = (uint32_t)(bw[g] >> (32 * (t >> 1)));
                bv[g] = expand_pm1((t & 1) ? (d >> 16) : d);
            }
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                const uint32_t d = (uint32_t)(cw[f] >> (32 * (t >> 1)));
                bf16x8 ah, al;
                expand_masked((t & 1) ? (d >> 16) : d, th, tl, ah, al);
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bv[g], acc[f][g], 0, 0, 0);
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bv[g], acc[f][g], 0, 0, 0);
            }
        }
    }
    float *Ep = E + split * l_pad * s_pad;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const int64_t col = (sb * FN + g) * 32 + r;
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const int64_t row = (ob * FM + f) * 32 + acc_row(a, h);
                Ep[row * s_pad + col] = acc[f][g][a];
            }
        }
}

// FP32 form: 32x32x2 products, lane l reads K value l / 32. The word is
// pre-shifted right by h, so K-step t (gates 2t, 2t+1) uses bit 2t. theta is
// split by gate parity: t32[h][32 w + t] = 2 theta'_{64 w + 2 t + h}.
template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_fwd_f32_kernel(
    const uint64_t *__restrict__ cbits, const uint64_t *__restrict__ bbits,
    const float *__restrict__ t32, int64_t m_pad, int64_t mw, int64_t n_ob, int64_t n_sb,
    int64_t units, int64_t wps, float *__restrict__ E, int64_t l_pad, int64_t s_pad) {
    const int lane = threadIdx.x & 63;
    const int64_t u = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave_id();
    if (u >= units) return;
    const int64_t sb = u % n_sb;
    const int64_t t0 = u / n_sb;
    const int64_t ob = t0 % n_ob;
    const int64_t split = t0 / n_ob;
    const int64_t w0 = split * wps;
    const int64_t w1 = (w0 + wps < mw) ? w0 + wps : mw;
    const int h = lane >> 5, r = lane & 31;
    const float4 *thp = reinterpret_cast<const float4 *>(t32 + h * (m_pad >> 1));

    const uint64_t *cp[FM];
    const uint64_t *bp[FN];
#pragma unroll
    for (int f = 0; f < FM; ++f) cp[f] = cbits + (ob * FM + f) * mw * 32 + r;
#pragma unroll
    for (int g = 0; g < FN; ++g) bp[g] = bbits + (sb * FN + g) * mw * 32 + r;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    for (int64_t w = w0; w < w1; ++w) {
        uint64_t cw[FM], bw[FN];
#pragma unroll
        for (int f = 0; f < FM; ++f) cw[f] = cp[f][w * 32] >> h;
#pragma unroll
        for (int g = 0; g < FN; ++g) bw[g] = bp[g][w * 32] >> h;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float4 tv = thp[8 * w + q];
            const float tq[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int t = 4 * q + e;
                float bv[FN];
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    bv[g] = __uint_as_float((((uint32_t)(bw[g] >> (2 * t)) & 1u) << 31) |
                                            0x3F800000u);
#pragma unroll
                for (int f = 0; f < FM; ++f) {
                    const uint32_t msk = 0u - ((uint32_t)(cw[f] >> (2 * t)) & 1u);
                    const float av = __uint_as_float(__float_as_uint(tq[e]) & msk);
#pragma unroll
                    for (int g = 0; g < FN; ++g)
                        acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[g], acc[f][g], 0, 0, 0);
                }
            }
        }
    }
    float *Ep = E + split * l_pad * s_pad;
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const int64_t col = (sb * FN + g) * 32 + r;
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const int64_t row = (ob * FM + f) * 32 + acc_row(a, h);
                Ep[row * s_pad + col] = acc[f][g][a];
            }
        }
}

template <int FM, int FN>
static void fwd_dispatch(const LaunchCtx &lc, int prec, const uint64_t *cbits,
                         const uint64_t *bbits, const uint16_t *thh, const uint16_t *thl,
                         const float *t32, int64_t m_pad, int64_t l_pad, int64_t s_pad,
                         int64_t splits, float *E) {
    const int64_t mw = m_pad / 64;
    const int64_t n_ob = l_pad / (32 * FM), n_sb = s_pad / (32 * FN);
    const int64_t wps = ceil_div(mw, splits);
    const int64_t units = n_ob * n_sb * splits;
    dim3 grid((unsigned)ceil_div(units, 4));
    if (prec == 1)
        hipLaunchKernelGGL((phase_fwd_bf16_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, cbits,
                           bbits, reinterpret_cast<const u32x4 *>(thh),
                           reinterpret_cast<const u32x4 *>(thl), mw, n_ob, n_sb, units, wps, E,
                           l_pad, s_pad);
    else
        hipLaunchKernelGGL((phase_fwd_f32_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, cbits,
                           bbits, t32, m_pad, mw, n_ob, n_sb, units, wps, E, l_pad, s_pad);
}

hipError_t launch_phase_fwd(const LaunchCtx &lc, int prec, int fm, int fn, const uint64_t *cbits,
                            const uint64_t *bbits, const uint16_t *thh, const uint16_t *thl,
                            const float *t32, int64_t m_pad, int64_t l_pad, int64_t s_pad,
                            int64_t splits, float *E) {
    hipEvent_t ev;
    timed_begin(lc, KF_FWD, &ev);
    if (fm == 4 && fn == 4)
        fwd_dispatch<4, 4>(lc, prec, cbits, bbits, thh, thl, t32, m_pad, l_pad, s_pad, splits, E);
    else if (fm == 2 && fn == 2)
        fwd_dispatch<2, 2>(lc, prec, cbits, bbits, thh, thl, t32, m_pad, l_pad, s_pad, splits, E);
    else if (fm == 2 && fn == 4)
        fwd_dispatch<2, 4>(lc, prec, cbits, bbits, thh, thl, t32, m_pad, l_pad, s_pad, splits, E);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_FWD, ev);
    return e;
}

// ---------------------------------------------------------------------------
// epilogue: one block per (observable k, chunk of kEpiChunk samples).
__device__ __forceinline__ double block_sum_256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void epilogue_kernel(const float *__restrict__ E, int64_t splits,
                                                       int64_t l, int64_t s, int64_t l_pad,
                                                       int64_t s_pad, int64_t nchunk,
                                                       float *__restrict__ phase_out,
                                                       double *__restrict__ part) {
    __shared__ double sh[256];
    const int64_t blk = blockIdx.x;
    const int64_t k = blk / nchunk, ch = blk - k * nchunk;
    double sc = 0.0, sc2 = 0.0;
#pragma unroll
    for (int q = 0; q < (int)(kEpiChunk / 256); ++q) {
        const int64_t i = ch * kEpiChunk + q * 256 + threadIdx.x;
        if (i < s) {
            double e = 0.0;
            for (int64_t sp = 0; sp < splits; ++sp) e += (double)E[(sp * l_pad + k) * s_pad + i];
            const double kk = rint(e * IQP_INV_TWO_PI);
            double rr = fma(-kk, IQP_TWO_PI_HI, e);
            rr = fma(-kk, IQP_TWO_PI_LO, rr);
            const float rf = (float)rr;
            const float c = cosf(rf);
            if (phase_out) phase_out[k * s + i] = rf;
            sc += (double)c;
            sc2 += (double)c * (double)c;
        }
    }
    sc = block_sum_256(sc, sh);
    sc2 = block_sum_256(sc2, sh);
    if (threadIdx.x == 0) {
        part[(k * nchunk + ch) * 2 + 0] = sc;
        part[(k * nchunk + ch) * 2 + 1] = sc2;
    }
}

hipError_t launch_epilogue(const LaunchCtx &lc, const float *E, int64_t splits, int64_t l,
                           int64_t s, int64_t l_pad, int64_t s_pad, float *phase_out,
                           double *part) {
    const int64_t nchunk = ceil_div(s, kEpiChunk);
    hipEvent_t ev;
    timed_begin(lc, KF_EPI, &ev);
    hipLaunchKernelGGL(epilogue_kernel, dim3((unsigned)(l * nchunk)), dim3(256), 0, lc.stream, E,
                       splits, l, s, l_pad, s_pad, nchunk, phase_out, part);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_EPI, ev);
    return e;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ part, int64_t l,
                                                       int64_t nchunk, int64_t s,
                                                       double *__restrict__ mean,
                                                       double *__restrict__ stderr_,
                                                       double *__restrict__ rowsum) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= l) return;
    double sc = 0.0, sc2 = 0.0;
    for (int64_t ch = 0; ch < nchunk; ++ch) {
        sc += part[(k * nchunk + ch) * 2 + 0];
        sc2 += part[(k * nchunk + ch) * 2 + 1];
    }
    const double S = (double)s;
    const double mu = sc / S;
    const double var = sc2 / S - mu * mu;
    if (mean) mean[k] = mu;
    if (stderr_) stderr_[k] = sqrt((var > 0.0 ? var : 0.0) / S);
    if (rowsum) {
        rowsum[2 * k + 0] = sc;
        rowsum[2 * k + 1] = sc2;
    }
}

hipError_t launch_finalize(const LaunchCtx &lc, const double *part, int64_t l, int64_t s,
                           double *mean, double *stderr_, double *rowsum) {
    const int64_t nchunk = ceil_div(s, kEpiChunk);
    hipEvent_t ev;
    timed_begin(lc, KF_FIN, &ev);
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0,
                       lc.stream, part, l, nchunk, s, mean, stderr_, rowsum);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_FIN, ev);
    return e;
}

// ---------------------------------------------------------------------------
// Backward weights. coef[2k] = alpha_k, coef[2k+1] = beta_k give
// dL/dc_ki = alpha_k + beta_k cos E_ki, and
//   S_ki = (alpha_k + beta_k cos E_ki) sin E_ki.
__global__ __launch_bounds__(256) void coef_plain_kernel(const double *__restrict__ u, int64_t l,
                                                         int64_t s, double *__restrict__ coef) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= l) return;
    coef[2 * k] = u[k] / (double)s;
    coef[2 * k + 1] = 0.0;
}

hipError_t launch_coef_plain(const LaunchCtx &lc, const double *grad_mean, int64_t l, int64_t s,
                             double *coef) {
    hipEvent_t ev;
    timed_begin(lc, KF_WEIGHTS, &ev);
    hipLaunchKernelGGL(coef_plain_kernel, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0,
                       lc.stream, grad_mean, l, s, coef);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_WEIGHTS, ev);
    return e;
}

// One block per 64 observables x 64 samples: S values are staged in LDS and
// written out in the register image of the backward product's B operand.
//   BF16: 16-byte unit ((ib * KT + kt) * 64 + h*32 + i%32) holds
//         S[i][16 kt + 8 h + e], e = 0..7 (ib = i / 32, KT = l_pad / 16)
//   FP32: float ((ib * KT2 + t) * 64 + h*32 + i%32) holds S[i][2 t + h]
//         (KT2 = l_pad / 2)
__global__ __launch_bounds__(256) void weights_kernel(const float *__restrict__ phase,
                                                      const double *__restrict__ coef, int64_t l,
                                                      int64_t s, int64_t l_pad, int prec,
                                                      uint16_t *__restrict__ shi,
                                                      uint16_t *__restrict__ slo,
                                                      float *__restrict__ s32) {
    __shared__ float tile[64][65];  // [obs][sample]
    const int64_t i0 = (int64_t)blockIdx.x * 64, k0 = (int64_t)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int kr = ty * 16 + q;
        const int64_t k = k0 + kr, i = i0 + tx;
        float v = 0.0f;
        if (k < l && i < s) {
            const float ph = phase[k * s + i];
            float sn, cs;
            sincosf(ph, &sn, &cs);
            const double a = coef[2 * k], b = coef[2 * k + 1];
            v = (float)((a + b * (double)cs) * (double)sn);
        }
        tile[kr][tx] = v;
    }
    __syncthreads();
    if (prec == 1) {
        const int64_t KT = l_pad / 16;
        // 64 samples x 8 groups of 8 observables = 512 units, 2 per thread
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int unit = q * 256 + threadIdx.x;
            const int il = unit & 63, kg = unit >> 6;  // kg = 0..7: observables 8 kg ..
            const int64_t i = i0 + il;
            const int64_t kabs = k0 + 8 * kg;
            const int64_t kt = kabs >> 4;
            const int hh = (int)((kabs >> 3) & 1);
            const int64_t idx = ((i >> 5) * KT + kt) * 64 + hh * 32 + (i & 31);
            uint32_t dh[4], dl[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uint16_t hv[2], lv[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float x = tile[8 * kg + 2 * v + e][il];
                    hv[e] = f2bf_rne(x);
                    lv[e] = f2bf_rne(x - bf2f(hv[e]));
                }
                dh[v] = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
                dl[v] = (uint32_t)lv[0] | ((uint32_t)lv[1] << 16);
            }
            reinterpret_cast<u32x4 *>(shi)[idx] = (u32x4){dh[0], dh[1], dh[2], dh[3]};
            reinterpret_cast<u32x4 *>(slo)[idx] = (u32x4){dl[0], dl[1], dl[2], dl[3]};
        }
    } else {
        const int64_t KT2 = l_pad / 2;
        // 64 samples x 64 observables = 4096 floats, 16 per thread
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int unit = q * 256 + threadIdx.x;
            const int il = unit & 63, kl = unit >> 6;
            const int64_t i = i0 + il, kabs = k0 + kl;
            const int64_t t = kabs >> 1;
            const int hh = (int)(kabs & 1);
            s32[((i >> 5) * KT2 + t) * 64 + hh * 32 + (i & 31)] = tile[kl][il];
        }
    }
}

hipError_t launch_weights(const LaunchCtx &lc, int prec, const float *phase, const double *coef,
                          int64_t l, int64_t s, int64_t l_pad, int64_t s_pad, uint16_t *shi,
                          uint16_t *slo, float *s32) {
    hipEvent_t ev;
    timed_begin(lc, KF_WEIGHTS, &ev);
    dim3 grid((unsigned)(s_pad / 64), (unsigned)(l_pad / 64));
    hipLaunchKernelGGL(weights_kernel, grid, dim3(256), 0, lc.stream, phase, coef, l, s, l_pad,
                       prec, shi, slo, s32);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_WEIGHTS, ev);
    return e;
}

// ---------------------------------------------------------------------------
// phase_bwd: D[j][i] = sum_k c_kj S_ki (gates x samples, K = observables),
// then per gate sum_i (-1)^{b_ij} D[j][i] over the wave's samples. A operand
// from tiled32 C^T bits (rows = gates, bits over observables), B operand the
// S register image. Units are (sample block, gate block), gate fastest, so
// the waves of an XCD share the S strip of one sample block.
template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_bwd_bf16_kernel(
    const uint64_t *__restrict__ ctbits, const u32x4 *__restrict__ shi,
    const u32x4 *__restrict__ slo, const uint64_t *__restrict__ bbits, int64_t lw, int64_t mw,
    int64_t n_jb, int64_t units, float *__restrict__ gpart, int64_t m_pad) {
    const int lane = threadIdx.x & 63;
    const int64_t u = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave_id();
    if (u >= units) return;
    const int64_t ib = u / n_jb, jb = u - ib * n_jb;
    const int h = lane >> 5, r = lane & 31;
    const int64_t KT = lw * 4;

    const uint64_t *cp[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) cp[f] = ctbits + (jb * FM + f) * lw * 32 + r;
    int64_t sp[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) sp[g] = (ib * FN + g) * KT * 64 + lane;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    uint64_t cwn[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) cwn[f] = cp[f][0];
    for (int64_t w = 0; w < lw; ++w) {
        uint64_t cw[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) cw[f] = cwn[f] >> (8 * h);
        if (w + 1 < lw) {
#pragma unroll
            for (int f = 0; f < FM; ++f) cwn[f] = cp[f][(w + 1) * 32];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t kt = 4 * w + t;
            bf16x8 bh[FN], bl[FN];
#pragma unroll
            for (int g = 0; g < FN; ++g) {
                bh[g] = __builtin_bit_cast(bf16x8, shi[sp[g] + kt * 64]);
                bl[g] = __builtin_bit_cast(bf16x8, slo[sp[g] + kt * 64]);
            }
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                const uint32_t d = (uint32_t)(cw[f] >> (32 * (t >> 1)));
                const bf16x8 av = expand_01((t & 1) ? (d >> 16) : d);
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bh[g], acc[f][g], 0, 0, 0);
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bl[g], acc[f][g], 0, 0, 0);
            }
        }
    }
    // epilogue: signs (-1)^{b_ij} from the tiled32 B bits of sample i
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const int64_t j0 = (jb * FM + f) * 32;
        const int64_t jw = j0 >> 6;
        const int jo = (int)(j0 & 63);
        float gs[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) gs[a] = 0.0f;
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const uint64_t bw = bbits[((ib * FN + g) * mw + jw) * 32 + r];
            const uint32_t b32 = (uint32_t)(bw >> jo) >> (4 * h);
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const uint32_t sgn = ((b32 >> (8 * (a >> 2) + (a & 3))) & 1u) << 31;
                gs[a] += __uint_as_float(__float_as_uint(acc[f][g][a]) ^ sgn);
            }
        }
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            float x = gs[a];
#pragma unroll
            for (int d = 1; d < 32; d <<= 1) x += __shfl_xor(x, d, 64);
            gs[a] = x;
        }
        if (r == 0) {
#pragma unroll
            for (int a = 0; a < 16; ++a) gpart[ib * m_pad + j0 + acc_row(a, h)] = gs[a];
        }
    }
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_bwd_f32_kernel(
    const uint64_t *__restrict__ ctbits, const float *__restrict__ s32,
    const uint64_t *__restrict__ bbits, int64_t lw, int64_t mw, int64_t n_jb, int64_t units,
    float *__restrict__ gpart, int64_t m_pad) {
    const int lane = threadIdx.x & 63;
    const int64_t u = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave_id();
    if (u >= units) return;
    const int64_t ib = u / n_jb, jb = u - ib * n_jb;
    const int h = lane >> 5, r = lane & 31;
    const int64_t KT2 = lw * 32;

    const uint64_t *cp[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) cp[f] = ctbits + (jb * FM + f) * lw * 32 + r;
    int64_t sp[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) sp[g] = (ib * FN + g) * KT2 * 64 + lane;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    for (int64_t w = 0; w < lw; ++w) {
        uint64_t cw[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) cw[f] = cp[f][w * 32] >> h;
#pragma unroll 8
        for (int t = 0; t < 32; ++t) {
            const int64_t kt = 32 * w + t;
            float bv[FN];
#pragma unroll
            for (int g = 0; g < FN; ++g) bv[g] = s32[sp[g] + kt * 64];
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                const float av = ((cw[f] >> (2 * t)) & 1ull) ? 1.0f : 0.0f;
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[g], acc[f][g], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const int64_t j0 = (jb * FM + f) * 32;
        const int64_t jw = j0 >> 6;
        const int jo = (int)(j0 & 63);
        float gs[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) gs[a] = 0.0f;
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const uint64_t bw = bbits[((ib * FN + g) * mw + jw) * 32 + r];
            const uint32_t b32 = (uint32_t)(bw >> jo) >> (4 * h);
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const uint32_t sgn = ((b32 >> (8 * (a >> 2) + (a & 3))) & 1u) << 31;
                gs[a] += __uint_as_float(__float_as_uint(acc[f][g][a]) ^ sgn);
            }
        }
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            float x = gs[a];
#pragma unroll
            for (int d = 1; d < 32; d <<= 1) x += __shfl_xor(x, d, 64);
            gs[a] = x;
        }
        if (r == 0) {
#pragma unroll
            for (int a = 0; a < 16; ++a) gpart[ib * m_pad + j0 + acc_row(a, h)] = gs[a];
        }
    }
}

template <int FM, int FN>
static void bwd_dispatch(const LaunchCtx &lc, int prec, const uint64_t *ctbits,
                         const uint16_t *shi, const uint16_t *slo, const float *s32,
                         const uint64_t *bbits, int64_t m_pad, int64_t l_pad, int64_t s_pad,
                         float *gpart) {
    const int64_t lw = l_pad / 64, mw = m_pad / 64;
    const int64_t n_jb = m_pad / (32 * FM), n_ib = s_pad / (32 * FN);
    const int64_t units = n_jb * n_ib;
    dim3 grid((unsigned)ceil_div(units, 4));
    if (prec == 1)
        hipLaunchKernelGGL((phase_bwd_bf16_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, ctbits,
                           reinterpret_cast<const u32x4 *>(shi),
                           reinterpret_cast<const u32x4 *>(slo), bbits, lw, mw, n_jb, units,
                           gpart, m_pad);
    else
        hipLaunchKernelGGL((phase_bwd_f32_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, ctbits,
                           s32, bbits, lw, mw, n_jb, units, gpart, m_pad);
}

hipError_t launch_phase_bwd(const LaunchCtx &lc, int prec, int fm, int fn, const uint64_t *ctbits,
                            const uint16_t *shi, const uint16_t *slo, const float *s32,
                            const uint64_t *bbits, int64_t m_pad, int64_t l_pad, int64_t s_pad,
                            float *gpart) {
    hipEvent_t ev;
    timed_begin(lc, KF_BWD, &ev);
    if (fm == 4 && fn == 4)
        bwd_dispatch<4, 4>(lc, prec, ctbits, shi, slo, s32, bbits, m_pad, l_pad, s_pad, gpart);
    else if (fm == 2 && fn == 2)
        bwd_dispatch<2, 2>(lc, prec, ctbits, shi, slo, s32, bbits, m_pad, l_pad, s_pad, gpart);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_BWD, ev);
    return e;
}

__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *__restrict__ gpart,
                                                          int64_t n_parts, int64_t m,
                                                          int64_t m_pad,
                                                          double *__restrict__ grad) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= m) return;
    double acc = 0.0;
    for (int64_t p = 0; p < n_parts; ++p) acc += (double)gpart[p * m_pad + j];
    grad[j] = -2.0 * acc;
}

hipError_t launch_grad_reduce(const LaunchCtx &lc, const float *gpart, int64_t n_parts,
                              int64_t m, int64_t m_pad, double *grad) {
    hipEvent_t ev;
    timed_begin(lc, KF_GRAD, &ev);
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0,
                       lc.stream, gpart, n_parts, m, m_pad, grad);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_GRAD, ev);
    return e;
}

// ---------------------------------------------------------------------------
// MMD^2 chain. data_stats: from row-major parity bits (rows = observables,
// bits over the N training strings) pstat[2k] = sum_n (-1)^{a_k . x_n} and
// pstat[2k+1] = p_k = that sum / N.
__global__ __launch_bounds__(256) void data_stats_kernel(const uint64_t *__restrict__ dbits,
                                                         int64_t l, int64_t Nw, int64_t N,
                                                         double *__restrict__ pstat) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= l) return;
    int64_t odd = 0;
    for (int64_t w = 0; w < Nw; ++w) odd += __popcll(dbits[k * Nw + w]);
    const double sv = (double)(N - 2 * odd);
    pstat[2 * k] = sv;
    pstat[2 * k + 1] = sv / (double)N;
}

hipError_t launch_data_stats(const LaunchCtx &lc, const uint64_t *dbits, int64_t l, int64_t Nw,
                             int64_t N, double *pstat) {
    hipEvent_t ev;
    timed_begin(lc, KF_MMD, &ev);
    hipLaunchKernelGGL(data_stats_kernel, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0,
                       lc.stream, dbits, l, Nw, N, pstat);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_MMD, ev);
    return e;
}

__global__ __launch_bounds__(256) void mmd_loss_kernel(const double *__restrict__ pstat,
                                                       const double *__restrict__ rowsum,
                                                       const double *__restrict__ w, int64_t l,
                                                       int64_t s, int64_t N, int unbiased,
                                                       double *__restrict__ loss) {
    __shared__ double sh[256];
    const double S = (double)s, Nd = (double)N;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < l; k += 256) {
        const double sv = pstat[2 * k], p = pstat[2 * k + 1];
        const double sc = rowsum[2 * k], sc2 = rowsum[2 * k + 1];
        const double q = sc / S;
        double term;
        if (unbiased) {
            const double P2 = (sv * sv - Nd) / (Nd * (Nd - 1.0));
            const double Q2 = (sc * sc - sc2) / (S * (S - 1.0));
            term = P2 - 2.0 * p * q + Q2;
        } else {
            term = (p - q) * (p - q);
        }
        acc += w[k] * term;
    }
    acc = block_sum_256(acc, sh);
    if (threadIdx.x == 0) loss[0] = acc;
}

hipError_t launch_mmd_loss(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int64_t N, int unbiased,
                           double *loss) {
    hipEvent_t ev;
    timed_begin(lc, KF_MMD, &ev);
    hipLaunchKernelGGL(mmd_loss_kernel, dim3(1), dim3(256), 0, lc.stream, pstat, rowsum,
                       op_weight, l, s, N, unbiased, loss);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_MMD, ev);
    return e;
}

// dL/dc_ki: unbiased w_k [-2 p_k / s + 2 (sum_i' c_ki' - c_ki) / (s (s-1))],
// plug-in w_k 2 (q_k - p_k) / s; written as alpha_k + beta_k c_ki.
__global__ __launch_bounds__(256) void coef_mmd_kernel(const double *__restrict__ pstat,
                                                       const double *__restrict__ rowsum,
                                                       const double *__restrict__ w, int64_t l,
                                                       int64_t s, int unbiased,
                                                       double *__restrict__ coef) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= l) return;
    const double S = (double)s;
    const double p = pstat[2 * k + 1], sc = rowsum[2 * k];
    if (unbiased) {
        const double d = S * (S - 1.0);
        coef[2 * k] = w[k] * (-2.0 * p / S + 2.0 * sc / d);
        coef[2 * k + 1] = -2.0 * w[k] / d;
    } else {
        coef[2 * k] = w[k] * 2.0 * (sc / S - p) / S;
        coef[2 * k + 1] = 0.0;
    }
}

hipError_t launch_coef_mmd(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int unbiased,
                           double *coef) {
    hipEvent_t ev;
    timed_begin(lc, KF_MMD, &ev);
    hipLaunchKernelGGL(coef_mmd_kernel, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0,
                       lc.stream, pstat, rowsum, op_weight, l, s, unbiased, coef);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_MMD, ev);
    return e;
}

}  // namespace iqp
