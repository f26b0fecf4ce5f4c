// gfx950 kernels of the IQP Monte Carlo expectation-value path.
//
//   theta_prep      theta -> 2 theta' (theta' = theta reduced to [-pi/2, pi/2]
//                   by whole multiples of pi), as FP32 or two / three BF16
//                   limbs
//   bitslice,       bit-exact popcount(row AND col) mod 2 matrices (the
//   parity_bs       exponents of B and C, Sec. 2.2) as XORs of per-qubit bit
//                   columns, with in-register 64x64 bit transposes
//   phase_fwd       E = C Theta B^T (eq. Emat) on the matrix cores, operands
//                   expanded from parity bits in registers
//   epilogue        FP64 reduction of E modulo 2 pi, cos, per-chunk sums of
//                   cos and cos^2 (eq. expvalsample)
//   finalize        mean and standard error per observable, fixed order
//   weights         S_ki = (alpha_k + beta_k cos E_ki) sin E_ki, written in
//                   the register image of the backward matrix-core operand
//   phase_bwd       T[k][j] = sum_i S_ki (-1)^{b_ij} on the matrix cores
//                   (K = samples), epilogue sum_k c_kj T[k][j] per gate
//   grad_reduce     dtheta_j = -2 sum over observable tiles, fixed order
//
// Every step is a body function over one problem and one block (or work
// unit). A plain launch runs one problem; a batched launch runs many problems
// of uneven size in one grid, and the two contractions also come as
// persistent kernels that take work units from a queue.
//   data_stats, mmd_loss, coef_*: the MMD^2 chain (eq. mmd_estimate)
//
// No float atomics anywhere: every reduction runs in a fixed order, so a call
// is bitwise reproducible.
#include "iqp_device.h"

#include <math.h>
#include <type_traits>

namespace iqp {

// OCP FP8 E4M3 (bias 7, 3 mantissa bits, no infinities) of a float, rounded
// to nearest even; |y| must be below 464 (the first value that would round
// past 448). Non-finite input gives the NaN code.
__device__ __forceinline__ uint32_t f32_to_e4m3(float y) {
    const uint32_t u = __float_as_uint(y);
    const uint32_t sgn = (u >> 24) & 0x80u;
    const uint32_t a = u & 0x7FFFFFFFu;
    if (a >= 0x7F800000u) return sgn | 0x7Fu;
    if (a < 0x3C800000u)  // below 2^-6: the subnormal grid of step 2^-9 (8 = 2^-6)
        return sgn | (uint32_t)rintf(__uint_as_float(a) * 512.0f);
    // keep 3 of the 23 mantissa bits, ties to even on the 20 dropped ones; a
    // carry moves into the exponent; rebias 127 -> 7
    const uint32_t r = a + 0x7FFFFu + ((a >> 20) & 1u);
    return sgn | ((r >> 20) - (120u << 3));
}

// ---------------------------------------------------------------------------
// theta_prep
__device__ __forceinline__ void theta_prep_body(const ThetaArgs &a, int64_t blk) {
    const int64_t i = blk * 256 + threadIdx.x;
    if (i >= a.m_pad) return;
    const double t = i < a.m ? gptr(a.theta)[i] : 0.0;
    const double tr = t - IQP_PI * rint(t * IQP_INV_PI);
    const double two = 2.0 * tr;
    if (a.prec == 2) {
        gptr(a.t32)[i] = (float)two;  // plain, for the sparse contraction
    } else if (a.prec == 1 || a.prec == 3 || a.prec == 4) {
        // each limb is the BF16 rounding of what the previous ones leave
        const uint16_t h = f2bf_rne((float)two);
        const double rem = two - (double)bf2f(h);
        const uint16_t l = f2bf_rne((float)rem);
        gptr(a.hi)[i] = h;
        if (a.prec != 3) {
            gptr(a.lo)[i] = l;
        } else {
            // third limb: E4M3 of the rest times 2^kLo8Exp (|rest| <= 2^-16 pi,
            // so below 2^kLo8Exp * 4.8e-5 ~ 50), the product scaled back by
            // 2^-kLo8Exp; one byte per gate, stored per 64-gate word in the
            // order the forward's lanes read it: byte 32 h + 8 t + e holds
            // gate 16 t + 8 h + e of the word
            gptr(a.mid)[i] = l;
            const double rest = rem - (double)bf2f(l);
            const int64_t gw = i & 63;
            const int64_t dst = (i - gw) + ((gw >> 3) & 1) * 32 + (gw >> 4) * 8 + (gw & 7);
            reinterpret_cast<uint8_t IQP_GLOBAL *>(gptr(a.lo))[dst] =
                (uint8_t)f32_to_e4m3((float)ldexp(rest, kLo8Exp));
        }
    } else {
        // split by gate parity: lane half h of the 32x32x2 product reads gate 2t + h
        gptr(a.t32)[(i & 1) * (a.m_pad >> 1) + (i >> 1)] = (float)two;
    }
}

hipError_t launch_theta_prep(const LaunchCtx &lc, const ThetaArgs &a) {
    return plain_launch<ThetaArgs, theta_prep_body>(lc, KF_THETA, a, blocks_of(a));
}

// ---------------------------------------------------------------------------
// Parity bits, bit-sliced. parity(x, g) = XOR over the qubits q of g of x_q,
// so with the rows transposed into per-qubit bit columns Xt[q] (bit r = qubit
// q of row r), the parities of one generator g against 64 rows are the XOR of
// |g| words. Cost grows with the weight of g (1..4 in the circuits of the
// paper), not with n.
//
// Xt[q * ldx + rw]: bit r = qubit q of row 64 rw + r (rows >= R read as 0),
// for q < 64 W and rw < ldx; row q = 64 W is all zero (the parity kernel
// reads it for absent support entries).
__device__ __forceinline__ void bitslice_body(const BitsliceArgs &a, int64_t blk) {
    const int lane = threadIdx.x & 63;
    const int64_t unit = blk * 4 + wave_id();
    if (unit >= a.ldx * a.W) return;
    const int64_t w = unit / a.ldx, rw = unit - w * a.ldx;
    const int64_t r = rw * 64 + lane;
    const uint64_t x = r < a.R ? gptr(a.rows)[r * a.W + w] : 0ull;
    gptr(a.Xt)[(w * 64 + lane) * a.ldx + rw] = transpose64(x, lane);
    if (unit == 0)
        for (int64_t c = lane; c < a.ldx; c += 64) gptr(a.Xt)[(int64_t)64 * a.W * a.ldx + c] = 0ull;
}

// Support lists, one lane per generator: the bit row is read once here, so
// the parity kernel touches only the listed qubits.
__device__ __forceinline__ void support_body(const SupportArgs &a, int64_t blk) {
    const int64_t j = blk * 256 + threadIdx.x;
    if (j >= a.rows) return;
    int32_t s[kSupCap];
#pragma unroll
    for (int k = 0; k < kSupCap; ++k) s[k] = -1;
    int cnt = 0;
    if (j < a.m) {
        for (int w = 0; w < a.W; ++w) {
            uint64_t x = gptr(a.gens)[j * a.W + w];
            while (x) {
                const int32_t q = w * 64 + __builtin_ctzll(x);
                x &= x - 1;
#pragma unroll
                for (int k = 0; k < kSupCap; ++k) s[k] = (cnt == k) ? q : s[k];
                ++cnt;
            }
        }
    }
    if (cnt > kSupCap) {
#pragma unroll
        for (int k = 0; k < kSupCap; ++k) s[k] = -1;
        s[0] = -2;
    }
    i32x4 IQP_GLOBAL *dst = reinterpret_cast<i32x4 IQP_GLOBAL *>(gptr(a.sup) + j * kSupCap);
    dst[0] = (i32x4){s[0], s[1], s[2], s[3]};
    dst[1] = (i32x4){s[4], s[5], s[6], s[7]};
}

// 64x64 bit transpose inside one lane: x[g] bit r -> x[r] bit g. At block
// size k, rows i and i + k (i & k == 0) swap the off-diagonal k x k blocks of
// their 2k x 2k block (mask m keeps the columns with bit k clear).
__device__ __forceinline__ void transpose64_regs(uint64_t (&x)[64]) {
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int k = 32 >> st;
        const uint64_t m = st == 0 ? 0x00000000FFFFFFFFull
                         : st == 1 ? 0x0000FFFF0000FFFFull
                         : st == 2 ? 0x00FF00FF00FF00FFull
                         : st == 3 ? 0x0F0F0F0F0F0F0F0Full
                         : st == 4 ? 0x3333333333333333ull
                                   : 0x5555555555555555ull;
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            if (i & k) continue;
            const uint64_t t = ((x[i] >> k) ^ x[i + k]) & m;
            x[i + k] ^= t;
            x[i] ^= t << k;
        }
    }
}

// One wave: 64 generators x 64 row words (lane rw). For generator j the
// parities against 64 rows are the XOR of the bit-column words
// Xt[q * ldx + rw] over q in supp(j): one coalesced 512-byte load per support
// qubit. The wave reads its 64 support lists once (lane g holds generator
// g's), and runs k-outer over the block's largest weight: entry k of every
// generator is moved to a scalar register and its 64 loads are independent,
// with absent entries reading the zero column. Generators heavier than the
// list walk their bit row afterwards.
//   LAYOUT 0: row-major    out[r * Gw + j/64], bit j%64
//   LAYOUT 1: tiled32      out[((r/32) * Gw + j/64) * 32 + r%32], bit j%64
//   LAYOUT 2: transposed tiled32 (rows = generators)
//             out[((j/32) * Rw + r/64) * 32 + j%32], bit r%64
//   LAYOUT 3: transposed row-major (rows = generators) out[j * Rw + r/64], bit r%64
// Layouts 0 and 1 transpose the lane's 64 x 64 block in registers; layouts 2
// and 3 store the XOR words as they are. Generators j >= m give zero bits.
template <int LAYOUT>
__device__ __forceinline__ void parity_bs_body(const ParityArgs &a, int64_t blk) {
    const uint64_t IQP_GLOBAL *__restrict__ Xt = gptr(a.Xt);
    uint64_t IQP_GLOBAL *__restrict__ out = gptr(a.out);
    const int64_t Rw = a.Rw, ldx = a.ldx, R_out = a.R_out, Gw = a.Gw;
    const int lane = threadIdx.x & 63;
    const int64_t unit = blk * 4 + wave_id();
    if (unit >= Gw * ceil_div(Rw, 64)) return;  // uniform over the wave
    const int64_t rc = unit / Gw, gb = unit - rc * Gw;
    const int64_t rw = rc * 64 + lane;
    const bool live = rw < Rw;
    const uint64_t IQP_GLOBAL *__restrict__ xcol = Xt + (live ? rw : 0);
    const int32_t zrow = 64 * a.W;

    const i32x4 IQP_GLOBAL *sp =
        reinterpret_cast<const i32x4 IQP_GLOBAL *>(gptr(a.sup) + (gb * 64 + lane) * kSupCap);
    const i32x4 s0 = sp[0], s1 = sp[1];
    const int32_t sv[kSupCap] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
    const uint64_t heavy = __ballot(sv[0] == -2);
    int32_t qv[kSupCap];
    int kmax = 0;
#pragma unroll
    for (int k = 0; k < kSupCap; ++k) {
        qv[k] = sv[k] >= 0 ? sv[k] : zrow;
        kmax += __ballot(sv[k] >= 0) != 0ull;  // lists fill from entry 0
    }
    uint64_t x[64];
#pragma unroll
    for (int g = 0; g < 64; ++g) x[g] = 0ull;
#pragma unroll
    for (int k = 0; k < kSupCap; ++k) {
        if (k >= kmax) break;
#pragma unroll
        for (int g = 0; g < 64; ++g) {
            const int32_t q = __builtin_amdgcn_readlane(qv[k], g);
            x[g] ^= xcol[(int64_t)q * ldx];
        }
    }
    if (heavy) {
#pragma unroll
        for (int g = 0; g < 64; ++g) {
            if (!((heavy >> g) & 1ull)) continue;
            const uint64_t IQP_GLOBAL *row = gptr(a.gens) + (gb * 64 + g) * a.W;
            for (int w = 0; w < a.W; ++w) {
                uint64_t bits = row[w];
                while (bits) {
                    const int64_t q = (int64_t)w * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1;
                    x[g] ^= xcol[q * ldx];
                }
            }
        }
    }
    if (!live) return;
    if (LAYOUT == 3) {
#pragma unroll
        for (int g = 0; g < 64; ++g) out[(gb * 64 + g) * Rw + rw] = x[g];
    } else if (LAYOUT == 2) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            uint64_t IQP_GLOBAL *dst = out + ((gb * 2 + hh) * Rw + rw) * 32;
#pragma unroll
            for (int g = 0; g < 32; g += 2)
                *reinterpret_cast<u64x2 IQP_GLOBAL *>(dst + g) = (u64x2){x[32 * hh + g], x[32 * hh + g + 1]};
        }
    } else {
        transpose64_regs(x);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int64_t r0 = rw * 64 + 32 * hh;
            if (r0 >= R_out) break;  // R_out is a multiple of 32 in layout 1
            if (LAYOUT == 1) {
                uint64_t IQP_GLOBAL *dst = out + ((r0 >> 5) * Gw + gb) * 32;
#pragma unroll
                for (int b = 0; b < 32; b += 2)
                    *reinterpret_cast<u64x2 IQP_GLOBAL *>(dst + b) = (u64x2){x[32 * hh + b], x[32 * hh + b + 1]};
            } else {
#pragma unroll
                for (int b = 0; b < 32; ++b)
                    if (r0 + b < R_out) out[(r0 + b) * Gw + gb] = x[32 * hh + b];
            }
        }
    }
}

hipError_t launch_bitslice(const LaunchCtx &lc, const BitsliceArgs &a) {
    return plain_launch<BitsliceArgs, bitslice_body>(lc, KF_PARITY, a, blocks_of(a));
}

hipError_t launch_support(const LaunchCtx &lc, const SupportArgs &a) {
    return plain_launch<SupportArgs, support_body>(lc, KF_PARITY, a, blocks_of(a));
}

hipError_t launch_parity_bs(const LaunchCtx &lc, int layout, const ParityArgs &a) {
    const int64_t nb = blocks_of(a);
    if (layout == 0) return plain_launch<ParityArgs, parity_bs_body<0>>(lc, KF_PARITY, a, nb);
    if (layout == 1) return plain_launch<ParityArgs, parity_bs_body<1>>(lc, KF_PARITY, a, nb);
    if (layout == 2) return plain_launch<ParityArgs, parity_bs_body<2>>(lc, KF_PARITY, a, nb);
    if (layout == 3) return plain_launch<ParityArgs, parity_bs_body<3>>(lc, KF_PARITY, a, nb);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Operand expansion from parity bits, in registers.
//
// A 32x32x16 BF16 product reads, in lane l, 8 consecutive K values
// 8*(l/32) + e, e = 0..7, packed two per dword (element 2v in the low half of
// dword v). `x` carries the lane's 8 parity bits in bits 0..7 of a 16-bit
// value (bits 8..15 are ignored). A packed 16-bit shift by (15 - 2v, 14 - 2v)
// moves bits 2v and 2v+1 to the sign positions 15 and 31 of dword v.

// B_ij = (-1)^{bit}: +1.0 = 0x3F80, -1.0 = 0xBF80. `ones` holds 0x3F803F80 in
// a vector register so that mask-and-or is one instruction.
__device__ __forceinline__ bf16x8 expand_pm1(uint32_t x16, uint32_t ones) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh = {(unsigned short)(15 - 2 * v), (unsigned short)(14 - 2 * v)};
        d[v] = (__builtin_bit_cast(uint32_t, (u16x2)(xv << sh)) & 0x80008000u) | ones;
    }
    return __builtin_bit_cast(bf16x8, d);
}

// C_kj theta_j / 2 = bit ? 2 theta'_j : 0 for each of the NL limbs; the sign
// bit is spread over its half by an arithmetic shift to make the mask.
template <int NL>
__device__ __forceinline__ void expand_masked(uint32_t x16, const u32x4 (&th)[NL],
                                              bf16x8 (&out)[NL]) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t d[NL][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh = {(unsigned short)(15 - 2 * v), (unsigned short)(14 - 2 * v)};
        const s16x2 sg = __builtin_bit_cast(s16x2, (u16x2)(xv << sh)) >> (s16x2){15, 15};
        const uint32_t msk = __builtin_bit_cast(uint32_t, sg);
#pragma unroll
        for (int L = 0; L < NL; ++L) d[L][v] = th[L][v] & msk;
    }
#pragma unroll
    for (int L = 0; L < NL; ++L) out[L] = __builtin_bit_cast(bf16x8, d[L]);
}

// The same with an FP8 third limb (IQP_SPLIT3_BF16): the two 16-bit-lane masks
// of gates (2v, 2v+1) and (2v+2, 2v+3) give, by one byte permute (their low
// bytes), the byte mask of those four gates, applied to the limb's bytes l8
// (dword u: gates 4u .. 4u+3 of the K-step).
template <int NL>
__device__ __forceinline__ void expand_masked_f8(uint32_t x16, const u32x4 (&th)[NL],
                                                 bf16x8 (&out)[NL], uint32_t l0, uint32_t l1,
                                                 uint32_t &a0, uint32_t &a1) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t d[NL][4], msk[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh = {(unsigned short)(15 - 2 * v), (unsigned short)(14 - 2 * v)};
        const s16x2 sg = __builtin_bit_cast(s16x2, (u16x2)(xv << sh)) >> (s16x2){15, 15};
        msk[v] = __builtin_bit_cast(uint32_t, sg);
#pragma unroll
        for (int L = 0; L < NL; ++L) d[L][v] = th[L][v] & msk[v];
    }
#pragma unroll
    for (int L = 0; L < NL; ++L) out[L] = __builtin_bit_cast(bf16x8, d[L]);
    a0 = __builtin_amdgcn_perm(msk[1], msk[0], 0x06040200u) & l0;
    a1 = __builtin_amdgcn_perm(msk[3], msk[2], 0x06040200u) & l1;
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

// Direct global -> LDS copy of 16 bytes per lane: lane l's bytes land at
// lds_block + 16 l. Completion is tracked by the vector-memory counter.
typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ void dma16(const void IQP_GLOBAL *gsrc, void *lds_block) {
    __builtin_amdgcn_global_load_lds(gsrc, (lds_void *)lds_block, 16, 0, 0);
}

// Wait for this wave's outstanding vector-memory operations (including the
// global -> LDS copies above), then synchronise the workgroup.
// (The builtin, unlike inline assembly, is visible to the compiler's own
// wait-count tracking, so it does not wait again for loads this covered.)
__device__ __forceinline__ void dma_wait_barrier() {
    // vmcnt(0), expcnt and lgkmcnt left at their maxima (gfx9 encoding)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
}

// A value the compiler must keep in a vector register.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// The 16 accumulators of a 32x32 product in lane l hold column l % 32 and
// rows 8*(a/4) + 4*(l/32) + (a%4), a = 0..15.
__device__ __forceinline__ int acc_row(int a, int h) { return 8 * (a >> 2) + 4 * h + (a & 3); }

// ---------------------------------------------------------------------------
// phase_fwd: E[k][i] = sum_j (c_kj * 2 theta'_j) * (-1)^{b_ij}.
// A workgroup is 4 waves that share a gate range (split) and an observable
// block and take 4 consecutive sample blocks; each wave computes a
// (32 FM) x (32 FN) tile. C and B parity bits are tiled32, so each 32-row
// fragment of a 64-gate word is 256 contiguous bytes. Within a word, K-step t
// (16 gates) uses byte 2t + h of the lane's word (h = lane / 32): the word is
// pre-shifted right by 8h.
//
// Memory discipline: the theta limbs, shared by the 4 waves, are staged
// through LDS in chunks of kChunkWords gate words (double-buffered, one
// barrier per chunk), so the only vector loads in the loop are the bit words
// of word w+1, requested at the start of word w and consumed in issue order;
// no wait on a later load ever covers them early.
constexpr int kChunkWords = 32;

// Interleave of one half-region of the pipeline: optional LDS reads for the
// next K-step first, then each matrix product followed by a few of the next
// K-step's expansion instructions, so the matrix core never waits for a run
// of VALU. A region issues the hi-limb products of all accumulators in one
// half and the lo-limb products in the other, fenced, so two products into
// the same accumulator are always a full pass apart.
template <int NDS, int NMFMA, int NVALU>
__device__ __forceinline__ void interleave_half() {
    if (NDS > 0) __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);  // LDS reads
#pragma unroll
    for (int i = 0; i < NMFMA; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix product
        if (NVALU > 0)
            __builtin_amdgcn_sched_group_barrier(0x002, (NVALU + NMFMA - 1) / NMFMA, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Operands of one K-step: the +-1 B fragments and the masked theta limb A
// fragments (limb 0 = hi, limb 1 = lo, or mid when an FP8 limb follows).
template <int FM, int FN, int NL>
struct FwdOps {
    bf16x8 bv[FN], a[NL][FM];
};

// Third theta limb in FP8 (IQP_SPLIT3_BF16): per 64-gate word one 32x32x64
// FP8 product per block, A = the limb's bytes masked by C, B = +-1.0 in
// E4M3, both built per K-step from the BF16 operands (two dwords, 8 gates,
// per K-step and row or column block): lane half h holds gates 16 t + 8 h +
// e of K-step t in bytes 8 t + e, the order the limb is stored in, so A and
// B pair the same gate in every lane and byte. l8: the word's limb bytes of
// the lane's half.
template <int FM, int FN>
struct F8Ops {
    uint32_t a[FM][8], b[FN][8], l8[8];
    uint32_t m80, c38;  // the E4M3 sign mask and +1.0, in vector registers
};
template <int FM, int FN, bool F8>
using F8State = typename std::conditional<F8, F8Ops<FM, FN>, char>::type;

template <int FM, int FN, int NL, int T, bool F8>
__device__ __forceinline__ void fwd_expand_b(FwdOps<FM, FN, NL> &o, const uint64_t (&bw)[FN],
                                             uint32_t ones, F8State<FM, FN, F8> &e8) {
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        const uint32_t d = (uint32_t)(bw[g] >> (32 * (T >> 1)));
        o.bv[g] = expand_pm1((T & 1) ? (d >> 16) : d, ones);
        if constexpr (F8) {
            // the high bytes of the +-1 BF16 pairs (0x3F / 0xBF) -> 0x38 / 0xB8
            const u32x4 q = __builtin_bit_cast(u32x4, o.bv[g]);
            e8.b[g][2 * T] = (__builtin_amdgcn_perm(q[1], q[0], 0x07050301u) & e8.m80) | e8.c38;
            e8.b[g][2 * T + 1] =
                (__builtin_amdgcn_perm(q[3], q[2], 0x07050301u) & e8.m80) | e8.c38;
        }
    }
}

template <int FM, int FN, int NL, int T, bool F8>
__device__ __forceinline__ void fwd_expand_a(FwdOps<FM, FN, NL> &o, const uint64_t (&cw)[FM],
                                             const u32x4 (&th)[NL], F8State<FM, FN, F8> &e8) {
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const uint32_t d = (uint32_t)(cw[f] >> (32 * (T >> 1)));
        bf16x8 x[NL];
        if constexpr (F8)
            expand_masked_f8<NL>((T & 1) ? (d >> 16) : d, th, x, e8.l8[2 * T], e8.l8[2 * T + 1],
                                 e8.a[f][2 * T], e8.a[f][2 * T + 1]);
        else
            expand_masked<NL>((T & 1) ? (d >> 16) : d, th, x);
#pragma unroll
        for (int L = 0; L < NL; ++L) o.a[L][f] = x[L];
    }
}

template <int FM, int FN, int NL, int T, bool F8>
__device__ __forceinline__ void fwd_expand(FwdOps<FM, FN, NL> &o, const uint64_t (&cw)[FM],
                                           const uint64_t (&bw)[FN], const u32x4 (&th)[NL],
                                           uint32_t ones, F8State<FM, FN, F8> &e8) {
    fwd_expand_b<FM, FN, NL, T, F8>(o, bw, ones, e8);
    fwd_expand_a<FM, FN, NL, T, F8>(o, cw, th, e8);
}

// the word's FP8 limb bytes of the lane's half (two 16-byte units)
template <int FM, int FN>
__device__ __forceinline__ void fwd_load_l8(F8Ops<FM, FN> &e8, const u32x4 *T8, int o8) {
    const u32x4 p0 = T8[o8], p1 = T8[o8 + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        e8.l8[i] = p0[i];
        e8.l8[4 + i] = p1[i];
    }
}

// the word's FP8 products, scaled by 2^-kLo8Exp
template <int FM, int FN>
__device__ __forceinline__ void fwd_mfma_f8(const F8Ops<FM, FN> &e8, f32x16 (&acc)[FM][FN]) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const i32x8 a = __builtin_bit_cast(i32x8, e8.a[f]);
            const i32x8 b = __builtin_bit_cast(i32x8, e8.b[g]);
            acc[f][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc[f][g], 0, 0, 0,
                                                                        127 - kLo8Exp, 0, 127);
        }
}

template <int FM, int FN, int NL, int LIMB>
__device__ __forceinline__ void fwd_mfma_limb(const FwdOps<FM, FN, NL> &o,
                                              f32x16 (&acc)[FM][FN]) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
            acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.a[LIMB][f], o.bv[g], acc[f][g],
                                                                0, 0, 0);
}

// The theta limbs of one K-step from LDS: limb L at Tp[L][off].
template <int NL>
__device__ __forceinline__ void fwd_theta(u32x4 (&th)[NL], const u32x4 *const (&Tp)[NL], int off) {
#pragma unroll
    for (int L = 0; L < NL; ++L) th[L] = Tp[L][off];
}

// One pipeline region: the products of K-step t (operands `cur`) while the
// operands of K-step T1 (theta limbs at offset `off`) are expanded into `nxt`.
// The products of each limb run as one pass over all accumulators, so two
// products into the same accumulator are always a full pass apart.
// With the FP8 third limb, region 0 (whose expansion starts the next word)
// first issues the finished word's FP8 products and reads the next word's
// limb bytes (at o8).
template <int FM, int FN, int NL, int T1, bool F8>
__device__ __forceinline__ void fwd_region(const FwdOps<FM, FN, NL> &cur, FwdOps<FM, FN, NL> &nxt,
                                           const uint64_t (&cw)[FM], const uint64_t (&bw)[FN],
                                           const u32x4 *const (&Tp)[NL], int off, uint32_t ones,
                                           f32x16 (&acc)[FM][FN], F8State<FM, FN, F8> &e8,
                                           const u32x4 *T8, int o8) {
    u32x4 th[NL];
    fwd_theta<NL>(th, Tp, off);
    if constexpr (F8) {
        if constexpr (T1 == 0) {
            fwd_mfma_f8<FM, FN>(e8, acc);
            fwd_load_l8<FM, FN>(e8, T8, o8);
        }
    }
    fwd_expand_b<FM, FN, NL, T1, F8>(nxt, bw, ones, e8);
    fwd_mfma_limb<FM, FN, NL, 0>(cur, acc);
    constexpr int kF8M = (F8 && T1 == 0) ? FM * FN : 0;
    constexpr int kF8V = F8 ? 4 * FN : 0;
    interleave_half<NL + (F8 && T1 == 0 ? 2 : 0), FM * FN + kF8M, 8 * FN + 4 + kF8V>();
    fwd_expand_a<FM, FN, NL, T1, F8>(nxt, cw, th, e8);
    fwd_mfma_limb<FM, FN, NL, 1>(cur, acc);
    interleave_half<0, FM * FN, 16 * FM + 4 + (F8 ? 4 * FM : 0)>();
}

// Decomposition shared by both forward kernels.
struct FwdUnit {
    int64_t sb, ob, split, w0, w1;
    bool active;
};

__device__ __forceinline__ bool fwd_unit(FwdUnit &U, int64_t gu, int64_t n_ob, int64_t n_sb,
                                         int64_t mw, int64_t wps) {
    const int64_t n_sbg = ceil_div(n_sb, 4);
    const int64_t sbg = gu % n_sbg;
    const int64_t t0 = gu / n_sbg;
    U.ob = t0 % n_ob;
    U.split = t0 / n_ob;
    U.sb = sbg * 4 + wave_id();
    U.active = U.sb < n_sb;
    U.w0 = U.split * wps;
    U.w1 = (U.w0 + wps < mw) ? U.w0 + wps : mw;
    return true;
}

template <int FM, int FN>
__device__ __forceinline__ void store_tile(const f32x16 (&acc)[FM][FN], float IQP_GLOBAL *Ep, int64_t ob,
                                           int64_t sb, int64_t s_pad, int h, int r) {
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

// NL = 2: IQP_SPLIT_BF16 and IQP_SPLIT_BF16_FP8 (hi, lo), or IQP_SPLIT3_BF16
// with F8 (hi, mid in BF16; the third limb in FP8).
template <int FM, int FN, int NL, bool F8>
__device__ __forceinline__ void fwd_bf16_body(const FwdArgs &a, int64_t gu, int tid) {
    // per word 8 units of 16 bytes per limb: K-step t, half h at 2t + h; the
    // FP8 limb 4 units per word: half h at 2h, 2h + 1
    __shared__ u32x4 lt[NL][2][kChunkWords * 8];
    __shared__ u32x4 lt8[F8 ? 2 : 1][F8 ? kChunkWords * 4 : 1];
    const uint64_t IQP_GLOBAL *__restrict__ cbits = gptr(a.cbits);
    const uint64_t IQP_GLOBAL *__restrict__ bbits = gptr(a.bbits);
    const u32x4 IQP_GLOBAL *thp[NL];
    static_assert(NL == 2, "two BF16 limbs, the second lo or (with F8) mid");
    thp[0] = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.thh));
    thp[1] = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(F8 ? a.thm : a.thl));
    const u32x4 IQP_GLOBAL *th8 = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.thl));
    float IQP_GLOBAL *__restrict__ E = gptr(a.E);
    const int64_t l_pad = a.l_pad, s_pad = a.s_pad, mw = a.m_pad / 64;
    const int64_t n_ob = l_pad / (32 * FM), n_sb = s_pad / (32 * FN);
    const int64_t wps = ceil_div(mw, a.splits);
    FwdUnit U;
    fwd_unit(U, gu, n_ob, n_sb, mw, wps);
    const int lane = tid & 63;
    const int h = lane >> 5, r = lane & 31;
    const uint32_t ones = in_vgpr(0x3F803F80u);
    const uint64_t IQP_GLOBAL *cbase = cbits + U.ob * FM * mw * 32;
    const uint64_t IQP_GLOBAL *bbase = bbits + (U.active ? U.sb : 0) * FN * mw * 32;
    const int64_t nwords = U.w1 > U.w0 ? U.w1 - U.w0 : 0;
    const int64_t nchunks = ceil_div(nwords, kChunkWords);

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    // stage a chunk: wave v copies units [64 v, 64 v + 64) of every limb
    const int wv = wave_id();
    auto stage = [&](int64_t cw0, int buf) {
        const int64_t src = cw0 * 8 + wv * 64 + lane;
        if (src < U.w1 * 8) {
#pragma unroll
            for (int L = 0; L < NL; ++L) dma16(thp[L] + src, &lt[L][buf][wv * 64]);
        }
        if constexpr (F8) {
            // the FP8 limb: wave v copies units [32 v, 32 v + 32) with lanes 0..31
            const int64_t s8 = cw0 * 4 + wv * 32 + lane;
            if (lane < 32 && s8 < U.w1 * 4) dma16(th8 + s8, &lt8[buf][wv * 32]);
        }
    };
    if (nchunks > 0) stage(U.w0, 0);
    uint64_t nxt_c[FM], nxt_b[FN], cur_c[FM], cur_b[FN];
    if (nwords > 0) {
#pragma unroll
        for (int f = 0; f < FM; ++f) nxt_c[f] = (cbase + (f * mw + U.w0) * 32)[r];
#pragma unroll
        for (int g = 0; g < FN; ++g) nxt_b[g] = (bbase + (g * mw + U.w0) * 32)[r];
    }
    dma_wait_barrier();
    FwdOps<FM, FN, NL> opA, opB;
    F8State<FM, FN, F8> e8;
    if constexpr (F8) {
        e8.m80 = in_vgpr(0x80808080u);
        e8.c38 = in_vgpr(0x38383838u);
    }
    for (int64_t c = 0; c < nchunks; ++c) {
        const int buf = (int)(c & 1);
        const int64_t cw0 = U.w0 + c * kChunkWords;
        const int64_t cw1 = (cw0 + kChunkWords < U.w1) ? cw0 + kChunkWords : U.w1;
        if (c + 1 < nchunks) stage(cw1, buf ^ 1);
        const u32x4 *Tp[NL];
#pragma unroll
        for (int L = 0; L < NL; ++L) Tp[L] = lt[L][buf] + h;
        const u32x4 *T8 = lt8[F8 ? buf : 0] + 2 * h;
        // K-step 0 of the chunk's first word (with the FP8 limb, the previous
        // chunk's last word has issued its FP8 products in its region 0)
#pragma unroll
        for (int f = 0; f < FM; ++f) cur_c[f] = nxt_c[f] >> (8 * h);
#pragma unroll
        for (int g = 0; g < FN; ++g) cur_b[g] = nxt_b[g] >> (8 * h);
        {
            u32x4 th[NL];
            fwd_theta<NL>(th, Tp, 0);
            if constexpr (F8) fwd_load_l8<FM, FN>(e8, T8, 0);
            fwd_expand<FM, FN, NL, 0, F8>(opA, cur_c, cur_b, th, ones, e8);
        }
        for (int64_t w = cw0; w < cw1; ++w) {
            const int o = (int)(w - cw0) * 8;
            if (w + 1 < U.w1) {
#pragma unroll
                for (int f = 0; f < FM; ++f) nxt_c[f] = (cbase + (f * mw + w + 1) * 32)[r];
#pragma unroll
                for (int g = 0; g < FN; ++g) nxt_b[g] = (bbase + (g * mw + w + 1) * 32)[r];
            }
            // region t: products of K-step t, expansion of K-step t+1
            fwd_region<FM, FN, NL, 1, F8>(opA, opB, cur_c, cur_b, Tp, o + 2, ones, acc, e8, T8, 0);
            fwd_region<FM, FN, NL, 2, F8>(opB, opA, cur_c, cur_b, Tp, o + 4, ones, acc, e8, T8, 0);
            fwd_region<FM, FN, NL, 3, F8>(opA, opB, cur_c, cur_b, Tp, o + 6, ones, acc, e8, T8, 0);
            // K-step 0 of word w+1, unconditionally so that it interleaves with
            // the products below: past the chunk's last word it reads inside
            // the chunk's buffer and is recomputed after the barrier
            const int on = (w + 1 < cw1) ? o + 8 : o;
#pragma unroll
            for (int f = 0; f < FM; ++f) cur_c[f] = nxt_c[f] >> (8 * h);
#pragma unroll
            for (int g = 0; g < FN; ++g) cur_b[g] = nxt_b[g] >> (8 * h);
            fwd_region<FM, FN, NL, 0, F8>(opB, opA, cur_c, cur_b, Tp, on, ones, acc, e8, T8,
                                          on / 2);
        }
        dma_wait_barrier();
    }
    if (U.active) store_tile<FM, FN>(acc, E + U.split * l_pad * s_pad, U.ob, U.sb, s_pad, h, r);
}

// FP32 form: 32x32x2 products, lane l reads K value l / 32. The word is
// pre-shifted right by h, so K-step t (gates 2t, 2t+1) uses bit 2t. theta is
// split by gate parity, t32[h][32 w + t] = 2 theta'_{64 w + 2 t + h}, and
// staged per word as 16 float4: half h at 8h + q holds K-steps 4q..4q+3.
template <int FM, int FN, int Q>
__device__ __forceinline__ void fwd32_group(const uint64_t (&cw)[FM], const uint64_t (&bw)[FN],
                                            const float4 &tv, f32x16 (&acc)[FM][FN]) {
    const float tq[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int t = 4 * Q + e;
        float bv[FN];
#pragma unroll
        for (int g = 0; g < FN; ++g)
            bv[g] = __uint_as_float((((uint32_t)(bw[g] >> (2 * t)) & 1u) << 31) | 0x3F800000u);
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

template <int FM, int FN>
__device__ __forceinline__ void fwd_f32_body(const FwdArgs &a, int64_t gu, int tid) {
    __shared__ float4 lt[2][kChunkWords * 16];
    const uint64_t IQP_GLOBAL *__restrict__ cbits = gptr(a.cbits);
    const uint64_t IQP_GLOBAL *__restrict__ bbits = gptr(a.bbits);
    const float IQP_GLOBAL *__restrict__ t32 = gptr(a.t32);
    float IQP_GLOBAL *__restrict__ E = gptr(a.E);
    const int64_t l_pad = a.l_pad, s_pad = a.s_pad, m_pad = a.m_pad, mw = m_pad / 64;
    const int64_t n_ob = l_pad / (32 * FM), n_sb = s_pad / (32 * FN);
    const int64_t wps = ceil_div(mw, a.splits);
    FwdUnit U;
    fwd_unit(U, gu, n_ob, n_sb, mw, wps);
    const int lane = tid & 63;
    const int h = lane >> 5, r = lane & 31;
    const float4 IQP_GLOBAL *tp4 = reinterpret_cast<const float4 IQP_GLOBAL *>(t32);
    const int64_t half4 = m_pad >> 3;  // float4 units per parity half
    const uint64_t IQP_GLOBAL *cbase = cbits + U.ob * FM * mw * 32;
    const uint64_t IQP_GLOBAL *bbase = bbits + (U.active ? U.sb : 0) * FN * mw * 32;
    const int64_t nwords = U.w1 > U.w0 ? U.w1 - U.w0 : 0;
    const int64_t nchunks = ceil_div(nwords, kChunkWords);

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    // staging unit u = 16 (word) + 8 hh + q  <-  t32 half hh, float4 8 w + q;
    // wave v copies units [64 (v + 4 k), +64) for k = 0, 1
    const int wv = wave_id();
    auto stage = [&](int64_t cw0, int buf) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int uidx = (wv + 4 * k) * 64 + lane;
            const int64_t w = cw0 + (uidx >> 4);
            const int hh = (uidx >> 3) & 1, q = uidx & 7;
            if (w < U.w1) dma16(tp4 + hh * half4 + 8 * w + q, &lt[buf][(wv + 4 * k) * 64]);
        }
    };
    if (nchunks > 0) stage(U.w0, 0);
    uint64_t nxt_c[FM], nxt_b[FN], cur_c[FM], cur_b[FN];
    if (nwords > 0) {
#pragma unroll
        for (int f = 0; f < FM; ++f) nxt_c[f] = (cbase + (f * mw + U.w0) * 32)[r];
#pragma unroll
        for (int g = 0; g < FN; ++g) nxt_b[g] = (bbase + (g * mw + U.w0) * 32)[r];
    }
    dma_wait_barrier();
    for (int64_t c = 0; c < nchunks; ++c) {
        const int buf = (int)(c & 1);
        const int64_t cw0 = U.w0 + c * kChunkWords;
        const int64_t cw1 = (cw0 + kChunkWords < U.w1) ? cw0 + kChunkWords : U.w1;
        if (c + 1 < nchunks) stage(cw1, buf ^ 1);
        for (int64_t w = cw0; w < cw1; ++w) {
#pragma unroll
            for (int f = 0; f < FM; ++f) cur_c[f] = nxt_c[f] >> h;
#pragma unroll
            for (int g = 0; g < FN; ++g) cur_b[g] = nxt_b[g] >> h;
            if (w + 1 < U.w1) {
#pragma unroll
                for (int f = 0; f < FM; ++f) nxt_c[f] = (cbase + (f * mw + w + 1) * 32)[r];
#pragma unroll
                for (int g = 0; g < FN; ++g) nxt_b[g] = (bbase + (g * mw + w + 1) * 32)[r];
            }
            {
                const float4 *tl = &lt[buf][(int)(w - cw0) * 16 + 8 * h];
                fwd32_group<FM, FN, 0>(cur_c, cur_b, tl[0], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 1>(cur_c, cur_b, tl[1], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 2>(cur_c, cur_b, tl[2], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 3>(cur_c, cur_b, tl[3], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 4>(cur_c, cur_b, tl[4], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 5>(cur_c, cur_b, tl[5], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 6>(cur_c, cur_b, tl[6], acc);
                __builtin_amdgcn_sched_barrier(0);
                fwd32_group<FM, FN, 7>(cur_c, cur_b, tl[7], acc);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        dma_wait_barrier();
    }
    if (U.active) store_tile<FM, FN>(acc, E + U.split * l_pad * s_pad, U.ob, U.sb, s_pad, h, r);
}

// Plain launch: one workgroup per unit, units spread over the XCDs in
// contiguous ranges. NL = number of theta limbs: 2 (BF16 hi, lo) or 3 (BF16
// hi, mid and the FP8 third limb).
template <int FM, int FN, int NL>
__global__ __launch_bounds__(256, 1) void phase_fwd_bf16_kernel(FwdArgs a, int64_t units) {
    const int64_t gu = xcd_remap(blockIdx.x, gridDim.x);
    if (gu >= units) return;  // uniform over the workgroup
    fwd_bf16_body<FM, FN, 2, NL == 3>(a, gu, (int)threadIdx.x);
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_fwd_f32_kernel(FwdArgs a, int64_t units) {
    const int64_t gu = xcd_remap(blockIdx.x, gridDim.x);
    if (gu >= units) return;
    fwd_f32_body<FM, FN>(a, gu, (int)threadIdx.x);
}

// Persistent launch over the units of a batch of problems.
template <int FM, int FN, int NL>
__global__ __launch_bounds__(256, 1) void phase_fwd_bf16_persistent(
    const FwdArgs *__restrict__ args, const int64_t *__restrict__ off, int np,
    unsigned long long *counter) {
    persistent_loop(off, np, counter,
                    [&](int p, int64_t u) {
                        fwd_bf16_body<FM, FN, 2, NL == 3>(args[p], u, opaque_tid());
                    });
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_fwd_f32_persistent(
    const FwdArgs *__restrict__ args, const int64_t *__restrict__ off, int np,
    unsigned long long *counter) {
    persistent_loop(off, np, counter, [&](int p, int64_t u) { fwd_f32_body<FM, FN>(args[p], u, opaque_tid()); });
}

template <int FM, int FN>
static hipError_t fwd_dispatch(const LaunchCtx &lc, int prec, const FwdArgs &a) {
    const int64_t units = fwd_units(a, FM, FN);
    if (units <= 0) return hipSuccess;
    if (units > kMaxBlocks) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)units);
    if (prec == 1 || prec == 4)
        hipLaunchKernelGGL((phase_fwd_bf16_kernel<FM, FN, 2>), grid, dim3(256), 0, lc.stream, a,
                           units);
    else if (prec == 3)
        hipLaunchKernelGGL((phase_fwd_bf16_kernel<FM, FN, 3>), grid, dim3(256), 0, lc.stream, a,
                           units);
    else
        hipLaunchKernelGGL((phase_fwd_f32_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, a, units);
    return hipGetLastError();
}

hipError_t launch_phase_fwd(const LaunchCtx &lc, int prec, int fm, int fn, const FwdArgs &a) {
    hipEvent_t ev;
    timed_begin(lc, KF_FWD, &ev);
    hipError_t e;
    if (fm == 4 && fn == 4) e = fwd_dispatch<4, 4>(lc, prec, a);
    else if (fm == 2 && fn == 2) e = fwd_dispatch<2, 2>(lc, prec, a);
    else if (fm == 2 && fn == 4) e = fwd_dispatch<2, 4>(lc, prec, a);
    else e = hipErrorInvalidValue;
    timed_end(lc, KF_FWD, ev);
    return e;
}

template <int FM, int FN>
static hipError_t fwd_persistent(const LaunchCtx &lc, int prec, const FwdArgs *args,
                                 const int64_t *off, int np, unsigned long long *counter,
                                 int grid) {
    if (prec == 1 || prec == 4)
        hipLaunchKernelGGL((phase_fwd_bf16_persistent<FM, FN, 2>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    else if (prec == 3)
        hipLaunchKernelGGL((phase_fwd_bf16_persistent<FM, FN, 3>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    else
        hipLaunchKernelGGL((phase_fwd_f32_persistent<FM, FN>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    return hipGetLastError();
}

hipError_t launch_phase_fwd_persistent(const LaunchCtx &lc, int prec, int fm, int fn,
                                       const FwdArgs *args, const int64_t *off, int np,
                                       unsigned long long *counter, int grid) {
    if (grid < 1 || np < 1) return hipErrorInvalidValue;
    hipEvent_t ev;
    timed_begin(lc, KF_FWD, &ev);
    hipError_t e;
    if (fm == 4 && fn == 4) e = fwd_persistent<4, 4>(lc, prec, args, off, np, counter, grid);
    else if (fm == 2 && fn == 2) e = fwd_persistent<2, 2>(lc, prec, args, off, np, counter, grid);
    else if (fm == 2 && fn == 4) e = fwd_persistent<2, 4>(lc, prec, args, off, np, counter, grid);
    else e = hipErrorInvalidValue;
    timed_end(lc, KF_FWD, ev);
    return e;
}

// ---------------------------------------------------------------------------
// epilogue: one block per (observable k, chunk of kEpiChunk samples).

__device__ __forceinline__ void epilogue_body(const EpiArgs &a, int64_t blk) {
    __shared__ double sh[256];
    const float IQP_GLOBAL *__restrict__ E = gptr(a.E);
    float IQP_GLOBAL *__restrict__ phase_out = gptr(a.phase_out);
    double IQP_GLOBAL *__restrict__ part = gptr(a.part);
    const int64_t splits = a.splits, s = a.s, l_pad = a.l_pad, s_pad = a.s_pad;
    const int64_t nchunk = ceil_div(s, kEpiChunk);
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

hipError_t launch_epilogue(const LaunchCtx &lc, const EpiArgs &a) {
    return plain_launch<EpiArgs, epilogue_body>(lc, KF_EPI, a, blocks_of(a));
}

__device__ __forceinline__ void finalize_body(const FinArgs &a, int64_t blk) {
    const double IQP_GLOBAL *__restrict__ part = gptr(a.part);
    double IQP_GLOBAL *__restrict__ mean = gptr(a.mean);
    double IQP_GLOBAL *__restrict__ stderr_ = gptr(a.stderr_);
    double IQP_GLOBAL *__restrict__ rowsum = gptr(a.rowsum);
    const int64_t s = a.s, nchunk = ceil_div(s, kEpiChunk);
    const int64_t k = blk * 256 + threadIdx.x;
    if (k >= a.l) return;
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

hipError_t launch_finalize(const LaunchCtx &lc, const FinArgs &a) {
    return plain_launch<FinArgs, finalize_body>(lc, KF_FIN, a, blocks_of(a));
}

// ---------------------------------------------------------------------------
// Backward weights. coef[2k] = alpha_k, coef[2k+1] = beta_k give
// dL/dc_ki = alpha_k + beta_k cos E_ki, and
//   S_ki = (alpha_k + beta_k cos E_ki) sin E_ki.
// Row scale of the fixed-point weights: |S_ki| <= |alpha_k| + |beta_k| since
// |cos|, |sin| <= 1.
__device__ __forceinline__ void coef_rowscale(double *sq, int32_t *nf, int64_t k, double al,
                                              double be) {
    if (sq) {
        gptr(sq)[k] = (fabs(al) + fabs(be)) / kI8Max;
        gptr(nf)[k] = 0;
    }
}

// Row exponent of the FP16 + FP8 weights: with bound_k = f 2^x, f in
// [1/2, 1), e_k = 15 - x puts bound_k 2^e_k in [2^14, 2^15), inside FP16's
// range with its normal numbers covering all weights above 2^-28 bound_k;
// 0 for a zero or non-finite bound (the row is zero, or its weights carry
// the NaN on).
__device__ __forceinline__ int f16_row_exp(double al, double be) {
    const double b = fabs(al) + fabs(be);
    if (!(b > 0.0) || !isfinite(b)) return 0;
    int x;
    (void)frexp(b, &x);
    const int e = 15 - x;
    return e < -120 ? -120 : (e > 120 ? 120 : e);
}

__device__ __forceinline__ void coef_plain_body(const CoefArgs &a, int64_t blk) {
    const int64_t k = blk * 256 + threadIdx.x;
    if (k >= a.l) return;
    const double al = gptr(a.grad_mean)[k] / (double)a.s;
    gptr(a.coef)[2 * k] = al;
    gptr(a.coef)[2 * k + 1] = 0.0;
    coef_rowscale(a.sq, a.nf, k, al, 0.0);
}

hipError_t launch_coef_plain(const LaunchCtx &lc, const CoefArgs &a) {
    return plain_launch<CoefArgs, coef_plain_body>(lc, KF_WEIGHTS, a, blocks_of(a));
}

// One block per 64 observables x 64 samples: S values are staged in LDS and
// written out in the register image of the backward product's A operand
// (rows = observables, K = samples):
//   BF16: 16-byte unit ((k/32) * KTs + i/16) * 64 + ((i/8)&1) * 32 + k%32 holds
//         S[k][i..i+7] (i a multiple of 8, KTs = s_pad / 16); hi and lo limbs
//         in two arrays
//   FP32: float (((k/32) * KT4s + i/8) * 64 + (i&1) * 32 + k%32) * 4 + (i/2)%4
//         holds S[k][i] (KT4s = s_pad / 8): four K-steps per 16-byte load
__device__ __forceinline__ void weights_body(const WeightsArgs &a, int64_t blk) {
    __shared__ float tile[64][65];  // [obs][sample]
    const float IQP_GLOBAL *__restrict__ phase = gptr(a.phase);
    const double IQP_GLOBAL *__restrict__ coef = gptr(a.coef);
    uint16_t IQP_GLOBAL *__restrict__ shi = gptr(a.shi);
    uint16_t IQP_GLOBAL *__restrict__ slo = gptr(a.slo);
    float IQP_GLOBAL *__restrict__ s32 = gptr(a.s32);
    const int64_t l = a.l, s = a.s, s_pad = a.s_pad;
    const int prec = a.prec;
    // blocks run sample tiles fastest
    const int64_t nsx = s_pad / 64;
    const int64_t by = blk / nsx;
    const int64_t i0 = (blk - by * nsx) * 64, k0 = by * 64;
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
    if (prec == 3) {
        // 16-bit fixed point per observable row: N = rint(S / q_k), split into
        // signed 8-bit limbs N = 256 hi + lo; 64 observables x 4 groups of 16
        // samples, one 16-byte unit of each limb per thread, at
        // ((k/32) * KTs + i/32) * 64 + ((i/16)&1) * 32 + k%32, KTs = s_pad / 32
        const int64_t KTs = s_pad / 32;
        const int kl = threadIdx.x & 63, sg = threadIdx.x >> 6;
        const int64_t k = k0 + kl, i = i0 + 16 * sg;
        double inv = 0.0;
        if (k < l) {
            const double sig = fabs(coef[2 * k]) + fabs(coef[2 * k + 1]);
            inv = sig > 0.0 ? kI8Max / sig : 0.0;
        }
        bool bad = false;
        uint32_t dh[4], dl[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            uint32_t ph = 0, pl = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float x = tile[kl][16 * sg + 4 * v + e];
                bad |= !isfinite(x);
                double nv = rint((double)x * inv);
                nv = nv > kI8Max ? kI8Max : (nv < -kI8Max - 1.0 ? -kI8Max - 1.0 : nv);
                const int32_t N = isfinite(nv) ? (int32_t)nv : 0;
                const int32_t hi = (N + 128) >> 8, lo = N - 256 * hi;
                ph |= ((uint32_t)hi & 0xFFu) << (8 * e);
                pl |= ((uint32_t)lo & 0xFFu) << (8 * e);
            }
            dh[v] = ph;
            dl[v] = pl;
        }
        const int64_t idx = ((k >> 5) * KTs + (i >> 5)) * 64 + ((i >> 4) & 1) * 32 + (k & 31);
        reinterpret_cast<u32x4 IQP_GLOBAL *>(shi)[idx] = (u32x4){dh[0], dh[1], dh[2], dh[3]};
        reinterpret_cast<u32x4 IQP_GLOBAL *>(slo)[idx] = (u32x4){dl[0], dl[1], dl[2], dl[3]};
        if (bad && k < l) gptr(a.nf)[k] = 1;  // every writer stores the same value
    } else if (prec == 4) {
        // x = S_ki 2^e_k: FP16 limb h = rn(x) in the BF16 form's image, and
        // FP8 limb rn_e4m3(x - h) (exact difference, |x - h| <= 8) in the
        // A-operand image of a 32x32x64 FP8 product: lane (l/32, l%32) holds
        // row l%32 and, in byte 8 t + e, sample 16 t + 8 (l/32) + e of a
        // sample word (the samples of the lane's four FP16 K-steps), as two
        // 16-byte units at (((k/32) * sw + i/64) * 2 + q) * 64 + l for bytes
        // 16 q .. 16 q + 15 (sw = s_pad / 64)
        const int kl = threadIdx.x & 63;
        const int64_t k = k0 + kl;
        int ex = 0;
        if (k < l) ex = f16_row_exp(coef[2 * k], coef[2 * k + 1]);
        const int64_t KTs = s_pad / 16;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int sg = (q * 256 + (int)threadIdx.x) >> 6;
            const int64_t i = i0 + 8 * sg;
            const int64_t idx = ((k >> 5) * KTs + (i >> 4)) * 64 + ((i >> 3) & 1) * 32 + (k & 31);
            uint32_t dh[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uint32_t hv[2];
#pragma unroll
                for (int e = 0; e < 2; ++e)
                    hv[e] = __builtin_bit_cast(uint16_t,
                                               (_Float16)ldexpf(tile[kl][8 * sg + 2 * v + e], ex));
                dh[v] = hv[0] | (hv[1] << 16);
            }
            reinterpret_cast<u32x4 IQP_GLOBAL *>(shi)[idx] = (u32x4){dh[0], dh[1], dh[2], dh[3]};
        }
        const int hq = threadIdx.x >> 6, hh = hq >> 1, q = hq & 1;
        uint32_t d8[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            uint32_t w = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // byte 16 q + 4 v + e of the lane: K-step 2 q + v / 2, sample
                // 8 (v % 2) + e of its half hh
                const int i = 32 * q + 16 * (v >> 1) + 8 * hh + 4 * (v & 1) + e;
                const float x = ldexpf(tile[kl][i], ex);
                const float h = (float)(_Float16)x;
                w |= f32_to_e4m3(x - h) << (8 * e);
            }
            d8[v] = w;
        }
        const int64_t sw = s_pad / 64;
        const int64_t idx8 = (((k >> 5) * sw + i0 / 64) * 2 + q) * 64 + hh * 32 + (k & 31);
        reinterpret_cast<u32x4 IQP_GLOBAL *>(slo)[idx8] = (u32x4){d8[0], d8[1], d8[2], d8[3]};
        if (i0 == 0 && hq == 0 && k < l) gptr(a.sq)[k] = ldexp(1.0, -ex);
    } else if (prec == 1) {
        const int64_t KTs = s_pad / 16;
        // 64 observables x 8 groups of 8 samples = 512 units, 2 per thread
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int unit = q * 256 + threadIdx.x;
            const int kl = unit & 63, sg = unit >> 6;
            const int64_t k = k0 + kl, i = i0 + 8 * sg;
            const int64_t idx = ((k >> 5) * KTs + (i >> 4)) * 64 + ((i >> 3) & 1) * 32 + (k & 31);
            uint32_t dh[4], dl[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uint16_t hv[2], lv[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float x = tile[kl][8 * sg + 2 * v + e];
                    hv[e] = f2bf_rne(x);
                    lv[e] = f2bf_rne(x - bf2f(hv[e]));
                }
                dh[v] = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
                dl[v] = (uint32_t)lv[0] | ((uint32_t)lv[1] << 16);
            }
            reinterpret_cast<u32x4 IQP_GLOBAL *>(shi)[idx] = (u32x4){dh[0], dh[1], dh[2], dh[3]};
            reinterpret_cast<u32x4 IQP_GLOBAL *>(slo)[idx] = (u32x4){dl[0], dl[1], dl[2], dl[3]};
        }
    } else {
        const int64_t KT4s = s_pad / 8;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int unit = q * 256 + threadIdx.x;
            const int kl = unit & 63, il = unit >> 6;
            const int64_t k = k0 + kl, i = i0 + il;
            s32[(((k >> 5) * KT4s + (i >> 3)) * 64 + (i & 1) * 32 + (k & 31)) * 4 + ((i >> 1) & 3)] =
                tile[kl][il];
        }
    }
}

hipError_t launch_weights(const LaunchCtx &lc, const WeightsArgs &a) {
    return plain_launch<WeightsArgs, weights_body>(lc, KF_WEIGHTS, a, blocks_of(a));
}

// ---------------------------------------------------------------------------
// phase_bwd: T[k][j] = sum_i S_ki (-1)^{b_ij} (observables x gates, K =
// samples), then dtheta_j = -2 sum_k c_kj T[k][j]. The contraction runs over
// the long sample dimension, so each tile amortises its prologue and
// epilogue; the epilogue is a masked sum over the tile's observable rows and
// one cross-lane add.
//   A operand: S in the register image written by weights_kernel
//   B operand: +-1 from the sample-contiguous B^T bits (transposed tiled32:
//              row = gate j, bits over samples), K-step t of a sample word
//              is byte 2t + h of the lane's word
//   epilogue:  c_kj from the C^T bits (row = gate j, bits over observables)
// A workgroup is 4 waves that share an observable block (the S strip,
// staged through LDS per sample word, double-buffered) and take 4
// consecutive gate blocks. Workgroups are ordered gate block fastest, so an
// XCD's workgroups share one S strip in L2. As in the forward, the last
// region of a word runs after the barrier that validates the next word's
// buffer, so it already expands the next word's first K-step.
// Work unit -> (observable block, gate-block group, sample split). Within a
// split the observable blocks run in groups of `grp`; inside a group the
// observable block changes fastest, so workgroups that run at the same time
// share both their S strips (grp of them) and their B^T strips (one per
// gate-block group), and each B^T strip is fetched about n_ob / grp times
// instead of n_ob times. The last group may be smaller.
__device__ __forceinline__ void bwd_unit(int64_t gu, int64_t n_ob, int64_t n_jbg, int64_t grp,
                                         int64_t &ob, int64_t &jbg, int64_t &ks) {
    const int64_t per_split = n_ob * n_jbg;
    ks = gu / per_split;
    const int64_t u = gu - ks * per_split;
    const int64_t G = grp < 1 ? 1 : (grp > n_ob ? n_ob : grp);
    const int64_t g = u / (G * n_jbg);
    const int64_t gsz = (g + 1) * G <= n_ob ? G : n_ob - g * G;
    const int64_t r = u - g * G * n_jbg;
    jbg = r / gsz;
    ob = g * G + (r - jbg * gsz);
}

template <int FM, int FN>
struct BwdOps {
    bf16x8 ah[FM], al[FM], bv[FN];
};

template <int FM, int FN, int T>
__device__ __forceinline__ void bwd_expand_a(BwdOps<FM, FN> &o, const u32x4 *ls, int lane) {
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        o.ah[f] = __builtin_bit_cast(bf16x8, ls[((0 * FM + f) * 4 + T) * 64 + lane]);
        o.al[f] = __builtin_bit_cast(bf16x8, ls[((1 * FM + f) * 4 + T) * 64 + lane]);
    }
}

template <int FM, int FN, int T, int G0, int G1>
__device__ __forceinline__ void bwd_expand_b(BwdOps<FM, FN> &o, const uint64_t (&bw)[FN],
                                             uint32_t ones) {
#pragma unroll
    for (int g = G0; g < G1; ++g) {
        const uint32_t d = (uint32_t)(bw[g] >> (32 * (T >> 1)));
        o.bv[g] = expand_pm1((T & 1) ? (d >> 16) : d, ones);
    }
}

template <int FM, int FN, int T>
__device__ __forceinline__ void bwd_expand(BwdOps<FM, FN> &o, const u32x4 *ls,
                                           const uint64_t (&bw)[FN], int lane, uint32_t ones) {
    bwd_expand_a<FM, FN, T>(o, ls, lane);
    bwd_expand_b<FM, FN, T, 0, FN>(o, bw, ones);
}

template <int FM, int FN, int LIMB>
__device__ __forceinline__ void bwd_mfma_half(const BwdOps<FM, FN> &o, f32x16 (&acc)[FM][FN]) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
            acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(LIMB ? o.al[f] : o.ah[f], o.bv[g],
                                                                acc[f][g], 0, 0, 0);
}

// One pipeline region: the products of K-step t (operands `cur`) while the
// operands of K-step T1 are read from `lsn` and expanded into `nxt`.
template <int FM, int FN, int T1>
__device__ __forceinline__ void bwd_region(const BwdOps<FM, FN> &cur, BwdOps<FM, FN> &nxt,
                                           const u32x4 *lsn, const uint64_t (&bw)[FN], int lane,
                                           uint32_t ones, f32x16 (&acc)[FM][FN]) {
    bwd_expand_a<FM, FN, T1>(nxt, lsn, lane);
    bwd_expand_b<FM, FN, T1, 0, FN / 2>(nxt, bw, ones);
    bwd_mfma_half<FM, FN, 0>(cur, acc);
    interleave_half<2 * FM, FM * FN, 4 * FN + 2>();
    bwd_expand_b<FM, FN, T1, FN / 2, FN>(nxt, bw, ones);
    bwd_mfma_half<FM, FN, 1>(cur, acc);
    interleave_half<0, FM * FN, 4 * FN + 2>();
}

// sum_k c_kj T[k][j] over this wave's observable rows, per gate column.
template <int FM, int FN>
__device__ __forceinline__ void bwd_epilogue(const f32x16 (&acc)[FM][FN],
                                             const uint64_t IQP_GLOBAL *__restrict__ ctbits, int64_t ob,
                                             int64_t jb, int64_t lw, int h, int r, bool active,
                                             float IQP_GLOBAL *__restrict__ gpart, int64_t m_pad) {
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        const int64_t j = (jb * FN + g) * 32 + r;
        float gs = 0.0f;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const int64_t k0 = (ob * FM + f) * 32;
            const uint64_t cw = ctbits[((j >> 5) * lw + (k0 >> 6)) * 32 + (j & 31)];
            const uint32_t c32 = (uint32_t)(cw >> (k0 & 63)) >> (4 * h);
#pragma unroll
            for (int a = 0; a < 16; ++a)
                gs += ((c32 >> (8 * (a >> 2) + (a & 3))) & 1u) ? acc[f][g][a] : 0.0f;
        }
        gs += __shfl_xor(gs, 32, 64);
        if (active && h == 0) gpart[ob * m_pad + j] = gs;
    }
}

template <int FM, int FN>
__device__ __forceinline__ void bwd_bf16_body(const BwdArgs &a, int64_t gu, int tid) {
    // one sample word: [limb][f][t][lane], 16 bytes each. The two buffers
    // are distinct objects selected at compile time (the word loop is
    // unrolled by two), so the compiler can tell that reads of one never
    // alias the global -> LDS copy in flight into the other.
    constexpr int kUnits = 2 * FM * 4 * 64;
    __shared__ u32x4 ls0[kUnits], ls1[kUnits];
    const u32x4 IQP_GLOBAL *__restrict__ shi = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.shi));
    const u32x4 IQP_GLOBAL *__restrict__ slo = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.slo));
    const uint64_t IQP_GLOBAL *__restrict__ btbits = gptr(a.btbits);
    const uint64_t IQP_GLOBAL *__restrict__ ctbits = gptr(a.ctbits);
    const int64_t m_pad = a.m_pad, sw = a.s_pad / 64, lw = a.l_pad / 64;
    const int64_t n_jb = m_pad / (32 * FN), n_ob = a.l_pad / (32 * FM);
    const int64_t n_jbg = ceil_div(n_jb, 4);
    int64_t jbg, ob, ks;
    bwd_unit(gu, n_ob, n_jbg, a.obgroup, ob, jbg, ks);
    const int64_t wps = ceil_div(sw, a.ksplits);
    const int64_t w0 = ks * wps, w1 = (w0 + wps < sw) ? w0 + wps : sw;
    float IQP_GLOBAL *__restrict__ gpart = gptr(a.gpart) + ks * n_ob * m_pad;
    const int64_t jb_raw = jbg * 4 + wave_id();
    const bool active = jb_raw < n_jb;
    const int64_t jb = active ? jb_raw : n_jb - 1;
    const int lane = tid & 63;
    const int h = lane >> 5, r = lane & 31;
    const uint32_t ones = in_vgpr(0x3F803F80u);
    const int64_t KTs = sw * 4;
    const uint64_t IQP_GLOBAL *bbase = btbits + jb * FN * sw * 32;
    const u32x4 IQP_GLOBAL *sbase_h = shi + ob * FM * KTs * 64;
    const u32x4 IQP_GLOBAL *sbase_l = slo + ob * FM * KTs * 64;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    // staging block b = (limb * FM + f) * 4 + t (64 units of 16 bytes)
    //   <- S(limb)[(f * KTs + 4 w + t) * 64 + ln]; wave v copies blocks v, v+4, ...
    const int wv = wave_id();
    auto stage = [&](int64_t w, u32x4 *dst) {
#pragma unroll
        for (int k = 0; k < kUnits / 256; ++k) {
            const int b = wv + 4 * k;
            const int t = b & 3, f = (b >> 2) % FM, limb = b / (4 * FM);
            const int64_t src = ((int64_t)f * KTs + 4 * w + t) * 64 + lane;
            dma16((limb ? sbase_l : sbase_h) + src, &dst[b * 64]);
        }
    };
    // every unit has w1 - w0 >= 1 sample words (the host picks the splits)
    stage(w0, ls0);
    if (w0 + 1 < w1) stage(w0 + 1, ls1);
    uint64_t nxt[FN], cur[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w0) * 32)[r];
    dma_wait_barrier();
#pragma unroll
    for (int g = 0; g < FN; ++g) cur[g] = nxt[g] >> (8 * h);
    if (w0 + 1 < w1) {
#pragma unroll
        for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w0 + 1) * 32)[r];
    }
    BwdOps<FM, FN> opA, opB;
    bwd_expand<FM, FN, 0>(opA, ls0, cur, lane, ones);
    // Word w reads `mine`; its last region runs after a barrier that makes
    // word w+1's buffer `other` valid, so that region already expands word
    // w+1's first K-step; the copy of word w+2 into `mine` is issued right
    // after that barrier.
    auto word = [&](int64_t w, u32x4 *mine, const u32x4 *other) {
        bwd_region<FM, FN, 1>(opA, opB, mine, cur, lane, ones, acc);
        bwd_region<FM, FN, 2>(opB, opA, mine, cur, lane, ones, acc);
        bwd_region<FM, FN, 3>(opA, opB, mine, cur, lane, ones, acc);
        dma_wait_barrier();
        if (w + 2 < w1) stage(w + 2, mine);
#pragma unroll
        for (int g = 0; g < FN; ++g) cur[g] = nxt[g] >> (8 * h);
        if (w + 2 < w1) {
#pragma unroll
            for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w + 2) * 32)[r];
        }
        // past the last word this expands a stale buffer and is never used
        bwd_region<FM, FN, 0>(opB, opA, other, cur, lane, ones, acc);
    };
    for (int64_t w = w0; w < w1; w += 2) {
        word(w, ls0, ls1);
        if (w + 1 < w1) word(w + 1, ls1, ls0);
    }
    bwd_epilogue<FM, FN>(acc, ctbits, ob, jb, lw, h, r, active, gpart, m_pad);
}

// FP32 form: A operand S[k][2t + h] from the float4 image (four K-steps per
// lane and load), staged per sample word as [f][q][lane]; B operand +-1.0f.
template <int FM, int FN>
__device__ __forceinline__ void bwd_f32_body(const BwdArgs &a, int64_t gu, int tid) {
    constexpr int kUnits = FM * 8 * 64;
    __shared__ float4 ls[2][kUnits];
    const float4 IQP_GLOBAL *__restrict__ s32 = reinterpret_cast<const float4 IQP_GLOBAL *>(gptr(a.s32));
    const uint64_t IQP_GLOBAL *__restrict__ btbits = gptr(a.btbits);
    const uint64_t IQP_GLOBAL *__restrict__ ctbits = gptr(a.ctbits);
    const int64_t m_pad = a.m_pad, sw = a.s_pad / 64, lw = a.l_pad / 64;
    const int64_t n_jb = m_pad / (32 * FN), n_ob = a.l_pad / (32 * FM);
    const int64_t n_jbg = ceil_div(n_jb, 4);
    int64_t jbg, ob, ks;
    bwd_unit(gu, n_ob, n_jbg, a.obgroup, ob, jbg, ks);
    const int64_t wps = ceil_div(sw, a.ksplits);
    const int64_t w0 = ks * wps, w1 = (w0 + wps < sw) ? w0 + wps : sw;
    float IQP_GLOBAL *__restrict__ gpart = gptr(a.gpart) + ks * n_ob * m_pad;
    const int64_t jb_raw = jbg * 4 + wave_id();
    const bool active = jb_raw < n_jb;
    const int64_t jb = active ? jb_raw : n_jb - 1;
    const int lane = tid & 63;
    const int h = lane >> 5, r = lane & 31;
    const int64_t KT4s = sw * 8;
    const uint64_t IQP_GLOBAL *bbase = btbits + jb * FN * sw * 32;
    const float4 IQP_GLOBAL *sbase = s32 + ob * FM * KT4s * 64;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int a = 0; a < 16; ++a) acc[f][g][a] = 0.0f;

    // staging block b = f * 8 + q (64 float4) <- S[(f * KT4s + 8 w + q) * 64 + ln]
    const int wv = wave_id();
    auto stage = [&](int64_t w, int buf) {
#pragma unroll
        for (int k = 0; k < kUnits / 256; ++k) {
            const int b = wv + 4 * k;
            const int q = b & 7, f = b >> 3;
            dma16(sbase + ((int64_t)f * KT4s + 8 * w + q) * 64 + lane, &ls[buf][b * 64]);
        }
    };
    stage(w0, 0);
    uint64_t nxt[FN], cur[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w0) * 32)[r];
    dma_wait_barrier();
    for (int64_t w = w0; w < w1; ++w) {
        const int buf = (int)((w - w0) & 1);
        const bool more = w + 1 < w1;
        if (more) stage(w + 1, buf ^ 1);
#pragma unroll
        for (int g = 0; g < FN; ++g) cur[g] = nxt[g] >> h;
        if (more) {
#pragma unroll
            for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w + 1) * 32)[r];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float4 sv[FM];
#pragma unroll
            for (int f = 0; f < FM; ++f) sv[f] = ls[buf][(f * 8 + q) * 64 + lane];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int t = 4 * q + e;
                float bv[FN];
#pragma unroll
                for (int g = 0; g < FN; ++g)
                    bv[g] = __uint_as_float((((uint32_t)(cur[g] >> (2 * t)) & 1u) << 31) |
                                            0x3F800000u);
#pragma unroll
                for (int f = 0; f < FM; ++f) {
                    const float av = e == 0 ? sv[f].x : e == 1 ? sv[f].y : e == 2 ? sv[f].z : sv[f].w;
#pragma unroll
                    for (int g = 0; g < FN; ++g)
                        acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv[g], acc[f][g], 0, 0, 0);
                }
            }
        }
        dma_wait_barrier();
    }
    bwd_epilogue<FM, FN>(acc, ctbits, ob, jb, lw, h, r, active, gpart, m_pad);
}

// ---------------------------------------------------------------------------
// INT8 form of the backward (IQP_SPLIT3_BF16). S is held per observable row in
// 16-bit fixed point, S_ki ~ q_k (256 hi_ki + lo_ki) with signed 8-bit limbs,
// written by weights_kernel as the A-operand image of a 32x32x32 INT8 product
// (lane l: row l % 32, K values 16 (l / 32) .. + 15). Each K-step (32
// samples) takes two INT8 products per 32x32 block, one per limb, into
// separate INT32 accumulators, so the sums are exact; the epilogue forms
// q_k (256 T_hi + T_lo) in FP64 per row before the masked sum over rows.
// Same work units, staging and pipeline as the BF16 form, with two K-steps
// per 64-sample word instead of four.
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

// B_ij = (-1)^{bit} as signed bytes (+1 = 0x01, -1 = 0xFF) for the 16 K values
// of the lane (bits 0..15 of x16). For dword v (bits 4v .. 4v+3), packed
// 16-bit shifts move bits 4v, 4v+1 to positions 15, 31 of one dword and bits
// 4v+2, 4v+3 to positions 15, 31 of another; the byte permute's
// sign-replicating selectors 8..11 turn those four sign positions into
// 0x00 / 0xFF bytes in order.
__device__ __forceinline__ i32x4 expand_pm1_i8(uint32_t x16) {
    const u16x2 xv = {(unsigned short)x16, (unsigned short)x16};
    uint32_t d[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const u16x2 sh1 = {(unsigned short)(15 - 4 * v), (unsigned short)(14 - 4 * v)};
        const u16x2 sh0 = {(unsigned short)(13 - 4 * v), (unsigned short)(12 - 4 * v)};
        const uint32_t s1 = __builtin_bit_cast(uint32_t, (u16x2)(xv << sh1));
        const uint32_t s0 = __builtin_bit_cast(uint32_t, (u16x2)(xv << sh0));
        d[v] = __builtin_amdgcn_perm(s0, s1, 0x0B0A0908u) | 0x01010101u;
    }
    return (i32x4){(int32_t)d[0], (int32_t)d[1], (int32_t)d[2], (int32_t)d[3]};
}

template <int FM, int FN>
struct BwdOpsI8 {
    i32x4 a[2][FM], bv[FN];
};

// A staged block is 128 samples (two sample words, four K-steps): K-step T
// uses bits 32 (T % 2) + 16 h .. + 15 of sample word T / 2 of the lane's
// B^T words (bw0, bw1, pre-shifted right by 16 h).
template <int FM, int FN, int T>
__device__ __forceinline__ void bwdi8_expand_a(BwdOpsI8<FM, FN> &o, const u32x4 *ls, int lane) {
#pragma unroll
    for (int L = 0; L < 2; ++L)
#pragma unroll
        for (int f = 0; f < FM; ++f)
            o.a[L][f] = __builtin_bit_cast(i32x4, ls[((L * FM + f) * 4 + T) * 64 + lane]);
}

template <int FM, int FN, int T, int G0, int G1>
__device__ __forceinline__ void bwdi8_expand_b(BwdOpsI8<FM, FN> &o, const uint64_t (&bw0)[FN],
                                               const uint64_t (&bw1)[FN]) {
#pragma unroll
    for (int g = G0; g < G1; ++g)
        o.bv[g] = expand_pm1_i8((uint32_t)((T < 2 ? bw0[g] : bw1[g]) >> (32 * (T & 1))));
}

template <int FM, int FN, int L>
__device__ __forceinline__ void bwdi8_mfma_limb(const BwdOpsI8<FM, FN> &o,
                                                i32x16 (&acc)[2][FM][FN]) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
            acc[L][f][g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(o.a[L][f], o.bv[g], acc[L][f][g],
                                                                 0, 0, 0);
}

// One pipeline region: the products of K-step t (operands `cur`) while the
// operands of K-step T1 are read from `lsn` and expanded into `nxt`.
template <int FM, int FN, int T1>
__device__ __forceinline__ void bwdi8_region(const BwdOpsI8<FM, FN> &cur, BwdOpsI8<FM, FN> &nxt,
                                             const u32x4 *lsn, const uint64_t (&bw0)[FN],
                                             const uint64_t (&bw1)[FN], int lane,
                                             i32x16 (&acc)[2][FM][FN]) {
    bwdi8_expand_a<FM, FN, T1>(nxt, lsn, lane);
    bwdi8_expand_b<FM, FN, T1, 0, FN / 2>(nxt, bw0, bw1);
    bwdi8_mfma_limb<FM, FN, 0>(cur, acc);
    interleave_half<2 * FM, FM * FN, 9 * FN + 2>();
    bwdi8_expand_b<FM, FN, T1, FN / 2, FN>(nxt, bw0, bw1);
    bwdi8_mfma_limb<FM, FN, 1>(cur, acc);
    interleave_half<0, FM * FN, 9 * FN + 2>();
}

// sum_k c_kj q_k (256 T_hi + T_lo)[k][j] over this wave's observable rows, per
// gate column; 256 T_hi + T_lo is exact in INT32 (a work unit covers at most
// kI8MaxSamplesPerUnit samples) and is then rounded to FP32 once, as the
// BF16 form's accumulators are. A row whose weights were not finite
// contributes NaN.
template <int FM, int FN>
__device__ __forceinline__ void bwdi8_epilogue(const i32x16 (&acc)[2][FM][FN],
                                               const uint64_t IQP_GLOBAL *__restrict__ ctbits,
                                               const double IQP_GLOBAL *__restrict__ sq,
                                               const int32_t IQP_GLOBAL *__restrict__ nf,
                                               int64_t ob, int64_t jb, int64_t lw, int h, int r,
                                               bool active, float IQP_GLOBAL *__restrict__ gpart,
                                               int64_t m_pad) {
    float gs[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) gs[g] = 0.0f;
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const int64_t k0 = (ob * FM + f) * 32;
        float q[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            const int64_t k = k0 + acc_row(a, h);
            q[a] = nf[k] ? NAN : (float)sq[k];
        }
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const int64_t j = (jb * FN + g) * 32 + r;
            const uint64_t cw = ctbits[((j >> 5) * lw + (k0 >> 6)) * 32 + (j & 31)];
            const uint32_t c32 = (uint32_t)(cw >> (k0 & 63)) >> (4 * h);
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                const int32_t t = acc[1][f][g][a] * 256 + acc[0][f][g][a];
                gs[g] += ((c32 >> (8 * (a >> 2) + (a & 3))) & 1u) ? q[a] * (float)t : 0.0f;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        const int64_t j = (jb * FN + g) * 32 + r;
        const float v = gs[g] + __shfl_xor(gs[g], 32, 64);
        if (active && h == 0) gpart[ob * m_pad + j] = v;
    }
}

template <int FM, int FN>
__device__ __forceinline__ void bwd_i8_body(const BwdArgs &a, int64_t gu, int tid) {
    // one block of 128 samples: [limb][f][t][lane], 16 bytes each, two buffers
    constexpr int kUnits = 2 * FM * 4 * 64;
    __shared__ u32x4 ls0[kUnits], ls1[kUnits];
    const u32x4 IQP_GLOBAL *__restrict__ shi = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.shi));
    const u32x4 IQP_GLOBAL *__restrict__ slo = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.slo));
    const uint64_t IQP_GLOBAL *__restrict__ btbits = gptr(a.btbits);
    const uint64_t IQP_GLOBAL *__restrict__ ctbits = gptr(a.ctbits);
    const int64_t m_pad = a.m_pad, sw = a.s_pad / 64, lw = a.l_pad / 64;
    const int64_t n_jb = m_pad / (32 * FN), n_ob = a.l_pad / (32 * FM);
    const int64_t n_jbg = ceil_div(n_jb, 4);
    int64_t jbg, ob, ks;
    bwd_unit(gu, n_ob, n_jbg, a.obgroup, ob, jbg, ks);
    // splits are whole blocks of two sample words (s_pad is a multiple of
    // 128, so sw is even)
    const int64_t nb2 = sw / 2, bps = ceil_div(nb2, a.ksplits);
    const int64_t b0 = ks * bps, b1 = (b0 + bps < nb2) ? b0 + bps : nb2;
    float IQP_GLOBAL *__restrict__ gpart = gptr(a.gpart) + ks * n_ob * m_pad;
    const int64_t jb_raw = jbg * 4 + wave_id();
    const bool active = jb_raw < n_jb;
    const int64_t jb = active ? jb_raw : n_jb - 1;
    const int lane = tid & 63;
    const int h = lane >> 5, r = lane & 31;
    const int64_t KTs = sw * 2;
    const uint64_t IQP_GLOBAL *bbase = btbits + jb * FN * sw * 32;
    const u32x4 IQP_GLOBAL *sbase_h = shi + ob * FM * KTs * 64;
    const u32x4 IQP_GLOBAL *sbase_l = slo + ob * FM * KTs * 64;

    i32x16 acc[2][FM][FN];
#pragma unroll
    for (int L = 0; L < 2; ++L)
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int g = 0; g < FN; ++g)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[L][f][g][e] = 0;

    // staging block q = (limb * FM + f) * 4 + t (64 units of 16 bytes)
    //   <- S(limb)[(f * KTs + 4 b + t) * 64 + ln]; limb 0 = lo, 1 = hi;
    // wave v copies blocks v, v+4, ...
    const int wv = wave_id();
    auto stage = [&](int64_t b, u32x4 *dst) {
#pragma unroll
        for (int k = 0; k < kUnits / 256; ++k) {
            const int q = wv + 4 * k;
            const int t = q & 3, f = (q >> 2) % FM, limb = q / (4 * FM);
            const int64_t src = ((int64_t)f * KTs + 4 * b + t) * 64 + lane;
            dma16((limb ? sbase_h : sbase_l) + src, &dst[q * 64]);
        }
    };
    auto load_bits = [&](int64_t b, uint64_t (&x0)[FN], uint64_t (&x1)[FN]) {
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            x0[g] = (bbase + (g * sw + 2 * b) * 32)[r];
            x1[g] = (bbase + (g * sw + 2 * b + 1) * 32)[r];
        }
    };
    // every unit has b1 - b0 >= 1 blocks (the host picks the splits)
    stage(b0, ls0);
    if (b0 + 1 < b1) stage(b0 + 1, ls1);
    uint64_t nxt0[FN], nxt1[FN], cur0[FN], cur1[FN];
    load_bits(b0, nxt0, nxt1);
    dma_wait_barrier();
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        cur0[g] = nxt0[g] >> (16 * h);
        cur1[g] = nxt1[g] >> (16 * h);
    }
    if (b0 + 1 < b1) load_bits(b0 + 1, nxt0, nxt1);
    BwdOpsI8<FM, FN> opA, opB;
    bwdi8_expand_a<FM, FN, 0>(opA, ls0, lane);
    bwdi8_expand_b<FM, FN, 0, 0, FN>(opA, cur0, cur1);
    // Block b reads `mine`; its last region runs after a barrier that makes
    // block b+1's buffer `other` valid, so that region already expands block
    // b+1's first K-step; the copy of block b+2 into `mine` is issued right
    // after that barrier.
    auto block = [&](int64_t b, u32x4 *mine, const u32x4 *other) {
        bwdi8_region<FM, FN, 1>(opA, opB, mine, cur0, cur1, lane, acc);
        bwdi8_region<FM, FN, 2>(opB, opA, mine, cur0, cur1, lane, acc);
        bwdi8_region<FM, FN, 3>(opA, opB, mine, cur0, cur1, lane, acc);
        dma_wait_barrier();
        if (b + 2 < b1) stage(b + 2, mine);
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            cur0[g] = nxt0[g] >> (16 * h);
            cur1[g] = nxt1[g] >> (16 * h);
        }
        if (b + 2 < b1) load_bits(b + 2, nxt0, nxt1);
        // past the last block this expands a stale buffer and is never used
        bwdi8_region<FM, FN, 0>(opB, opA, other, cur0, cur1, lane, acc);
    };
    int64_t b = b0;
    do {  // b1 > b0: the accumulators always pass through the loop
        block(b, ls0, ls1);
        if (b + 1 < b1) block(b + 1, ls1, ls0);
        b += 2;
    } while (b < b1);
    bwdi8_epilogue<FM, FN>(acc, ctbits, gptr(a.sq), gptr(a.nf), ob, jb, lw, h, r, active, gpart,
                           m_pad);
}

// The 64 x 64 wave tile fits two waves per SIMD (its INT32 accumulators in
// VGPRs, no AGPRs), which hides the per-block barrier and load latency.
// ---------------------------------------------------------------------------
// FP16 + FP8 form of the backward (IQP_SPLIT_BF16_FP8). Row k of S is scaled
// by 2^e_k and held as an FP16 limb plus an FP8 E4M3 limb (weights_kernel).
// Per 64-sample word and 32x32 block: four 32x32x16 FP16 products of the
// FP16 limb (K-steps as in the BF16 form, B = +-1.0 in FP16) and one
// 32x32x64 FP8 product of the FP8 limb (B = +-1.0 in E4M3), all into the
// same FP32 accumulators; the FP8 product takes the matrix-core time of two
// FP16 ones, so a word costs 6 instead of the 8 of two BF16 limbs. The
// epilogue multiplies each row by 2^-e_k (sq) before the masked sum over
// rows. Same work units, staging (one sample word per buffer) and pipeline
// as the BF16 form. The FP8 B operand is built per K-step from the FP16 one
// (the high bytes of its +-1 pairs, 0x3C / 0xBC, by one byte permute, then
// 0x38 / 0xB8), so lane half h holds samples 16 t + 8 h + e of K-step t in
// bytes 8 t + e, the order the weights kernel writes the FP8 limb in; a
// word's FP8 products are issued at the start of its last region (after the
// word's barrier), before that region's expansion starts the next word.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int FM, int FN>
struct BwdOpsH {
    f16x8 ah[FM], bv[FN];
};
// the FP8 limb of the word's S strip and the word's +-1 FP8 operands
template <int FM, int FN>
struct BwdLoF8 {
    i32x8 a[FM];
    uint32_t b[FN][8];
    uint32_t m80, c38;  // the E4M3 sign mask and +1.0, in vector registers
};

template <int FM, int FN, int T>
__device__ __forceinline__ void bwdh_expand_a(BwdOpsH<FM, FN> &o, const u32x4 *ls, int lane) {
#pragma unroll
    for (int f = 0; f < FM; ++f)
        o.ah[f] = __builtin_bit_cast(f16x8, ls[(f * 4 + T) * 64 + lane]);
}

template <int FM, int FN, int T>
__device__ __forceinline__ void bwdh_expand_b(BwdOpsH<FM, FN> &o, const uint64_t (&bw)[FN],
                                              uint32_t ones, BwdLoF8<FM, FN> &lo) {
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        const uint32_t d = (uint32_t)(bw[g] >> (32 * (T >> 1)));
        const bf16x8 v = expand_pm1((T & 1) ? (d >> 16) : d, ones);
        o.bv[g] = __builtin_bit_cast(f16x8, v);
        const u32x4 q = __builtin_bit_cast(u32x4, v);
        lo.b[g][2 * T] = (__builtin_amdgcn_perm(q[1], q[0], 0x07050301u) & lo.m80) | lo.c38;
        lo.b[g][2 * T + 1] = (__builtin_amdgcn_perm(q[3], q[2], 0x07050301u) & lo.m80) | lo.c38;
    }
}

// One pipeline region: the FP16 products of K-step t (operands `cur`) while
// the operands of K-step T1 are read from `lsn` and expanded into `nxt`.
// Region 1 also reads the word's FP8 limb; region 0 (after the word's
// barrier) first issues the word's FP8 products.
template <int FM, int FN, int R>
__device__ __forceinline__ void bwdh_region(const BwdOpsH<FM, FN> &cur, BwdOpsH<FM, FN> &nxt,
                                            const u32x4 *lsn, const uint64_t (&bw)[FN], int lane,
                                            uint32_t ones, BwdLoF8<FM, FN> &lo,
                                            f32x16 (&acc)[FM][FN]) {
    if constexpr (R == 1) {
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const u32x4 p0 = lsn[(4 * FM + 2 * f) * 64 + lane];
            const u32x4 p1 = lsn[(4 * FM + 2 * f + 1) * 64 + lane];
            lo.a[f] = (i32x8){(int32_t)p0[0], (int32_t)p0[1], (int32_t)p0[2], (int32_t)p0[3],
                              (int32_t)p1[0], (int32_t)p1[1], (int32_t)p1[2], (int32_t)p1[3]};
        }
    }
    if constexpr (R == 0) {
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int g = 0; g < FN; ++g)
                acc[f][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    lo.a[f], __builtin_bit_cast(i32x8, lo.b[g]), acc[f][g], 0, 0, 0, 127, 0, 127);
    }
    bwdh_expand_a<FM, FN, R>(nxt, lsn, lane);
    bwdh_expand_b<FM, FN, R>(nxt, bw, ones, lo);
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
            acc[f][g] = __builtin_amdgcn_mfma_f32_32x32x16_f16(cur.ah[f], cur.bv[g], acc[f][g], 0, 0,
                                                               0);
    constexpr int kM = FM * FN * (R == 0 ? 2 : 1);
    constexpr int kV = 12 * FN + 2;
    interleave_half<FM + (R == 1 ? 2 * FM : 0), kM, kV>();
}

// sum_k c_kj 2^-e_k T[k][j] over this wave's observable rows, per gate column
template <int FM, int FN>
__device__ __forceinline__ void bwdh_epilogue(const f32x16 (&acc)[FM][FN],
                                              const uint64_t IQP_GLOBAL *__restrict__ ctbits,
                                              const double IQP_GLOBAL *__restrict__ sq, int64_t ob,
                                              int64_t jb, int64_t lw, int h, int r, bool active,
                                              float IQP_GLOBAL *__restrict__ gpart, int64_t m_pad) {
    float gs[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) gs[g] = 0.0f;
#pragma unroll
    for (int f = 0; f < FM; ++f) {
        const int64_t k0 = (ob * FM + f) * 32;
        float q[16];
#pragma unroll
        for (int a = 0; a < 16; ++a) q[a] = (float)sq[k0 + acc_row(a, h)];
#pragma unroll
        for (int g = 0; g < FN; ++g) {
            const int64_t j = (jb * FN + g) * 32 + r;
            const uint64_t cw = ctbits[((j >> 5) * lw + (k0 >> 6)) * 32 + (j & 31)];
            const uint32_t c32 = (uint32_t)(cw >> (k0 & 63)) >> (4 * h);
#pragma unroll
            for (int a = 0; a < 16; ++a)
                gs[g] += ((c32 >> (8 * (a >> 2) + (a & 3))) & 1u) ? q[a] * acc[f][g][a] : 0.0f;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int g = 0; g < FN; ++g) {
        const int64_t j = (jb * FN + g) * 32 + r;
        const float v = gs[g] + __shfl_xor(gs[g], 32, 64);
        if (active && h == 0) gpart[ob * m_pad + j] = v;
    }
}

template <int FM, int FN>
__device__ __forceinline__ void bwd_f16f8_body(const BwdArgs &a, int64_t gu, int tid) {
    // one sample word: [f][t][lane] FP16 blocks, then [f][q][lane] FP8 blocks,
    // 16 bytes each; two buffers as in the BF16 form
    constexpr int kUnits = 6 * FM * 64;
    __shared__ u32x4 ls0[kUnits], ls1[kUnits];
    const u32x4 IQP_GLOBAL *__restrict__ shi = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.shi));
    const u32x4 IQP_GLOBAL *__restrict__ slo = reinterpret_cast<const u32x4 IQP_GLOBAL *>(gptr(a.slo));
    const uint64_t IQP_GLOBAL *__restrict__ btbits = gptr(a.btbits);
    const uint64_t IQP_GLOBAL *__restrict__ ctbits = gptr(a.ctbits);
    const int64_t m_pad = a.m_pad, sw = a.s_pad / 64, lw = a.l_pad / 64;
    const int64_t n_jb = m_pad / (32 * FN), n_ob = a.l_pad / (32 * FM);
    const int64_t n_jbg = ceil_div(n_jb, 4);
    int64_t jbg, ob, ks;
    bwd_unit(gu, n_ob, n_jbg, a.obgroup, ob, jbg, ks);
    const int64_t wps = ceil_div(sw, a.ksplits);
    const int64_t w0 = ks * wps, w1 = (w0 + wps < sw) ? w0 + wps : sw;
    float IQP_GLOBAL *__restrict__ gpart = gptr(a.gpart) + ks * n_ob * m_pad;
    const int64_t jb_raw = jbg * 4 + wave_id();
    const bool active = jb_raw < n_jb;
    const int64_t jb = active ? jb_raw : n_jb - 1;
    const int lane = tid & 63;
    const int h = lane >> 5, r = lane & 31;
    const uint32_t ones = in_vgpr(0x3C003C00u);  // +1.0 in FP16, twice
    const int64_t KTs = sw * 4;
    const uint64_t IQP_GLOBAL *bbase = btbits + jb * FN * sw * 32;
    const u32x4 IQP_GLOBAL *sbase_h = shi + ob * FM * KTs * 64;
    const u32x4 IQP_GLOBAL *sbase_8 = slo + ob * FM * sw * 2 * 64;

    f32x16 acc[FM][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int g = 0; g < FN; ++g)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[f][g][e] = 0.0f;

    // staging block b < 4 FM: FP16 limb, f = b / 4, t = b % 4
    //   <- shi[(f * KTs + 4 w + t) * 64 + ln];
    // b >= 4 FM: FP8 limb, f = (b - 4 FM) / 2, q = (b - 4 FM) % 2
    //   <- slo[((f * sw + w) * 2 + q) * 64 + ln]; wave v copies blocks v, v+4, ...
    const int wv = wave_id();
    auto stage = [&](int64_t w, u32x4 *dst) {
#pragma unroll
        for (int k = 0; k < kUnits / 256; ++k) {
            const int b = wv + 4 * k;
            if (b < 4 * FM) {
                const int t = b & 3, f = b >> 2;
                dma16(sbase_h + ((int64_t)f * KTs + 4 * w + t) * 64 + lane, &dst[b * 64]);
            } else {
                const int f = (b - 4 * FM) >> 1, q = (b - 4 * FM) & 1;
                dma16(sbase_8 + (((int64_t)f * sw + w) * 2 + q) * 64 + lane, &dst[b * 64]);
            }
        }
    };
    // every unit has w1 - w0 >= 1 sample words (the host picks the splits)
    stage(w0, ls0);
    if (w0 + 1 < w1) stage(w0 + 1, ls1);
    uint64_t nxt[FN], cur[FN];
#pragma unroll
    for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w0) * 32)[r];
    dma_wait_barrier();
#pragma unroll
    for (int g = 0; g < FN; ++g) cur[g] = nxt[g] >> (8 * h);
    if (w0 + 1 < w1) {
#pragma unroll
        for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w0 + 1) * 32)[r];
    }
    BwdOpsH<FM, FN> opA, opB;
    BwdLoF8<FM, FN> lo;
    lo.m80 = in_vgpr(0x80808080u);
    lo.c38 = in_vgpr(0x38383838u);
    bwdh_expand_a<FM, FN, 0>(opA, ls0, lane);
    bwdh_expand_b<FM, FN, 0>(opA, cur, ones, lo);
    auto word = [&](int64_t w, u32x4 *mine, const u32x4 *other) {
        bwdh_region<FM, FN, 1>(opA, opB, mine, cur, lane, ones, lo, acc);
        bwdh_region<FM, FN, 2>(opB, opA, mine, cur, lane, ones, lo, acc);
        bwdh_region<FM, FN, 3>(opA, opB, mine, cur, lane, ones, lo, acc);
        dma_wait_barrier();
        if (w + 2 < w1) stage(w + 2, mine);
#pragma unroll
        for (int g = 0; g < FN; ++g) cur[g] = nxt[g] >> (8 * h);
        if (w + 2 < w1) {
#pragma unroll
            for (int g = 0; g < FN; ++g) nxt[g] = (bbase + (g * sw + w + 2) * 32)[r];
        }
        // past the last word this expands a stale buffer and is never used
        bwdh_region<FM, FN, 0>(opB, opA, other, cur, lane, ones, lo, acc);
    };
    for (int64_t w = w0; w < w1; w += 2) {
        word(w, ls0, ls1);
        if (w + 1 < w1) word(w + 1, ls1, ls0);
    }
    bwdh_epilogue<FM, FN>(acc, ctbits, gptr(a.sq), ob, jb, lw, h, r, active, gpart, m_pad);
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 2) void phase_bwd_f16f8_kernel(BwdArgs a, int64_t units) {
    const int64_t gu = xcd_remap(blockIdx.x, gridDim.x);
    if (gu >= units) return;  // uniform over the workgroup
    bwd_f16f8_body<FM, FN>(a, gu, (int)threadIdx.x);
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 2) void phase_bwd_f16f8_persistent(
    const BwdArgs *__restrict__ args, const int64_t *__restrict__ off, int np,
    unsigned long long *counter) {
    persistent_loop(off, np, counter,
                    [&](int p, int64_t u) { bwd_f16f8_body<FM, FN>(args[p], u, opaque_tid()); });
}

template <int FN>
constexpr int kI8Waves = FN == 2 ? 2 : 1;

template <int FM, int FN>
__global__ __launch_bounds__(256, kI8Waves<FN>) void phase_bwd_i8_kernel(BwdArgs a, int64_t units) {
    const int64_t gu = xcd_remap(blockIdx.x, gridDim.x);
    if (gu >= units) return;  // uniform over the workgroup
    bwd_i8_body<FM, FN>(a, gu, (int)threadIdx.x);
}

template <int FM, int FN>
__global__ __launch_bounds__(256, kI8Waves<FN>) void phase_bwd_i8_persistent(
    const BwdArgs *__restrict__ args, const int64_t *__restrict__ off, int np,
    unsigned long long *counter) {
    persistent_loop(off, np, counter,
                    [&](int p, int64_t u) { bwd_i8_body<FM, FN>(args[p], u, opaque_tid()); });
}

// Both BF16 backward tiles fit two waves per SIMD (the 64 x 128 one with its
// accumulators in VGPRs).
template <int FM, int FN>
__global__ __launch_bounds__(256, 2) void phase_bwd_bf16_kernel(BwdArgs a, int64_t units) {
    const int64_t gu = xcd_remap(blockIdx.x, gridDim.x);
    if (gu >= units) return;  // uniform over the workgroup
    bwd_bf16_body<FM, FN>(a, gu, (int)threadIdx.x);
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_bwd_f32_kernel(BwdArgs a, int64_t units) {
    const int64_t gu = xcd_remap(blockIdx.x, gridDim.x);
    if (gu >= units) return;
    bwd_f32_body<FM, FN>(a, gu, (int)threadIdx.x);
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 2) void phase_bwd_bf16_persistent(
    const BwdArgs *__restrict__ args, const int64_t *__restrict__ off, int np,
    unsigned long long *counter) {
    persistent_loop(off, np, counter, [&](int p, int64_t u) { bwd_bf16_body<FM, FN>(args[p], u, opaque_tid()); });
}

template <int FM, int FN>
__global__ __launch_bounds__(256, 1) void phase_bwd_f32_persistent(
    const BwdArgs *__restrict__ args, const int64_t *__restrict__ off, int np,
    unsigned long long *counter) {
    persistent_loop(off, np, counter, [&](int p, int64_t u) { bwd_f32_body<FM, FN>(args[p], u, opaque_tid()); });
}

template <int FM, int FN>
static hipError_t bwd_dispatch(const LaunchCtx &lc, int prec, const BwdArgs &a) {
    const int64_t units = bwd_units(a, FM, FN);
    if (units <= 0) return hipSuccess;
    if (units > kMaxBlocks) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)units);
    if (prec == 1)
        hipLaunchKernelGGL((phase_bwd_bf16_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, a, units);
    else if (prec == 3)
        hipLaunchKernelGGL((phase_bwd_i8_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, a, units);
    else if (prec == 4)
        hipLaunchKernelGGL((phase_bwd_f16f8_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, a,
                           units);
    else
        hipLaunchKernelGGL((phase_bwd_f32_kernel<FM, FN>), grid, dim3(256), 0, lc.stream, a, units);
    return hipGetLastError();
}

// the 128 x 64 wave tile, FP16 + FP8 form only
template <int FM, int FN>
static hipError_t bwd_f16f8_dispatch(const LaunchCtx &lc, const BwdArgs &a) {
    const int64_t units = bwd_units(a, FM, FN);
    if (units <= 0) return hipSuccess;
    if (units > kMaxBlocks) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((phase_bwd_f16f8_kernel<FM, FN>), dim3((unsigned)units), dim3(256), 0,
                       lc.stream, a, units);
    return hipGetLastError();
}

// (a 128x128 backward tile cannot hold the double-buffered pipeline in 512
// registers without spilling, so it is not offered)
hipError_t launch_phase_bwd(const LaunchCtx &lc, int prec, int fm, int fn, const BwdArgs &a) {
    hipEvent_t ev;
    timed_begin(lc, KF_BWD, &ev);
    hipError_t e;
    if (fm == 2 && fn == 2) e = bwd_dispatch<2, 2>(lc, prec, a);
    else if (fm == 2 && fn == 4) e = bwd_dispatch<2, 4>(lc, prec, a);
    else if (fm == 4 && fn == 2 && prec == 4) e = bwd_f16f8_dispatch<4, 2>(lc, a);
    else e = hipErrorInvalidValue;
    timed_end(lc, KF_BWD, ev);
    return e;
}

template <int FM, int FN>
static hipError_t bwd_persistent(const LaunchCtx &lc, int prec, const BwdArgs *args,
                                 const int64_t *off, int np, unsigned long long *counter,
                                 int grid) {
    if (prec == 1)
        hipLaunchKernelGGL((phase_bwd_bf16_persistent<FM, FN>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    else if (prec == 3)
        hipLaunchKernelGGL((phase_bwd_i8_persistent<FM, FN>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    else if (prec == 4)
        hipLaunchKernelGGL((phase_bwd_f16f8_persistent<FM, FN>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    else
        hipLaunchKernelGGL((phase_bwd_f32_persistent<FM, FN>), dim3(grid), dim3(256), 0,
                           lc.stream, args, off, np, counter);
    return hipGetLastError();
}

hipError_t launch_phase_bwd_persistent(const LaunchCtx &lc, int prec, int fm, int fn,
                                       const BwdArgs *args, const int64_t *off, int np,
                                       unsigned long long *counter, int grid) {
    if (grid < 1 || np < 1) return hipErrorInvalidValue;
    hipEvent_t ev;
    timed_begin(lc, KF_BWD, &ev);
    hipError_t e;
    if (fm == 2 && fn == 2) e = bwd_persistent<2, 2>(lc, prec, args, off, np, counter, grid);
    else if (fm == 2 && fn == 4) e = bwd_persistent<2, 4>(lc, prec, args, off, np, counter, grid);
    else if (fm == 4 && fn == 2 && prec == 4) {
        hipLaunchKernelGGL((phase_bwd_f16f8_persistent<4, 2>), dim3(grid), dim3(256), 0, lc.stream,
                           args, off, np, counter);
        e = hipGetLastError();
    } else e = hipErrorInvalidValue;
    timed_end(lc, KF_BWD, ev);
    return e;
}

// Resident workgroups of a kernel on the current device.
template <typename K>
static int resident_grid(K kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess)
        return 0;
    return (per_cu > 0 ? per_cu : 1) * cus;
}

int persistent_grid(bool fwd, int prec, int fm, int fn) {
#define IQP_GRID3(K2, K3, KF) \
    (prec == 1 ? resident_grid(K2) : prec == 3 ? resident_grid(K3) : resident_grid(KF))
    if (fwd && prec == 4) prec = 1;  // the same forward kernels
    if (!fwd && prec == 4) {
        if (fm == 2 && fn == 2) return resident_grid(phase_bwd_f16f8_persistent<2, 2>);
        if (fm == 2 && fn == 4) return resident_grid(phase_bwd_f16f8_persistent<2, 4>);
        if (fm == 4 && fn == 2) return resident_grid(phase_bwd_f16f8_persistent<4, 2>);
        return 0;
    }
    if (fwd) {
        if (fm == 4 && fn == 4)
            return IQP_GRID3((phase_fwd_bf16_persistent<4, 4, 2>),
                             (phase_fwd_bf16_persistent<4, 4, 3>), (phase_fwd_f32_persistent<4, 4>));
        if (fm == 2 && fn == 2)
            return IQP_GRID3((phase_fwd_bf16_persistent<2, 2, 2>),
                             (phase_fwd_bf16_persistent<2, 2, 3>), (phase_fwd_f32_persistent<2, 2>));
        if (fm == 2 && fn == 4)
            return IQP_GRID3((phase_fwd_bf16_persistent<2, 4, 2>),
                             (phase_fwd_bf16_persistent<2, 4, 3>), (phase_fwd_f32_persistent<2, 4>));
        return 0;
    }
    if (fm == 2 && fn == 2)
        return IQP_GRID3((phase_bwd_bf16_persistent<2, 2>), (phase_bwd_i8_persistent<2, 2>),
                         (phase_bwd_f32_persistent<2, 2>));
    if (fm == 2 && fn == 4)
        return IQP_GRID3((phase_bwd_bf16_persistent<2, 4>), (phase_bwd_i8_persistent<2, 4>),
                         (phase_bwd_f32_persistent<2, 4>));
#undef IQP_GRID3
    return 0;
}

__global__ __launch_bounds__(64) void reset_counters_kernel(unsigned long long *c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0ull;
}

hipError_t launch_reset_counters(const LaunchCtx &lc, unsigned long long *c, int n) {
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, lc.stream, c, n);
    return hipGetLastError();
}

__device__ __forceinline__ void grad_reduce_body(const GradArgs &a, int64_t blk) {
    const int64_t j = blk * 256 + threadIdx.x;
    if (j >= a.m) return;
    double acc = 0.0;
    for (int64_t p = 0; p < a.n_parts; ++p) acc += (double)gptr(a.gpart)[p * a.m_pad + j];
    gptr(a.grad)[j] = -2.0 * acc;
}

hipError_t launch_grad_reduce(const LaunchCtx &lc, const GradArgs &a) {
    return plain_launch<GradArgs, grad_reduce_body>(lc, KF_GRAD, a, blocks_of(a));
}

// ---------------------------------------------------------------------------
// Batched launches of the per-step bodies.
template <typename A, void (*F)(const A &, int64_t)>
static void batched(const LaunchCtx &lc, const void *args, const int64_t *off, int np,
                    int64_t total) {
    hipLaunchKernelGGL((batched_kernel<A, F>), dim3((unsigned)total), dim3(256), 0, lc.stream,
                       static_cast<const A *>(args), off, np);
}

hipError_t launch_batched(const LaunchCtx &lc, int kind, const void *args, const int64_t *off,
                          int np, int64_t total) {
    if (total <= 0) return hipSuccess;
    if (total > kMaxBlocks || np < 1) return hipErrorInvalidConfiguration;
    static const int family[SK_COUNT] = {KF_THETA, KF_PARITY,  KF_PARITY,  KF_PARITY,
                                         KF_PARITY, KF_EPI,    KF_FIN,     KF_WEIGHTS,
                                         KF_WEIGHTS, KF_GRAD,  KF_PARITY};
    if (kind < 0 || kind >= SK_COUNT) return hipErrorInvalidValue;
    hipEvent_t ev;
    timed_begin(lc, family[kind], &ev);
    switch (kind) {
        case SK_THETA: batched<ThetaArgs, theta_prep_body>(lc, args, off, np, total); break;
        case SK_BITSLICE: batched<BitsliceArgs, bitslice_body>(lc, args, off, np, total); break;
        case SK_PARITY0: batched<ParityArgs, parity_bs_body<0>>(lc, args, off, np, total); break;
        case SK_PARITY1: batched<ParityArgs, parity_bs_body<1>>(lc, args, off, np, total); break;
        case SK_PARITY2: batched<ParityArgs, parity_bs_body<2>>(lc, args, off, np, total); break;
        case SK_EPI: batched<EpiArgs, epilogue_body>(lc, args, off, np, total); break;
        case SK_FIN: batched<FinArgs, finalize_body>(lc, args, off, np, total); break;
        case SK_COEF: batched<CoefArgs, coef_plain_body>(lc, args, off, np, total); break;
        case SK_WEIGHTS: batched<WeightsArgs, weights_body>(lc, args, off, np, total); break;
        case SK_GRAD: batched<GradArgs, grad_reduce_body>(lc, args, off, np, total); break;
        case SK_SUPPORT: batched<SupportArgs, support_body>(lc, args, off, np, total); break;
    }
    hipError_t e = hipGetLastError();
    timed_end(lc, family[kind], ev);
    return e;
}

// ---------------------------------------------------------------------------
// MMD^2 chain. data_stats: pstat[2k] = sum_n (-1)^{a_k . x_n} and
// pstat[2k+1] = p_k = that sum / N (eq. mmd_estimate's data term), counted
// directly by AND + popcount: both operands may be dense (the observables of
// a narrow kernel bandwidth, Bernoulli training strings), where bit columns
// would not pay. A wave takes kStatOps observables, read as scalars; lane n
// walks data rows n, n + 64, ...; the per-lane odd counts are summed across
// the wave in a fixed butterfly order (integers: exact).
constexpr int kStatOps = 8;

__global__ __launch_bounds__(256) void data_stats_kernel(const uint64_t *__restrict__ ops,
                                                         int64_t l,
                                                         const uint64_t *__restrict__ data,
                                                         int64_t N, int W,
                                                         double *__restrict__ pstat) {
    const int lane = threadIdx.x & 63;
    const int64_t k0 = ((int64_t)blockIdx.x * 4 + wave_id()) * kStatOps;
    if (k0 >= l) return;  // uniform over the wave
    int cnt[kStatOps];
#pragma unroll
    for (int i = 0; i < kStatOps; ++i) cnt[i] = 0;
    for (int64_t n0 = 0; n0 < N; n0 += 64) {
        const int64_t n = n0 + lane;
        const bool live = n < N;
        uint32_t par[kStatOps];
#pragma unroll
        for (int i = 0; i < kStatOps; ++i) par[i] = 0;
        for (int w = 0; w < W; ++w) {
            const uint64_t x = live ? data[n * W + w] : 0ull;
#pragma unroll
            for (int i = 0; i < kStatOps; ++i) {
                const uint64_t av = (k0 + i < l) ? ops[(k0 + i) * W + w] : 0ull;
                par[i] ^= (uint32_t)__popcll(av & x);
            }
        }
#pragma unroll
        for (int i = 0; i < kStatOps; ++i) cnt[i] += (int)(par[i] & 1u);
    }
#pragma unroll
    for (int i = 0; i < kStatOps; ++i) {
        int c = cnt[i];
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) c += __shfl_xor(c, s, 64);
        cnt[i] = c;
    }
#pragma unroll
    for (int i = 0; i < kStatOps; ++i) {
        if (lane == i && k0 + i < l) {
            const double sv = (double)(N - 2 * (int64_t)cnt[i]);
            pstat[2 * (k0 + i)] = sv;
            pstat[2 * (k0 + i) + 1] = sv / (double)N;
        }
    }
}

hipError_t launch_data_stats(const LaunchCtx &lc, const uint64_t *ops, int64_t l,
                             const uint64_t *data, int64_t N, int W, double *pstat) {
    const int64_t blocks = ceil_div(l, 4 * kStatOps);
    if (blocks > kMaxBlocks) return hipErrorInvalidConfiguration;
    hipEvent_t ev;
    timed_begin(lc, KF_MMD, &ev);
    hipLaunchKernelGGL(data_stats_kernel, dim3((unsigned)blocks), dim3(256), 0, lc.stream, ops,
                       l, data, N, W, pstat);
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
                                                       double *__restrict__ coef, double *sq,
                                                       int32_t *nf) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= l) return;
    const double S = (double)s;
    const double p = pstat[2 * k + 1], sc = rowsum[2 * k];
    double al, be;
    if (unbiased) {
        const double d = S * (S - 1.0);
        al = w[k] * (-2.0 * p / S + 2.0 * sc / d);
        be = -2.0 * w[k] / d;
    } else {
        al = w[k] * 2.0 * (sc / S - p) / S;
        be = 0.0;
    }
    coef[2 * k] = al;
    coef[2 * k + 1] = be;
    coef_rowscale(sq, nf, k, al, be);
}

hipError_t launch_coef_mmd(const LaunchCtx &lc, const double *pstat, const double *rowsum,
                           const double *op_weight, int64_t l, int64_t s, int unbiased,
                           double *coef, double *sq, int32_t *nf) {
    hipEvent_t ev;
    timed_begin(lc, KF_MMD, &ev);
    hipLaunchKernelGGL(coef_mmd_kernel, dim3((unsigned)ceil_div(l, 256)), dim3(256), 0,
                       lc.stream, pstat, rowsum, op_weight, l, s, unbiased, coef, sq, nf);
    hipError_t e = hipGetLastError();
    timed_end(lc, KF_MMD, ev);
    return e;
}

// ---------------------------------------------------------------------------
// Stochastic bitflip circuits (Prop. 3, eq. expval_bitflip): the exact
// <Z_{a_k}> = prod_{j in J_k} cos(2 theta_j) over the generators that
// anticommute with Z_{a_k}, all in FP64. The product is kept as a sum of
// logarithms, a sign parity and a count of exact-zero factors, so that the
// product leaving out any one factor (the gradient) needs no division.
//   enc_j = copysign(-log|cos 2 theta_j|, cos 2 theta_j)  (+-inf for a zero)
__device__ __forceinline__ void bitflip_prep_body(const BitflipPrepArgs &a, int64_t blk) {
    const int64_t j = blk * 256 + threadIdx.x;
    if (j >= a.m) return;
    const double c = cos(2.0 * gptr(a.theta)[j]);
    gptr(a.enc)[j] = copysign(c == 0.0 ? (double)INFINITY : -log(fabs(c)), c);
}

hipError_t launch_bitflip_prep(const LaunchCtx &lc, const BitflipPrepArgs &a) {
    return plain_launch<BitflipPrepArgs, bitflip_prep_body>(lc, KF_THETA, a, blocks_of(a));
}

// One wave per observable k: lane v walks gate words v, v + 64, ... of the
// tiled32 row of C and sums the encoded factors in gate order; the lanes'
// (sum, sign parity, zero count) are then combined by a fixed butterfly.
// stat[k] = (S_k = sum of log|c| over non-zero factors, sign of those
// factors times 1 + min(zero factors, 2)); mean[k] = the product.
__device__ __forceinline__ void bitflip_fwd_body(const BitflipFwdArgs &a, int64_t blk) {
    const int64_t k = blk * 4 + wave_id();
    if (k >= a.l) return;  // uniform over the wave
    const int lane = threadIdx.x & 63;
    const uint64_t IQP_GLOBAL *crow = gptr(a.cbits) + (k >> 5) * a.mw * 32 + (k & 31);
    const double IQP_GLOBAL *enc = gptr(a.enc);
    double S = 0.0;
    int neg = 0, zeros = 0;
    for (int64_t w = lane; w < a.mw; w += 64) {
        uint64_t bits = crow[w * 32];
        while (bits) {
            const int64_t j = w * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
            const double e = enc[j];
            if (isinf(e)) {
                ++zeros;
            } else {
                S -= fabs(e);
                neg ^= (int)signbit(e) & 1;
            }
        }
    }
#pragma unroll
    for (int st = 32; st >= 1; st >>= 1) {
        S += __shfl_xor(S, st, 64);
        neg ^= __shfl_xor(neg, st, 64);
        zeros += __shfl_xor(zeros, st, 64);
    }
    if (lane == 0) {
        const double sgn = neg ? -1.0 : 1.0;
        gptr(a.mean)[k] = zeros ? 0.0 : sgn * exp(S);
        if (a.stderr_) gptr(a.stderr_)[k] = 0.0;
        double IQP_GLOBAL *st = gptr(a.stat) + 2 * k;
        st[0] = S;
        st[1] = sgn * (double)(zeros < 2 ? 1 + zeros : 3);
    }
}

hipError_t launch_bitflip_fwd(const LaunchCtx &lc, const BitflipFwdArgs &a) {
    return plain_launch<BitflipFwdArgs, bitflip_fwd_body>(lc, KF_FWD, a, blocks_of(a));
}

// One lane per gate j: walks the transposed tiled32 row of C^T (observable
// words) and sums u_k times the product over J_k without factor j:
//   c_j = 0:  (zero count of k is 1) ? sign_k exp(S_k) : 0
//   else:     (no zero factor in k) ? sign_k sgn(c_j) exp(S_k - log|c_j|) : 0
// then dtheta_j = -2 sin(2 theta_j) times that sum.
__device__ __forceinline__ void bitflip_grad_body(const BitflipGradArgs &a, int64_t blk) {
    const int64_t j = blk * 256 + threadIdx.x;
    if (j >= a.m) return;
    const uint64_t IQP_GLOBAL *crow = gptr(a.ctbits) + (j >> 5) * a.lw * 32 + (j & 31);
    const double IQP_GLOBAL *stat = gptr(a.stat);
    const double IQP_GLOBAL *u = gptr(a.grad_mean);
    const double e = gptr(a.enc)[j];
    const bool jzero = isinf(e);
    const double Lj = -fabs(e), sj = signbit(e) ? -1.0 : 1.0;
    double acc = 0.0;
    for (int64_t w = 0; w < a.lw; ++w) {
        uint64_t bits = crow[w * 32];
        while (bits) {
            const int64_t k = w * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
            const double S = stat[2 * k], code = stat[2 * k + 1];
            const double z = fabs(code) - 1.0;  // zero factors: 0, 1, or 2 for >= 2
            const double sk = code < 0.0 ? -1.0 : 1.0;
            double p = 0.0;
            if (jzero) p = (z == 1.0) ? sk * exp(S) : 0.0;
            else p = (z == 0.0) ? sk * sj * exp(S - Lj) : 0.0;
            acc += u[k] * p;
        }
    }
    gptr(a.grad)[j] = -2.0 * sin(2.0 * gptr(a.theta)[j]) * acc;
}

hipError_t launch_bitflip_grad(const LaunchCtx &lc, const BitflipGradArgs &a) {
    return plain_launch<BitflipGradArgs, bitflip_grad_body>(lc, KF_BWD, a, blocks_of(a));
}

}  // namespace iqp
