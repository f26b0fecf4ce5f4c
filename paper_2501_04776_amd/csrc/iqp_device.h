// Device-side helpers shared by the kernel sources: vector types, the 2 pi
// constants of the phase reduction, global-address-space pointers, wave and
// lane utilities, and the plain / batched launch templates of the per-step
// body functions.
#pragma once

#include "iqp_internal.h"

#include <math.h>

namespace iqp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x8 __attribute__((ext_vector_type(8)));
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

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

// A pointer read from an argument struct in memory is generic (flat) to the
// compiler. The kernels hold such pointers in the global address space
// (`glb<T>`), so every access through them is a global memory instruction,
// which, unlike a flat one, never waits on LDS or scalar-memory counters.
#define IQP_GLOBAL __attribute__((address_space(1)))
template <typename T>
using glb = T IQP_GLOBAL *;
template <typename T>
__device__ __forceinline__ glb<T> gptr(T *p) {
    return (glb<T>)p;
}

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ int64_t uniform64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Problem p of a batch owns blocks off[p] .. off[p+1]-1 (off[0] = 0, b <
// off[np]); empty problems have off[p] = off[p+1] and are skipped.
__device__ __forceinline__ int find_slot(const int64_t *__restrict__ off, int np, int64_t b) {
    int lo = 0, hi = np;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename A, void (*F)(const A &, int64_t)>
__global__ __launch_bounds__(256) void plain_kernel(A a) {
    F(a, (int64_t)blockIdx.x);
}

template <typename A, void (*F)(const A &, int64_t)>
__global__ __launch_bounds__(256) void batched_kernel(const A *__restrict__ args,
                                                      const int64_t *__restrict__ off, int np) {
    const int64_t b = (int64_t)blockIdx.x;
    const int p = find_slot(off, np, b);
    const A a = args[p];
    F(a, b - off[p]);
}

// 256-thread blocks: a grid stays below 2^32 work-items.
constexpr int64_t kMaxBlocks = ((int64_t)1 << 24) - 1;

template <typename A, void (*F)(const A &, int64_t)>
static hipError_t plain_launch(const LaunchCtx &lc, int family, const A &a, int64_t blocks) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > kMaxBlocks) return hipErrorInvalidConfiguration;
    hipEvent_t ev;
    timed_begin(lc, family, &ev);
    hipLaunchKernelGGL((plain_kernel<A, F>), dim3((unsigned)blocks), dim3(256), 0, lc.stream, a);
    hipError_t e = hipGetLastError();
    timed_end(lc, family, ev);
    return e;
}

// threadIdx.x, hidden from loop-invariant code motion: a persistent kernel
// then recomputes lane-derived values per work unit instead of keeping them
// live across units (the contraction bodies need every register).
__device__ __forceinline__ int opaque_tid() {
    int t = (int)threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// Work-queue loop of the persistent kernels: the workgroup takes the next
// unit from `counter` until the units run out. Every workgroup reaches the
// exit, whatever the order in which units are taken.
template <typename Body>
__device__ __forceinline__ void persistent_loop(const int64_t *__restrict__ off, int np,
                                                unsigned long long *counter, Body body) {
    __shared__ unsigned long long slot;
    const int64_t total = off[np];
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(counter, 1ull);
        __syncthreads();
        const int64_t u = uniform64(slot);
        __syncthreads();
        if (u >= total) break;
        const int p = find_slot(off, np, u);
        body(p, u - off[p]);
    }
}


// 64x64 bit transpose across the lanes of a wave.
// transpose64: lane r holds row r of a 64x64 bit matrix (bit c = column c)
// and receives row r of its transpose. Six butterfly stages: at block size k
// lanes r and r^k swap the off-diagonal k x k blocks of their 2k x 2k block
// (the lane with bit k clear keeps its low blocks and takes the partner's
// low blocks shifted up; the other keeps its high blocks and takes the
// partner's high blocks shifted down). The lane exchanges use gfx950's
// cross-lane moves rather than LDS permutes: the 32- and 16-lane stages swap
// whole registers between the wave's halves / alternate 16-lane rows; in the
// stages 8, 2 and 1 apart a DPP move fetches the partner's dword, 4 apart a
// swizzle. There each lane first rotates its dword right by k (left by k
// where its lane index has the bit of value k set), so the partner's blocks
// arrive where they belong, and a bit-field insert keeps its own blocks.
// 35 VALU instructions and 2 swizzles per transpose.
template <int K>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
    if constexpr (K == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
    if constexpr (K == 4) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);
    if constexpr (K == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    if constexpr (K == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    return v;
}

template <int K, int LOGK, uint32_t M>
__device__ __forceinline__ void small_stage(uint32_t &lo, uint32_t &hi, int lane) {
    const bool up = (lane >> LOGK) & 1;
    const uint32_t keep = up ? ~M : M;
    const uint32_t amt = up ? 32 - K : K;
    const uint32_t rl = lane_xor<K>(__builtin_amdgcn_alignbit(lo, lo, amt));
    const uint32_t rh = lane_xor<K>(__builtin_amdgcn_alignbit(hi, hi, amt));
    lo = (lo & keep) | (rl & ~keep);
    hi = (hi & keep) | (rh & ~keep);
}

__device__ __forceinline__ uint64_t transpose64(uint64_t x, int lane) {
    uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
    {  // 32 apart: lanes 32..63 take the high dword of lanes 0..31 as their
       // low dword, lanes 0..31 the low dword of lanes 32..63 as their high
        const auto r = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
        lo = r[0];
        hi = r[1];
    }
    {  // 16 apart: gather the low and the high 16-bit halves of the two
       // dwords, swap the odd rows of the first with the even rows of the
       // second, spread them back
        uint32_t a = (lo & 0xFFFFu) | (hi << 16), b = (lo >> 16) | (hi & 0xFFFF0000u);
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
        lo = (a & 0xFFFFu) | (b << 16);
        hi = (a >> 16) | (b & 0xFFFF0000u);
    }
    small_stage<8, 3, 0x00FF00FFu>(lo, hi, lane);
    small_stage<4, 2, 0x0F0F0F0Fu>(lo, hi, lane);
    small_stage<2, 1, 0x33333333u>(lo, hi, lane);
    small_stage<1, 0, 0x55555555u>(lo, hi, lane);
    return ((uint64_t)hi << 32) | lo;
}

// Sum of one double per thread over a 256-thread block, in a fixed order.
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

}  // namespace iqp
