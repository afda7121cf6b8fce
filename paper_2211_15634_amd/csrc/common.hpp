// Device-side building blocks shared by the diff3d kernels: storage/compute
// types of each dtype, BF16 conversions, the Philox4x32-10 generator behind
// stochastic rounding, vector loads/stores and the XCD-aware block mapping.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "diff3d.h"

namespace diff3d {

// ----------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of the 4x32 Philox S-box with the
// Weyl key schedule.  Counter-based, so every (seed, step, point) gets its
// own random word without state.
struct u32x4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)M0 * c.x;
        const uint64_t p1 = (uint64_t)M1 * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// Random bits for point `idx` at step `step`: one Philox call covers the 8
// consecutive points idx & ~7 (the two 16-bit halves of its four 32-bit
// words), so every kernel variant draws the same bits for the same point.
struct SrState {
    uint32_t k0, k1;     // seed
    uint32_t s0, s1;     // step index
};

__device__ inline u32x4 sr_block(const SrState& st, size_t group)
{
    return philox4x32_10(u32x4{(uint32_t)group, (uint32_t)(group >> 32), st.s0, st.s1}, st.k0, st.k1);
}

// The 16 random bits of point j = idx & 7, placed in the upper half of the
// word (the half the rounding instruction reads).
__device__ inline uint32_t sr_word(const u32x4& r, unsigned j)
{
    const uint32_t w = (j >> 1) == 0 ? r.x : (j >> 1) == 1 ? r.y : (j >> 1) == 2 ? r.z : r.w;
    return (j & 1) ? (w & 0xFFFF0000u) : (w << 16);
}

// ----------------------------------------------------------------- BF16
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ inline float bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

// Round to nearest even (v_cvt_pk_bf16_f32 on gfx950; NaN stays NaN).
__device__ inline uint16_t f32_to_bf16_rne(float f)
{
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

// Stochastic rounding (v_cvt_sr_bf16_f32): the instruction adds the upper 16
// bits of `rnd` below the kept mantissa and truncates, so a value rounds up
// with probability equal to the discarded fraction of an ulp (unbiased in
// expectation); NaN and infinities are kept.
__device__ inline uint16_t f32_to_bf16_sr(float f, uint32_t rnd)
{
    const bf16x2_t v = __builtin_amdgcn_cvt_sr_bf16_f32(bf16x2_t{}, f, rnd, false);
    return (uint16_t)(__builtin_bit_cast(uint32_t, v) & 0xFFFFu);
}

// ----------------------------------------------------------------- dtypes
// Storage type S, compute type C, and the conversion at load and store.
template <int DT>
struct Traits;

template <>
struct Traits<DIFF3D_F64> {
    using S = double;
    using C = double;
    static constexpr bool sr = false;
    __device__ static C load(S v) { return v; }
    __device__ static S store(C v, uint32_t) { return v; }
};

template <>
struct Traits<DIFF3D_F32> {
    using S = float;
    using C = float;
    static constexpr bool sr = false;
    __device__ static C load(S v) { return v; }
    __device__ static S store(C v, uint32_t) { return v; }
};

template <>
struct Traits<DIFF3D_BF16> {
    using S = uint16_t;
    using C = float;
    static constexpr bool sr = true;
    __device__ static C load(S v) { return bf16_to_f32(v); }
    __device__ static S store(C v, uint32_t rnd) { return f32_to_bf16_sr(v, rnd); }
};

template <>
struct Traits<DIFF3D_BF16_RNE> {
    using S = uint16_t;
    using C = float;
    static constexpr bool sr = false;
    __device__ static C load(S v) { return bf16_to_f32(v); }
    __device__ static S store(C v, uint32_t) { return f32_to_bf16_rne(v); }
};

// ----------------------------------------------------------------- vectors
// V consecutive elements of S moved as one naturally aligned load/store of
// V*sizeof(S) bytes (2, 4, 8 or 16).  NT selects the non-temporal form
// (streaming data that is not re-read by this launch).
typedef unsigned int u32v2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32v4 __attribute__((ext_vector_type(4)));
template <int BYTES>
struct RawVec;
template <> struct RawVec<2> { using T = uint16_t; };
template <> struct RawVec<4> { using T = uint32_t; };
template <> struct RawVec<8> { using T = u32v2; };
template <> struct RawVec<16> { using T = u32v4; };

template <class S, int V, bool NT = false>
__device__ inline void vload(const S* p, S (&out)[V])
{
    using R = typename RawVec<V * sizeof(S)>::T;
    R r;
    if (NT)
        r = __builtin_nontemporal_load(reinterpret_cast<const R*>(p));
    else
        r = *reinterpret_cast<const R*>(p);
    __builtin_memcpy(out, &r, sizeof(R));
}

template <class S, int V, bool NT = false>
__device__ inline void vstore(S* p, const S (&in)[V])
{
    using R = typename RawVec<V * sizeof(S)>::T;
    R r;
    __builtin_memcpy(&r, in, sizeof(R));
    if (NT)
        __builtin_nontemporal_store(r, reinterpret_cast<R*>(p));
    else
        *reinterpret_cast<R*>(p) = r;
}

// ----------------------------------------------------------------- mapping
// Workgroups of a 1-D grid are dispatched round-robin over the 8 XCDs
// (block b runs on XCD b % 8).  Returning a contiguous range of logical
// tiles to each XCD keeps tiles that share halo rows on one L2.
constexpr int kNumXcd = 8;

__device__ inline unsigned xcd_remap(unsigned b, unsigned nb)
{
    const unsigned per = nb / kNumXcd, rem = nb % kNumXcd;
    const unsigned xcd = b % kNumXcd, j = b / kNumXcd;
    return xcd * per + (xcd < rem ? xcd : rem) + j;
}

// The value of the next (UP) or previous lane of the wave (DPP wave shift by
// one lane; the end lanes read zero).
template <class T, bool UP>
__device__ inline T lane_shift(T v)
{
    constexpr int ctrl = UP ? 0x130 : 0x138;     // wave_shl:1 / wave_shr:1
    if constexpr (sizeof(T) == 8) {
        const int2 w = __builtin_bit_cast(int2, v);
        const int lo = __builtin_amdgcn_mov_dpp(w.x, ctrl, 0xF, 0xF, true);
        const int hi = __builtin_amdgcn_mov_dpp(w.y, ctrl, 0xF, 0xF, true);
        return __builtin_bit_cast(T, int2{lo, hi});
    } else {
        const int w = __builtin_bit_cast(int, v);
        return __builtin_bit_cast(T, __builtin_amdgcn_mov_dpp(w, ctrl, 0xF, 0xF, true));
    }
}

// LDS-only workgroup barrier: waits for this wave's LDS traffic and meets
// the other waves, without waiting for outstanding global loads (those are
// software-pipelined across the barrier).
__device__ inline void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

}  // namespace diff3d
