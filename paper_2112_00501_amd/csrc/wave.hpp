// Exchanges among the 64 lanes of one wave held in registers: DPP moves
// inside each row of 16 lanes and the gfx950 permlane swaps between rows.
// None of them goes through LDS, so they neither queue behind LDS traffic nor
// wait on it.  Every lane of the wave must take part.
#pragma once

#include <hip/hip_runtime.h>

namespace cs {

namespace wave_detail {

// DPP controls: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror
enum { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

template <int CTRL>
__device__ __forceinline__ int dpp(int x) {
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(dpp<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)dpp<CTRL>((int)(unsigned)b), hi = (unsigned)dpp<CTRL>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v_permlane32_swap on (a, b): afterwards a holds lanes 0..31 of a then lanes
// 0..31 of b, and b holds lanes 32..63 of a then lanes 32..63 of b.
// v_permlane16_swap does the same with rows of 16 inside each half of 32.
template <int W>
__device__ __forceinline__ void swap_u32(unsigned& a, unsigned& b) {
    if constexpr (W == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}

// v of this lane plus v of the lane W away (lane ^ W), the same bits in both
template <int W>
__device__ __forceinline__ float cross_add(float v) {
    unsigned a = __float_as_uint(v), b = a;
    swap_u32<W>(a, b);
    return __uint_as_float(a) + __uint_as_float(b);
}
template <int W>
__device__ __forceinline__ double cross_add(double v) {
    const unsigned long long x = (unsigned long long)__double_as_longlong(v);
    unsigned alo = (unsigned)x, blo = alo, ahi = (unsigned)(x >> 32), bhi = ahi;
    swap_u32<W>(alo, blo);
    swap_u32<W>(ahi, bhi);
    const double a = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
    const double b = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
    return a + b;
}

}  // namespace wave_detail

// Sum over the wave; every lane receives bitwise the same total.  Within a
// row: neighbours, pairs, mirrored halves of 8, mirrored halves of 16; then
// row 0 + row 1 and row 2 + row 3, then the two halves.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    using namespace wave_detail;
    v += dpp_move<DPP_XOR1>(v);
    v += dpp_move<DPP_XOR2>(v);
    v += dpp_move<DPP_HALF_MIRROR>(v);
    v += dpp_move<DPP_MIRROR>(v);
    v = cross_add<16>(v);
    return cross_add<32>(v);
}

// Lane pairs (i, i + 32), i < 32.  Both lanes of a pair receive from_lo = v
// of lane i and from_hi = v of lane i + 32.
__device__ __forceinline__ void pair_share(float v, float& from_lo, float& from_hi) {
    unsigned a = __float_as_uint(v), b = a;
    wave_detail::swap_u32<32>(a, b);
    from_lo = __uint_as_float(a);
    from_hi = __uint_as_float(b);
}

// Lane pairs (i, i + 32), i < 32: lane i receives u(i) + u(i + 32) and lane
// i + 32 receives l(i) + l(i + 32).
__device__ __forceinline__ float pair_split_sum(float u, float l) {
    unsigned a = __float_as_uint(u), b = __float_as_uint(l);
    wave_detail::swap_u32<32>(a, b);
    return __uint_as_float(a) + __uint_as_float(b);
}

}  // namespace cs
