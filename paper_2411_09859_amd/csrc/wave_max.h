// Wave-level helpers shared by the panel and batched kernels: reading a
// double from one lane, the largest key over a wave with DPP moves (no
// LDS), and FP64 FMAs whose second factor is broadcast inside 16-lane rows.
#pragma once

#include <hip/hip_runtime.h>

namespace skl {

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One step of a 32-bit unsigned max over lanes with a DPP data movement
// (row_mask selects the rows that take the moved value; others keep theirs).
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_max_u32(unsigned x)
{
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, ROWS, 0xf, false);
    return (o > x) ? o : x;
}

// Largest value over lanes 0 .. CL-1 (CL = 16, 32 or 64), as a uniform
// value: pairs and quads (quad_perm), 8 and 16 lanes (row half mirror, row
// mirror), then lane 15 of each row into the next and lane 31 into the upper
// half (row_bcast 15 / 31), the maximum ending in lane 0 (CL = 16), 31 or
// 63.  All VALU, no LDS.
template <int CL>
__device__ __forceinline__ unsigned lanes_max_u32(unsigned x)
{
    static_assert(CL == 16 || CL == 32 || CL == 64, "lane count");
    x = dpp_max_u32<0xb1, 0xf>(x);
    x = dpp_max_u32<0x4e, 0xf>(x);
    x = dpp_max_u32<0x141, 0xf>(x);
    x = dpp_max_u32<0x140, 0xf>(x);
    if constexpr (CL == 16)
        return (unsigned)__builtin_amdgcn_readlane((int)x, 0);
    x = dpp_max_u32<0x142, 0xa>(x);
    if constexpr (CL == 32)
        return (unsigned)__builtin_amdgcn_readlane((int)x, 31);
    x = dpp_max_u32<0x143, 0xc>(x);
    return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

// acc[i & 3] += Lr[Q0 + i] * h[i] for the slots i < N of one 16-slot block,
// h[i] being lane i of the row of hb: one FP64 FMA per slot with the row
// broadcast as its DPP source operand (64-bit VALU operations accept DPP
// with row_newbcast only).  The first of a block waits the two wait states a
// DPP read needs after a VALU write of its source; volatile keeps that one
// first.  Same product and rounding as fma(Lr, h, acc).  Every lane of the
// wave must be active (each reads its row's source lane).
template <int I, int N, int Q0, int LEN>
__device__ __forceinline__ void bcast_fma(double (&acc)[4], const double (&Lr)[LEN], double hb)
{
    if constexpr (I < N && Q0 + I < LEN) {
        if constexpr (I == 0)
            asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                         : "+v"(acc[I & 3])
                         : "v"(hb), "v"(Lr[Q0 + I]), "i"(I));
        else
            asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
                         : "+v"(acc[I & 3])
                         : "v"(hb), "v"(Lr[Q0 + I]), "i"(I));
        bcast_fma<I + 1, N, Q0, LEN>(acc, Lr, hb);
    }
}

}  // namespace skl
