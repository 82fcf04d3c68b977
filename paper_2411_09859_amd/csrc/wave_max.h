// Wave-level helpers shared by the panel, unpivoted and batched kernels:
// waiting for the wave's memory operations, sums across lanes by lane swaps
// and DPP moves, reading a double from one lane, the largest key over a wave
// with DPP moves (no LDS), and FP64 FMAs whose second factor is broadcast
// inside 16-lane rows.
#pragma once

#include <hip/hip_runtime.h>

namespace skl {

// Wait until this wave's outstanding memory operations have completed
// (s_waitcnt vmcnt(0)).
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ double dbl_of(unsigned lo, unsigned hi)
{
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One step of an xor butterfly over the lanes OFF = 32 or 16 apart: every
// lane gets s + s(lane ^ OFF), with the gfx950 lane-swap instructions (VALU,
// no LDS).  Swapping a register with itself leaves, in the two outputs, the
// lane's own half and the partner half, so their sum is the butterfly step
// (the same sum as s + shfl_xor(s, OFF): addition commutes).
template <int OFF>
__device__ __forceinline__ double xor_add(double s)
{
    static_assert(OFF == 32 || OFF == 16, "swap distance");
    const unsigned long long b = (unsigned long long)__double_as_longlong(s);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    if constexpr (OFF == 32) {
        const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return dbl_of(l2[0], h2[0]) + dbl_of(l2[1], h2[1]);
    } else {
        const auto l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        return dbl_of(l2[0], h2[0]) + dbl_of(l2[1], h2[1]);
    }
}

// one DPP move of a double (both dwords through the same pattern CTRL)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    return dbl_of((unsigned)lo, (unsigned)hi);
}

// Sum of s over the 64 lanes of a wave, the same bits in every lane: inside
// each 16-lane row lanes are paired by DPP moves (xor 1 and xor 2 by quad
// permutations, then the half-row and row mirrors, which pair lanes whose
// partial sums are by then equal within their quad and half-row), then the
// rows by the lane swaps 16 and 32 apart.  At every step a lane adds its
// own partial sum and its partner's, which the partner adds the other way
// round: addition commutes, so all lanes keep equal bits.  All VALU, no LDS.
__device__ __forceinline__ double wave_sum_f64(double s)
{
    s = s + dpp_f64<0xB1>(s);  // quad_perm [1,0,3,2]
    s = s + dpp_f64<0x4E>(s);  // quad_perm [2,3,0,1]
    s = s + dpp_f64<0x141>(s); // row_half_mirror
    s = s + dpp_f64<0x140>(s); // row_mirror
    s = xor_add<16>(s);
    return xor_add<32>(s);
}

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Largest value over lanes 0 .. CL-1 (CL = 16, 32 or 64), as a uniform
// value: pairs and quads (quad_perm), 8 and 16 lanes (row half mirror, row
// mirror), then lane 15 of each row into the next and lane 31 into the upper
// half (row_bcast 15 / 31 with row masks), the maximum ending in lane 15
// (CL = 16), 31 or 63.  Each step is one v_max_u32 whose first operand is
// the DPP-moved register, x = max(x[moved], x); rows outside the row mask,
// and lanes without a source lane, keep x.  A DPP read of a register written
// by the previous VALU instruction needs two wait states (the s_nop 1s).
// All VALU, no LDS.
template <int CL>
__device__ __forceinline__ unsigned lanes_max_u32(unsigned x)
{
    static_assert(CL == 16 || CL == 32 || CL == 64, "lane count");
    asm volatile("s_nop 1\n\t"
                 "v_max_u32_dpp %0, %0, %0 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1\n\t"
                 "v_max_u32_dpp %0, %0, %0 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1\n\t"
                 "v_max_u32_dpp %0, %0, %0 row_half_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1\n\t"
                 "v_max_u32_dpp %0, %0, %0 row_mirror row_mask:0xf bank_mask:0xf\n\t"
                 "s_nop 1"
                 : "+v"(x));
    if constexpr (CL == 16)
        return (unsigned)__builtin_amdgcn_readlane((int)x, 15);
    asm volatile("v_max_u32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
                 "s_nop 1"
                 : "+v"(x));
    if constexpr (CL == 32)
        return (unsigned)__builtin_amdgcn_readlane((int)x, 31);
    asm volatile("v_max_u32_dpp %0, %0, %0 row_bcast:31 row_mask:0xc bank_mask:0xf\n\t"
                 "s_nop 1"
                 : "+v"(x));
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
