// Images of start indices under the pivot transpositions tau_r = (r ipiv[r])
// of the factorization (ipiv[r] >= r, absolute indices), applied for r
// descending: the composition that maps a row of the factored order back to
// the row it came from (the pivot matrices of Sec. 3.7.1, stored as in
// Sec. 4.1).
//
// Following one start index i: while r > i nothing moves it (r != i and
// ipiv[r] >= r > i); at r = i it becomes ipiv[i] >= i; from then on its value
// v stays above r, so it moves (to r) exactly at the steps with ipiv[r] == v.
// A wave follows kWalkI start indices at once over chunks of 64 pivots
// (lane = step r): per index and chunk one compare and one ballot, plus one
// more per move.  A chunk step costs a few instructions, so a whole map takes
// about n / 64 of them instead of n dependent selects per index.
#pragma once

#include <hip/hip_runtime.h>

namespace skl {

constexpr int kWalkI = 16;       // start indices per wave
constexpr int kWalkStage = 8192; // pivots staged in LDS at a time

// One chunk of steps r = R, R-1, ..., R-len+1 (lane l holds pr = ipiv[R-l];
// lanes >= len hold anything).  v[k] is the current image of start index
// i0 + k; every value here is wave-uniform.
__device__ __forceinline__ void walk_chunk(int (&v)[kWalkI], int i0, int R, int len, int pr)
{
    const unsigned long long in_len = (len >= 64) ? ~0ull : ((1ull << len) - 1ull);
    const int rb = R - len + 1;
    if (R < i0) {
        // the common case: every index of the wave is past its own step, so
        // only a pivot equal to one of the current values can move anything
        unsigned long long any = 0;
#pragma unroll
        for (int k = 0; k < kWalkI; ++k)
            any |= __ballot(pr == v[k]);
        if ((any & in_len) == 0)
            return;
    }
#pragma unroll
    for (int k = 0; k < kWalkI; ++k) {
        const int i = i0 + k;
        if (i < rb)
            continue; // step r = i comes in a later chunk
        unsigned long long live = in_len;
        if (i <= R) { // step r = i is in this chunk: i -> ipiv[i]
            const int li = R - i;
            v[k] = __builtin_amdgcn_readlane(pr, li);
            live &= ~((2ull << li) - 1ull); // only the later steps (lanes > li)
        }
        unsigned long long m = __ballot(pr == v[k]) & live;
        while (m) {
            const int l0 = __builtin_ctzll(m); // the first matching step
            v[k] = R - l0;
            live &= ~((2ull << l0) - 1ull);
            m = __ballot(pr == v[k]) & live;
        }
    }
}

// Copies ipiv[lo .. hi] (at most kWalkStage entries) to sp, eight loads in
// flight per thread; the caller synchronizes around it.
__device__ __forceinline__ void walk_stage(const int *__restrict__ ipiv, int lo, int hi,
                                           int *__restrict__ sp)
{
    constexpr int U = 8;
    const int nt = blockDim.x;
    for (int base = lo + (int)threadIdx.x; base <= hi; base += U * nt) {
        int x[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            x[u] = ipiv[min(base + u * nt, hi)];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * nt <= hi)
                sp[base + u * nt - lo] = x[u];
    }
}

// Writes the kWalkI images of a wave with one vector store (lane k < kWalkI
// writes start index i0 + k, if below n).
__device__ __forceinline__ void walk_store(const int (&v)[kWalkI], int i0, int n, int lane,
                                           int *__restrict__ out)
{
    int x = 0;
#pragma unroll
    for (int k = 0; k < kWalkI; ++k)
        x = (lane == k) ? v[k] : x;
    if (lane < kWalkI && i0 + lane < n)
        out[i0 + lane] = x;
}

}  // namespace skl
