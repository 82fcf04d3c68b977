// Finalization: deferred row exchanges of earlier L columns, and the
// Pfaffian read off T and P.
//
// Paper (arXiv 2411.09859): after each panel the blocked pivoted algorithm
// applies the panel's pivots to the rows of all earlier columns of L
// (pivot_rows in the code of Fig. "C++ implementation", Sec. 4.2); the paper
// measures this as its largest pivoted overhead because rows are exchanged in
// column-major storage (Sec. 5.3).  The right-looking update never reads those
// columns again, so here every column of L receives all of its later
// exchanges at once at the end: column j gets the composition of the
// transpositions of all steps after the panel that last wrote it, applied as
// one gather per column held in registers (read the column once, write it
// once, coalesced).
//
// Pfaffian: Pf(A) = det(P) * prod_i T[2i][2i+1] (definition in Sec. 1 with
// Pf(B X B^T) = det(B) Pf(X), T of Sec. 1 / eq. (TvsS): T[2i][2i+1] = -t[2i]).
#include "common.h"
#include "pivot_walk.h"

#include <cmath>

namespace skl {

__global__ void fill_zero_kernel(uint32_t *p, size_t words)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void set_int_kernel(int *p, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        *p = v;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    const size_t words = bytes / 4;
    if (!words)
        return hipSuccess;
    (void)hipGetLastError(); // report this launch only
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t *)p,
                       words);
    return hipGetLastError();
}

hipError_t launch_set_int(int *p, int v, hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(64), 0, s, p, v);
    return hipGetLastError();
}

// gmap[B][i] = the row whose entry lands in row i when the exchanges of all
// steps after block B are applied to a column (composition of
// transpositions, last step innermost).  Block B covers steps
// [B*b, min((B+1)*b, n-1)).
__global__ __launch_bounds__(256) void suffix_map_kernel(const int *__restrict__ ipiv, int n,
                                                         int b, int nblk,
                                                         int *__restrict__ gmap)
{
    // the steps c >= (B+1) b of the map of block B are the transpositions
    // r = c + 1 >= (B+1) b + 1; one walk over r = n-1 .. b+1 takes a
    // snapshot at each block boundary (chunks end on the boundaries)
    __shared__ int sp[kWalkStage];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i0 = (blockIdx.x * 4 + wave) * kWalkI;
    const int imax = i0 + kWalkI - 1;
    int v[kWalkI];
#pragma unroll
    for (int k = 0; k < kWalkI; ++k)
        v[k] = i0 + k;
    walk_store(v, i0, n, lane, gmap + (size_t)(nblk - 1) * n);
    int B = nblk - 2;
    int bnd = (B + 1) * b + 1; // lowest transposition of the map of block B
    for (int hi = n - 1; hi >= b + 1; hi -= kWalkStage) {
        const int lo = max(b + 1, hi - kWalkStage + 1);
        __syncthreads();
        walk_stage(ipiv, lo, hi, sp);
        __syncthreads();
        for (int R = hi; R >= lo;) {
            const int bot = max(max(lo, R - 63), bnd);
            if (bot <= imax && i0 < n) {
                const int pr = sp[max(R - lane, bot) - lo];
                walk_chunk(v, i0, R, R - bot + 1, pr);
            }
            R = bot - 1;
            if (bot == bnd) {
                walk_store(v, i0, n, lane, gmap + (size_t)B * n);
                --B;
                bnd -= b;
            }
        }
    }
}

// Column a (holding L column j = a + 1) of block B = j / b receives the
// exchanges of the steps after block B: rows >= lo take row gmap[B][row].
struct GatherCol {
    int B, lo, len;
};
__device__ __forceinline__ GatherCol gather_col(int a, int n, int b, int nblk)
{
    GatherCol g;
    const int j = a + 1;
    g.B = j / b;
    const int s = min((g.B + 1) * b, n - 1);
    g.lo = s + 1;
    g.len = (g.B >= nblk - 1) ? 0 : n - g.lo; // the last block has no later exchanges
    return g;
}

// One 1024-thread workgroup per column, the column held in registers (E per
// thread): every source is read before the barrier and every destination
// written after it, so the in-place permutation needs no staging buffer.
template <int E>
__global__ __launch_bounds__(1024) void gather_reg_kernel(double *__restrict__ A, int lda, int n,
                                                          int b, int nblk,
                                                          const int *__restrict__ gmap)
{
    const int a = blockIdx.x;
    const GatherCol gc = gather_col(a, n, b, nblk);
    if (gc.len <= 0)
        return;
    double *cp = A + (size_t)a * lda + gc.lo;
    const int *g = gmap + (size_t)gc.B * n + gc.lo;
    double v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = threadIdx.x + e * 1024;
        v[e] = 0.0;
        if (q < gc.len) {
            int src = g[q] - gc.lo;
            if (src < 0 || src >= gc.len)
                src = q; // cannot happen for valid pivots; keeps the read in range
            v[e] = cp[src];
        }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int q = threadIdx.x + e * 1024;
        if (q < gc.len)
            cp[q] = v[e];
    }
}

// One 1024-thread workgroup per column, the column staged in LDS: read
// once in order (coalesced), then every entry written in order from its
// permuted source in LDS.  The register form above reads its sources at
// permuted addresses, one 8-byte entry per memory granule when the
// permutation scatters (it does, after thousands of pivots).
constexpr int kGatherLdsMax = 20480; // doubles: 160 KB of LDS
__global__ __launch_bounds__(1024) void gather_lds_kernel(double *__restrict__ A, int lda, int n,
                                                          int b, int nblk,
                                                          const int *__restrict__ gmap)
{
    extern __shared__ double col[];
    const int a = blockIdx.x;
    const GatherCol gc = gather_col(a, n, b, nblk);
    if (gc.len <= 0)
        return;
    double *cp = A + (size_t)a * lda + gc.lo;
    const int *g = gmap + (size_t)gc.B * n + gc.lo;
    for (int q = threadIdx.x; q < gc.len; q += blockDim.x)
        col[q] = cp[q];
    __syncthreads();
    for (int q = threadIdx.x; q < gc.len; q += blockDim.x) {
        int src = g[q] - gc.lo;
        if (src < 0 || src >= gc.len)
            src = q; // cannot happen for valid pivots; keeps the read in range
        __builtin_nontemporal_store(col[src], &cp[q]);
    }
}

// Columns longer than the register version holds: gather into a scratch
// column of the (no longer needed) work matrix, then copy back.
__global__ __launch_bounds__(1024) void gather_scratch_kernel(double *__restrict__ A, int lda,
                                                              int n, int b, int nblk,
                                                              const int *__restrict__ gmap,
                                                              double *__restrict__ scratch,
                                                              int lds_)
{
    const int a = blockIdx.x;
    const GatherCol gc = gather_col(a, n, b, nblk);
    if (gc.len <= 0)
        return;
    double *cp = A + (size_t)a * lda + gc.lo;
    double *tmp = scratch + (size_t)a * lds_;
    const int *g = gmap + (size_t)gc.B * n + gc.lo;
    for (int q = threadIdx.x; q < gc.len; q += blockDim.x) {
        int src = g[q] - gc.lo;
        if (src < 0 || src >= gc.len)
            src = q;
        tmp[q] = cp[src];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < gc.len; q += blockDim.x)
        cp[q] = tmp[q];
}

void finalize_init_attrs()
{
    (void)hipFuncSetAttribute((const void *)gather_lds_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              kGatherLdsMax * (int)sizeof(double));
}

hipError_t launch_finalize(double *A, int lda, int n, int b, const int *ipiv,
                           const FactorWs &ws, hipStream_t s)
{
    const int nsteps = n - 1;
    if (nsteps <= 0)
        return hipSuccess;
    const int nblk = (nsteps + b - 1) / b;
    if (nblk <= 1)
        return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(suffix_map_kernel, dim3((n + 4 * kWalkI - 1) / (4 * kWalkI)), dim3(256), 0,
                       s, ipiv, n, b,
                       nblk, ws.gmap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int maxlen = n - (b + 1);
    if (maxlen <= 0)
        return hipSuccess;
    const dim3 grid(n - 2 > 0 ? n - 2 : 1), blk(1024);
    const int *gm = ws.gmap;
    if (maxlen > 4 * 1024 && maxlen <= kGatherLdsMax)
        hipLaunchKernelGGL(gather_lds_kernel, grid, blk, (size_t)maxlen * sizeof(double), s, A,
                           lda, n, b, nblk, gm);
    else if (maxlen <= 4 * 1024)
        hipLaunchKernelGGL(gather_reg_kernel<4>, grid, blk, 0, s, A, lda, n, b, nblk, gm);
    else if (maxlen <= 8 * 1024)
        hipLaunchKernelGGL(gather_reg_kernel<8>, grid, blk, 0, s, A, lda, n, b, nblk, gm);
    else if (maxlen <= 16 * 1024)
        hipLaunchKernelGGL(gather_reg_kernel<16>, grid, blk, 0, s, A, lda, n, b, nblk, gm);
    else if (maxlen <= 32 * 1024)
        hipLaunchKernelGGL(gather_reg_kernel<32>, grid, blk, 0, s, A, lda, n, b, nblk, gm);
    else
        hipLaunchKernelGGL(gather_scratch_kernel, grid, blk, 0, s, A, lda, n, b, nblk, gm,
                           ws.W[0], ws.ldw);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void pfaffian_kernel(int n, const double *__restrict__ t,
                                                       const int *__restrict__ ipiv,
                                                       double *__restrict__ log_abs_pf,
                                                       int *__restrict__ sign)
{
    __shared__ double sl[256];
    __shared__ int sneg[256], szero[256];
    const int tid = threadIdx.x;
    if (n % 2 != 0) {
        if (tid == 0) {
            *log_abs_pf = -INFINITY;
            *sign = 0;
        }
        return;
    }
    double acc = 0.0;
    int neg = 0, zero = 0;
    // det(P): one factor -1 per non-trivial transposition
    for (int i = tid; i < n; i += 256)
        neg += (ipiv[i] != i) ? 1 : 0;
    // prod_i T[2i][2i+1] = prod_i (-t[2i])
    for (int i = tid; i < n / 2; i += 256) {
        const double f = -t[2 * i];
        if (f == 0.0)
            zero = 1;
        else {
            if (f < 0.0)
                ++neg;
            acc += log(fabs(f));
        }
    }
    sl[tid] = acc;
    sneg[tid] = neg;
    szero[tid] = zero;
    __syncthreads();
    for (int st = 128; st >= 1; st >>= 1) {
        if (tid < st) {
            sl[tid] += sl[tid + st];
            sneg[tid] += sneg[tid + st];
            szero[tid] |= szero[tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (szero[0]) {
            *log_abs_pf = -INFINITY;
            *sign = 0;
        } else {
            *log_abs_pf = sl[0];
            *sign = (sneg[0] & 1) ? -1 : 1;
        }
    }
}

hipError_t launch_pfaffian(int n, const double *t, const int *ipiv, double *log_abs_pf, int *sign,
                           hipStream_t s)
{
    (void)hipGetLastError();
    hipLaunchKernelGGL(pfaffian_kernel, dim3(1), dim3(256), 0, s, n, t, ipiv, log_abs_pf, sign);
    return hipGetLastError();
}

}  // namespace skl
