// Finalization: deferred row exchanges of earlier L columns, and the
// Pfaffian read off T and P.
//
// Paper (arXiv 2411.09859): after each panel the blocked pivoted algorithm
// applies the panel's pivots to the rows of all earlier columns of L
// (pivot_rows in the code of Fig. "C++ implementation", Sec. 4.2); the paper
// measures this as its largest pivoted overhead because rows are exchanged in
// column-major storage (Sec. 5.2).  The right-looking update never reads those
// columns again, so here every column of L receives all of its later
// exchanges at once at the end: column j gets the composition of the
// transpositions of all steps after the panel that last wrote it, applied as
// one gather through LDS (read the column once, write it once, coalesced).
//
// Pfaffian: Pf(A) = det(P) * prod_i T[2i][2i+1] (definition in Sec. 1 with
// Pf(B X B^T) = det(B) Pf(X), T of Sec. 1 / eq. (TvsS): T[2i][2i+1] = -t[2i]).
#include "common.h"

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
__global__ void suffix_map_kernel(const int *__restrict__ ipiv, int n, int b, int nblk,
                                  int *__restrict__ gmap)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int v = i;
    gmap[(size_t)(nblk - 1) * n + i] = v;
    for (int B = nblk - 2; B >= 0; --B) {
        const int s_lo = (B + 1) * b;                       // first step of block B+1
        const int s_hi = min((B + 2) * b, n - 1);           // end of block B+1
        for (int c = s_hi - 1; c >= s_lo; --c) {
            const int rr = c + 1;
            const int pp = ipiv[rr];
            if (v == rr)
                v = pp;
            else if (v == pp)
                v = rr;
        }
        gmap[(size_t)B * n + i] = v;
    }
}

// One workgroup per stored column a = j-1 of L column j.
__global__ __launch_bounds__(256) void gather_kernel(double *__restrict__ A, int lda, int n,
                                                     int b, int nblk,
                                                     const int *__restrict__ gmap)
{
    extern __shared__ double col[];
    const int a = blockIdx.x; // A column, holds L column j = a + 1
    const int j = a + 1;
    const int B = j / b;
    if (B >= nblk - 1)
        return; // the last block has no later exchanges
    const int s = min((B + 1) * b, n - 1);
    const int lo = s + 1; // rows >= lo can move
    const int len = n - lo;
    if (len <= 0)
        return;
    double *cp = A + (size_t)a * lda + lo;
    for (int q = threadIdx.x; q < len; q += blockDim.x)
        col[q] = cp[q];
    __syncthreads();
    const int *g = gmap + (size_t)B * n + lo;
    for (int q = threadIdx.x; q < len; q += blockDim.x) {
        int src = g[q] - lo;
        if (src < 0 || src >= len)
            src = q; // cannot happen for valid pivots; keeps the LDS read in range
        cp[q] = col[src];
    }
}

void finalize_init_attrs()
{
    (void)hipFuncSetAttribute((const void *)gather_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        160 * 1024);
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
    hipLaunchKernelGGL(suffix_map_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ipiv, n, b,
                       nblk, ws.gmap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int maxlen = n - (b + 1);
    if (maxlen <= 0)
        return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)maxlen;
    hipLaunchKernelGGL(gather_kernel, dim3(n - 2 > 0 ? n - 2 : 1), dim3(256), lds, s, A, lda, n,
                       b, nblk, (const int *)ws.gmap);
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
