// Full skew storage of the input for the factorization's work matrix.
//
// The caller's matrix is given by its strict lower triangle (the implicit
// skew structure of Sec. 2.4 of arXiv 2411.09859).  The factorization keeps
// its trailing matrix in a separate buffer holding both triangles,
// W[i][j] = -W[j][i], W[i][i] = 0, so that any row of it is also a column
// and the pivot column of every step is one coalesced read.
#include "common.h"

namespace skl {

constexpr int TT = 64;

// One 64x64 lower tile (I >= J) of A per workgroup, staged in LDS: it is
// written to W at (I, J) and, negated and transposed, at (J, I).
__global__ __launch_bounds__(256) void init_full_kernel(const double *__restrict__ A, int lda,
                                                        int n, double *__restrict__ W, int ldw)
{
    __shared__ double tile[TT][TT + 1]; // tile[c][r] = A[i0 + r][j0 + c]
    int I, J;
    tile_of(blockIdx.x, &I, &J);
    const int i0 = I * TT, j0 = J * TT;
    const int tid = threadIdx.x;
    const int r = tid % TT;
    for (int c = tid / TT; c < TT; c += 256 / TT) {
        const int gi = i0 + r, gj = j0 + c;
        double v = 0.0;
        if (gi < n && gj < n && gi > gj)
            v = A[(size_t)gj * lda + gi];
        tile[c][r] = v;
    }
    __syncthreads();
    for (int c = tid / TT; c < TT; c += 256 / TT) {
        const int gi = i0 + r, gj = j0 + c;
        if (gi < n && gj < n) {
            double v;
            if (I > J || r > c)
                v = tile[c][r];
            else if (r < c)
                v = -tile[r][c]; // diagonal tile: upper entry from the lower one
            else
                v = 0.0;
            __builtin_nontemporal_store(v, &W[(size_t)gj * ldw + gi]);
        }
    }
    if (I == J)
        return;
    // W[j0 + r][i0 + c] = -A[i0 + c][j0 + r]
    for (int c = tid / TT; c < TT; c += 256 / TT) {
        const int wi = j0 + r, wj = i0 + c;
        if (wi < n && wj < n)
            __builtin_nontemporal_store(-tile[r][c], &W[(size_t)wj * ldw + wi]);
    }
}

hipError_t launch_init_full(const double *A, int lda, int n, double *W, int ldw, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int nt = (n + TT - 1) / TT;
    const int ntiles = nt * (nt + 1) / 2;
    (void)hipGetLastError(); // report this launch only
    hipLaunchKernelGGL(init_full_kernel, dim3(ntiles), dim3(256), 0, s, A, lda, n, W, ldw);
    return hipGetLastError();
}

}  // namespace skl
