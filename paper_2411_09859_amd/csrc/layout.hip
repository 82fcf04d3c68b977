// Lower-triangle work copy of the input for the factorization.
//
// The caller's matrix is given by its strict lower triangle (the implicit
// skew structure of Sec. 2.4 of arXiv 2411.09859).  The factorization keeps
// its trailing matrix in a separate buffer in the same storage (entry (i, j)
// at column j, row i for i > j; the upper entries are their negations and
// are read there), so the caller's matrix is only read.
#include "common.h"

namespace skl {

constexpr int TT = 64;

// One 64x64 lower tile (I >= J) of A per workgroup: the strict lower entries
// are copied, the diagonal is set to zero, the upper entries of diagonal
// tiles are not written.
__global__ __launch_bounds__(256) void init_lower_kernel(const double *__restrict__ A, int lda,
                                                         int n, double *__restrict__ W, int ldw)
{
    int I, J;
    tile_of(blockIdx.x, &I, &J);
    const int i0 = I * TT, j0 = J * TT;
    const int tid = threadIdx.x;
    const int r = tid % TT;
    for (int c = tid / TT; c < TT; c += 256 / TT) {
        const int gi = i0 + r, gj = j0 + c;
        if (gi < n && gj < n && gi >= gj) {
            const double v = (gi > gj) ? A[(size_t)gj * lda + gi] : 0.0;
            __builtin_nontemporal_store(v, &W[(size_t)gj * ldw + gi]);
        }
    }
}

hipError_t launch_init_lower(const double *A, int lda, int n, double *W, int ldw, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int nt = (n + TT - 1) / TT;
    const int ntiles = nt * (nt + 1) / 2;
    (void)hipGetLastError(); // report this launch only
    hipLaunchKernelGGL(init_lower_kernel, dim3(ntiles), dim3(256), 0, s, A, lda, n, W, ldw);
    return hipGetLastError();
}

}  // namespace skl
