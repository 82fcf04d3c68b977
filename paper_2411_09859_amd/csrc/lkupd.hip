// Left-looking panel update of the blocked left-looking algorithm (Variant 3,
// Sec. 3.6.4, from Invariant 3 of Sec. 3.4; the level-3 operation there is
// skew_tridiag_gemm, Sec. 3.6.6), unpivoted.
//
// Each earlier panel P contributes the skew rank-2k term U_P V_P^T -
// V_P U_P^T (the same operands the right-looking update applies at once,
// Theorem "TandS" of Sec. 2.2 with W formed after the panel, Sec. 3.6.5).
// The left-looking algorithm applies them only when a panel is reached, and
// only to that panel's columns: with every earlier panel's [U | V] appended
// to opI and [-V | U] to opJ (K columns in all),
//     W[i][j] += sum_k opI[i][k] opJ[j][k]
// for the panel's columns j (at most one 128-wide tile column) and every row
// i > j of the trailing block.  The product is a tall, thin GEMM with a long
// K, so K is split over several workgroups (each adds its partial product
// with device-scope floating-point atomics, so the summation order, and the
// last bits, may differ between runs), giving the GPU enough workgroups even
// where the trailing block has few tile rows.
#include "common.h"
#include "mfma_tile.h"

namespace skl {

__global__ __launch_bounds__(256, 2) void lkupd_kernel(double *__restrict__ W, int ldw, int n,
                                                       int c0, int nb,
                                                       const double *__restrict__ opI,
                                                       const double *__restrict__ opJ, int ldo,
                                                       int K, int S, int ksplit)
{
    typedef MfmaT<double>::acc4 acc4;
    constexpr size_t kOpBytes = sizeof(double) * 2 * KC * TMP;
    __shared__ __attribute__((aligned(16))) char smem[2 * kOpBytes];
    double(*sI)[KC][TMP] = reinterpret_cast<double(*)[KC][TMP]>(smem);
    double(*sJ)[KC][TMP] = reinterpret_cast<double(*)[KC][TMP]>(smem + kOpBytes);

    // split s of tile row ti (the splits of one K range sit on one XCD when
    // S divides 8: workgroup ids are dealt to the XCDs round-robin)
    const int s = blockIdx.x % S;
    const int ti = blockIdx.x / S;
    const int i0 = c0 + ti * TM;
    const int j0 = c0;
    const int kb = s * ksplit;
    const int ke = min(K, kb + ksplit);
    if (i0 >= n || kb >= ke)
        return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave & 1, wj = wave >> 1;
    const int ib = i0 + wi * 64;
    const int jb = j0 + wj * 64;
    // the diagonal tile's quarter strictly above the diagonal has no work;
    // neither has a quarter of columns past the panel
    const bool active = !(ti == 0 && wi == 0 && wj == 1) && (jb < c0 + nb);
    const int lrow = lane & 15;
    const int lk = lane >> 4;

    TileK<double> tk(sI, sJ, opI + (size_t)kb * ldo, opJ + (size_t)kb * ldo, ldo, n, i0, j0,
                     ke - kb);
    tk.prologue();
    acc4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[bi][bj][q] = 0.0;
    tk.run(acc, active, wi, wj, lrow, lk);
    if (!active)
        return;
    // D[m][nn] (m = drow(lane/16, q): column j, nn = lane%16: row i); only
    // strictly lower entries of the panel's columns are read later
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int gi = ib + bi * 16 + lrow;
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gj = jb + bj * 16 + MfmaT<double>::drow(lk, q);
                if (gi < n && gj < gi && gj < c0 + nb) {
                    double *p = &W[(size_t)gj * ldw + gi];
                    if (S == 1)
                        *p += acc[bi][bj][q];
                    else
                        unsafeAtomicAdd(p, acc[bi][bj][q]);
                }
            }
        }
    }
}

hipError_t launch_lkupd(double *W, int ldw, int n, int c0, int nb, const double *opI,
                        const double *opJ, int ldo, int K, hipStream_t s)
{
    if (K <= 0 || nb <= 0 || c0 >= n)
        return hipSuccess;
    if (nb > TM)
        return hipErrorInvalidValue;
    const int nti = (n - c0 + TM - 1) / TM;
    // enough workgroups for two per CU, each split at least 16 K-chunks long
    int S = (512 + nti - 1) / nti;
    const int smax = (K + 16 * KC - 1) / (16 * KC);
    if (S > smax)
        S = smax;
    if (S > 8)
        S = 8;
    if (S < 1)
        S = 1;
    int ks = (K + S - 1) / S;
    ks = (ks + KC - 1) / KC * KC;
    (void)hipGetLastError();
    hipLaunchKernelGGL(lkupd_kernel, dim3((unsigned)(nti * S)), dim3(256), 0, s, W, ldw, n, c0, nb,
                       opI, opJ, ldo, K, S, ks);
    return hipGetLastError();
}

}  // namespace skl
