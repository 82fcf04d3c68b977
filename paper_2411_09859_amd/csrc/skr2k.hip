// Skew-symmetric rank-2k trailing update on MFMA.
//
// Paper (arXiv 2411.09859): the trailing update C := C - A T A^T of the fused
// blocked right-looking algorithm (Sec. 3.6.3, T of order b+1) becomes a skew
// rank-2k update C := C - (W A^T - A W^T) with W = A S (Theorem "TandS" of
// Sec. 2.2, eq. (TvsS); Sec. 3.6.5 "Forming W after the panel
// factorization"), the skew_rank2k operation of the level-3 table in
// Sec. 3.5.4/3.6.6.  Only the odd columns of W are non-zero, so with
// U = W[:, odd] and V = A[:, odd] the update is C -= U V^T - V U^T with
// k = floor((b+1)/2) columns each.
//
// The panel kernel writes the operands once, column-major with leading
// dimension n, as [U | V | -V | U]; then C += [U | V] [-V | U]^T is a plain
// GEMM with K = 2k restricted to the strict lower triangle of the trailing
// block (rows and columns cp..n-1, the first column included).
//
// The trailing matrix is held as its lower triangle, and the panel does not
// apply its row/column exchanges to it; this kernel does.  It reads
// C[i][j] = Wc[perm[i]][perm[j]] (perm: row of the panel-start matrix that
// position i holds after the panel's exchanges; an upper source entry is
// read as the negation of its lower mirror) and writes the updated lower
// entry (i, j) of the other buffer Wn, so each panel's permutation costs no
// extra pass over the matrix.
//
// Tiling: a 128x128 output tile per 512-thread workgroup, eight waves of
// 64x32 (64 rows, 32 columns), each a 4x2 grid of 16x16 MFMA blocks.  With
// 121 registers per lane two workgroups share a CU, so four waves per SIMD
// issue FP64 MFMAs: the FP64 matrix pipe of a SIMD needs two issuing waves
// to run at full rate, and with four, one wave's barrier, C gather or stores
// no longer halve it (four waves of 64x64 at two per SIMD: 40 TFLOP/s on
// the largest update of n = 16384; eight of 64x32: 48).  The MFMA computes
// the transposed tile, D[j][i], so that each lane's four accumulator values
// lie in four columns at one row i and sixteen consecutive lanes cover
// sixteen consecutive rows: loads of C and stores are 128-byte segments; all
// C stores are streaming (non-temporal): the next reader is the next panel
// or update, long after.
// Tiles are enumerated over the lower triangle only; a diagonal tile skips
// the waves whose 64x32 piece lies strictly above the diagonal and masks the
// rest.
// Consecutive tile indices go to one XCD (workgroup ids are dealt to the 8
// XCDs round-robin) and follow a blocked order (4 x 4 tile blocks), so the
// tiles an XCD works on at once share operand panels in its L2 (measured:
// fewer operand re-reads, 6-10 % faster on large trailing blocks).
// Small trailing blocks (fewer 128-tiles than the chip has CUs, at the end
// of a factorization) take 64x64 tiles instead: four waves of 32x32 per
// 256-thread workgroup, so four times as many workgroups share the work.  A
// 128-tile alone on a CU takes about 52 us whatever the trailing order; the
// small tiles finish sooner.  Every element is summed over K in the same
// order by both tilings, so the results are bit for bit the same.
#include "skltlt.h"
#include "common.h"
#include "mfma_tile.h"

namespace skl {

// The update of one output tile of TMV x TMV by NT threads, waves of WR rows
// by WC columns; TMPV: padded LDS row of the operand stage.
template <typename T, int TMV, int TMPV, int NT, int WR, int WC>
__device__ __forceinline__ void skr2k_tile(const double *__restrict__ Wc, double *__restrict__ Wn,
                                           int ldw, const int *__restrict__ perm, int n, int cp,
                                           int K, const T *__restrict__ uv, int ntiles)
{
    typedef typename MfmaT<T>::acc4 acc4;
    constexpr int BR = WR / 16, BC = WC / 16; // 16x16 blocks per wave tile
    constexpr int WPR = TMV / WR;             // waves along the rows
    static_assert(WPR * (TMV / WC) * 64 == NT, "waves cover the tile");
    // LDS: double-buffered operand chunks, k-major, rows padded so that the
    // four k-rows read by one fragment load fall in different LDS banks.
    constexpr size_t kOpBytes = sizeof(T) * 2 * KC * TMPV;
    __shared__ __attribute__((aligned(16))) char smem[2 * kOpBytes];
    T(*sI)[KC][TMPV] = reinterpret_cast<T(*)[KC][TMPV]>(smem);            // [U|V] rows i
    T(*sJ)[KC][TMPV] = reinterpret_cast<T(*)[KC][TMPV]>(smem + kOpBytes); // [-V|U] rows j
    __shared__ int sPi[TMV], sPj[TMV]; // source rows of the tile's rows and columns

    // XCD-grouped tile order
    const int nwg = gridDim.x;
    const int per_xcd = (nwg + 7) / 8;
    const int bid = blockIdx.x;
    const int tau = (bid & 7) * per_xcd + (bid >> 3);
    if (tau >= ntiles)
        return;
    int ti, tj;
    tile_of_blocked<4>(tau, (n - cp + TMV - 1) / TMV, &ti, &tj);
    const int i0 = cp + ti * TMV;
    const int j0 = cp + tj * TMV;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave % WPR, wj = wave / WPR;
    const int ib = i0 + wi * WR; // this wave's rows
    const int jb = j0 + wj * WC; // this wave's columns
    const bool active = !(ti == tj && jb >= ib + WR);

    const int lrow = lane & 15; // row inside a 16-block
    const int lk = lane >> 4;   // k inside a 4-step, or row group of D

    // Source rows of the tile's rows and columns (loaded first, their latency
    // overlaps the first operand chunk).
    for (int q = tid; q < 2 * TMV; q += NT) {
        if (q < TMV) {
            const int g = i0 + q;
            sPi[q] = (g < n) ? perm[g] : 0;
        } else {
            const int g = j0 + q - TMV;
            sPj[q - TMV] = (g < n) ? perm[g] : 0;
        }
    }
    constexpr bool kF64 = sizeof(T) == 8;
    // C[gi][gj] from the lower-triangle source (rows/columns past n have
    // source row 0: still in range)
    auto cval = [&](int gi, int gj) -> double {
        bool neg;
        const double v = Wc[skew_at(sPi[gi - i0], sPj[gj - j0], ldw, neg)];
        return neg ? -v : v;
    };

    TileStage<T, NT, TMV, TMPV> tk(sI, sJ, uv, uv + (size_t)K * n, n, n, i0, j0, K);
    tk.prologue();

    // Accumulators.  FP64: start from the (permuted) C tile; FP32: start from
    // zero and add the fp32 product to C in fp64 at the end.
    acc4 acc[BR][BC];
#pragma unroll
    for (int bi = 0; bi < BR; ++bi) {
        const int gi = ib + bi * 16 + lrow;
#pragma unroll
        for (int bj = 0; bj < BC; ++bj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gj = jb + bj * 16 + MfmaT<T>::drow(lk, q);
                T v = 0;
                if (kF64) {
                    const double cv = cval(gi, gj);
                    v = (active && gi < n && gj < gi) ? (T)cv : (T)0;
                }
                acc[bi][bj][q] = v;
            }
        }
    }
    tk.template run<BR, BC>(acc, active, wi * WR, wj * WC, lrow, lk);
    if (!active)
        return;

    // D[m][nn] (m = MfmaT::drow(lane/16, q) : column j, nn = lane%16 : row i):
    // sixteen lanes write 128 consecutive bytes of column j.
#pragma unroll
    for (int bi = 0; bi < BR; ++bi) {
        const int gi = ib + bi * 16 + lrow;
#pragma unroll
        for (int bj = 0; bj < BC; ++bj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gj = jb + bj * 16 + MfmaT<T>::drow(lk, q);
                if (gi < n && gj < gi) {
                    const double v =
                        kF64 ? (double)acc[bi][bj][q] : cval(gi, gj) + (double)acc[bi][bj][q];
                    __builtin_nontemporal_store(v, &Wn[(size_t)gj * ldw + gi]);
                }
            }
        }
    }
}

// 128x128 tiles, eight waves of 64x32, two workgroups per CU
constexpr int kSkThreads = 512;
template <typename T>
__global__ __launch_bounds__(kSkThreads, 2) void skr2k_kernel(const double *__restrict__ Wc,
                                                              double *__restrict__ Wn, int ldw,
                                                              const int *__restrict__ perm,
                                                              int n, int cp, int K,
                                                              const T *__restrict__ uv,
                                                              int ntiles)
{
    skr2k_tile<T, TM, TMP, kSkThreads, 64, 32>(Wc, Wn, ldw, perm, n, cp, K, uv, ntiles);
}

// 64x64 tiles (LDS rows padded to 80: k-rows 640 B apart, banks shift by
// 128 B), four waves of 32x32
constexpr int kSkSmallThreads = 256;
constexpr int kSmallTM = 64;
template <typename T>
__global__ __launch_bounds__(kSkSmallThreads) void skr2k_small_kernel(
    const double *__restrict__ Wc, double *__restrict__ Wn, int ldw,
    const int *__restrict__ perm, int n, int cp, int K, const T *__restrict__ uv, int ntiles)
{
    skr2k_tile<T, kSmallTM, 80, kSkSmallThreads, 32, 32>(Wc, Wn, ldw, perm, n, cp, K, uv, ntiles);
}

// Trailing blocks with fewer 128-tiles than this take the 64x64 tiles.
static int g_small_tiles = -1;

hipError_t launch_skr2k(const double *Wc, double *Wn, int n, int cp, int nq,
                        const FactorWs &ws, int precision, hipStream_t s)
{
    const int m = n - cp;
    if (m < 2 || nq <= 0)
        return hipSuccess;
    if (g_small_tiles < 0)
        g_small_tiles = device_cu_count();
    const int nt = (m + TM - 1) / TM;
    const bool small = nt * (nt + 1) / 2 < g_small_tiles;
    const int ntm = small ? (m + kSmallTM - 1) / kSmallTM : nt;
    const int ntiles = ntm * (ntm + 1) / 2;
    const int per_xcd = (ntiles + 7) / 8;
    const int grid = per_xcd * 8;
    const int K = 2 * nq;
    (void)hipGetLastError(); // report this launch only
    if (small) {
        if (precision == 1)
            hipLaunchKernelGGL(skr2k_small_kernel<float>, dim3(grid), dim3(kSkSmallThreads), 0, s,
                               Wc, Wn, ws.ldw, (const int *)ws.perm, n, cp, K,
                               (const float *)ws.uv32, ntiles);
        else
            hipLaunchKernelGGL(skr2k_small_kernel<double>, dim3(grid), dim3(kSkSmallThreads), 0, s,
                               Wc, Wn, ws.ldw, (const int *)ws.perm, n, cp, K,
                               (const double *)ws.uv, ntiles);
    } else if (precision == 1) {
        hipLaunchKernelGGL(skr2k_kernel<float>, dim3(grid), dim3(kSkThreads), 0, s, Wc, Wn, ws.ldw,
                           (const int *)ws.perm, n, cp, K, (const float *)ws.uv32, ntiles);
    } else {
        hipLaunchKernelGGL(skr2k_kernel<double>, dim3(grid), dim3(kSkThreads), 0, s, Wc, Wn, ws.ldw,
                           (const int *)ws.perm, n, cp, K, (const double *)ws.uv, ntiles);
    }
    return hipGetLastError();
}

// Sets the 128-tile count below which the 64x64 tiles are used (0: never;
// negative: the default, the device's CU count).
void skr2k_set_small_tiles(int t) { g_small_tiles = t < 0 ? device_cu_count() : t; }

}  // namespace skl

extern "C" int skltlt_tune_skr2k_small_tiles(int tiles)
{
    skl::skr2k_set_small_tiles(tiles);
    return SKLTLT_OK;
}
