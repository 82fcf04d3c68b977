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
// The trailing matrix is held in full skew storage, and the panel does not
// apply its row/column exchanges to it; this kernel does.  It reads
// C[i][j] = Wc[perm[i]][perm[j]] (perm: row of the panel-start matrix that
// position i holds after the panel's exchanges) and writes the updated entry
// and its negation to (i, j) and (j, i) of the other buffer Wn, so each
// panel's permutation costs no extra pass over the matrix.
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
// sixteen consecutive rows: loads of C and stores of the lower entries are
// 128-byte segments, and the mirrored upper entries go out through an LDS
// transpose as 256-byte column pieces; all C stores are streaming
// (non-temporal): the next reader is the next panel or update, long after.
// Tiles are enumerated over the lower triangle only; a diagonal tile skips
// the waves whose 64x32 piece lies strictly above the diagonal and masks the
// rest.
// Consecutive tile indices go to one XCD (workgroup ids are dealt to the 8
// XCDs round-robin) and follow a blocked order (4 x 4 tile blocks), so the
// tiles an XCD works on at once share operand panels in its L2 (measured:
// fewer operand re-reads, 6-10 % faster on large trailing blocks).
#include "common.h"
#include "mfma_tile.h"

namespace skl {

constexpr int kSkThreads = 512;
constexpr int kWR = 64, kWC = 32;  // wave tile: rows i, columns j
constexpr int TRS = kWC + 2;       // LDS row of the epilogue transpose (spreads banks)

template <typename T>
__global__ __launch_bounds__(kSkThreads, 2) void skr2k_kernel(const double *__restrict__ Wc,
                                                              double *__restrict__ Wn, int ldw,
                                                              const int *__restrict__ perm,
                                                              int n, int cp, int K,
                                                              const T *__restrict__ uv,
                                                              int ntiles)
{
    typedef typename MfmaT<T>::acc4 acc4;
    constexpr int BR = kWR / 16, BC = kWC / 16; // 16x16 blocks per wave tile
    constexpr int WPR = TM / kWR;                // waves along the rows
    // LDS: double-buffered operand chunks during the K loop, k-major, rows
    // padded so that the four k-rows read by one fragment load fall in
    // different LDS banks; afterwards each wave reuses 16 x TRS doubles of
    // the same space to transpose its mirrored (upper) stores.
    constexpr size_t kOpBytes = sizeof(T) * 2 * KC * TMP;
    constexpr size_t kTrBytes = sizeof(double) * (kSkThreads / 64) * 16 * TRS;
    constexpr size_t kLds = (2 * kOpBytes > kTrBytes) ? 2 * kOpBytes : kTrBytes;
    __shared__ __attribute__((aligned(16))) char smem[kLds];
    T(*sI)[KC][TMP] = reinterpret_cast<T(*)[KC][TMP]>(smem);            // [U|V] rows i
    T(*sJ)[KC][TMP] = reinterpret_cast<T(*)[KC][TMP]>(smem + kOpBytes); // [-V|U] rows j
    __shared__ int sPi[TM], sPj[TM]; // source rows of the tile's rows and columns

    // XCD-grouped tile order
    const int nwg = gridDim.x;
    const int per_xcd = (nwg + 7) / 8;
    const int bid = blockIdx.x;
    const int tau = (bid & 7) * per_xcd + (bid >> 3);
    if (tau >= ntiles)
        return;
    int ti, tj;
    tile_of_blocked<4>(tau, (n - cp + TM - 1) / TM, &ti, &tj);
    const int i0 = cp + ti * TM;
    const int j0 = cp + tj * TM;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wi = wave % WPR, wj = wave / WPR;
    const int ib = i0 + wi * kWR; // this wave's rows
    const int jb = j0 + wj * kWC; // this wave's columns
    const bool active = !(ti == tj && jb >= ib + kWR);

    const int lrow = lane & 15; // row inside a 16-block
    const int lk = lane >> 4;   // k inside a 4-step, or row group of D

    // Source rows of the tile's rows and columns (loaded first, their latency
    // overlaps the first operand chunk).
    if (tid < TM) {
        const int g = i0 + tid;
        sPi[tid] = (g < n) ? perm[g] : 0;
    } else if (tid < 2 * TM) {
        const int g = j0 + tid - TM;
        sPj[tid - TM] = (g < n) ? perm[g] : 0;
    }
    constexpr bool kF64 = sizeof(T) == 8;
    auto csrc = [&](int gi, int gj) -> const double * {
        return Wc + (size_t)sPj[gj - j0] * ldw + sPi[gi - i0];
    };

    TileStage<T, kSkThreads> tk(sI, sJ, uv, uv + (size_t)K * n, n, n, i0, j0, K);
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
                    // rows/columns past n have source row 0: still in range
                    const double cv = *csrc(gi, gj);
                    v = (active && gi < n && gj < gi) ? (T)cv : (T)0;
                }
                acc[bi][bj][q] = v;
            }
        }
    }
    tk.template run<BR, BC>(acc, active, wi * kWR, wj * kWC, lrow, lk);
    if (!active)
        return;

    // D[m][nn] (m = MfmaT::drow(lane/16, q) : column j, nn = lane%16 : row i).
    // Lower entries (i, j) go straight out: sixteen lanes write 128
    // consecutive bytes of column j.  Their negations at (j, i) lie along
    // column i, so each 16-row block is staged in this wave's LDS rows and
    // written back one column i at a time: 32 consecutive j per half wave,
    // two columns i per store.
    double *tr = reinterpret_cast<double *>(smem) + wave * 16 * TRS;
    const int jl2 = lane % kWC;
#pragma unroll
    for (int bi = 0; bi < BR; ++bi) {
        const int gi = ib + bi * 16 + lrow;
#pragma unroll
        for (int bj = 0; bj < BC; ++bj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int jl = bj * 16 + MfmaT<T>::drow(lk, q);
                const int gj = jb + jl;
                double v = 0.0;
                if (gi < n && gj < gi) {
                    v = kF64 ? (double)acc[bi][bj][q] : *csrc(gi, gj) + (double)acc[bi][bj][q];
                    __builtin_nontemporal_store(v, &Wn[(size_t)gj * ldw + gi]);
                }
                tr[lrow * TRS + jl] = v;
            }
        }
        // the wave's own LDS writes are visible to its later reads (LDS
        // instructions of one wave execute in order)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int gj = jb + jl2;
#pragma unroll
        for (int r0 = 0; r0 < 16; r0 += 64 / kWC) {
            const int rr = r0 + lane / kWC;
            const int gi2 = ib + bi * 16 + rr;
            const double v = tr[rr * TRS + jl2];
            if (gi2 < n && gj < gi2)
                __builtin_nontemporal_store(-v, &Wn[(size_t)gi2 * ldw + gj]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

hipError_t launch_skr2k(const double *Wc, double *Wn, int n, int cp, int nq,
                        const FactorWs &ws, int precision, hipStream_t s)
{
    const int m = n - cp;
    if (m < 2 || nq <= 0)
        return hipSuccess;
    const int nt = (m + TM - 1) / TM;
    const int ntiles = nt * (nt + 1) / 2;
    const int per_xcd = (ntiles + 7) / 8;
    const int grid = per_xcd * 8;
    const int K = 2 * nq;
    (void)hipGetLastError(); // report this launch only
    if (precision == 1) {
        hipLaunchKernelGGL(skr2k_kernel<float>, dim3(grid), dim3(kSkThreads), 0, s, Wc, Wn, ws.ldw,
                           (const int *)ws.perm, n, cp, K, (const float *)ws.uv32, ntiles);
    } else {
        hipLaunchKernelGGL(skr2k_kernel<double>, dim3(grid), dim3(kSkThreads), 0, s, Wc, Wn, ws.ldw,
                           (const int *)ws.perm, n, cp, K, (const double *)ws.uv, ntiles);
    }
    return hipGetLastError();
}

}  // namespace skl
