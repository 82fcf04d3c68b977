// MFMA tile machinery shared by the trailing update (skr2k) and the
// left-looking panel update: a 128 x 128 output tile per workgroup, split
// into wave tiles that are grids of 16 x 16 MFMA blocks (skr2k: eight waves
// of 64 x 32; the panel update: four waves of 64 x 64), operands streamed
// through a double-buffered LDS stage in K-chunks of KC.  The operands are column-major with leading dimension ldo: opI
// holds the tile's rows i (columns = k), opJ the tile's columns j.  The MFMA
// computes the transposed tile D[j][i] += sum_k opJ[j][k] opI[i][k].
#pragma once

#include <hip/hip_runtime.h>

namespace skl {

constexpr int TM = 128;    // tile rows (i) and columns (j)
constexpr int TMP = 144;   // padded LDS row (k-rows 1152 B apart: banks shift by 128 B)
constexpr int KC = 16;     // K chunk staged in LDS

template <typename T> struct MfmaT;
// Output layout of the 16x16 MFMA result held by lane l (value q of 4),
// measured on gfx950: fp64 holds rows (l/16) + 4q, fp32 rows 4(l/16) + q;
// the column is l%16 for both.
template <> struct MfmaT<double> {
    typedef double __attribute__((ext_vector_type(4))) acc4;
    static __device__ __forceinline__ acc4 mma(double a, double b, acc4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int lk, int q) { return lk + 4 * q; }
};
template <> struct MfmaT<float> {
    typedef float __attribute__((ext_vector_type(4))) acc4;
    static __device__ __forceinline__ acc4 mma(float a, float b, acc4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int drow(int lk, int q) { return 4 * lk + q; }
};


// Operand staging of one TMV x TMV tile (128 unless stated; LDS rows padded
// to TMPV) shared by NT threads (NT / 64 waves): K-chunks of the two
// operands move from HBM to registers and from registers to a
// double-buffered LDS stage.  Every load is issued
// unconditionally (clamped address) and masked only when the chunk is
// written to LDS: with a fixed number of loads per chunk and no use right
// after them, the compiler waits for the chunk that is due while the
// prefetched one stays in flight (loads skipped by branches, or used at
// once, make it wait for all of them).
template <typename T, int NT, int TMV = TM, int TMPV = TMP>
struct TileStage {
    static constexpr int PER = (KC * TMV) / NT; // elements per thread per operand and chunk
    static_assert(PER * NT == KC * TMV, "threads divide a chunk");
    T (*sI)[KC][TMPV];
    T (*sJ)[KC][TMPV];
    const T *opI;
    const T *opJ;
    int ldo, n, i0, j0, K, nk, tid;
    T ri[PER], rj[PER];

    __device__ __forceinline__ TileStage(T (*sI_)[KC][TMPV], T (*sJ_)[KC][TMPV], const T *opI_,
                                         const T *opJ_, int ldo_, int n_, int i0_, int j0_, int K_)
        : sI(sI_), sJ(sJ_), opI(opI_), opJ(opJ_), ldo(ldo_), n(n_), i0(i0_), j0(j0_), K(K_),
          nk((K_ + KC - 1) / KC), tid(threadIdx.x)
    {
    }
    __device__ __forceinline__ void load_chunk(int kc)
    {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * NT;
            const int rr = e % TMV;
            const int k = kc * KC + e / TMV;
            const int kk = (k < K) ? k : 0;
            ri[q] = opI[(size_t)kk * ldo + min(i0 + rr, n - 1)];
            rj[q] = opJ[(size_t)kk * ldo + min(j0 + rr, n - 1)];
        }
    }
    __device__ __forceinline__ void store_chunk(int buf, int kc)
    {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = tid + q * NT;
            const int rr = e % TMV;
            const bool kok = kc * KC + e / TMV < K;
            sI[buf][e / TMV][rr] = (kok && i0 + rr < n) ? ri[q] : (T)0;
            sJ[buf][e / TMV][rr] = (kok && j0 + rr < n) ? rj[q] : (T)0;
        }
    }
    // the first chunk in LDS, the second in flight
    __device__ __forceinline__ void prologue()
    {
        load_chunk(0);
        store_chunk(0, 0);
        if (nk > 1)
            load_chunk(1);
        __syncthreads();
    }
    // acc[bi][bj] (16 x 16 block bi of this wave's WR rows, bj of its WC
    // columns; the wave's rows start at wr0 and its columns at wc0 inside
    // the tile) += the product over all K; ends with a barrier
    template <int BR, int BC, typename Acc>
    __device__ __forceinline__ void run(Acc (&acc)[BR][BC], bool active, int wr0, int wc0,
                                        int lrow, int lk)
    {
        for (int kc = 0; kc < nk; ++kc) {
            const int cur = kc & 1;
            if (kc + 1 < nk) {
                store_chunk(cur ^ 1, kc + 1); // buffer freed by the barrier ending step kc-1
                if (kc + 2 < nk)
                    load_chunk(kc + 2); // in flight during this chunk's MFMAs
            }
            if (active) {
#pragma unroll
                for (int ks = 0; ks < KC; ks += 4) {
                    T fa[BC], fb[BR];
#pragma unroll
                    for (int bj = 0; bj < BC; ++bj)
                        fa[bj] = sJ[cur][ks + lk][wc0 + bj * 16 + lrow];
#pragma unroll
                    for (int bi = 0; bi < BR; ++bi)
                        fb[bi] = sI[cur][ks + lk][wr0 + bi * 16 + lrow];
#pragma unroll
                    for (int bi = 0; bi < BR; ++bi)
#pragma unroll
                        for (int bj = 0; bj < BC; ++bj)
                            acc[bi][bj] = MfmaT<T>::mma(fa[bj], fb[bi], acc[bi][bj]);
                }
            }
            __syncthreads();
        }
    }
};

// The four-wave form (256 threads, 64 x 64 per wave) used by the
// left-looking panel update.
template <typename T>
struct TileK : TileStage<T, 256> {
    using TileStage<T, 256>::TileStage;
    template <typename Acc>
    __device__ __forceinline__ void run(Acc (&acc)[4][4], bool active, int wi, int wj, int lrow,
                                        int lk)
    {
        TileStage<T, 256>::template run<4, 4>(acc, active, wi * 64, wj * 64, lrow, lk);
    }
};

}  // namespace skl
