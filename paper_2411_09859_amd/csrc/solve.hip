// Solving A X = B with the factors of the pivoted LTL^T.
//
// Paper (arXiv 2411.09859): the factorization P A P^T = L T L^T (Sec. 3.2,
// pivoting Sec. 3.7) is used to solve skew-symmetric systems (Sec. 1), so
//     X = P^T L^{-T} T^{-1} L^{-1} P B.
// Stages, each a kernel (or a block-sequential chain of them):
//   1. the row permutation: (P B)[i] = B[q[i]], q the identity with the
//      transpositions (r, ipiv[r]) applied for r = 1 .. n-1 in order;
//   2. the unit lower solve, in blocks of kSB columns: the block's triangle
//      is solved in LDS by one workgroup, then the rows below are updated by
//      a column-coalesced product with the solved block;
//   3. the skew tridiagonal solve: with T[i+1][i] = t[i] = -T[i][i+1], the
//      even rows give the odd unknowns by a forward recurrence and the odd
//      rows the even unknowns by a backward one (n even);
//   4. the L^T solve, blocks from the bottom: the block's rows are updated
//      with the solved part below (one workgroup per column, deterministic
//      reduction), then the block's triangle is solved in LDS;
//   5. the inverse permutation: X[q[i]] = Y[i].
// L is read where the factorization left it: L[i][j] = LT[i][j-1] for
// i > j >= 1, L[i][0] = 0 for i > 0, unit diagonal.
#include "common.h"
#include "pivot_walk.h"

namespace skl {

constexpr int kSB = 128;  // solve block (columns of L per block)
constexpr int kRC = 8;    // right-hand sides per pass
constexpr int kSBP = kSB + 1;

__device__ __forceinline__ double lval(const double *__restrict__ LT, int lda, int i, int j)
{
    // L[i][j] for i > j
    return (j >= 1) ? LT[(size_t)(j - 1) * lda + i] : 0.0;
}

// q[i] = image of i under the transpositions applied last to first (one
// wave per kWalkI indices, pivots staged in LDS).
__global__ __launch_bounds__(256) void perm_map_kernel(const int *__restrict__ ipiv, int n,
                                                       int *__restrict__ q)
{
    __shared__ int sp[kWalkStage];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i0 = (blockIdx.x * 4 + wave) * kWalkI;
    const int imax = i0 + kWalkI - 1;
    int v[kWalkI];
#pragma unroll
    for (int k = 0; k < kWalkI; ++k)
        v[k] = i0 + k;
    for (int hi = n - 1; hi >= 1; hi -= kWalkStage) {
        const int lo = max(1, hi - kWalkStage + 1);
        __syncthreads();
        walk_stage(ipiv, lo, hi, sp);
        __syncthreads();
        if (i0 < n) {
            for (int R = min(hi, imax); R >= lo; R -= 64) {
                const int len = min(64, R - lo + 1);
                const int pr = sp[max(R - lane, lo) - lo];
                walk_chunk(v, i0, R, len, pr);
            }
        }
    }
    walk_store(v, i0, n, lane, q);
}

// Y[i][k] = B[q[i]][k] (gather) or B[q[i]][k] = Y[i][k] (scatter).
__global__ void permute_rows_kernel(double *__restrict__ B, int ldb, double *__restrict__ Y,
                                    int ldy, const int *__restrict__ q, int n, int nrhs,
                                    int scatter)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n * nrhs)
        return;
    const int i = (int)(e % n), k = (int)(e / n);
    int src = q[i];
    if (src < 0 || src >= n)
        src = i; // cannot happen for pivots of a factorization; keeps the access in range
    if (scatter)
        B[(size_t)k * ldb + src] = Y[(size_t)k * ldy + i];
    else
        Y[(size_t)k * ldy + i] = B[(size_t)k * ldb + src];
}

// Triangle of the block [c0, c0+bs): Lb[j][i] = L[c0+i][c0+j] for i > j.
__device__ __forceinline__ void load_block_triangle(double *Lb, const double *__restrict__ LT,
                                                    int lda, int c0, int bs)
{
    for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
        const int j = e / bs, i = e - j * bs;
        Lb[j * kSBP + i] = (i > j) ? lval(LT, lda, c0 + i, c0 + j) : 0.0;
    }
}

// Forward solve of the block's unit lower triangle, in place on Y.
__global__ __launch_bounds__(256) void trsv_lower_block_kernel(const double *__restrict__ LT,
                                                               int lda, int c0, int bs,
                                                               double *__restrict__ Y, int ldy,
                                                               int nrhs)
{
    extern __shared__ double lds[];
    double *Lb = lds;                 // kSB x kSBP
    double *yb = lds + kSB * kSBP;    // kRC x kSB
    load_block_triangle(Lb, LT, lda, c0, bs);
    for (int k0 = 0; k0 < nrhs; k0 += kRC) {
        const int kc = min(kRC, nrhs - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < kc * bs; e += blockDim.x) {
            const int kk = e / bs, i = e - kk * bs;
            yb[kk * kSB + i] = Y[(size_t)(k0 + kk) * ldy + c0 + i];
        }
        __syncthreads();
        for (int j = 0; j + 1 < bs; ++j) {
            for (int e = threadIdx.x; e < kc * bs; e += blockDim.x) {
                const int kk = e / bs, i = e - kk * bs;
                if (i > j)
                    yb[kk * kSB + i] -= Lb[j * kSBP + i] * yb[kk * kSB + j];
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < kc * bs; e += blockDim.x) {
            const int kk = e / bs, i = e - kk * bs;
            Y[(size_t)(k0 + kk) * ldy + c0 + i] = yb[kk * kSB + i];
        }
    }
}

// Rows below the block: Y[i] -= L[i][c0:c0+bs] * Y[c0:c0+bs] for i >= c0+bs.
__global__ __launch_bounds__(256) void lower_update_kernel(const double *__restrict__ LT, int lda,
                                                           int n, int c0, int bs,
                                                           double *__restrict__ Y, int ldy,
                                                           int nrhs)
{
    __shared__ double zb[kRC][kSB];
    const int i = c0 + bs + blockIdx.x * blockDim.x + threadIdx.x;
    for (int k0 = 0; k0 < nrhs; k0 += kRC) {
        const int kc = min(kRC, nrhs - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < kRC * kSB; e += blockDim.x) {
            const int kk = e / kSB, j = e - kk * kSB;
            zb[kk][j] = (kk < kc && j < bs) ? Y[(size_t)(k0 + kk) * ldy + c0 + j] : 0.0;
        }
        __syncthreads();
        if (i < n) {
            double acc[kRC];
#pragma unroll
            for (int kk = 0; kk < kRC; ++kk)
                acc[kk] = 0.0;
            for (int j = 0; j < bs; ++j) {
                const double l = lval(LT, lda, i, c0 + j);
#pragma unroll
                for (int kk = 0; kk < kRC; ++kk)
                    acc[kk] += l * zb[kk][j];
            }
            for (int kk = 0; kk < kc; ++kk)
                Y[(size_t)(k0 + kk) * ldy + i] -= acc[kk];
        }
    }
}

// T U = Y for the skew tridiagonal T (n even):
//   even row 2i:  t[2i-1] u[2i-1] - t[2i] u[2i+1] = y[2i]
//   odd row 2i+1: t[2i] u[2i] - t[2i+1] u[2i+2] = y[2i+1]   (u[n] = 0)
// One workgroup per (right-hand side, chain): the odd unknowns run forward
// from the even rows, the even unknowns backward from the odd rows.  For a
// chunk of the chain the workgroup forms each step as an affine map
// u = a u_prev + c (a = t_side / t[2i], c = -+ y / t[2i]) in parallel, then
// thread 0 runs the chain (one FMA per step) and the workgroup writes the
// chunk back.
constexpr int kTC = 2048; // chain steps per chunk
__global__ __launch_bounds__(256) void tridiag_skew_solve_kernel(const double *__restrict__ t,
                                                                 int n,
                                                                 const double *__restrict__ Y,
                                                                 int ldy, double *__restrict__ U,
                                                                 int ldu, int nrhs)
{
    __shared__ double ca[kTC], cc[kTC], us[kTC];
    const int k = blockIdx.x >> 1;
    const bool fwd = (blockIdx.x & 1) == 0;
    if (k >= nrhs)
        return;
    const double *y = Y + (size_t)k * ldy;
    double *u = U + (size_t)k * ldu;
    const int half = n / 2;
    double carry = 0.0; // u[2i-1] (forward) or u[2i+2] (backward)
    for (int s0 = 0; s0 < half; s0 += kTC) {
        const int len = min(kTC, half - s0);
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            const int i = fwd ? s0 + q : half - 1 - (s0 + q);
            const double piv = t[2 * i];
            if (fwd) {
                ca[q] = ((i > 0) ? t[2 * i - 1] : 0.0) / piv;
                cc[q] = -y[2 * i] / piv;
            } else {
                ca[q] = ((2 * i + 1 < n - 1) ? t[2 * i + 1] : 0.0) / piv;
                cc[q] = y[2 * i + 1] / piv;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // batches of 16 coefficients are read ahead of their FMAs
            int q = 0;
            for (; q + 16 <= len; q += 16) {
                double a[16], c[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    a[j] = ca[q + j];
                    c[j] = cc[q + j];
                }
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    carry = fma(a[j], carry, c[j]);
                    us[q + j] = carry;
                }
            }
            for (; q < len; ++q) {
                carry = fma(ca[q], carry, cc[q]);
                us[q] = carry;
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < len; q += blockDim.x) {
            const int i = fwd ? s0 + q : half - 1 - (s0 + q);
            u[fwd ? 2 * i + 1 : 2 * i] = us[q];
        }
        __syncthreads();
    }
}

// Rows of the block from the solved part below: U[j] -= sum_{i >= c0+bs}
// L[i][j] U[i] for j in [c0, c0+bs); one workgroup per column j.
__global__ __launch_bounds__(256) void upper_update_kernel(const double *__restrict__ LT, int lda,
                                                           int n, int c0, int bs,
                                                           double *__restrict__ U, int ldu,
                                                           int nrhs)
{
    __shared__ double red[kRC][256];
    const int j = c0 + blockIdx.x;
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < nrhs; k0 += kRC) {
        const int kc = min(kRC, nrhs - k0);
        double acc[kRC];
#pragma unroll
        for (int kk = 0; kk < kRC; ++kk)
            acc[kk] = 0.0;
        for (int i = c0 + bs + tid; i < n; i += 256) {
            const double l = lval(LT, lda, i, j);
#pragma unroll
            for (int kk = 0; kk < kRC; ++kk)
                acc[kk] += (kk < kc) ? l * U[(size_t)(k0 + kk) * ldu + i] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kRC; ++kk)
            red[kk][tid] = acc[kk];
        __syncthreads();
        for (int s = 128; s >= 1; s >>= 1) {
            if (tid < s) {
#pragma unroll
                for (int kk = 0; kk < kRC; ++kk)
                    red[kk][tid] += red[kk][tid + s];
            }
            __syncthreads();
        }
        if (tid < kc)
            U[(size_t)(k0 + tid) * ldu + j] -= red[tid][0];
    }
}

// Backward solve of the block's triangle with L^T (unit upper), in place.
__global__ __launch_bounds__(256) void trsv_upper_block_kernel(const double *__restrict__ LT,
                                                               int lda, int c0, int bs,
                                                               double *__restrict__ U, int ldu,
                                                               int nrhs)
{
    extern __shared__ double lds[];
    double *Lb = lds;
    double *ub = lds + kSB * kSBP;
    load_block_triangle(Lb, LT, lda, c0, bs);
    for (int k0 = 0; k0 < nrhs; k0 += kRC) {
        const int kc = min(kRC, nrhs - k0);
        __syncthreads();
        for (int e = threadIdx.x; e < kc * bs; e += blockDim.x) {
            const int kk = e / bs, i = e - kk * bs;
            ub[kk * kSB + i] = U[(size_t)(k0 + kk) * ldu + c0 + i];
        }
        __syncthreads();
        // x_j final; then u_i -= L[c0+j][c0+i] x_j for i < j
        for (int j = bs - 1; j >= 1; --j) {
            for (int e = threadIdx.x; e < kc * bs; e += blockDim.x) {
                const int kk = e / bs, i = e - kk * bs;
                if (i < j)
                    ub[kk * kSB + i] -= Lb[i * kSBP + j] * ub[kk * kSB + j];
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < kc * bs; e += blockDim.x) {
            const int kk = e / bs, i = e - kk * bs;
            U[(size_t)(k0 + kk) * ldu + c0 + i] = ub[kk * kSB + i];
        }
    }
}

// ---- single-launch triangular solves ---------------------------------------
// One workgroup per block of kFB rows (all resident: cooperative launch).
// The solution goes to a separate array that is filled beforehand with a
// "pending" marker, a signaling NaN, which arithmetic never produces; a
// value other than the marker is final.  Workgroup b takes the contributions
// of the other blocks as their values appear, then solves its own diagonal
// block in one wave per right-hand side (lane = row, the pivot value
// broadcast with readlane, no barriers) and stores it.  A consumer polls the
// values it needs directly, so the chain between consecutive blocks is one
// store-to-load round trip plus the 64-step in-register solve; everything
// else (reading L once, 8 n^2 / 2 bytes) overlaps with it.  Bounded waits: a
// block that never appears poisons the result with a quiet NaN instead of
// hanging.
constexpr int kFB = 64;
constexpr long kSolveSpin = 1L << 22;
constexpr unsigned long long kPending = 0xfff7a5a5a5a5a5a5ull;

__device__ __forceinline__ double ld_dev(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool is_pending(double x)
{
    return (unsigned long long)__double_as_longlong(x) == kPending;
}
__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__global__ void fill_pending_kernel(double *__restrict__ p, size_t count)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = __longlong_as_double((long long)kPending);
}

// Loads the 16 x NR values z[k][jj] = X[k * ldx + idx(jj)] of another block
// once none of them is pending (false if the wait runs out).
template <int NR, class Idx>
__device__ __forceinline__ bool poll16(const double *X, int ldx, Idx idx, double (&z)[NR][16])
{
    for (long spins = 0;; ++spins) {
        bool pend = false;
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                z[k][jj] = ld_dev(&X[(size_t)k * ldx + idx(jj)]);
                pend |= is_pending(z[k][jj]);
            }
        if (__ballot(pend) == 0)
            return true;
        if (spins > kSolveSpin)
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
}
// Per lane: the value at p once no lane's value is pending.
__device__ __forceinline__ bool poll_lane(const double *p, double *z)
{
    for (long spins = 0;; ++spins) {
        *z = ld_dev(p);
        if (__ballot(is_pending(*z)) == 0)
            return true;
        if (spins > kSolveSpin)
            return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Forward: Z[b] := L_bb^{-1} (Y[b] - sum_{c<b} L_bc Z[c]), blocks ascending.
// Wave w takes columns 16w .. 16w+15 of every earlier block but the last
// (lane = row); the last one is on the critical path and taken by the waves
// that solve, one per right-hand side.
template <int NR>
__global__ __launch_bounds__(256) void trsv_lower_sf_kernel(const double *__restrict__ LT, int lda,
                                                            int n, const double *__restrict__ Y,
                                                            int ldy, double *__restrict__ Z, int ldz)
{
    __shared__ double Ld[kFB][kFB + 1]; // Ld[j][i] = L[r0+i][r0+j]
    __shared__ double part[4][NR][kFB];
    __shared__ int fail;
    const int b = blockIdx.x, r0 = b * kFB, h = min(kFB, n - r0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0)
        fail = 0;
    for (int e = tid; e < kFB * kFB; e += 256) {
        const int j = e / kFB, i = e - j * kFB;
        Ld[j][i] = (i > j && i < h) ? lval(LT, lda, r0 + i, r0 + j) : 0.0;
    }
    const int row = min(r0 + lane, n - 1);
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k)
        acc[k] = 0.0;
    bool ok = true;
    for (int c = 0; c + 1 < b && ok; ++c) {
        const int c0 = c * kFB + wave * 16;
        double l[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            l[jj] = lval(LT, lda, row, c0 + jj); // row >= r0 > column: below the diagonal
        double z[NR][16];
        ok = poll16<NR>(Z, ldz, [&](int jj) { return c0 + jj; }, z);
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int jj = 0; jj < 16; ++jj)
                acc[k] += l[jj] * z[k][jj];
    }
    if (!ok)
        fail = 1;
#pragma unroll
    for (int k = 0; k < NR; ++k)
        part[wave][k][lane] = acc[k];
    __syncthreads();
    if (wave < NR) {
        const int k = wave;
        bool bad = fail != 0;
        double y = 0.0;
        if (lane < h)
            y = Y[(size_t)k * ldy + r0 + lane] - ((part[0][k][lane] + part[1][k][lane]) +
                                                  (part[2][k][lane] + part[3][k][lane]));
        // the block just before: its L rows are read before waiting, its
        // solution with one load per lane, then applied column by column
        // with the value broadcast by readlane
        if (b >= 1) {
            const int c0 = (b - 1) * kFB;
            double l[kFB];
#pragma unroll
            for (int jj = 0; jj < kFB; ++jj)
                l[jj] = lval(LT, lda, row, c0 + jj);
            double zv;
            if (!poll_lane(&Z[(size_t)k * ldz + c0 + lane], &zv))
                bad = true;
#pragma unroll
            for (int jj = 0; jj < kFB; ++jj)
                y -= l[jj] * readlane_f64(zv, jj);
        }
        for (int j = 0; j + 1 < h; ++j) {
            const double zj = readlane_f64(y, j);
            if (lane > j)
                y -= Ld[j][lane] * zj;
        }
        if (bad)
            y = __longlong_as_double(0x7ff8000000000000ll);
        if (lane < h)
            st_dev(&Z[(size_t)k * ldz + r0 + lane], y);
    }
}

// Backward: X[b] := L_bb^{-T} (U[b] - sum_{c>b} L_cb^T X[c]), blocks
// descending.  Wave w takes rows 16w .. 16w+15 of every later block but the
// nearest; lane = column of block b (the 16 rows of one column are one
// 128-byte line).
template <int NR>
__global__ __launch_bounds__(256) void trsv_upper_sf_kernel(const double *__restrict__ LT, int lda,
                                                            int n, const double *__restrict__ U,
                                                            int ldu, double *__restrict__ X, int ldx)
{
    __shared__ double Ld[kFB][kFB + 1]; // Ld[j][i] = L[r0+i][r0+j]
    __shared__ double part[4][NR][kFB];
    __shared__ int fail;
    const int nb = gridDim.x;
    const int b = blockIdx.x, r0 = b * kFB, h = min(kFB, n - r0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0)
        fail = 0;
    for (int e = tid; e < kFB * kFB; e += 256) {
        const int j = e / kFB, i = e - j * kFB;
        Ld[j][i] = (i > j && i < h) ? lval(LT, lda, r0 + i, r0 + j) : 0.0;
    }
    const int col = min(r0 + lane, n - 1);
    double acc[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k)
        acc[k] = 0.0;
    bool ok = true;
    for (int c = nb - 1; c > b + 1 && ok; --c) {
        const int i0 = c * kFB + wave * 16;
        const int cnt = min(16, n - i0); // rows of this slice that exist
        double l[16];
        // rows past n (last block) are clamped and their terms dropped, so
        // no address leaves the matrix even if a load is speculated
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) {
            const double lv = lval(LT, lda, min(i0 + ii, n - 1), col);
            l[ii] = (ii < cnt) ? lv : 0.0;
        }
        double x[NR][16];
        ok = poll16<NR>(X, ldx, [&](int ii) { return min(i0 + ii, n - 1); }, x);
#pragma unroll
        for (int k = 0; k < NR; ++k)
#pragma unroll
            for (int ii = 0; ii < 16; ++ii)
                acc[k] += l[ii] * x[k][ii];
    }
    if (!ok)
        fail = 1;
#pragma unroll
    for (int k = 0; k < NR; ++k)
        part[wave][k][lane] = acc[k];
    __syncthreads();
    if (wave < NR) {
        const int k = wave;
        bool bad = fail != 0;
        double y = 0.0;
        if (lane < h)
            y = U[(size_t)k * ldu + r0 + lane] - ((part[0][k][lane] + part[1][k][lane]) +
                                                  (part[2][k][lane] + part[3][k][lane]));
        // the block just after (lane = column of block b; row i of block
        // b+1 of that column, read before waiting)
        if (b + 1 < nb) {
            const int i0 = (b + 1) * kFB;
            const int cnt = min(kFB, n - i0);
            double l[kFB];
#pragma unroll
            for (int ii = 0; ii < kFB; ++ii) {
                const double lv = lval(LT, lda, min(i0 + ii, n - 1), col);
                l[ii] = (ii < cnt) ? lv : 0.0;
            }
            double xv;
            if (!poll_lane(&X[(size_t)k * ldx + min(i0 + lane, n - 1)], &xv))
                bad = true;
#pragma unroll
            for (int ii = 0; ii < kFB; ++ii)
                y -= l[ii] * readlane_f64(xv, ii);
        }
        // x_j final (j descending); u_i -= L[r0+j][r0+i] x_j for i < j
        for (int j = h - 1; j >= 1; --j) {
            const double xj = readlane_f64(y, j);
            if (lane < j)
                y -= Ld[lane][j] * xj;
        }
        if (bad)
            y = __longlong_as_double(0x7ff8000000000000ll);
        if (lane < h)
            st_dev(&X[(size_t)k * ldx + r0 + lane], y);
    }
}

// Launch one single-launch solve for up to 4 right-hand sides (In -> Out,
// Out filled with the pending marker); returns
// hipErrorCooperativeLaunchTooLarge (or another error) when it cannot run.
static hipError_t launch_sf(bool lower, int nr, const double *LT, int lda, int n, const double *In,
                            double *Out, int ld, hipStream_t s)
{
    const int nb = (n + kFB - 1) / kFB;
    const size_t cnt = (size_t)ld * nr;
    hipLaunchKernelGGL(fill_pending_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                       Out, cnt);
    void *args[] = {(void *)&LT, (void *)&lda, (void *)&n, (void *)&In,
                    (void *)&ld, (void *)&Out, (void *)&ld};
    const void *fn = nullptr;
    switch (nr) {
    case 1: fn = lower ? (const void *)trsv_lower_sf_kernel<1> : (const void *)trsv_upper_sf_kernel<1>; break;
    case 2: fn = lower ? (const void *)trsv_lower_sf_kernel<2> : (const void *)trsv_upper_sf_kernel<2>; break;
    case 3: fn = lower ? (const void *)trsv_lower_sf_kernel<3> : (const void *)trsv_upper_sf_kernel<3>; break;
    default: fn = lower ? (const void *)trsv_lower_sf_kernel<4> : (const void *)trsv_upper_sf_kernel<4>; break;
    }
    return hipLaunchCooperativeKernel(fn, dim3(nb), dim3(256), args, 0, s);
}

// Whether every block of the single-launch solves for nr right-hand sides
// can be resident at once.
static bool sf_fits(int n, int nr)
{
    static int per_cu[5] = {-1, -1, -1, -1, -1};
    if (nr < 1 || nr > 4)
        return false;
    if (per_cu[nr] < 0) {
        const void *lo = nullptr, *up = nullptr;
        switch (nr) {
        case 1: lo = (const void *)trsv_lower_sf_kernel<1>; up = (const void *)trsv_upper_sf_kernel<1>; break;
        case 2: lo = (const void *)trsv_lower_sf_kernel<2>; up = (const void *)trsv_upper_sf_kernel<2>; break;
        case 3: lo = (const void *)trsv_lower_sf_kernel<3>; up = (const void *)trsv_upper_sf_kernel<3>; break;
        default: lo = (const void *)trsv_lower_sf_kernel<4>; up = (const void *)trsv_upper_sf_kernel<4>; break;
        }
        int a = 0, c = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, lo, 256, 0) != hipSuccess)
            a = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c, up, 256, 0) != hipSuccess)
            c = 0;
        per_cu[nr] = a < c ? a : c;
    }
    const int nb = (n + kFB - 1) / kFB;
    return per_cu[nr] > 0 && (long)nb <= (long)per_cu[nr] * device_cu_count();
}

static const size_t kSolveLds = sizeof(double) * (size_t)(kSB * kSBP + kRC * kSB);

void solve_init_attrs()
{
    (void)hipFuncSetAttribute((const void *)trsv_lower_block_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSolveLds);
    (void)hipFuncSetAttribute((const void *)trsv_upper_block_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSolveLds);
}

size_t solve_ws_layout(int n, int nrhs, SolveWs *ws, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = (off + bytes + kAlign - 1) / kAlign * kAlign;
        return base ? base + o : nullptr;
    };
    SolveWs w{};
    w.ld = n > 0 ? n : 1;
    w.q = (int *)take(sizeof(int) * (size_t)w.ld);
    w.Y = (double *)take(sizeof(double) * (size_t)w.ld * (size_t)(nrhs > 0 ? nrhs : 1));
    w.U = (double *)take(sizeof(double) * (size_t)w.ld * (size_t)(nrhs > 0 ? nrhs : 1));
    w.bytes = off;
    if (ws)
        *ws = w;
    return off;
}

hipError_t launch_solve(int n, int nrhs, const double *LT, int lda, const double *t,
                        const int *ipiv, double *B, int ldb, const SolveWs &ws, hipStream_t s)
{
    // single-launch path: P B -> Y, L^{-1} Y -> U, T^{-1} U -> Y, L^{-T} Y -> U
    // block path:         P B -> Y, L^{-1} in place, T^{-1} Y -> U, L^{-T} in place
    // then the solution in U goes back through P^T
    (void)hipGetLastError(); // report these launches only
    const int ld = ws.ld;
    const size_t tot = (size_t)n * nrhs;
    const unsigned pgrid = (unsigned)((tot + 255) / 256);
    const bool sf = nrhs <= 4 && sf_fits(n, nrhs);
    hipLaunchKernelGGL(perm_map_kernel, dim3((n + 4 * kWalkI - 1) / (4 * kWalkI)), dim3(256), 0,
                       s, ipiv, n, ws.q);
    hipLaunchKernelGGL(permute_rows_kernel, dim3(pgrid), dim3(256), 0, s, B, ldb, ws.Y, ld,
                       (const int *)ws.q, n, nrhs, 0);
    if (sf) {
        hipError_t e = launch_sf(true, nrhs, LT, lda, n, ws.Y, ws.U, ld, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(tridiag_skew_solve_kernel, dim3(2 * nrhs), dim3(256), 0, s, t, n,
                           (const double *)ws.U, ld, ws.Y, ld, nrhs);
        e = launch_sf(false, nrhs, LT, lda, n, ws.Y, ws.U, ld, s);
        if (e != hipSuccess)
            return e;
    } else {
        for (int c0 = 0; c0 < n; c0 += kSB) {
            const int bs = min(kSB, n - c0);
            hipLaunchKernelGGL(trsv_lower_block_kernel, dim3(1), dim3(256), kSolveLds, s, LT, lda,
                               c0, bs, ws.Y, ld, nrhs);
            const int below = n - c0 - bs;
            if (below > 0)
                hipLaunchKernelGGL(lower_update_kernel, dim3((below + 255) / 256), dim3(256), 0, s,
                                   LT, lda, n, c0, bs, ws.Y, ld, nrhs);
        }
        hipLaunchKernelGGL(tridiag_skew_solve_kernel, dim3(2 * nrhs), dim3(256), 0, s, t, n,
                           (const double *)ws.Y, ld, ws.U, ld, nrhs);
        const int nbs = (n + kSB - 1) / kSB;
        for (int B_ = nbs - 1; B_ >= 0; --B_) {
            const int c0 = B_ * kSB, bs = min(kSB, n - c0);
            if (n - c0 - bs > 0)
                hipLaunchKernelGGL(upper_update_kernel, dim3(bs), dim3(256), 0, s, LT, lda, n, c0,
                                   bs, ws.U, ld, nrhs);
            hipLaunchKernelGGL(trsv_upper_block_kernel, dim3(1), dim3(256), kSolveLds, s, LT, lda,
                               c0, bs, ws.U, ld, nrhs);
        }
    }
    hipLaunchKernelGGL(permute_rows_kernel, dim3(pgrid), dim3(256), 0, s, B, ldb, ws.U, ld,
                       (const int *)ws.q, n, nrhs, 1);
    return hipGetLastError();
}

}  // namespace skl
