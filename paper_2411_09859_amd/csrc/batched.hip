// Batched small factorizations: many independent pivoted LTL^T + Pfaffians
// in one persistent launch.
//
// Paper (arXiv 2411.09859): each matrix is factored with the fused blocked
// right-looking algorithm (Sec. 3.6.3) with a small panel width bs: the panel
// is the pivoted left-looking algorithm over the whole trailing matrix
// (Sec. 3.7.3, skew_tridiag_gemv of Sec. 3.5.4), the trailing update is the
// skew rank-2k form C -= U V^T - V U^T of Theorem "TandS" (Sec. 2.2) and
// Sec. 3.6.5; with bs = 2 this is the two-step algorithm of Sec. 3.5.2.  The
// Pfaffian is det(P) * prod_i T[2i][2i+1] (Sec. 1).
//
// One workgroup of 256 threads handles one matrix at a time (n <= 256, thread
// i owns trailing row i).  The workgroups take matrices from a device queue
// (one atomic per matrix), so the whole batch is one launch with no host
// synchronization and the launch can be captured in a hipGraph.  The
// trailing matrix stays in the caller's buffer (L2-resident at these sizes);
// the panel rows of L, the operands U and V and the pivots live in LDS.  The
// arithmetic of a matrix depends only on that matrix and on bs, never on
// which workgroup runs it or on the other matrices.
#include "../../include/skltlt.h"
#include "batched_table.h"
#include "common.h"

#include <climits>
#include <cmath>

namespace skl {

constexpr int kBT = 256;     // threads per workgroup = largest order
constexpr int kBMaxBs = 16;  // largest panel width (2 workgroups per CU)
constexpr int kBLd = kBMaxBs + 2;

__device__ __forceinline__ bool beats_b(double av, int ai, double bv, int bi)
{
    const double aa = fabs(av), bb = fabs(bv);
    return (aa > bb) || (aa == bb && ai < bi);
}

// Panel width for order n (block_size = 0): from the tuning table.
__device__ __host__ inline int batched_bs_for(int n)
{
    for (const BatchedTune &e : kBatchedTune)
        if (n <= e.n_max)
            return e.bs;
    return kBMaxBs;
}

struct BatchShared {
    double Lp[kBT][kBLd]; // panel rows of L, rows indexed by trailing row
    double U[kBT][kBMaxBs / 2 + 1];
    double V[kBT][kBMaxBs / 2 + 1];
    double hrow[kBLd];
    double hv[kBLd];
    double tl[kBT];
    int pv[kBT];
    int gmap[kBT];
    double red_v[kBT / 64];
    int red_i[kBT / 64];
    double bc_tau, bc_xr;
    int bc_p;
    int bc_idx;
    double rsum[kBT / 64];
    int rneg[kBT / 64], rzero[kBT / 64];
};

__device__ void factor_one(BatchShared &sh, double *__restrict__ A, int lda, int n,
                           double *__restrict__ t, int *__restrict__ ipiv, int bs)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0 && n >= 1)
        ipiv[0] = 0;
    if (n < 2)
        return;

    for (int k0 = 0; k0 < n - 1; k0 += bs) {
        const int nb = min(bs, n - 1 - k0);
        const int base = k0 + 1;
        const int i = tid; // this thread's row
        const bool valid = (i >= base) && (i < n);
        // panel start: column 0 of the panel is the carried column, kept in
        // Lp[.][nb_prev] of the previous panel (moved to column 0 below)
        __syncthreads();
        if (valid) {
            const double carried = (k0 == 0) ? 0.0 : sh.Lp[i][kBLd - 1];
            sh.Lp[i][0] = carried;
        }
        for (int a = tid; a < kBLd; a += kBT)
            sh.hrow[a] = 0.0;
        double ycol = valid ? A[(size_t)k0 * lda + i] : 0.0;
        __syncthreads();

        for (int j = 0; j < nb; ++j) {
            const int c = k0 + j;
            const int r = c + 1;
            const bool last = (r == k0 + nb);
            // h = T_p L[c, panel]^T (L[c][j] = 1)
            if (tid <= j) {
                const int a = tid;
                double v = 0.0;
                if (a + 1 <= j)
                    v -= sh.tl[k0 + a] * ((a + 1 < j) ? sh.hrow[a + 1] : 1.0);
                if (a >= 1)
                    v += sh.tl[k0 + a - 1] * sh.hrow[a - 1];
                sh.hv[a] = v;
            }
            __syncthreads();
            const bool cand = valid && (i >= r);
            double x = 0.0;
            if (cand) {
                double s = 0.0;
                for (int a = 0; a <= j; ++a)
                    s += sh.Lp[i][a] * sh.hv[a];
                x = ycol - s;
            }
            // argmax over the workgroup (first index on ties)
            double cv = cand ? x : 0.0;
            int ci = cand ? i : INT_MAX;
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(cv, off, 64);
                const int oi = __shfl_xor(ci, off, 64);
                if (beats_b(ov, oi, cv, ci)) {
                    cv = ov;
                    ci = oi;
                }
            }
            if (lane == 0) {
                sh.red_v[wave] = cv;
                sh.red_i[wave] = ci;
            }
            __syncthreads();
            if (tid == 0) {
                double bv = sh.red_v[0];
                int bi = sh.red_i[0];
                for (int q = 1; q < kBT / 64; ++q)
                    if (beats_b(sh.red_v[q], sh.red_i[q], bv, bi)) {
                        bv = sh.red_v[q];
                        bi = sh.red_i[q];
                    }
                if (bi < r || bi >= n) { // cannot happen: row r is a candidate
                    bi = r;
                    bv = __longlong_as_double(0x7ff8000000000000ll);
                }
                sh.bc_tau = bv;
                sh.bc_p = bi;
                sh.tl[c] = bv;
                sh.pv[r] = bi;
            }
            __syncthreads();
            const int p = sh.bc_p;
            const double tau = sh.bc_tau;
            // pivot row of L for the next step's h (row p before the
            // exchange); row r hands its x to row p
            if (tid <= j)
                sh.hrow[tid] = sh.Lp[p][tid];
            if (i == r)
                sh.bc_xr = x;
            __syncthreads();
            if (p != r && tid <= j) {
                // exchange rows r and p of the panel's L (columns 0..j)
                const double tmp = sh.Lp[r][tid];
                sh.Lp[r][tid] = sh.Lp[p][tid];
                sh.Lp[p][tid] = tmp;
            }
            if (i == p && p != r)
                x = sh.bc_xr;
            // symmetric exchange r <-> p of the trailing matrix (lower
            // storage), then ycol = Y'[i, r]
            if (valid && i > r) {
                double *colr = A + (size_t)r * lda;
                double ynew;
                if (p == r) {
                    ynew = colr[i];
                } else if (i > p) {
                    double *colp = A + (size_t)p * lda;
                    const double av = colr[i];
                    const double bv = colp[i];
                    colp[i] = av;
                    if (last)
                        colr[i] = bv;
                    ynew = bv;
                } else if (i < p) {
                    double *pi = A + (size_t)i * lda + p;
                    const double av = colr[i];
                    const double bv = *pi;
                    *pi = -av;
                    if (last)
                        colr[i] = -bv;
                    ynew = -bv;
                } else {
                    const double av = colr[p];
                    if (last)
                        colr[p] = -av;
                    ynew = -av;
                }
                ycol = ynew;
            }
            // new column of L
            if (valid && i > r)
                sh.Lp[i][j + 1] = (tau != 0.0) ? x / tau : 0.0;
            if (tid == r)
                sh.Lp[r][j + 1] = 1.0;
            __syncthreads();
        }

        // panel end: L into A (shifted one column left), t on the
        // subdiagonal, and the operands of the trailing update
        const int cp = k0 + nb;
        if (valid) {
            for (int a = 0; a <= nb; ++a) {
                const int col = k0 + a;
                if (col >= 1 && i >= col + 1)
                    A[(size_t)(col - 1) * lda + i] = sh.Lp[i][a];
            }
        }
        if (tid < nb) {
            A[(size_t)(k0 + tid) * lda + (k0 + tid + 1)] = sh.tl[k0 + tid];
            t[k0 + tid] = sh.tl[k0 + tid];
            ipiv[k0 + tid + 1] = sh.pv[k0 + tid + 1];
        }
        const int nq = (nb + 1) / 2;
        if (valid && i >= cp) {
            for (int q = 0; q < nq; ++q) {
                double u = -sh.tl[k0 + 2 * q] * sh.Lp[i][2 * q];
                if (2 * q + 2 <= nb)
                    u += sh.tl[k0 + 2 * q + 1] * sh.Lp[i][2 * q + 2];
                sh.U[i][q] = u;
                sh.V[i][q] = sh.Lp[i][2 * q + 1];
            }
        }
        __syncthreads();
        // C -= U V^T - V U^T on the strict lower triangle of rows/cols >= cp
        if (cp < n - 1) {
            for (int jj = cp; jj < n - 1; ++jj) {
                double uj[kBMaxBs / 2 + 1], vj[kBMaxBs / 2 + 1];
#pragma unroll
                for (int q = 0; q < kBMaxBs / 2 + 1; ++q) {
                    uj[q] = (q < nq) ? sh.U[jj][q] : 0.0;
                    vj[q] = (q < nq) ? sh.V[jj][q] : 0.0;
                }
                const int ii = tid;
                if (ii > jj && ii < n) {
                    double acc = 0.0;
#pragma unroll
                    for (int q = 0; q < kBMaxBs / 2 + 1; ++q)
                        if (q < nq)
                            acc += sh.U[ii][q] * vj[q] - sh.V[ii][q] * uj[q];
                    double *cptr = A + (size_t)jj * lda + ii;
                    *cptr -= acc;
                }
            }
        }
        // carry the last column of L into the next panel
        if (valid && i >= cp + 1)
            sh.Lp[i][kBLd - 1] = sh.Lp[i][nb];
        __syncthreads();
    }

    // deferred row exchanges of earlier L columns: walk the blocks backwards
    // composing the later transpositions; column j (stored in A column j-1)
    // of block B receives all exchanges of the steps after block B.
    const int nsteps = n - 1;
    const int nblk = (nsteps + bs - 1) / bs;
    sh.gmap[tid] = tid;
    __syncthreads();
    for (int B = nblk - 1; B >= 0; --B) {
        const int s = min((B + 1) * bs, nsteps); // first later step
        if (B < nblk - 1) {
            for (int j = max(1, B * bs); j < min((B + 1) * bs, n - 1); ++j) {
                const int col = j - 1;
                double v = 0.0;
                const int i = tid;
                const bool mv = (i > s) && (i < n);
                if (mv)
                    v = A[(size_t)col * lda + sh.gmap[i]];
                __syncthreads();
                if (mv)
                    A[(size_t)col * lda + i] = v;
                __syncthreads();
            }
        }
        // g := (transpositions of block B, last step innermost) o g
        const int lo = B * bs;
        {
            int v = sh.gmap[tid];
            for (int c = s - 1; c >= lo; --c) {
                const int rr = c + 1, pp = sh.pv[rr];
                if (v == rr)
                    v = pp;
                else if (v == pp)
                    v = rr;
            }
            __syncthreads();
            sh.gmap[tid] = v;
            __syncthreads();
        }
    }
}

__device__ void pfaffian_one(BatchShared &sh, int n, double *log_abs_pf, int *sign)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    if (n % 2 != 0) {
        if (tid == 0) {
            *log_abs_pf = -INFINITY;
            *sign = 0;
        }
        return;
    }
    double acc = 0.0;
    int neg = 0, zero = 0;
    if (tid < n && sh.pv[tid] != tid && tid >= 1)
        ++neg;
    if (tid < n / 2) {
        const double f = -sh.tl[2 * tid];
        if (f == 0.0)
            zero = 1;
        else {
            if (f < 0.0)
                ++neg;
            acc = log(fabs(f));
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        neg += __shfl_xor(neg, off, 64);
        zero |= __shfl_xor(zero, off, 64);
    }
    if (lane == 0) {
        sh.rsum[wave] = acc;
        sh.rneg[wave] = neg;
        sh.rzero[wave] = zero;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0;
        int ng = 0, z = 0;
        for (int q = 0; q < kBT / 64; ++q) {
            a += sh.rsum[q];
            ng += sh.rneg[q];
            z |= sh.rzero[q];
        }
        if (z) {
            *log_abs_pf = -INFINITY;
            *sign = 0;
        } else {
            *log_abs_pf = a;
            *sign = (ng & 1) ? -1 : 1;
        }
    }
}

__global__ __launch_bounds__(kBT) void batched_kernel(int batch, const int *__restrict__ nv,
                                                      double *const *__restrict__ Av,
                                                      const int *__restrict__ ldav,
                                                      double *const *__restrict__ tv,
                                                      int *const *__restrict__ ipv,
                                                      double *__restrict__ log_abs_pf,
                                                      int *__restrict__ sign,
                                                      int *__restrict__ info, int max_n,
                                                      int block_size, int *__restrict__ queue)
{
    extern __shared__ double smem_b[];
    BatchShared &sh = *reinterpret_cast<BatchShared *>(smem_b);
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0)
            sh.bc_idx = atomicAdd(queue, 1);
        __syncthreads();
        const int idx = sh.bc_idx;
        __syncthreads();
        if (idx >= batch)
            break;
        const int n = nv[idx];
        const int lda = ldav[idx];
        const bool ok = (n >= 0) && (n <= max_n) && (n <= kBT) && (lda >= (n > 1 ? n : 1));
        if (info && tid == 0)
            info[idx] = ok ? 0 : -1;
        if (!ok)
            continue;
        const int bs = block_size > 0 ? block_size : batched_bs_for(n);
        for (int q = tid; q < kBT; q += kBT) {
            sh.tl[q] = 0.0;
            sh.pv[q] = q;
        }
        __syncthreads();
        factor_one(sh, Av[idx], lda, n, tv[idx], ipv[idx], bs);
        __syncthreads();
        if (log_abs_pf && sign)
            pfaffian_one(sh, n, &log_abs_pf[idx], &sign[idx]);
        __syncthreads();
    }
}

static hipError_t launch_batched(int batch, const int *n, double *const *A, const int *lda,
                                 double *const *t, int *const *ipiv, double *log_abs_pf,
                                 int *sign, int *info, int max_n, int block_size, int *queue,
                                 hipStream_t s)
{
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)batched_kernel,
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)sizeof(BatchShared));
        attr = true;
    }
    (void)hipGetLastError(); // a refused attribute is not a launch failure
    hipError_t e = launch_fill_zero(queue, 256, s);
    if (e != hipSuccess)
        return e;
    int cus = device_cu_count();
    if (cus <= 0)
        cus = 256;
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)batched_kernel, kBT,
                                                     sizeof(BatchShared)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int grid = cus * per_cu;
    if (grid > batch)
        grid = batch;
    if (grid < 1)
        return hipSuccess;
    void *args[] = {&batch, &n, &A, &lda, &t, &ipiv, &log_abs_pf, &sign, &info, &max_n,
                    &block_size, &queue};
    return hipLaunchKernel((const void *)batched_kernel, dim3(grid), dim3(kBT), args,
                           sizeof(BatchShared), s);
}

}  // namespace skl

using namespace skl;

extern "C" int skltlt_batched_max_n(void) { return kBT; }

extern "C" int skltlt_batched_workspace_size(int batch, size_t *bytes)
{
    if (batch < 0 || !bytes)
        return SKLTLT_EINVAL;
    *bytes = 256; // the work-queue counter
    return SKLTLT_OK;
}

extern "C" int skltlt_batched(int batch, const int *n, double *const *A, const int *lda,
                              double *const *t, int *const *ipiv, double *log_abs_pf, int *sign,
                              int *info, int max_n, int block_size, int precision, void *work,
                              size_t work_bytes, void *stream)
{
    if (batch < 0 || max_n < 0 || max_n > kBT || block_size < 0 || block_size > kBMaxBs)
        return block_size > kBMaxBs || max_n > kBT ? SKLTLT_ENOTSUP : SKLTLT_EINVAL;
    if (precision == SKLTLT_FP32_UPDATE)
        return SKLTLT_ENOTSUP;
    if (precision != SKLTLT_FP64)
        return SKLTLT_EINVAL;
    if ((log_abs_pf == nullptr) != (sign == nullptr))
        return SKLTLT_EINVAL;
    if (batch == 0)
        return SKLTLT_OK;
    if (!n || !A || !lda || !t || !ipiv || !work || work_bytes < 256 ||
        ((uintptr_t)work % 4) != 0)
        return SKLTLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int ti = tm_begin(SKLTLT_K_BATCHED, s);
    const hipError_t e = launch_batched(batch, n, A, lda, t, ipiv, log_abs_pf, sign, info, max_n,
                                        block_size, (int *)work, s);
    if (e != hipSuccess)
        return device_error(e, "batched launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}
