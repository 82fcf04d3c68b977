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
// the panel rows of L (for the update, U in place of their even columns, V
// in the odd ones) and the pivots live in LDS.  The
// arithmetic of a matrix depends only on that matrix and on bs, never on
// which workgroup runs it or on the other matrices.
#include "../../include/skltlt.h"
#include "batched_table.h"
#include "common.h"
#include "wave_max.h"

#include <climits>
#include <cmath>
#include <mutex>

namespace skl {

constexpr int kBT = 256;     // threads per workgroup = largest order
// largest panel width: the workgroup's LDS (the panel rows of L, 8 (kBMaxBs
// + 1) bytes per row, 39 KB in all) then lets four workgroups share a CU
// (with at most 128 VGPRs per thread: the launch bound below), which hides
// more of each column step's latency than wider panels gain (measured on the
// 4096-matrix batch: 3.12 ms at a largest width of 32 with two workgroups
// per CU, 2.46 ms at 20 with three, 2.28 ms at 16 with four)
constexpr int kBMaxBs = 16;
constexpr int kBPerCu = 4;
// LDS row of the panel's L: columns 0 .. kBMaxBs; the last slot also holds
// the carried column between panels (moved to column 0 at the next panel's
// start).  An odd number of doubles puts the rows read by one wave's lanes in
// different bank pairs.
constexpr int kBLd = kBMaxBs + 1;

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
            return e.bs < kBMaxBs ? e.bs : kBMaxBs;
    return kBMaxBs;
}

// Persistent workgroups per CU for a batch whose largest order is max_n:
// from the tuning table (entry of max_n's class), or the tuner's override.
static int g_wgpc_override = 0;
static int batched_wgpc_for(int max_n)
{
    if (g_wgpc_override > 0)
        return g_wgpc_override;
    for (const BatchedTune &e : kBatchedTune)
        if (max_n <= e.n_max)
            return e.wgpc;
    return kBPerCu;
}

struct BatchShared {
    double Lp[kBT][kBLd]; // panel rows of L, rows indexed by trailing row
    double hv[kBLd];
    double tl[kBT];
    int pv[kBT];
    int gmap[kBT];
    double red_v[kBT / 64];
    int red_i[kBT / 64];
    double bc_xr;
    int bc_idx;
    double rsum[kBT / 64];
    int rneg[kBT / 64], rzero[kBT / 64];
};

// The per-matrix pointers arrive through arrays, so the compiler cannot tell
// that they point to device memory: generic (flat) accesses also count
// against the LDS wait counter, and every wait for an LDS result would then
// wait for the outstanding matrix accesses too.  factor_one takes them in
// the global address space.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) int gint;

// Matrix accesses of the column steps and the trailing update go through a
// bounds-checked buffer resource over the matrix (the entry point rejects a
// member that spans 2 GiB or more): a lane with nothing to access passes the
// end of the buffer as its offset, so its load returns 0 and its store is
// dropped, and every lane issues the same loads and stores.  With the
// accesses in branches the compiler's waits (which must hold on every path)
// waited for each store to complete before the next access.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double ld_m(__amdgpu_buffer_rsrc_t rs, int off)
{
    const u32x2 d = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
    return __longlong_as_double((long long)(((unsigned long long)d.y << 32) | d.x));
}
__device__ __forceinline__ void st_m(__amdgpu_buffer_rsrc_t rs, int off, double v)
{
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    u32x2 d;
    d.x = (unsigned)bits;
    d.y = (unsigned)(bits >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(d, rs, off, 0, 0);
}
// bytes a member spans, and whether the buffer accesses can reach all of it
__device__ __host__ inline size_t member_span(int n, int lda)
{
    return ((size_t)(n > 1 ? n - 1 : 0) * (size_t)lda + (size_t)n) * sizeof(double);
}
constexpr size_t kMaxMemberSpan = 0x7fffffff;

__device__ void factor_one(BatchShared &sh, gdouble *__restrict__ A, int lda, int n,
                           gdouble *__restrict__ t, gint *__restrict__ ipiv, int bs)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid == 0 && n >= 1)
        ipiv[0] = 0;
    if (n < 2)
        return;
    const int span = __builtin_amdgcn_readfirstlane((int)member_span(n, lda));
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(double *)A, (short)0, span, 0x00020000);
    // (unsigned arithmetic: lanes past n form offsets they never use)
    auto moff = [&](int col, int row) {
        return (int)(((unsigned)col * (unsigned)lda + (unsigned)row) * (unsigned)sizeof(double));
    };

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
        // h of the first step is zero (column 0 has no earlier panel column)
        for (int a = tid; a < kBLd; a += kBT)
            sh.hv[a] = 0.0;
        double ycol = valid ? A[(size_t)k0 * lda + i] : 0.0;
        // nothing in flight when the steps begin (a load pending from here
        // makes the compiler wait for every access at each step's start)
        wait_vm();
        __syncthreads();

        for (int j = 0; j < nb; ++j) {
            const int c = k0 + j;
            const int r = c + 1;
            const bool last = (r == k0 + nb);
            // x = Y[., c] - L_p h, h = T_p L[c, panel]^T formed in the
            // previous step (zero at j = 0).  Per block of 16 terms each lane
            // reads one entry of h (lane m of a 16-lane row: term m) and the
            // row's own 16 entries of L_p; every product is one FMA with the
            // h entry broadcast inside the row as its DPP operand (one LDS
            // read of h per 16 terms instead of one per term).  Every lane
            // computes (the broadcast reads other lanes); rows that are not
            // candidates discard the result.  Terms past column j are zero
            // on both sides (LDS there may hold anything); four partial sums,
            // term a into sum a % 4.
            const bool cand = valid && (i >= r);
            double sacc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int a0 = 0; a0 <= j; a0 += 16) { // uniform
                const int am = a0 + (lane & 15);
                const double hb = (am <= j) ? sh.hv[am] : 0.0;
                double lv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    lv[u] = (a0 + u <= j) ? sh.Lp[i][a0 + u] : 0.0;
                bcast_fma<0, 16, 0, 16>(sacc, lv, hb);
            }
            double x = cand ? ycol - ((sacc[0] + sacc[1]) + (sacc[2] + sacc[3])) : 0.0;
            // argmax over the workgroup (first index on ties).  Per wave: the
            // largest |x| as its bit pattern (monotone for non-negative
            // doubles) by DPP moves, then the first candidate lane holding it
            // by a ballot (lanes are rows in order); then every thread
            // reduces the wave results in the same order (no serial step, no
            // extra barrier).
            // (the largest high dword first, the low dwords compared only
            // when several candidates share it)
            const unsigned long long key =
                cand ? (unsigned long long)__double_as_longlong(fabs(x)) : 0ull;
            // The DPP maxima run with every lane active (each reads other
            // lanes), outside any condition.
            const unsigned khi = (unsigned)(key >> 32);
            const unsigned mh = lanes_max_u32<64>(khi);
            const bool tophi = cand && (khi == mh);
            unsigned long long top = __ballot(tophi);
            if (__popcll(top) > 1) { // uniform
                const unsigned klo = (unsigned)key;
                const unsigned ml = lanes_max_u32<64>(tophi ? klo : 0u);
                top = __ballot(tophi && klo == ml);
            }
            double cv = 0.0;
            int ci = INT_MAX;
            if (top != 0) {
                const int wl = __ffsll((long long)top) - 1;
                cv = readlane_f64(x, wl);
                ci = wave * 64 + wl;
            }
            if (lane == 0) {
                sh.red_v[wave] = cv;
                sh.red_i[wave] = ci;
            }
            __syncthreads();
            double tau = sh.red_v[0];
            int p = sh.red_i[0];
#pragma unroll
            for (int q = 1; q < kBT / 64; ++q)
                if (beats_b(sh.red_v[q], sh.red_i[q], tau, p)) {
                    tau = sh.red_v[q];
                    p = sh.red_i[q];
                }
            if (p < r || p >= n) { // cannot happen: row r is a candidate
                p = r;
                tau = __longlong_as_double(0x7ff8000000000000ll);
            }
            if (tid == 0) {
                sh.tl[c] = tau;
                sh.pv[r] = p;
            }
            // h of the next step from the pivot row of L (row p before the
            // exchange, entry j+1 the unit diagonal) and t; hv is no longer
            // read in this step
            if (tid <= j + 1 && j + 1 < nb) {
                const int a = tid;
                double v = 0.0;
                if (a <= j)
                    v -= ((a == j) ? tau : sh.tl[k0 + a]) * ((a < j) ? sh.Lp[p][a + 1] : 1.0);
                if (a >= 1)
                    v += ((a - 1 == j) ? tau : sh.tl[k0 + a - 1]) * sh.Lp[p][a - 1];
                sh.hv[a] = v;
            }
            // the exchange's reads of this row's entries (their addresses are
            // known with the pivot; every entry is read and written by one
            // thread only): issued here, their latency overlaps the rest of
            // the step up to the barrier
            // (one load instruction for bv whichever side of p the row is
            // on: loads in alternative branches into one register made the
            // second wait for the first)
            const bool xrow = valid && i > r;
            // entry (i, r), and the entry this row exchanges with (i, p) or
            // (p, i) of the lower triangle
            const bool xch = xrow && p != r && i != p;
            const int off_r = moff(r, i);
            const int off_x = (i > p) ? moff(p, i) : moff(i, p);
            const double av = ld_m(rs, xrow ? off_r : span);
            const double bv = ld_m(rs, xch ? off_x : span);
            // row r hands its x to row p
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
            // storage), then ycol = Y'[i, r]: entry (i, r) moves to (p, i)
            // (i > p) or, negated, to (i, p) (i < p); the new (i, r) is the
            // old (p, i) (i > p), minus the old (i, p) (i < p), or minus the
            // old (p, r) at i = p, and is written back only at the panel's
            // last column (later columns read it from ycol).  ycol is set
            // before the stores are issued.
            const double ynew = (p == r) ? av : ((i > p) ? bv : ((i < p) ? -bv : -av));
            if (xrow)
                ycol = ynew;
            st_m(rs, xch ? off_x : span, (i > p) ? av : -av);
            st_m(rs, (xrow && p != r && last) ? off_r : span, ynew);
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
        // U = W[:, odd] replaces the even columns of the row's L in place
        // (column 2q is read for the last time by U_q, column nb, the
        // carried one, is never overwritten); V = L[:, odd] stays in the odd
        // columns.
        const int nq = (nb + 1) / 2;
        if (valid && i >= cp) {
            for (int q = 0; q < nq; ++q) {
                double u = -sh.tl[k0 + 2 * q] * sh.Lp[i][2 * q];
                if (2 * q + 2 <= nb)
                    u += sh.tl[k0 + 2 * q + 1] * sh.Lp[i][2 * q + 2];
                sh.Lp[i][2 * q] = u;
            }
        }
        __syncthreads();
        // C -= U V^T - V U^T on the strict lower triangle of rows/cols >= cp,
        // written as C -= A B^T with K = 2 nq: A[i][k] = L'[i][k] (U_q at
        // k = 2q, V_q at 2q + 1, the row's LDS entries as they now stand) and
        // B[j][k] = L'[j][k + 1] for even k, -L'[j][k - 1] for odd k.  On
        // 16 x 16 blocks with the FP64 MFMA (per 16x16x4 step a lane supplies
        // entry k = l / 16 of row or column l % 16; the result's lane l, value
        // q is column (l / 16) + 4q at row l % 16): a block reads 2 operand
        // values per lane and k-step from LDS, where a thread per row read
        // every column's operands for each of its products.  Each wave takes
        // every fourth block, kGrp at a time, their C loads issued before the
        // products.
        // C -= ... (loads and stores through the buffer resource)
        if (cp < n - 1) {
            constexpr int kGrp = 2; // (4 spilled two VGPRs at four workgroups per CU)
            const int m = n - cp;
            const int nt = (m + 15) / 16;
            const int nblk = nt * (nt + 1) / 2;
            const int K = 2 * nq;
            const int lrow = lane & 15, lk = lane >> 4;
            for (int t0 = wave; t0 < nblk; t0 += 4 * kGrp) {
                double cv[kGrp][4];
                int gi[kGrp], j0[kGrp];
                bool ok[kGrp];
#pragma unroll
                for (int u = 0; u < kGrp; ++u) {
                    const int tb = t0 + 4 * u;
                    ok[u] = tb < nblk;
                    int bI, bJ;
                    tile_of(ok[u] ? tb : 0, &bI, &bJ);
                    gi[u] = cp + 16 * bI + lrow;
                    j0[u] = cp + 16 * bJ;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int gj = j0[u] + lk + 4 * q;
                        cv[u][q] = ld_m(rs, (ok[u] && gi[u] < n && gj < gi[u]) ? moff(gj, gi[u])
                                                                               : span);
                    }
                }
#pragma unroll
                for (int u = 0; u < kGrp; ++u) {
                    typedef double __attribute__((ext_vector_type(4))) acc4;
                    acc4 acc = {0.0, 0.0, 0.0, 0.0};
                    const int ri = min(gi[u], n - 1);            // row side
                    const int rj = min(j0[u] + lrow, n - 1);     // column side
                    const bool rok = gi[u] < n, cok = j0[u] + lrow < n;
                    for (int ks = 0; ks < K; ks += 4) {
                        const int k = ks + lk;
                        const bool kok = k < K;
                        const int kb = (k & 1) ? k - 1 : k + 1;
                        const double av = sh.Lp[ri][kok ? k : 0];
                        const double bv = sh.Lp[rj][kok ? kb : 0];
                        const double fb = (kok && rok) ? av : 0.0;
                        const double fa = (kok && cok) ? ((k & 1) ? -bv : bv) : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, fb, acc, 0, 0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int gj = j0[u] + lk + 4 * q;
                        st_m(rs, (ok[u] && gi[u] < n && gj < gi[u]) ? moff(gj, gi[u]) : span,
                             cv[u][q] - acc[q]);
                    }
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
            // all columns of the block at once (bs <= kBMaxBs): every load
            // is issued before the barrier, every store after it
            const int jlo = max(1, B * bs), jhi = min((B + 1) * bs, n - 1);
            const int i = tid;
            const bool mv = (i > s) && (i < n);
            const int src = mv ? sh.gmap[i] : 0;
            double v[kBMaxBs];
#pragma unroll
            for (int u = 0; u < kBMaxBs; ++u) {
                const int j = jlo + u;
                v[u] = (mv && j < jhi) ? A[(size_t)(j - 1) * lda + src] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kBMaxBs; ++u) {
                const int j = jlo + u;
                if (mv && j < jhi)
                    A[(size_t)(j - 1) * lda + i] = v[u];
            }
            __syncthreads();
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

// Processing order, largest matrices first (longest-processing-time-first
// list scheduling: the persistent workgroups then finish within about one
// small matrix of each other instead of one large one): a counting sort of
// the batch indices by order n, descending, in one workgroup.  Orders outside
// [0, kBT] (rejected later) go last.  Within one order the positions follow
// the atomics' arrival; a matrix's arithmetic does not depend on it.
constexpr int kOrdT = 1024;
__global__ __launch_bounds__(kOrdT) void batch_order_kernel(int batch, const int *__restrict__ nv,
                                                            int *__restrict__ order)
{
    constexpr int kKeys = kBT + 2; // key 0: invalid order, key n + 1: order n
    __shared__ int cnt[kKeys];
    const int tid = threadIdx.x;
    for (int k = tid; k < kKeys; k += kOrdT)
        cnt[k] = 0;
    __syncthreads();
    auto key_of = [&](int i) {
        const int n = nv[i];
        return (n >= 0 && n <= kBT) ? n + 1 : 0;
    };
    for (int i = tid; i < batch; i += kOrdT)
        atomicAdd(&cnt[key_of(i)], 1);
    __syncthreads();
    if (tid == 0) { // first position of each key, largest key first
        int run = 0;
        for (int k = kKeys - 1; k >= 0; --k) {
            const int c = cnt[k];
            cnt[k] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = tid; i < batch; i += kOrdT)
        order[atomicAdd(&cnt[key_of(i)], 1)] = i;
}

__global__ __launch_bounds__(kBT, kBPerCu) void batched_kernel(int batch, const int *__restrict__ nv,
                                                      double *const *__restrict__ Av,
                                                      const int *__restrict__ ldav,
                                                      double *const *__restrict__ tv,
                                                      int *const *__restrict__ ipv,
                                                      double *__restrict__ log_abs_pf,
                                                      int *__restrict__ sign,
                                                      int *__restrict__ info, int max_n,
                                                      int block_size, int *__restrict__ queue,
                                                      const int *__restrict__ order)
{
    extern __shared__ double smem_b[];
    BatchShared &sh = *reinterpret_cast<BatchShared *>(smem_b);
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const int k = atomicAdd(queue, 1);
            sh.bc_idx = (k < batch) ? order[k] : batch;
        }
        __syncthreads();
        const int idx = sh.bc_idx;
        __syncthreads();
        if (idx >= batch)
            break;
        const int n = nv[idx];
        const int lda = ldav[idx];
        const bool ok = (n >= 0) && (n <= max_n) && (n <= kBT) && (lda >= (n > 1 ? n : 1)) &&
                        member_span(n, lda) < kMaxMemberSpan;
        if (info && tid == 0)
            info[idx] = ok ? 0 : -1;
        if (!ok) {
            // a rejected member's matrix, t and ipiv are not touched; its
            // Pfaffian outputs say that there is no result
            if (log_abs_pf && sign && tid == 0) {
                log_abs_pf[idx] = __longlong_as_double(0x7ff8000000000000ll);
                sign[idx] = 0;
            }
            continue;
        }
        const int bs = block_size > 0 ? block_size : batched_bs_for(n);
        for (int q = tid; q < kBT; q += kBT) {
            sh.tl[q] = 0.0;
            sh.pv[q] = q;
        }
        __syncthreads();
        factor_one(sh, (gdouble *)Av[idx], lda, n, (gdouble *)tv[idx], (gint *)ipv[idx], bs);
        __syncthreads();
        if (log_abs_pf && sign)
            pfaffian_one(sh, n, &log_abs_pf[idx], &sign[idx]);
        __syncthreads();
    }
}

static hipError_t launch_batched(int batch, const int *n, double *const *A, const int *lda,
                                 double *const *t, int *const *ipiv, double *log_abs_pf,
                                 int *sign, int *info, int max_n, int block_size, int *queue,
                                 int *order, hipStream_t s)
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
    {
        void *oargs[] = {&batch, &n, &order};
        e = hipLaunchKernel((const void *)batch_order_kernel, dim3(1), dim3(kOrdT), oargs, 0, s);
        if (e != hipSuccess)
            return e;
    }
    int cus = device_cu_count();
    if (cus <= 0)
        cus = 256;
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)batched_kernel, kBT,
                                                     sizeof(BatchShared)) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int want = batched_wgpc_for(max_n);
    if (want < per_cu)
        per_cu = want;
    int grid = cus * per_cu;
    if (grid > batch)
        grid = batch;
    if (grid < 1)
        return hipSuccess;
    void *args[] = {&batch, &n, &A, &lda, &t, &ipiv, &log_abs_pf, &sign, &info, &max_n,
                    &block_size, &queue, &order};
    return hipLaunchKernel((const void *)batched_kernel, dim3(grid), dim3(kBT), args,
                           sizeof(BatchShared), s);
}

}  // namespace skl

using namespace skl;

extern "C" int skltlt_batched_max_n(void) { return kBT; }

extern "C" int skltlt_tune_batched_wgpc(int wgpc)
{
    if (wgpc < 0 || wgpc > kBPerCu)
        return SKLTLT_EINVAL;
    g_wgpc_override = wgpc;
    return SKLTLT_OK;
}

// the work-queue counter (256 bytes), then the processing order (one int per
// matrix), rounded up to 256 bytes
static size_t batched_work_bytes(int batch)
{
    return 256 + (((size_t)batch * sizeof(int) + 255) / 256) * 256;
}

extern "C" int skltlt_batched_workspace_size(int batch, size_t *bytes)
{
    if (batch < 0 || !bytes)
        return SKLTLT_EINVAL;
    *bytes = batched_work_bytes(batch);
    return SKLTLT_OK;
}

// Argument checks shared by both batched entry points.
static int batched_check(int batch, const int *n, double *const *A, const int *lda,
                         double *const *t, int *const *ipiv, const double *log_abs_pf,
                         const int *sign, int max_n, int block_size, int precision)
{
    if (batch < 0 || max_n < 0 || max_n > kBT || block_size < 0 || block_size > kBMaxBs)
        return block_size > kBMaxBs || max_n > kBT ? SKLTLT_ENOTSUP : SKLTLT_EINVAL;
    if (precision == SKLTLT_FP32_UPDATE)
        return SKLTLT_ENOTSUP;
    if (precision != SKLTLT_FP64)
        return SKLTLT_EINVAL;
    if ((log_abs_pf == nullptr) != (sign == nullptr))
        return SKLTLT_EINVAL;
    if (batch > 0 && (!n || !A || !lda || !t || !ipiv))
        return SKLTLT_EINVAL;
    return SKLTLT_OK;
}

extern "C" int skltlt_batched(int batch, const int *n, double *const *A, const int *lda,
                              double *const *t, int *const *ipiv, double *log_abs_pf, int *sign,
                              int *info, int max_n, int block_size, int precision, void *work,
                              size_t work_bytes, void *stream)
{
    int st = batched_check(batch, n, A, lda, t, ipiv, log_abs_pf, sign, max_n, block_size,
                           precision);
    if (st != SKLTLT_OK || batch == 0)
        return st;
    if (!work || work_bytes < batched_work_bytes(batch) || ((uintptr_t)work % 4) != 0)
        return SKLTLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int ti = tm_begin(SKLTLT_K_BATCHED, s);
    const hipError_t e = launch_batched(batch, n, A, lda, t, ipiv, log_abs_pf, sign, info, max_n,
                                        block_size, (int *)work, (int *)((char *)work + 256), s);
    if (e != hipSuccess)
        return device_error(e, "batched launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}

// ---- allocation-free variant ------------------------------------------------
// The queue counter and the processing order live in a file-scope device
// array instead of a caller's workspace: one copy per device, held by the
// process until it ends.  In host code `scratch` only names the symbol; its
// device address is looked up once per device with hipGetSymbolAddress and
// that address is what the kernels receive.
constexpr int kNoAllocMaxBatch = 1 << 18;
constexpr size_t kNoAllocScratchBytes = 256 + (size_t)kNoAllocMaxBatch * sizeof(int);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static void *g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (looked up on the first
// call made with that device current).
static int scratch_of_current_device(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return device_error(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return SKLTLT_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return device_error(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p % 256) != 0)
            return device_error(hipErrorInvalidSymbol, "scratch address");
        g_scratch_dev[dev] = p;
    }
    *out = (char *)g_scratch_dev[dev];
    return SKLTLT_OK;
}

extern "C" int skltlt_batched_noalloc_max_batch(void) { return kNoAllocMaxBatch; }

extern "C" int skltlt_batched_noalloc(int batch, const int *n, double *const *A, const int *lda,
                                      double *const *t, int *const *ipiv, double *log_abs_pf,
                                      int *sign, int *info, int max_n, int block_size,
                                      int precision, void *stream)
{
    int st = batched_check(batch, n, A, lda, t, ipiv, log_abs_pf, sign, max_n, block_size,
                           precision);
    if (st != SKLTLT_OK || batch == 0)
        return st;
    if (batch > kNoAllocMaxBatch)
        return SKLTLT_ENOTSUP;
    char *sp = nullptr;
    if ((st = scratch_of_current_device(&sp)) != SKLTLT_OK)
        return st;
    hipStream_t s = (hipStream_t)stream;
    const int ti = tm_begin(SKLTLT_K_BATCHED, s);
    // the queue counter (first 256 bytes) is cleared by a kernel in
    // launch_batched; the order array is rewritten entirely by every call
    const hipError_t e = launch_batched(batch, n, A, lda, t, ipiv, log_abs_pf, sign, info, max_n,
                                        block_size, (int *)sp, (int *)(sp + 256), s);
    if (e != hipSuccess)
        return device_error(e, "batched launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}
