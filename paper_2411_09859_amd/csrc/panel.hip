// Pivoted left-looking panel of the fused blocked right-looking LTL^T.
//
// Paper (arXiv 2411.09859): the panel of a pivoted blocked right-looking
// algorithm must be factored by a left-looking unblocked algorithm over the
// whole trailing matrix (Sec. 3.7.3); the left-looking column update is the
// skew_tridiag_gemv y := y - A T x of Sec. 3.5.3/3.5.4; pivoting uses iamax
// and the symmetric exchange P(pi) of Sec. 3.7.1-3.7.2; the last Gauss
// transform of the previous panel is carried into this one (fused variant,
// Sec. 3.6.3); L and t are kept outside X while factoring and t is moved
// onto the subdiagonal afterwards (Sec. 4.1).
//
// One cooperative launch handles one panel of nb column steps.  Workgroup w
// owns the trailing rows k0+1+w*R .. k0+1+(w+1)*R-1 and keeps their panel
// rows of L (the carried column and the nb new ones) in LDS.  Each column
// step c (r = c+1):
//   1. h = T_p * L[c, panel]^T from the previous pivot row (all groups
//      compute it redundantly from the same data);
//   2. x_i = Y[i, c] - L[i, panel] . h for owned rows i >= r (Y is the
//      trailing matrix as of the panel start, with this panel's symmetric
//      exchanges applied in place);
//   3. local argmax of |x_i| (first index on ties), published in a slot
//      whose stamp is stored last with release semantics;
//   4. every group polls all stamps, then reduces the slots identically:
//      pivot p, tau = x_p;
//   5. exchange rows/columns r <-> p of the trailing matrix (lower storage
//      rule, one element per owned row), exchange the LDS rows r and p,
//      and form the new column of L, l = x / tau (0 if tau = 0).
// Panel rows are mirrored row-major in HBM under a physical-row indirection:
// an exchange swaps the owners' physical indices instead of moving data, so
// no mirror row that another group may still be reading is ever rewritten.
#include "common.h"

#include <climits>

namespace skl {

__device__ __forceinline__ bool beats(double av, int ai, double bv, int bi)
{
    const double aa = fabs(av), bb = fabs(bv);
    return (aa > bb) || (aa == bb && ai < bi);
}

__global__ __launch_bounds__(kPanelThreads) void panel_kernel(
    double *__restrict__ A, int lda, int n, int k0, int nb, int b,
    double *__restrict__ t, int *__restrict__ ipiv, double *__restrict__ mirror,
    int ldm, double *__restrict__ lcar, double *__restrict__ uv,
    float *__restrict__ uv32, int want32, Slot *__restrict__ slots, int G, int R)
{
    extern __shared__ double smem[];
    const int ldl = b + 2;
    double *Lp = smem;                  // R x ldl
    double *hrow = Lp + (size_t)R * ldl; // b+2: pivot row of the previous step
    double *rrow = hrow + (b + 2);      // b+2: old row r (owner of p only)
    double *hv = rrow + (b + 2);        // b+2: h
    double *xl = hv + (b + 2);          // R
    double *tl = xl + R;                // b
    int *perm = (int *)(tl + b);        // R

    __shared__ double red_v[kPanelThreads / 64];
    __shared__ int red_i[kPanelThreads / 64];
    __shared__ int red_ph[kPanelThreads / 64];
    __shared__ double bc_tau, bc_xr;
    __shared__ int bc_p, bc_physp, bc_physr;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int w = blockIdx.x;
    const int base = k0 + 1;          // first trailing row
    const int row0 = base + w * R;    // first row owned by this group
    const int TPR = kPanelThreads / R; // threads per row (power of two)
    const int lr = tid / TPR;
    const int sub = tid - lr * TPR;
    const int myrow = row0 + lr;
    const bool rowvalid = (lr < R) && (myrow < n);

    // ---- panel start: carried column, physical indices, first column of Y
    double ycol = 0.0;
    if (rowvalid && sub == 0) {
        const double l0 = (k0 == 0) ? 0.0 : lcar[myrow];
        Lp[(size_t)lr * ldl] = l0;
        perm[lr] = myrow - base;
        mirror[(size_t)(myrow - base) * ldm] = l0;
        ycol = A[(size_t)k0 * lda + myrow];
    }
    __syncthreads();

    for (int j = 0; j < nb; ++j) {
        const int c = k0 + j;
        const int r = c + 1;
        const int par = c & 1;
        const bool last = (r == k0 + nb);

        // 1. h[a] = sum_b T[a][b] L[c][b] over the panel columns a, b in 0..j,
        //    T tridiagonal with T[a+1][a] = t_a, T[a][a+1] = -t_a, L[c][j] = 1.
        if (tid <= j) {
            const int a = tid;
            double v = 0.0;
            if (a + 1 <= j)
                v -= tl[a] * ((a + 1 < j) ? hrow[a + 1] : 1.0);
            if (a >= 1)
                v += tl[a - 1] * hrow[a - 1];
            hv[a] = v;
        }
        __syncthreads();

        // 2. x_i = Y[i, c] - sum_a L[i][a] h[a] for owned rows i >= r.
        const bool cand = rowvalid && (myrow >= r);
        double s = 0.0;
        if (cand) {
            const double *Lrow = Lp + (size_t)lr * ldl;
            for (int a = sub; a <= j; a += TPR)
                s += Lrow[a] * hv[a];
        }
        for (int off = TPR >> 1; off >= 1; off >>= 1)
            s += __shfl_xor(s, off, 64);
        double xv = 0.0;
        if (cand && sub == 0) {
            xv = ycol - s;
            xl[lr] = xv;
        }

        // 3. local argmax: largest |x|, smallest row index on ties.
        double cv = 0.0;
        int ci = INT_MAX, cph = 0;
        if (cand && sub == 0) {
            cv = xv;
            ci = myrow;
            cph = perm[lr];
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(cv, off, 64);
            const int oi = __shfl_xor(ci, off, 64);
            const int oph = __shfl_xor(cph, off, 64);
            if (beats(ov, oi, cv, ci)) {
                cv = ov;
                ci = oi;
                cph = oph;
            }
        }
        if (lane == 0) {
            red_v[wave] = cv;
            red_i[wave] = ci;
            red_ph[wave] = cph;
        }
        __syncthreads();

        const int wr = (r - base) / R; // group owning row r
        if (tid == 0) {
            double bv = red_v[0];
            int bi = red_i[0], bph = red_ph[0];
            for (int q = 1; q < kPanelThreads / 64; ++q) {
                if (beats(red_v[q], red_i[q], bv, bi)) {
                    bv = red_v[q];
                    bi = red_i[q];
                    bph = red_ph[q];
                }
            }
            Slot *sl = &slots[par * kMaxPanelGroups + w];
            sl->xval = bv;
            sl->idx = bi;
            sl->phys = bph;
            if (w == wr) {
                const int lrr = (r - base) - w * R;
                sl->xr = xl[lrr];
                sl->phys_r = perm[lrr];
            }
            __hip_atomic_store(&sl->stamp, (unsigned)(c + 1), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }

        // 4. wait for every group's slot of this step.
        if (wave == 0) {
            for (int q = lane; q < G; q += 64) {
                const Slot *s2 = &slots[par * kMaxPanelGroups + q];
                while (__hip_atomic_load(&s2->stamp, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT) != (unsigned)(c + 1))
                    __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

        // global winner, reduced identically in every group
        {
            double gv = 0.0;
            int gi = INT_MAX, gph = 0;
            for (int q = tid; q < G; q += kPanelThreads) {
                const Slot *s2 = &slots[par * kMaxPanelGroups + q];
                const double v2 = s2->xval;
                const int i2 = s2->idx;
                if (beats(v2, i2, gv, gi)) {
                    gv = v2;
                    gi = i2;
                    gph = s2->phys;
                }
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(gv, off, 64);
                const int oi = __shfl_xor(gi, off, 64);
                const int oph = __shfl_xor(gph, off, 64);
                if (beats(ov, oi, gv, gi)) {
                    gv = ov;
                    gi = oi;
                    gph = oph;
                }
            }
            __syncthreads(); // red_* reuse
            if (lane == 0) {
                red_v[wave] = gv;
                red_i[wave] = gi;
                red_ph[wave] = gph;
            }
            __syncthreads();
            if (tid == 0) {
                double bv = red_v[0];
                int bi = red_i[0], bph = red_ph[0];
                for (int q = 1; q < kPanelThreads / 64; ++q) {
                    if (beats(red_v[q], red_i[q], bv, bi)) {
                        bv = red_v[q];
                        bi = red_i[q];
                        bph = red_ph[q];
                    }
                }
                bc_tau = bv;
                bc_p = bi;
                bc_physp = bph;
                const Slot *srr = &slots[par * kMaxPanelGroups + wr];
                bc_xr = srr->xr;
                bc_physr = srr->phys_r;
            }
            __syncthreads();
        }
        const int p = bc_p;
        const double tau = bc_tau;
        const int physp = bc_physp, physr = bc_physr;
        const int wp = (p - base) / R;

        // 5a. pivot row content (L[p][panel] before the exchange), and the old
        //     row r for the owner of p.
        if (tid <= j)
            hrow[tid] = mirror[(size_t)physp * ldm + tid];
        if (w == wp && p != r && tid <= j)
            rrow[tid] = mirror[(size_t)physr * ldm + tid];

        // 5b. symmetric exchange r <-> p of the trailing matrix in lower
        //     storage, one owned row i > r per thread; ycol becomes Y'[i, r].
        if (rowvalid && sub == 0 && myrow > r) {
            const size_t cr = (size_t)r * lda, cpv = (size_t)p * lda;
            double ynew;
            if (p == r) {
                ynew = A[cr + myrow];
            } else if (myrow > p) {
                const double av = A[cr + myrow];
                const double bvv = A[cpv + myrow];
                A[cpv + myrow] = av;
                if (last)
                    A[cr + myrow] = bvv;
                ynew = bvv;
            } else if (myrow < p) {
                const double av = A[cr + myrow];
                const size_t pi = (size_t)myrow * lda + p;
                const double bvv = A[pi];
                A[pi] = -av;
                if (last)
                    A[cr + myrow] = -bvv;
                ynew = -bvv;
            } else {
                const double av = A[cr + p];
                if (last)
                    A[cr + p] = -av;
                ynew = -av;
            }
            ycol = ynew;
        }
        __syncthreads();

        // 5c. exchange the LDS rows r and p and their physical indices.
        if (w == wr) {
            const int lrr = (r - base) - w * R;
            if (lr == lrr) {
                for (int a = sub; a <= j; a += TPR)
                    Lp[(size_t)lrr * ldl + a] = hrow[a];
                if (sub == 0) {
                    Lp[(size_t)lrr * ldl + j + 1] = 1.0;
                    perm[lrr] = physp;
                }
            }
        }
        if (w == wp && p != r) {
            const int lrp = (p - base) - w * R;
            if (lr == lrp) {
                for (int a = sub; a <= j; a += TPR)
                    Lp[(size_t)lrp * ldl + a] = rrow[a];
                if (sub == 0) {
                    perm[lrp] = physr;
                    xl[lrp] = bc_xr;
                }
            }
        }
        if (tid == 0)
            tl[j] = tau;
        if (w == 0 && tid == 0) {
            t[c] = tau;
            ipiv[r] = p;
        }
        __syncthreads();

        // 5d. new column of L: l_i = x_i / tau for owned rows i > r.
        if (rowvalid && sub == 0 && myrow > r) {
            const double l = (tau != 0.0) ? xl[lr] / tau : 0.0;
            Lp[(size_t)lr * ldl + j + 1] = l;
            mirror[(size_t)perm[lr] * ldm + j + 1] = l;
        }
        __syncthreads();
    }

    // ---- panel end: L into A (shifted one column left), t onto the
    //      subdiagonal, the carried column, and the skr2k operands.
    if (rowvalid) {
        const double *Lrow = Lp + (size_t)lr * ldl;
        for (int a = sub; a <= nb; a += TPR) {
            const int col = k0 + a;
            if (col >= 1 && myrow >= col + 1)
                A[(size_t)(col - 1) * lda + myrow] = Lrow[a];
        }
        const int cp = k0 + nb;
        if (sub == 0 && myrow >= cp + 1)
            lcar[myrow] = Lrow[nb];
        if (myrow >= cp && cp < n - 1) {
            const int nq = (nb + 1) / 2;
            for (int q = sub; q < nq; q += TPR) {
                const double vq = Lrow[2 * q + 1];
                double uq = -tl[2 * q] * Lrow[2 * q];
                if (2 * q + 2 <= nb)
                    uq += tl[2 * q + 1] * Lrow[2 * q + 2];
                uv[(size_t)q * n + myrow] = uq;
                uv[(size_t)(nq + q) * n + myrow] = vq;
                uv[(size_t)(2 * nq + q) * n + myrow] = -vq;
                uv[(size_t)(3 * nq + q) * n + myrow] = uq;
                if (want32) {
                    uv32[(size_t)q * n + myrow] = (float)uq;
                    uv32[(size_t)(nq + q) * n + myrow] = (float)vq;
                    uv32[(size_t)(2 * nq + q) * n + myrow] = -(float)vq;
                    uv32[(size_t)(3 * nq + q) * n + myrow] = (float)uq;
                }
            }
        }
    }
    if (w == 0) {
        for (int a = tid; a < nb; a += kPanelThreads)
            A[(size_t)(k0 + a) * lda + (k0 + a + 1)] = tl[a];
    }
}

PanelShape panel_shape(int n, int k0, int b, int max_groups)
{
    PanelShape sh;
    const int m = n - k0 - 1;
    int R = 64;
    while ((m + R - 1) / R > max_groups && R < kPanelThreads)
        R *= 2;
    sh.R = R;
    sh.G = (m + R - 1) / R;
    if (sh.G < 1)
        sh.G = 1;
    sh.lds = sizeof(double) * ((size_t)R * (b + 2) + 3 * (size_t)(b + 2) + R + b) +
             sizeof(int) * (size_t)R;
    return sh;
}

hipError_t launch_panel(double *A, int lda, int n, int k0, int nb, int b, double *t,
                        int *ipiv, const FactorWs &ws, int want32, const PanelShape &sh,
                        hipStream_t s)
{
    double *mirror = ws.mirror;
    int ldm = ws.ldm;
    double *lcar = ws.lcar;
    double *uv = ws.uv;
    float *uv32 = ws.uv32;
    Slot *slots = ws.slots;
    int G = sh.G, R = sh.R;
    void *args[] = {&A, &lda, &n, &k0, &nb, &b, &t, &ipiv, &mirror, &ldm, &lcar,
                    &uv, &uv32, &want32, &slots, &G, &R};
    return hipLaunchCooperativeKernel((const void *)panel_kernel, dim3(sh.G),
                                      dim3(kPanelThreads), args, (unsigned)sh.lds, s);
}

void panel_init_attrs()
{
    (void)hipFuncSetAttribute((const void *)panel_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                        160 * 1024);
}

int panel_max_groups(size_t lds_bytes)
{
    static int cached_cus = 0;
    if (!cached_cus)
        cached_cus = device_cu_count();
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)panel_kernel,
                                                     kPanelThreads, lds_bytes) != hipSuccess)
        return 0;
    long g = (long)per_cu * cached_cus;
    if (g > kMaxPanelGroups)
        g = kMaxPanelGroups;
    return (int)g;
}

}  // namespace skl
