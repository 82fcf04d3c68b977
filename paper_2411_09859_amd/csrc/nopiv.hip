// Unpivoted panel of the fused blocked right-looking LTL^T (the blocked
// algorithms of Sec. 3.6 without the pivoting of Sec. 3.7, for inputs known
// to need none; in exact arithmetic the unblocked algorithm of Sec. 2.4,
// eq. (1), with P = I).
//
// The panel's state and step are those of the pivoted panel with the pivot
// fixed at row r = c + 1: for panel step j (column c = k0 + j) and every
// trailing row i,
//   h_j[a] = -t_{k0+a} L[c][a+1] + t_{k0+a-1} L[c][a-1]   (a = 0..j,
//            L[c][j] = 1; T_p tridiagonal, the skew_tridiag_gemv of 3.5.4)
//   x_j[i] = Y[i][c] - sum_{a <= j} L[i][a] h_j[a]
//   t_c = x_j[r],  L[i][j+1] = x_j[i] / t_c  (i > r),  L[r][j+1] = 1,
// where L[i][a] is column k0 + a of L (a = 0: the carried column of the
// previous panel, Sec. 3.6.3).  Without exchanges, h_j and t_c depend only
// on the panel's top rows k0+1 .. k0+nb (the rows that receive the steps'
// subdiagonal entries), so:
//   * one workgroup runs the nb dependent steps over the top rows alone
//     (rows in registers, h from LDS, two barriers per step) and stores every
//     h_j and t_c;
//   * every other row then runs its own recurrence against the stored h_j
//     and t_c, independently of all other rows (no exchange between groups).
// The serial chain is nb steps inside one workgroup instead of nb device
// round trips.  Both kernels write L into A (shifted one column left,
// Sec. 4.1), the carried column and the skr2k operands U, V exactly as the
// pivoted panel does; the trailing update is the same skr2k (identity
// permutation).
#include "common.h"
#include "wave_max.h"

namespace skl {

constexpr int kNpNT = 256;   // threads per workgroup
constexpr int kNpTPR = 2;    // threads per row
constexpr int kNpR = kNpNT / kNpTPR; // rows per workgroup (128)
constexpr int kNpNS = 65;    // register slots per thread: 130 >= nb + 1 columns
constexpr int kNpMaxB = 128; // widest panel
constexpr int kNpD = 8;      // Y columns in flight per row (a column per step)

// L slot q of thread `sub` holds column sub + TPR q; new columns go into a
// ring of kRing registers flushed into the slots once a ring group is full
// (an indexed insert into the slot array needs a select over every slot).
struct NpRow {
    static constexpr int kRing = 4;
    static constexpr int kNSR = ((kNpNS + kRing - 1) / kRing) * kRing;
    static constexpr int NA = kNSR * kNpTPR;
    double Lreg[kNpNS];
    double Lnew[kRing];
    int grc;

    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int q = 0; q < kNpNS; ++q)
            Lreg[q] = 0.0;
#pragma unroll
        for (int i = 0; i < kRing; ++i)
            Lnew[i] = 0.0;
        grc = 0;
    }
    __device__ __forceinline__ void flush(int g)
    {
#pragma unroll
        for (int q = 0; q < kNpNS; ++q)
            Lreg[q] = (q / kRing == g) ? Lnew[q % kRing] : Lreg[q];
#pragma unroll
        for (int i = 0; i < kRing; ++i)
            Lnew[i] = 0.0;
    }
    // column a (uniform) := v in the thread that keeps it
    __device__ __forceinline__ void insert(int a, double v, int sub)
    {
        const int g = (a / kNpTPR) / kRing;
        if (g != grc) {
            flush(grc);
            grc = g;
        }
        if (sub == a % kNpTPR) {
            const int slot = (a / kNpTPR) % kRing;
#pragma unroll
            for (int i = 0; i < kRing; ++i)
                Lnew[i] = (i == slot) ? v : Lnew[i];
        }
    }
    // sum_a L[a] h[a] over this thread's filled columns (h in LDS, zero
    // beyond the filled ones), summed over the row's TPR threads.  Per block
    // of 16 slots each lane reads one entry of h (lane m of a 16-lane row:
    // slot m of the block, for the row's column class) and every product is
    // one FMA with that entry broadcast inside the row as its DPP operand;
    // slots of the unflushed ring group in Lreg are 0.  Needs the lane
    // layout of np_lane_row (a 16-lane row holds one column class) and every
    // lane active.
    __device__ __forceinline__ double dot(const double *h, int sub) const
    {
        const int lane = threadIdx.x & 63;
        const int hl = lane & 15;
        constexpr int kNB = (kNpNS + 15) / 16;
        static_assert(kNB <= 5, "h blocks");
        double hb[kNB];
#pragma unroll
        for (int k = 0; k < kNB; ++k) // uniform conditions; in-range index
            hb[k] = (16 * k < grc * kRing) ? h[min(sub + kNpTPR * (16 * k + hl), NA - 1)] : 0.0;
        const double hr = h[sub + kNpTPR * (grc * kRing + (lane & (kRing - 1)))];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (0 < grc * kRing)
            bcast_fma<0, 16, 0, kNpNS>(acc, Lreg, hb[0]);
        if constexpr (kNB > 1)
            if (16 < grc * kRing)
                bcast_fma<0, 16, 16, kNpNS>(acc, Lreg, hb[1 % kNB]);
        if constexpr (kNB > 2)
            if (32 < grc * kRing)
                bcast_fma<0, 16, 32, kNpNS>(acc, Lreg, hb[2 % kNB]);
        if constexpr (kNB > 3)
            if (48 < grc * kRing)
                bcast_fma<0, 16, 48, kNpNS>(acc, Lreg, hb[3 % kNB]);
        if constexpr (kNB > 4)
            if (64 < grc * kRing)
                bcast_fma<0, 16, 64, kNpNS>(acc, Lreg, hb[4 % kNB]);
        bcast_fma<0, kRing, 0, kRing>(acc, Lnew, hr);
        double s = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        static_assert(64 / kNpTPR == 32, "the row's two threads are 32 lanes apart");
        s = xor_add<32>(s); // the row's other thread (lane swap, no LDS)
        return s;
    }
    // after the last insert: every column in Lreg
    __device__ __forceinline__ void finish() { flush(grc); }
};

// Register row and column class of thread tid: the TPR threads of a row are
// 64 / TPR lanes apart, so each 16-lane row of a wave holds one column class
// (the broadcast of NpRow::dot).
__device__ __forceinline__ void np_lane_row(int tid, int &lr, int &sub)
{
    constexpr int RL = 64 / kNpTPR;
    lr = (tid >> 6) * RL + (tid & 63) % RL;
    sub = (tid & 63) / RL;
}

// The row's outputs once its panel columns 0..nb are final: L columns into
// A (column k0 + a is stored in A column k0 + a - 1, rows >= k0 + a + 1), the
// carried column (column nb) for rows > cp, and U_q = -t_2q L[2q] +
// t_2q+1 L[2q+2], V_q = L[2q+1] for rows >= cp.  With two threads per row
// the even columns are all in thread 0 and the odd ones in thread 1, so each
// thread forms its own operand (U or V) from its own slots.
static_assert(kNpTPR == 2, "operand formation assumes even/odd column threads");
__device__ __forceinline__ void np_row_outputs(const NpRow &L, int i, int sub, int k0, int nb,
                                               const double *tl, double *A, int lda, int n,
                                               double *lcar, double *uv, float *uv32, int want32)
{
    const int cp = k0 + nb;
#pragma unroll
    for (int q = 0; q < kNpNS; ++q) {
        const int a = sub + kNpTPR * q;
        const int col = k0 + a;
        if (a <= nb && col >= 1 && i >= col + 1)
            A[(size_t)(col - 1) * lda + i] = L.Lreg[q];
        if (a == nb && i >= cp + 1)
            lcar[i] = L.Lreg[q];
    }
    if (i < cp)
        return;
    const int nq = (nb + 1) / 2;
#pragma unroll
    for (int q = 0; q < kNpNS; ++q) {
        if (q >= nq)
            continue;
        if (sub == 0) { // U_q from columns 2q and 2q+2 (slots q and q+1)
            double uq = -tl[2 * q] * L.Lreg[q];
            if (2 * q + 2 <= nb && q + 1 < kNpNS)
                uq += tl[2 * q + 1] * L.Lreg[(q + 1 < kNpNS) ? q + 1 : q];
            uv[(size_t)q * n + i] = uq;
            uv[(size_t)(3 * nq + q) * n + i] = uq;
            if (want32) {
                uv32[(size_t)q * n + i] = (float)uq;
                uv32[(size_t)(3 * nq + q) * n + i] = (float)uq;
            }
        } else { // V_q = column 2q+1 (slot q)
            const double vq = L.Lreg[q];
            uv[(size_t)(nq + q) * n + i] = vq;
            uv[(size_t)(2 * nq + q) * n + i] = -vq;
            if (want32) {
                uv32[(size_t)(nq + q) * n + i] = (float)vq;
                uv32[(size_t)(2 * nq + q) * n + i] = -(float)vq;
            }
        }
    }
}

// The top rows k0+1 .. k0+nb and the steps' h_j, t_c (one workgroup).
// H[j * ldh + a] = h_j[a] for a <= j.
__global__ __launch_bounds__(kNpNT) void nopiv_top_kernel(
    double *__restrict__ A, int lda, const double *__restrict__ W, int ldw, int n, int k0,
    int nb, double *__restrict__ t, double *__restrict__ lcar, double *__restrict__ H, int ldh,
    double *__restrict__ uv, float *__restrict__ uv32, int want32)
{
    constexpr int NA = NpRow::NA;
    __shared__ double hv[NA];
    __shared__ double tl[kNpMaxB];
    __shared__ double rtl[kNpMaxB]; // 1 / t (0 where t = 0)
    extern __shared__ double ltop[]; // nb x (nb + 2): the top rows' L, row-major
    const int ldt = nb + 2;
    const int tid = threadIdx.x;
    int lr, sub;
    np_lane_row(tid, lr, sub);
    const int base = k0 + 1;
    const int i = base + lr; // this thread's row
    const bool mine = lr < nb;

    NpRow L;
    L.init();
    const double l0 = (mine && k0 > 0) ? lcar[i] : 0.0;
    L.insert(0, l0, sub);
    for (int a = tid; a < NA; a += kNpNT)
        hv[a] = 0.0;
    if (mine && sub == 0)
        ltop[lr * ldt] = l0;
    // Y[i][k0 + j] for the next kNpD steps (the columns are known in advance:
    // no exchanges); a row needs the columns of the steps j <= lr
    // Every lane loads (clamped addresses, unused values where the row does
    // not need the column): loads skipped by branches make the compiler wait
    // for all outstanding loads before the first use.
    const int ic = mine ? i : base;
    double yq[kNpD];
#pragma unroll
    for (int u = 0; u < kNpD; ++u)
        yq[u] = W[(size_t)(k0 + min(u, nb - 1)) * ldw + ic];
    __syncthreads();

    auto step = [&](int j, double &yslot) {
        const int c = k0 + j;
        // x_j for the rows at or below r (lr >= j); the slot is consumed
        // before it is refilled (same register, no copies at the loop's end)
        const double x = yslot - L.dot(hv, sub);
        yslot = W[(size_t)(k0 + min(j + kNpD, nb - 1)) * ldw + ic];
        if (mine && lr == j && sub == 0) {
            tl[j] = x;
            rtl[j] = (x != 0.0) ? 1.0 / x : 0.0;
            t[c] = x;
            A[(size_t)c * lda + c + 1] = x; // t on the subdiagonal
        }
        if (tid <= j)
            H[(size_t)j * ldh + tid] = hv[tid];
        __syncthreads();
        // new column j+1: x / t below r (as x times 1/t), the unit at r,
        // zero above
        const double rt = rtl[j];
        double l = 0.0;
        if (mine && lr > j)
            l = x * rt;
        else if (mine && lr == j)
            l = 1.0;
        L.insert(j + 1, l, sub);
        if (mine && lr >= j && sub == (j + 1) % kNpTPR)
            ltop[lr * ldt + j + 1] = l;
        // h of step j+1 from row c+1 (top row j: its columns 0..j are final
        // and in ltop; column j+1 is its unit)
        if (j + 1 < nb && tid <= j + 1) {
            const int a = tid, jj = j + 1;
            const double *row = ltop + (size_t)j * ldt;
            double hn = 0.0;
            if (a + 1 <= jj)
                hn -= tl[a] * ((a + 1 < jj) ? row[a + 1] : 1.0);
            if (a >= 1)
                hn += tl[a - 1] * row[a - 1];
            hv[a] = hn;
        }
        __syncthreads();
    };
    // whole groups of kNpD steps without conditions, then the remainder
    int j0 = 0;
    for (; j0 + kNpD <= nb; j0 += kNpD) {
#pragma unroll
        for (int u = 0; u < kNpD; ++u)
            step(j0 + u, yq[u]);
    }
#pragma unroll
    for (int u = 0; u < kNpD; ++u)
        if (j0 + u < nb)
            step(j0 + u, yq[u]);
    L.finish();
    if (mine)
        np_row_outputs(L, i, sub, k0, nb, tl, A, lda, n, lcar, uv, uv32, want32);
}

// Every trailing row below the top rows: its own recurrence against the
// stored h_j and t_c (kNpR rows per workgroup, nothing shared between groups).
__global__ __launch_bounds__(kNpNT) void nopiv_rows_kernel(
    double *__restrict__ A, int lda, const double *__restrict__ W, int ldw, int n, int k0,
    int nb, const double *__restrict__ t, double *__restrict__ lcar,
    const double *__restrict__ H, int ldh, double *__restrict__ uv, float *__restrict__ uv32,
    int want32)
{
    constexpr int NA = NpRow::NA;
    extern __shared__ double sh[]; // H staged: nb x NA
    __shared__ double tl[kNpMaxB];
    __shared__ double rtl[kNpMaxB]; // 1 / t (0 where t = 0)
    const int tid = threadIdx.x;
    int lr, sub;
    np_lane_row(tid, lr, sub);
    const int cp = k0 + nb;
    const int i = cp + 1 + blockIdx.x * kNpR + lr;
    const bool mine = i < n;

    double *hs = sh;
    for (int e = tid; e < nb * NA; e += kNpNT) {
        const int j = e / NA, a = e - j * NA;
        hs[e] = (a <= j) ? H[(size_t)j * ldh + a] : 0.0;
    }
    for (int j = tid; j < nb; j += kNpNT) {
        const double tj = t[k0 + j];
        tl[j] = tj;
        rtl[j] = (tj != 0.0) ? 1.0 / tj : 0.0;
    }

    NpRow L;
    L.init();
    const double l0 = (mine && k0 > 0) ? lcar[i] : 0.0;
    L.insert(0, l0, sub);
    // Y[i][k0 + j] for the next kNpD steps; every lane loads (clamped
    // addresses), so the compiler can count the loads in flight
    const int ic = mine ? i : n - 1;
    double yq[kNpD];
#pragma unroll
    for (int u = 0; u < kNpD; ++u)
        yq[u] = W[(size_t)(k0 + min(u, nb - 1)) * ldw + ic];
    __syncthreads();
    auto step = [&](int j, double y) {
        const double x = y - L.dot(hs + (size_t)j * NA, sub);
        L.insert(j + 1, mine ? x * rtl[j] : 0.0, sub);
    };
    // groups of kNpD steps; the next group's columns are requested when a
    // group starts, so they have a whole group's time to arrive (the
    // hand-over at the group's end waits for them)
    int j0 = 0;
    for (; j0 + kNpD <= nb; j0 += kNpD) {
        double nx[kNpD];
#pragma unroll
        for (int u = 0; u < kNpD; ++u)
            nx[u] = W[(size_t)(k0 + min(j0 + kNpD + u, nb - 1)) * ldw + ic];
#pragma unroll
        for (int u = 0; u < kNpD; ++u)
            step(j0 + u, yq[u]);
#pragma unroll
        for (int u = 0; u < kNpD; ++u)
            yq[u] = nx[u];
    }
#pragma unroll
    for (int u = 0; u < kNpD; ++u)
        if (j0 + u < nb)
            step(j0 + u, yq[u]);
    L.finish();
    if (mine)
        np_row_outputs(L, i, sub, k0, nb, tl, A, lda, n, lcar, uv, uv32, want32);
}

size_t nopiv_top_lds(int nb) { return sizeof(double) * (size_t)nb * (size_t)(nb + 2); }
size_t nopiv_rows_lds(int nb) { return sizeof(double) * (size_t)nb * NpRow::NA; }

void nopiv_init_attrs()
{
    (void)hipFuncSetAttribute((const void *)nopiv_top_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)nopiv_rows_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

int nopiv_max_block() { return kNpMaxB; }

static hipError_t launch_nopiv_top(double *A, int lda, const double *W, int n, int k0, int nb,
                                   double *t, const FactorWs &ws, int want32, hipStream_t s)
{
    if (nb < 1 || nb > kNpMaxB)
        return hipErrorInvalidValue;
    (void)hipGetLastError();
    hipLaunchKernelGGL(nopiv_top_kernel, dim3(1), dim3(kNpNT), nopiv_top_lds(nb), s, A, lda, W,
                       ws.ldw, n, k0, nb, t, ws.lcar, ws.mirror, (int)NpRow::NA, ws.uv, ws.uv32,
                       want32);
    return hipGetLastError();
}

static hipError_t launch_nopiv_rows(double *A, int lda, const double *W, int n, int k0, int nb,
                                    const double *t, const FactorWs &ws, int want32,
                                    hipStream_t s)
{
    if (nb < 1 || nb > kNpMaxB)
        return hipErrorInvalidValue;
    const int below = n - (k0 + nb + 1);
    if (below <= 0)
        return hipSuccess;
    (void)hipGetLastError();
    const dim3 grid((unsigned)((below + kNpR - 1) / kNpR));
    hipLaunchKernelGGL(nopiv_rows_kernel, grid, dim3(kNpNT), nopiv_rows_lds(nb), s, A, lda, W,
                       ws.ldw, n, k0, nb, t, ws.lcar, (const double *)ws.mirror, (int)NpRow::NA,
                       ws.uv, ws.uv32, want32);
    return hipGetLastError();
}

// The whole panel: the top rows (one workgroup; h and t into the mirror
// buffer), then every other row.
hipError_t launch_nopiv_panel(double *A, int lda, const double *W, int n, int k0, int nb,
                              double *t, const FactorWs &ws, int want32, hipStream_t s)
{
    hipError_t e = launch_nopiv_top(A, lda, W, n, k0, nb, t, ws, want32, s);
    if (e != hipSuccess)
        return e;
    return launch_nopiv_rows(A, lda, W, n, k0, nb, t, ws, want32, s);
}

// perm[i] = i (the skr2k's gather becomes the identity)
__global__ void iota_kernel(int *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = i;
}

hipError_t launch_iota(int *p, int n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    (void)hipGetLastError();
    hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace skl
