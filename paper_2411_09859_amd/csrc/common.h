// Internal declarations shared by the translation units of libskltlt.so.
// Not part of the public ABI (that is include/skltlt.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace skl {

constexpr int kPanelThreads = 512;   // threads per panel workgroup
constexpr int kMaxPanelGroups = 1024; // slot array capacity per parity
constexpr int kMaxBlock = 256;       // largest supported panel width
// one slot per panel workgroup and step parity
constexpr int kSlotsPerParity = kMaxPanelGroups;
constexpr size_t kAlign = 256;

// Pivot exchange slots: one 16-byte record per panel workgroup and step
// parity (layout in the panel kernel), one L2 line apart, then one 4-byte
// record per workgroup for the launch's XCD check.
constexpr int kSlotBytes = 128;
constexpr size_t kSlotArrayBytes = (size_t)kSlotBytes * 3 * kSlotsPerParity;
struct Slot {
    unsigned int w[4];
};

// Device workspace of skltlt_factor, carved from the caller's buffer.
struct FactorWs {
    double *W[2];      // the trailing matrix's lower triangle (ping-pong), ld = ldw
    int ldw;
    int *perm;         // panel permutation: perm[pos] = row at the panel start
    double *mirror;    // physical panel rows, row-major, ld = ldm
    int ldm;
    double *lcar;      // carried L column (n doubles)
    double *uv;        // skr2k operands, column-major n x (4*nq): [U | V | -V | U]
    float *uv32;       // same in fp32
    Slot *slots;       // kSlotArrayBytes: 2 parities x kMaxPanelGroups, XCD check
    int *gmap;         // nblocks x n suffix gather maps
    int *blk_k0;       // nblocks + 1 block starts (device copy not needed: args)
    size_t bytes;
};

size_t factor_ws_layout(int n, int b, FactorWs *ws, char *base);

// Device workspace of skltlt_solve.
struct SolveWs {
    int *q;      // row permutation (n)
    double *Y;   // P B and later stages (n x nrhs, ld)
    double *U;   // later stages, last the solution before the inverse permutation
    int ld;
    size_t bytes;
};
size_t solve_ws_layout(int n, int nrhs, SolveWs *ws, char *base);
hipError_t launch_solve(int n, int nrhs, const double *LT, int lda, const double *t,
                        const int *ipiv, double *B, int ldb, const SolveWs &ws, hipStream_t s);
void solve_init_attrs();

// ---- launchers (return hipError_t) -----------------------------------------
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_set_int(int *p, int v, hipStream_t s);

struct PanelShape {
    int G;  // workgroups
    int R;  // rows per workgroup (power of two, <= kPanelThreads)
    size_t lds;
};
PanelShape panel_shape(int n, int k0, int b, int max_groups);
// W: the trailing matrix as of the panel start, its lower triangle (read only).
hipError_t launch_panel(double *A, int lda, const double *W, int n, int k0, int nb, int b,
                        double *t, int *ipiv, const FactorWs &ws, int want32,
                        const PanelShape &sh, hipStream_t s);

// Pfaffian-only panel: pairs of columns, one pivot per pair (nb even).
hipError_t launch_panel_pair(const double *W, int n, int k0, int nb, int b, double *t, int *ipiv,
                             const FactorWs &ws, int want32, const PanelShape &sh, hipStream_t s);

// Unpivoted panel (top rows, then all other rows), nb <= nopiv_max_block().
hipError_t launch_nopiv_panel(double *A, int lda, const double *W, int n, int k0, int nb,
                              double *t, const FactorWs &ws, int want32, hipStream_t s);
int nopiv_max_block();
void nopiv_init_attrs();
// p[i] = i for i < n
hipError_t launch_iota(int *p, int n, hipStream_t s);

// W[i][j] += sum_k opI[i][k] opJ[j][k] for the columns c0 .. c0+nb-1 (nb <=
// 128) and rows i > j (the left-looking panel update).
hipError_t launch_lkupd(double *W, int ldw, int n, int c0, int nb, const double *opI,
                        const double *opJ, int ldo, int K, hipStream_t s);

// Wn[i][j] = Wc[perm[i]][perm[j]] - (U V^T - V U^T)[i][j] for i != j >= cp.
void skr2k_set_small_tiles(int t);
hipError_t launch_skr2k(const double *Wc, double *Wn, int n, int cp, int nq,
                        const FactorWs &ws, int precision, hipStream_t s);

// Lower triangle of W = A's strict lower triangle, zero diagonal.
hipError_t launch_init_lower(const double *A, int lda, int n, double *W, int ldw, hipStream_t s);

hipError_t launch_finalize(double *A, int lda, int n, int b, const int *ipiv,
                           const FactorWs &ws, hipStream_t s);

hipError_t launch_pfaffian(int n, const double *t, const int *ipiv,
                           double *log_abs_pf, int *sign, hipStream_t s);

// Entry (row, col) of a skew-symmetric matrix kept as its lower triangle
// (column-major, leading dimension ld): the offset of the stored entry, and
// in neg whether the entry is its negation (an upper entry, row < col).  The
// diagonal maps to the stored diagonal.
__device__ __forceinline__ size_t skew_at(int row, int col, int ld, bool &neg)
{
    neg = row < col;
    return neg ? (size_t)row * ld + col : (size_t)col * ld + row;
}

// Lower-triangle tile enumeration: tau = I (I + 1) / 2 + J with 0 <= J <= I.
__device__ __forceinline__ void tile_of(int tau, int *ti, int *tj)
{
    int I = (int)((sqrtf(8.0f * (float)tau + 1.0f) - 1.0f) * 0.5f);
    while ((I + 1) * (I + 2) / 2 <= tau)
        ++I;
    while (I * (I + 1) / 2 > tau)
        --I;
    *ti = I;
    *tj = tau - I * (I + 1) / 2;
}

// The same tiles in blocks of S tile rows x S tile columns: block rows in
// order, inside a block row the full blocks left to right (column-major
// inside a block) and the triangular diagonal block last, so that tiles
// processed together share operand panels in L2 (nt: tiles per side).
template <int S>
__device__ __forceinline__ void tile_of_blocked(int tau, int nt, int *ti, int *tj)
{
    int r, c;
    tile_of(tau, &r, &c); // block rows are contiguous in both orders
    const int r0 = (r / S) * S;
    const int h = min(S, nt - r0);
    int t = tau - r0 * (r0 + 1) / 2;
    const int full = r0 * h;
    if (t < full) {
        const int BJ = t / (S * h);
        const int q = t - BJ * S * h;
        *ti = r0 + q % h;
        *tj = BJ * S + q / h;
    } else {
        t -= full;
        int a = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while ((a + 1) * (a + 2) / 2 <= t)
            ++a;
        while (a * (a + 1) / 2 > t)
            --a;
        *ti = r0 + a;
        *tj = r0 + (t - a * (a + 1) / 2);
    }
}

int device_cu_count();
// Records the HIP error behind an SKLTLT_EDEVICE; returns SKLTLT_EDEVICE.
int device_error(hipError_t e, const char *where);
int tm_begin(int cls, hipStream_t s);
void tm_end(int idx, hipStream_t s, double flops);
void panel_init_attrs();
void finalize_init_attrs();
int panel_max_groups(size_t lds_bytes, bool pair);

}  // namespace skl
