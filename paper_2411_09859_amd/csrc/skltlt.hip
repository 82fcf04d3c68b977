// C ABI of libskltlt.so (declared in include/skltlt.h): argument checks,
// workspace layout and the enqueue sequence of the blocked factorization.
//
// Sequence per call (paper arXiv 2411.09859, Sec. 3.6.3 fused blocked
// right-looking algorithm with the pivoting of Sec. 3.7.3, code of Sec. 4.2):
//   copy the input's lower triangle into W0; for each panel of b columns:
//   panel kernel (pivot search, L columns, t, permutation, operands U and
//   V; reads W only), then the skr2k kernel, which applies the panel's
//   permutation and the update while writing the next trailing matrix into
//   the other W buffer; after the last panel: the deferred row exchanges of
//   the earlier L columns.  Pivot choices stay on the device; the host never
//   synchronizes with the stream.
#include "../../include/skltlt.h"
#include "common.h"
#include "factor_table.h"

#include <cstdio>
#include <mutex>

namespace skl {

static size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

static thread_local char g_last_err[256] = "";

int device_error(hipError_t e, const char *where)
{
    snprintf(g_last_err, sizeof(g_last_err), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
    return SKLTLT_EDEVICE;
}

int device_cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

// Leading dimension of the W buffers: n rounded up to 32 doubles plus 32, so
// that columns do not sit at a power-of-two stride.
static int work_ld(int n) { return ((n + 31) / 32) * 32 + 32; }

// Workspace: two work matrices (n x ldw fp64 each, the lower triangle used), the panel
// permutation (n), mirror ((n + 512) x (b+2) fp64, row-major), carried
// column (n), operands [U|V|-V|U] (n x 4k fp64) and their fp32 copy, slots,
// gather maps.
size_t factor_ws_layout(int n, int b, FactorWs *ws, char *base)
{
    const int nq = (b + 1) / 2;
    const int nblk = n > 1 ? (n - 1 + b - 1) / b : 1;
    size_t off = 0;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return base ? base + o : nullptr;
    };
    FactorWs w{};
    w.ldw = work_ld(n);
    w.W[0] = (double *)take(sizeof(double) * nn * (size_t)w.ldw);
    w.W[1] = (double *)take(sizeof(double) * nn * (size_t)w.ldw);
    w.perm = (int *)take(sizeof(int) * nn);
    w.ldm = b + 2;
    w.mirror = (double *)take(sizeof(double) * (nn + 512) * (size_t)(b + 2));
    w.lcar = (double *)take(sizeof(double) * nn);
    w.uv = (double *)take(sizeof(double) * nn * (size_t)(4 * nq));
    w.uv32 = (float *)take(sizeof(float) * nn * (size_t)(4 * nq));
    w.slots = (Slot *)take(kSlotArrayBytes);
    w.gmap = (int *)take(sizeof(int) * nn * (size_t)nblk);
    w.blk_k0 = nullptr;
    w.bytes = off;
    if (ws)
        *ws = w;
    return off;
}

}  // namespace skl

using namespace skl;

static void init_device_attrs()
{
    static std::once_flag once;
    std::call_once(once, [] {
        panel_init_attrs();
        finalize_init_attrs();
        nopiv_init_attrs();
        solve_init_attrs();
        (void)hipGetLastError();
    });
}

static const size_t kLdsCap = 160 * 1024;

extern "C" const char *skltlt_last_device_error(void) { return skl::g_last_err; }

extern "C" const char *skltlt_status_string(int status)
{
    switch (status) {
    case SKLTLT_OK: return "SKLTLT_OK";
    case SKLTLT_EINVAL: return "SKLTLT_EINVAL: invalid argument";
    case SKLTLT_ENOMEM: return "SKLTLT_ENOMEM: out of memory";
    case SKLTLT_EDEVICE: return "SKLTLT_EDEVICE: HIP call or kernel launch failed";
    case SKLTLT_ENOTSUP: return "SKLTLT_ENOTSUP: size or option not supported";
    default: return "SKLTLT: unknown status";
    }
}

// The tuned width for order n (factor_table.h, written by tune_factor.py:
// the fastest measured width at the nearest measured order).
extern "C" int skltlt_default_block_size(int n)
{
    for (const FactorTune &e : kFactorTune)
        if (n <= e.n_max)
            return e.b;
    return kFactorTune[sizeof(kFactorTune) / sizeof(kFactorTune[0]) - 1].b;
}

static int resolve_block(int n, int block_size)
{
    return block_size > 0 ? block_size : skltlt_default_block_size(n);
}

// Supported: panel widths up to kMaxBlock, and orders whose panel fits the
// slot array (256 rows per group at most 1024 groups).  Whether the panel's
// groups can all be resident is checked when the factorization runs.
static int check_supported(int n, int b)
{
    if (b < 1 || b > kMaxBlock)
        return SKLTLT_ENOTSUP;
    if (n > 256 * kMaxPanelGroups)
        return SKLTLT_ENOTSUP;
    return SKLTLT_OK;
}

extern "C" int skltlt_workspace_size(int n, int block_size, int precision, size_t *bytes)
{
    if (n < 0 || block_size < 0 || !bytes || (precision != SKLTLT_FP64 && precision != SKLTLT_FP32_UPDATE))
        return SKLTLT_EINVAL;
    const int b = resolve_block(n, block_size);
    int st = check_supported(n, b);
    if (st != SKLTLT_OK)
        return st;
    *bytes = factor_ws_layout(n, b, nullptr, nullptr);
    return SKLTLT_OK;
}

// pivot = 0: the unpivoted algorithm (panel width at most nopiv_max_block()).
static int factor_impl(int n, double *A, int lda, double *t, int *ipiv, int block_size,
                       int precision, void *work, size_t work_bytes, hipStream_t s,
                       bool pivot = true)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || block_size < 0)
        return SKLTLT_EINVAL;
    if (precision != SKLTLT_FP64 && precision != SKLTLT_FP32_UPDATE)
        return SKLTLT_EINVAL;
    if (n >= 1 && (!A || !ipiv))
        return SKLTLT_EINVAL;
    if (n >= 2 && !t)
        return SKLTLT_EINVAL;
    const int b0 = resolve_block(n, block_size);
    int st = check_supported(n, b0);
    if (st != SKLTLT_OK)
        return st;
    if (n == 0)
        return SKLTLT_OK;
    // the workspace is laid out for the requested width (what the size
    // query reports); the unpivoted panel may use a narrower one
    const size_t need = factor_ws_layout(n, b0, nullptr, nullptr);
    const int b = pivot ? b0 : (b0 < nopiv_max_block() ? b0 : nopiv_max_block());
    if (!work || work_bytes < need || ((uintptr_t)work % kAlign) != 0)
        return SKLTLT_EINVAL;
    init_device_attrs();

    FactorWs ws;
    factor_ws_layout(n, b0, &ws, (char *)work);

    {
        const int ti = tm_begin(SKLTLT_K_OTHER, s);
        hipError_t e = pivot ? launch_set_int(ipiv, 0, s) : launch_iota(ipiv, n, s);
        if (e != hipSuccess)
            return device_error(e, "set ipiv");
        if (!pivot && (e = launch_iota(ws.perm, n, s)) != hipSuccess)
            return device_error(e, "identity permutation");
        if (n > 1 && (e = launch_fill_zero(ws.slots, kSlotArrayBytes, s)) !=
                         hipSuccess)
            return device_error(e, "clear slots");
        if (n > 1 && (e = launch_init_lower(A, lda, n, ws.W[0], ws.ldw, s)) != hipSuccess)
            return device_error(e, "full copy");
        tm_end(ti, s, 0.0);
    }
    if (n == 1)
        return SKLTLT_OK;

    const int want32 = (precision == SKLTLT_FP32_UPDATE);
    // panel geometry: as many groups as the device keeps resident
    int maxg = 0;
    if (pivot) {
        PanelShape probe = panel_shape(n, 0, b, kMaxPanelGroups);
        maxg = panel_max_groups(probe.lds, false);
        if (maxg <= 0)
            return device_error(hipErrorInvalidValue, "panel occupancy query");
    }

    int cur = 0; // W buffer holding the current trailing matrix
    for (int k0 = 0; k0 < n - 1; k0 += b) {
        const int nb = (b < n - 1 - k0) ? b : (n - 1 - k0);
        int ti = tm_begin(SKLTLT_K_PANEL, s);
        hipError_t e;
        if (pivot) {
            PanelShape sh = panel_shape(n, k0, b, maxg);
            if (sh.lds > kLdsCap || sh.G > maxg || 8L * sh.G > 8L * maxg)
                return SKLTLT_ENOTSUP;
            e = launch_panel(A, lda, ws.W[cur], n, k0, nb, b, t, ipiv, ws, want32, sh, s);
        } else {
            e = launch_nopiv_panel(A, lda, ws.W[cur], n, k0, nb, t, ws, want32, s);
        }
        if (e != hipSuccess)
            return device_error(e, "panel launch");
        tm_end(ti, s, 0.0);
        const int cp = k0 + nb;
        if (cp < n - 1) {
            const int nq = (nb + 1) / 2;
            const double m = (double)(n - cp);
            ti = tm_begin(SKLTLT_K_SKR2K, s);
            if ((e = launch_skr2k(ws.W[cur], ws.W[cur ^ 1], n, cp, nq, ws, precision, s)) !=
                hipSuccess)
                return device_error(e, "skr2k launch");
            cur ^= 1;
            // strict lower triangle of the m x m trailing block, K = 2*nq
            tm_end(ti, s, m * (m - 1.0) * 0.5 * 2.0 * (2.0 * nq));
        }
    }
    if (pivot) {
        const int ti = tm_begin(SKLTLT_K_FINALIZE, s);
        hipError_t e = launch_finalize(A, lda, n, b, ipiv, ws, s);
        if (e != hipSuccess)
            return device_error(e, "finalize launch");
        tm_end(ti, s, 0.0);
    }
    return SKLTLT_OK;
}

extern "C" int skltlt_factor(int n, double *A, int lda, double *t, int *ipiv, int block_size,
                             int precision, void *work, size_t work_bytes, void *stream)
{
    return factor_impl(n, A, lda, t, ipiv, block_size, precision, work, work_bytes,
                       (hipStream_t)stream);
}

extern "C" int skltlt_pfaffian(int n, double *A, int lda, double *t, int *ipiv,
                               double *log_abs_pf, int *sign, int block_size, int precision,
                               void *work, size_t work_bytes, void *stream)
{
    if (!log_abs_pf || !sign)
        return SKLTLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = factor_impl(n, A, lda, t, ipiv, block_size, precision, work, work_bytes, s);
    if (st != SKLTLT_OK)
        return st;
    const int ti = tm_begin(SKLTLT_K_PFAFFIAN, s);
    hipError_t e = launch_pfaffian(n, t, ipiv, log_abs_pf, sign, s);
    if (e != hipSuccess)
        return device_error(e, "pfaffian launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}

extern "C" int skltlt_factor_nopiv(int n, double *A, int lda, double *t, int *ipiv,
                                   int block_size, int precision, void *work, size_t work_bytes,
                                   void *stream)
{
    return factor_impl(n, A, lda, t, ipiv, block_size, precision, work, work_bytes,
                       (hipStream_t)stream, false);
}

extern "C" int skltlt_pfaffian_nopiv(int n, double *A, int lda, double *t, int *ipiv,
                                     double *log_abs_pf, int *sign, int block_size, int precision,
                                     void *work, size_t work_bytes, void *stream)
{
    if (!log_abs_pf || !sign)
        return SKLTLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = factor_impl(n, A, lda, t, ipiv, block_size, precision, work, work_bytes, s, false);
    if (st != SKLTLT_OK)
        return st;
    const int ti = tm_begin(SKLTLT_K_PFAFFIAN, s);
    hipError_t e = launch_pfaffian(n, t, ipiv, log_abs_pf, sign, s);
    if (e != hipSuccess)
        return device_error(e, "pfaffian launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}

// ---- left-looking (Variant 3), unpivoted ------------------------------------
// Operand columns the left-looking update accumulates: every panel but the
// last appends 2 * ceil((nb+1)/2) columns to each of opI and opJ.
static size_t left_kcap(int n, int b)
{
    size_t k = 0;
    for (int k0 = 0; k0 < n - 1; k0 += b) {
        const int nb = (b < n - 1 - k0) ? b : (n - 1 - k0);
        if (k0 + nb < n - 1)
            k += 2 * (size_t)((nb + 1) / 2);
    }
    return k;
}

static int left_block(int n, int block_size)
{
    const int b = resolve_block(n, block_size);
    return b < nopiv_max_block() ? b : nopiv_max_block();
}

// Workspace: the factorization's (for the requested width), then opI and
// opJ (n x kcap fp64 each).
static size_t left_ws_bytes(int n, int block_size, size_t *opoff)
{
    const int b0 = resolve_block(n, block_size);
    const size_t base = align_up(factor_ws_layout(n, b0, nullptr, nullptr));
    if (opoff)
        *opoff = base;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    const size_t kc = left_kcap(n, left_block(n, block_size));
    return base + 2 * align_up(sizeof(double) * nn * (kc > 0 ? kc : 1));
}

extern "C" int skltlt_left_workspace_size(int n, int block_size, size_t *bytes)
{
    if (n < 0 || block_size < 0 || !bytes)
        return SKLTLT_EINVAL;
    int st = check_supported(n, resolve_block(n, block_size));
    if (st != SKLTLT_OK)
        return st;
    *bytes = left_ws_bytes(n, block_size, nullptr);
    return SKLTLT_OK;
}

static int left_impl(int n, double *A, int lda, double *t, int *ipiv, int block_size,
                     int precision, void *work, size_t work_bytes, hipStream_t s)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || block_size < 0)
        return SKLTLT_EINVAL;
    if (precision != SKLTLT_FP64 && precision != SKLTLT_FP32_UPDATE)
        return SKLTLT_EINVAL;
    if (precision != SKLTLT_FP64)
        return SKLTLT_ENOTSUP;
    if (n >= 1 && (!A || !ipiv))
        return SKLTLT_EINVAL;
    if (n >= 2 && !t)
        return SKLTLT_EINVAL;
    const int b0 = resolve_block(n, block_size);
    int st = check_supported(n, b0);
    if (st != SKLTLT_OK)
        return st;
    if (n == 0)
        return SKLTLT_OK;
    size_t opoff = 0;
    const size_t need = left_ws_bytes(n, block_size, &opoff);
    if (!work || work_bytes < need || ((uintptr_t)work % kAlign) != 0)
        return SKLTLT_EINVAL;
    init_device_attrs();
    FactorWs ws;
    factor_ws_layout(n, b0, &ws, (char *)work);
    const int b = left_block(n, block_size);
    const size_t kcap = left_kcap(n, b);
    double *opI = (double *)((char *)work + opoff);
    double *opJ = opI + align_up(sizeof(double) * (size_t)n * (kcap > 0 ? kcap : 1)) / sizeof(double);
    {
        const int ti = tm_begin(SKLTLT_K_OTHER, s);
        hipError_t e = launch_iota(ipiv, n, s);
        if (e == hipSuccess)
            e = launch_iota(ws.perm, n, s);
        if (e == hipSuccess && n > 1)
            e = launch_init_lower(A, lda, n, ws.W[0], ws.ldw, s);
        if (e != hipSuccess)
            return device_error(e, "left-looking set-up");
        tm_end(ti, s, 0.0);
    }
    if (n == 1)
        return SKLTLT_OK;
    size_t kcur = 0;
    for (int k0 = 0; k0 < n - 1; k0 += b) {
        const int nb = (b < n - 1 - k0) ? b : (n - 1 - k0);
        hipError_t e = hipSuccess;
        if (kcur > 0) {
            // every earlier panel's update, on this panel's columns only
            const double m = (double)(n - k0);
            const int ti = tm_begin(SKLTLT_K_SKR2K, s);
            e = launch_lkupd(ws.W[0], ws.ldw, n, k0, nb, opI, opJ, n, (int)kcur, s);
            tm_end(ti, s, 2.0 * (double)kcur * (m * nb - 0.5 * nb * (nb + 1.0)));
            if (e != hipSuccess)
                return device_error(e, "left-looking update launch");
        }
        const int tp = tm_begin(SKLTLT_K_PANEL, s);
        e = launch_nopiv_panel(A, lda, ws.W[0], n, k0, nb, t, ws, 0, s);
        tm_end(tp, s, 0.0);
        if (e != hipSuccess)
            return device_error(e, "panel launch");
        const int cp = k0 + nb;
        if (cp < n - 1) {
            // this panel's [U | V] and [-V | U] join the accumulated operands
            const int nq = (nb + 1) / 2;
            const size_t bytes = sizeof(double) * (size_t)n * (size_t)(2 * nq);
            e = hipMemcpyAsync(opI + kcur * (size_t)n, ws.uv, bytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(opJ + kcur * (size_t)n, ws.uv + (size_t)(2 * nq) * n, bytes,
                                   hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess)
                return device_error(e, "operand copy");
            kcur += 2 * (size_t)nq;
        }
    }
    return SKLTLT_OK;
}

extern "C" int skltlt_factor_left(int n, double *A, int lda, double *t, int *ipiv, int block_size,
                                  int precision, void *work, size_t work_bytes, void *stream)
{
    return left_impl(n, A, lda, t, ipiv, block_size, precision, work, work_bytes,
                     (hipStream_t)stream);
}

extern "C" int skltlt_pfaffian_left(int n, double *A, int lda, double *t, int *ipiv,
                                    double *log_abs_pf, int *sign, int block_size, int precision,
                                    void *work, size_t work_bytes, void *stream)
{
    if (!log_abs_pf || !sign)
        return SKLTLT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int st = left_impl(n, A, lda, t, ipiv, block_size, precision, work, work_bytes, s);
    if (st != SKLTLT_OK)
        return st;
    const int ti = tm_begin(SKLTLT_K_PFAFFIAN, s);
    hipError_t e = launch_pfaffian(n, t, ipiv, log_abs_pf, sign, s);
    if (e != hipSuccess)
        return device_error(e, "pfaffian launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}

extern "C" int skltlt_pfaffian_partial(int n, const double *A, int lda, double *t, int *ipiv,
                                       double *log_abs_pf, int *sign, int block_size,
                                       int precision, void *work, size_t work_bytes, void *stream)
{
    if (n < 0 || lda < (n > 1 ? n : 1) || block_size < 0 || !log_abs_pf || !sign)
        return SKLTLT_EINVAL;
    if (precision != SKLTLT_FP64 && precision != SKLTLT_FP32_UPDATE)
        return SKLTLT_EINVAL;
    if (n >= 1 && (!A || !ipiv))
        return SKLTLT_EINVAL;
    if (n >= 2 && !t)
        return SKLTLT_EINVAL;
    const int b0 = resolve_block(n, block_size);
    int st = check_supported(n, b0);
    if (st != SKLTLT_OK)
        return st;
    const int b = (b0 >= 2) ? (b0 & ~1) : 2; // pairs of columns
    hipStream_t s = (hipStream_t)stream;
    if (n >= 1) {
        const size_t need = factor_ws_layout(n, b0, nullptr, nullptr);
        if (!work || work_bytes < need || ((uintptr_t)work % kAlign) != 0)
            return SKLTLT_EINVAL;
    }
    init_device_attrs();
    FactorWs ws{};
    if (n >= 1)
        factor_ws_layout(n, b0, &ws, (char *)work);
    if (n >= 1) {
        const int ti = tm_begin(SKLTLT_K_OTHER, s);
        hipError_t e = launch_set_int(ipiv, 0, s);
        if (e != hipSuccess)
            return device_error(e, "set ipiv[0]");
        if (n > 1 && (e = launch_fill_zero(ws.slots, kSlotArrayBytes, s)) !=
                         hipSuccess)
            return device_error(e, "clear slots");
        if (n > 1 && (e = launch_init_lower(A, lda, n, ws.W[0], ws.ldw, s)) != hipSuccess)
            return device_error(e, "full copy");
        tm_end(ti, s, 0.0);
    }
    if (n > 1) {
        const int want32 = (precision == SKLTLT_FP32_UPDATE);
        PanelShape probe = panel_shape(n, 0, b, kMaxPanelGroups);
        int maxg = panel_max_groups(probe.lds, true);
        if (maxg <= 0)
            return device_error(hipErrorInvalidValue, "panel occupancy query");
        int cur = 0;
        for (int k0 = 0; k0 + 1 < n; k0 += b) {
            const int pairs_left = (n - k0) / 2;
            const int nb = (b < 2 * pairs_left) ? b : 2 * pairs_left;
            PanelShape sh = panel_shape(n, k0, b, maxg);
            if (sh.lds > kLdsCap || sh.G > maxg)
                return SKLTLT_ENOTSUP;
            int ti = tm_begin(SKLTLT_K_PANEL, s);
            hipError_t e = launch_panel_pair(ws.W[cur], n, k0, nb, b, t, ipiv, ws, want32, sh, s);
            if (e != hipSuccess)
                return device_error(e, "pair panel launch");
            tm_end(ti, s, 0.0);
            const int cp = k0 + nb;
            if (cp < n - 1) {
                const int nq = nb / 2;
                const double m = (double)(n - cp);
                ti = tm_begin(SKLTLT_K_SKR2K, s);
                if ((e = launch_skr2k(ws.W[cur], ws.W[cur ^ 1], n, cp, nq, ws, precision, s)) !=
                    hipSuccess)
                    return device_error(e, "skr2k launch");
                cur ^= 1;
                tm_end(ti, s, m * (m - 1.0) * 0.5 * 2.0 * (2.0 * nq));
            }
        }
    }
    const int ti = tm_begin(SKLTLT_K_PFAFFIAN, s);
    hipError_t e = launch_pfaffian(n, t, ipiv, log_abs_pf, sign, s);
    if (e != hipSuccess)
        return device_error(e, "pfaffian launch");
    tm_end(ti, s, 0.0);
    return SKLTLT_OK;
}

extern "C" int skltlt_solve_workspace_size(int n, int nrhs, size_t *bytes)
{
    if (n < 0 || nrhs < 1 || !bytes)
        return SKLTLT_EINVAL;
    *bytes = solve_ws_layout(n, nrhs, nullptr, nullptr);
    return SKLTLT_OK;
}

extern "C" int skltlt_solve(int n, int nrhs, const double *LT, int lda, const double *t,
                            const int *ipiv, double *B, int ldb, void *work, size_t work_bytes,
                            void *stream)
{
    if (n < 0 || (n & 1) || nrhs < 1)
        return SKLTLT_EINVAL;
    if (n == 0)
        return SKLTLT_OK;
    if (lda < n || ldb < n || !LT || !t || !ipiv || !B)
        return SKLTLT_EINVAL;
    const size_t need = solve_ws_layout(n, nrhs, nullptr, nullptr);
    if (!work || work_bytes < need || ((uintptr_t)work % kAlign) != 0)
        return SKLTLT_EINVAL;
    init_device_attrs();
    SolveWs ws;
    solve_ws_layout(n, nrhs, &ws, (char *)work);
    hipStream_t s = (hipStream_t)stream;
    const int ti = tm_begin(SKLTLT_K_SOLVE, s);
    hipError_t e = launch_solve(n, nrhs, LT, lda, t, ipiv, B, ldb, ws, s);
    if (e != hipSuccess)
        return device_error(e, "solve launch");
    // L^{-1}, L^{-T}: n^2 each per right-hand side; T^{-1}: O(n)
    tm_end(ti, s, 2.0 * (double)n * (double)n * nrhs);
    return SKLTLT_OK;
}
