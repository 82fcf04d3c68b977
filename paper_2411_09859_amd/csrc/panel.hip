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
// One launch handles one panel of nb column steps.  A workgroup
// of 512 threads owns R = 512/TPR consecutive trailing rows; the TPR threads
// of a row (64/TPR lanes apart in a wave) hold that row of the panel's L (the
// carried column and the nb new ones, column a in thread a % TPR, register
// a / TPR) in registers, so a
// group covers 256 rows at b = 128 and the whole n = 16384 trailing matrix
// needs only 64 groups (the cost of the per-step exchange grows with the
// number of groups).  Each column step c (r = c+1):
//   1. h = T_p * L[c, panel]^T from the previous pivot row (computed
//      redundantly by every group from the same data);
//   2. x_i = Y[i, c] - L[i, panel] . h for owned rows i >= r, where Y is the
//      trailing matrix as of the panel start with this panel's symmetric
//      exchanges applied;
//   3. argmax of |x_i| (first index on ties) over the group;
//   4. with several groups: each group publishes its candidate in a slot of
//      self-validating words (every 8-byte word carries the step stamp) and
//      polls all slots; every group reduces them to the same pivot p;
//   5. exchange rows/columns r <-> p: relabel the register rows of r and p,
//      load the next column, and form the new column of L, l = x / tau
//      (0 if tau = 0).
// The exchanges are never applied to memory here.  A register row always
// holds the same row of the panel-start matrix Y0 (its "original" row) and
// only the label it stands for changes: the one that held r continues as p
// with its x, the one that held p becomes row r, final for this panel.
// Entry (label i, label r) of the exchanged matrix is Y0[orig(i), orig(r)]:
// one column of Y0 per step, read from its lower triangle (the trailing
// matrix is kept as its lower triangle; rows above orig(r) read the mirrored
// entry, negated).  The skr2k kernel applies the panel's permutation when it
// forms the next trailing matrix.  The panel writes
// nothing but its outputs: L, t, pivots, the permutation, the operands.
// Other groups read the pivot row of L from a row-major mirror in HBM indexed
// by register row, which is written once per column and never rewritten.
// Cross-group words (slots, the mirror) are relaxed device-scope atomics:
// coherent across XCDs without L2 write-back or invalidation.
#include "common.h"
#include "wave_max.h"

#include <climits>
#include <cstdint>
#include <mutex>

namespace skl {


// Pivot order: larger |x| wins, the smaller row index on ties (evaluated
// without branches).
__device__ __forceinline__ bool beats(double av, int ai, double bv, int bi)
{
    const double aa = fabs(av), bb = fabs(bv);
    return (aa > bb) | ((aa == bb) & (ai < bi));
}

// Wave-wide argmax in the pivot order over the candidates in lanes
// 0 .. CL-1 (CL = 16, 32 or 64; other lanes are ignored); every lane
// receives the winner's (v, idx, ph).  The bit pattern of |v| orders
// non-negative doubles, so the largest is found on its high dword first (one
// 32-bit DPP max); the lanes holding that high dword are found with a
// ballot, and only when several do are their low dwords compared, and only
// on an exact tie the indices.  Lanes without a candidate hold v = 0,
// idx = INT_MAX.
template <int CL>
__device__ __forceinline__ void wave_argmax(double &v, int &idx, int &ph)
{
    const bool in = (CL == 64) || ((int)(threadIdx.x & 63) < CL);
    const unsigned long long key =
        in ? (unsigned long long)__double_as_longlong(fabs(v)) : 0ull;
    const unsigned khi = (unsigned)(key >> 32), klo = (unsigned)key;
    const unsigned mh = lanes_max_u32<CL>(khi);
    bool top = in && (khi == mh);
    unsigned long long m = __ballot(top);
    if (__popcll(m) != 1) {
        const unsigned ml = lanes_max_u32<CL>(top ? klo : 0u);
        top = top && (klo == ml);
        m = __ballot(top);
        if (__popcll(m) != 1) {
            int ci = top ? idx : INT_MAX;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const int o = __shfl_xor(ci, off, 64);
                ci = (o < ci) ? o : ci;
            }
            m = __ballot(top && idx == ci);
        }
    }
    const int wl = __ffsll((long long)m) - 1;
    v = readlane_f64(v, wl);
    idx = __builtin_amdgcn_readlane(idx, wl);
    ph = __builtin_amdgcn_readlane(ph, wl);
}

__device__ __forceinline__ double ld_dev(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A store read by other groups: plain when every working group shares this
// XCD (checked at the launch's start; the shared L2 makes it visible to their
// device-scope reads), device scope otherwise.
__device__ __forceinline__ void st_xcd(double *p, double v, bool local)
{
    if (local)
        *p = v;
    else
        st_dev(p, v);
}

// Stores into the row-major mirror of L through a bounds-checked buffer
// resource.  Every thread issues both forms of the store of a step, plain
// and device scope, and passes the end of the buffer as the offset of the
// one it does not use (or of both, with nothing to store), which the
// hardware drops.  So each step issues the same memory instructions on
// every path, and the compiler's waits for the step's earlier loads do not
// have to cover the later ones (with a store issued on some paths only, its
// wait for the mirror loads also waited for the next column's HBM load).
struct MirrorIO {
    __amdgpu_buffer_rsrc_t rs;
    int nrec;   // bytes covered; an offset of nrec is out of range
    bool local; // plain stores (every working group on this XCD)

    // bytes < 2^31 (the supported orders, n <= 2^18, keep the mirror below
    // 0.6 GB); readfirstlane keeps the
    // resource in scalar registers (a resource the compiler cannot prove
    // uniform is applied lane by lane in a loop)
    __device__ __forceinline__ MirrorIO(double *mirror, int bytes, bool local_)
        : nrec(__builtin_amdgcn_readfirstlane(bytes)), local(local_)
    {
        rs = __builtin_amdgcn_make_buffer_rsrc((void *)mirror, (short)0, nrec, 0x00020000);
    }
    // entry (row, col) when on, else nothing
    __device__ __forceinline__ void store(bool on, int row, int ldm, int col, double v) const
    {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        u32x2 d;
        d.x = (unsigned)b;
        d.y = (unsigned)(b >> 32);
        const int off = (row * ldm + col) * (int)sizeof(double);
        __builtin_amdgcn_raw_buffer_store_b64(d, rs, (on && local) ? off : nrec, 0, 0);
        // device scope (sc1)
        __builtin_amdgcn_raw_buffer_store_b64(d, rs, (on && !local) ? off : nrec, 0, 16);
    }
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// The pivot exchange between groups.  A slot is one 16-byte access.  Each
// of its four dwords carries the step stamp (4 bits: a slot is rewritten
// every second step, so the stale contents it can hold are one write old)
// above 28 payload bits: the candidate value (64 bits), its row relative to
// the panel base (24 bits, 0xffffff: none) and its register row (24 bits).
// A reader accepts the slot when all four stamps match, so a read that mixes
// two writes is never taken for a complete one.  Each slot has a 128-byte
// L2 line of its own: slots that share a line make writers on different
// XCDs contend for it (measured slower).
struct SlotIO {
    __amdgpu_buffer_rsrc_t srs;
    int base;   // the panel's first trailing row
    bool local; // every working group on this XCD (checked at the launch's start)

    __device__ __forceinline__ SlotIO(Slot *slots, int base_, bool local_)
        : srs(__builtin_amdgcn_make_buffer_rsrc((void *)slots, (short)0,
                                                (int)(kSlotBytes * 2 * kSlotsPerParity),
                                                0x00020000)),
          base(base_), local(local_)
    {
    }
    __device__ __forceinline__ void publish(int q, unsigned stamp, double v, int idx,
                                            int ph) const
    {
        const unsigned long long xb = (unsigned long long)__double_as_longlong(v);
        const unsigned vhi = (unsigned)(xb >> 32), vlo = (unsigned)xb;
        const unsigned ib = (idx == INT_MAX) ? 0xffffffu : (unsigned)(idx - base);
        const unsigned st = (stamp & 0xfu) << 28;
        u32x4 d;
        d.x = st | (vhi >> 4);
        d.y = st | ((vhi & 0xfu) << 24) | (vlo >> 8);
        d.z = st | ((vlo & 0xffu) << 20) | (ib >> 4);
        d.w = st | ((ib & 0xfu) << 24) | ((unsigned)ph & 0xffffffu);
        if (local)
            __builtin_amdgcn_raw_buffer_store_b128(d, srs, q * kSlotBytes, 0, 0);
        else // device scope (sc1): visible to other XCDs without an L2 write-back
            __builtin_amdgcn_raw_buffer_store_b128(d, srs, q * kSlotBytes, 0, 16);
    }
    __device__ __forceinline__ u32x4 load(int q) const
    {
        return __builtin_amdgcn_raw_buffer_load_b128(srs, q * kSlotBytes, 0, 16);
    }
    __device__ static __forceinline__ bool ready(u32x4 d, unsigned stamp)
    {
        const unsigned s4 = stamp & 0xfu;
        return ((d.x >> 28) == s4) & ((d.y >> 28) == s4) & ((d.z >> 28) == s4) &
               ((d.w >> 28) == s4);
    }
    // Folds a slot's candidate into (gv, gi, gph) in the pivot order.
    __device__ __forceinline__ void fold(u32x4 d, double &gv, int &gi, int &gph) const
    {
        const unsigned vhi = ((d.x & 0x0fffffffu) << 4) | ((d.y >> 24) & 0xfu);
        const unsigned vlo = ((d.y & 0x00ffffffu) << 8) | ((d.z >> 20) & 0xffu);
        const unsigned ib = ((d.z & 0x000fffffu) << 4) | ((d.w >> 24) & 0xfu);
        const double v2 = __longlong_as_double((long long)(((unsigned long long)vhi << 32) | vlo));
        const int i2 = (ib == 0xffffffu) ? INT_MAX : base + (int)ib;
        const bool wn = beats(v2, i2, gv, gi);
        gv = wn ? v2 : gv;
        gi = wn ? i2 : gi;
        gph = wn ? (int)(d.w & 0x00ffffffu) : gph;
    }
};

// bounded waits: a stuck peer never hangs the GPU (the result is poisoned)
constexpr long kSpinLimit = 1L << 20;

// LDS state of a group's pivot search.
template <int NW>
struct PivotLds {
    double red_v[NW];
    int red_i[NW], red_ph[NW];
    double bc_tau;
    int bc_p, bc_physp, bc_fail;
};

// Reduces the per-wave candidates (waves without one hold v = 0,
// idx = INT_MAX) in the pivot order; one thread.
template <int NW>
__device__ __forceinline__ void reduce_waves(const double *red_v, const int *red_i,
                                             const int *red_ph, double &bv, int &bi, int &bph)
{
    double rv[NW];
    int ri[NW], rph[NW];
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        rv[q] = red_v[q];
        ri[q] = red_i[q];
        rph[q] = red_ph[q];
    }
    bv = rv[0];
    bi = ri[0];
    bph = rph[0];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
        const bool wn = beats(rv[q], ri[q], bv, bi);
        bv = wn ? rv[q] : bv;
        bi = wn ? ri[q] : bi;
        bph = wn ? rph[q] : bph;
    }
}

// The step's pivot, broadcast through LDS; an index that does not name an
// existing candidate row can only follow a failed wait and poisons the
// result (tau = NaN) while keeping every later access in range.
template <int NW>
__device__ __forceinline__ void set_pivot(PivotLds<NW> &pl, double v, int idx, int ph, int r_cur,
                                          int n, int G, int R, int base)
{
    if (idx < r_cur || idx >= n || ph < 0 || ph >= G * R || base + ph >= n) {
        pl.bc_p = r_cur;
        pl.bc_physp = 0;
        pl.bc_fail = 1;
    } else {
        pl.bc_p = idx;
        pl.bc_physp = ph;
    }
    pl.bc_tau = v;
}

// Group argmax of the candidates (cv, ci, cph) (lanes without one hold
// v = 0, idx = INT_MAX) and, with several groups, the exchange through the
// slots: each group publishes its candidate and polls all slots of this
// parity, and every group reduces them to the same pivot.  Ends with a
// barrier after which pl.bc_* hold the pivot.  The caller's mirror stores
// (this wave's) are complete before the slot is published.
template <int NT, int CL>
__device__ __forceinline__ void find_pivot(PivotLds<NT / 64> &pl, const SlotIO &sio, bool multi,
                                           int G, int w, int par, unsigned stamp, int r_cur, int n,
                                           int R, double cv, int ci, int cph)
{
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    static_assert(NW <= 16, "waves per group");
    wave_argmax<CL>(cv, ci, cph);
    if (lane == 0) {
        pl.red_v[wave] = cv;
        pl.red_i[wave] = ci;
        pl.red_ph[wave] = cph;
    }
    // this wave's mirror stores of the previous step must be complete
    // before the group's slot is published
    if (multi)
        wait_vm();
    __syncthreads();
    // the group's candidate: wave 0 reduces the per-wave ones (lane q holds
    // wave q's), then publishes it or, alone, takes it as the pivot
    if (wave == 0) {
        double bv = 0.0;
        int bi = INT_MAX, bph = 0;
        if (lane < NW) {
            bv = pl.red_v[lane];
            bi = pl.red_i[lane];
            bph = pl.red_ph[lane];
        }
        wave_argmax<16>(bv, bi, bph);
        if (lane == 0) {
            if (multi)
                sio.publish(par * kSlotsPerParity + w, stamp, bv, bi, bph);
            else
                set_pivot<NW>(pl, bv, bi, bph, r_cur, n, G, R, sio.base);
        }
    }

    // several groups: poll all slots and reduce them identically in every
    // group
    if (multi && G <= 128) {
        // wave 0 alone: lane l polls slots l and l + 64 (a slot already
        // seen complete is not read again; both reads of a round are in
        // flight together), then one wave argmax gives the pivot
        if (wave == 0) {
            const int q0 = lane, q1 = lane + 64;
            const bool use0 = q0 < G, use1 = q1 < G;
            const int sb = par * kSlotsPerParity;
            u32x4 d0 = {0u, 0u, 0u, 0u}, d1 = {0u, 0u, 0u, 0u};
            bool ok0 = !use0, ok1 = !use1;
            long spins = 0;
            for (;;) {
                // compiler-only fence: the slot loads are ordinary
                // intrinsics and would otherwise be hoisted out of the spin
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                if (!ok0)
                    d0 = sio.load(sb + q0);
                if (!ok1)
                    d1 = sio.load(sb + q1);
                ok0 = ok0 || SlotIO::ready(d0, stamp);
                ok1 = ok1 || SlotIO::ready(d1, stamp);
                if (ok0 && ok1)
                    break;
                if (pl.bc_fail || ++spins > kSpinLimit) {
                    pl.bc_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            double gv = 0.0;
            int gi = INT_MAX, gph = 0;
            if (use0)
                sio.fold(d0, gv, gi, gph);
            if (use1)
                sio.fold(d1, gv, gi, gph);
            wave_argmax<64>(gv, gi, gph);
            if (lane == 0)
                set_pivot<NW>(pl, gv, gi, gph, r_cur, n, G, R, sio.base);
        }
    } else if (multi) {
        double gv = 0.0;
        int gi = INT_MAX, gph = 0;
        for (int q = tid; q < G; q += NT) {
            u32x4 d;
            long spins = 0;
            for (;;) {
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                d = sio.load(par * kSlotsPerParity + q);
                if (SlotIO::ready(d, stamp))
                    break;
                if (pl.bc_fail || ++spins > kSpinLimit) {
                    pl.bc_fail = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            sio.fold(d, gv, gi, gph);
        }
        {
            if (wave * 64 < G)
                wave_argmax<64>(gv, gi, gph);
            __syncthreads(); // red_* of the group argmax were consumed by thread 0
            if (lane == 0) {
                pl.red_v[wave] = gv;
                pl.red_i[wave] = gi;
                pl.red_ph[wave] = gph;
            }
            __syncthreads();
            if (tid == 0) {
                double bv;
                int bi, bph;
                reduce_waves<NW>(pl.red_v, pl.red_i, pl.red_ph, bv, bi, bph);
                set_pivot<NW>(pl, bv, bi, bph, r_cur, n, G, R, sio.base);
            }
        }
    }
    __syncthreads();
}


// Whether every working group of this launch runs on one XCD: each group
// publishes its XCC_ID (hardware register) tagged with the panel's first
// column and reads all the others' (device scope).  Every group reaches the
// same answer from the same records.  The exchange then uses plain stores,
// which the XCD's shared L2 makes visible to the device-scope reads of its
// other groups; otherwise every cross-group store is device scope.  A failed
// wait answers "no" and poisons the panel.
__device__ __forceinline__ bool groups_share_xcd(Slot *slots, int G, int w, int k0, int &fail)
{
    __shared__ int same;
    const int tid = threadIdx.x;
    if (tid < 64) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)((char *)slots + (size_t)2 * kSlotsPerParity * kSlotBytes), (short)0,
            (int)(kSlotBytes * kSlotsPerParity), 0x00020000);
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
        const unsigned tag = ((unsigned)(k0 + 1) & 0x0fffffffu) << 4;
        if (tid == 0)
            __builtin_amdgcn_raw_buffer_store_b32(tag | (xcc & 0xfu), rs, w * kSlotBytes, 0, 16);
        bool ok = true, lfail = false;
        for (int q = tid; q < G; q += 64) {
            unsigned v = 0;
            long spins = 0;
            for (;;) {
                __atomic_signal_fence(__ATOMIC_SEQ_CST);
                v = __builtin_amdgcn_raw_buffer_load_b32(rs, q * kSlotBytes, 0, 16);
                if ((v & ~0xfu) == tag)
                    break;
                if (++spins > kSpinLimit) {
                    lfail = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            ok = ok && !lfail && ((v & 0xfu) == (xcc & 0xfu));
        }
        const bool all = __ballot(!ok) == 0;
        if (__ballot(lfail) != 0 && tid == 0)
            fail = 1;
        if (tid == 0)
            same = all ? 1 : 0;
    }
    __syncthreads();
    // the same value in every lane; readfirstlane lets the compiler branch
    // on it with scalar branches
    return __builtin_amdgcn_readfirstlane(same) != 0;
}

template <int NT, int TPR, int kNS>
__global__ __launch_bounds__(NT) void panel_kernel(
    double *__restrict__ A, int lda, const double *__restrict__ W, int ldw, int n, int k0,
    int nb, int b, double *__restrict__ t, int *__restrict__ ipiv, int *__restrict__ perm,
    double *__restrict__ mirror,
    int ldm, double *__restrict__ lcar, double *__restrict__ uv,
    float *__restrict__ uv32, int want32, Slot *__restrict__ slots, int G, int one_xcd)
{
    constexpr int R = NT / TPR;
    constexpr int NW = NT / 64;
    // New columns are inserted into a ring of kRing registers; a full ring
    // group is flushed into Lreg once (kRing * TPR column steps).  Inserting
    // into Lreg directly needs a select over every slot at every step.
    constexpr int kRing = 8;
    constexpr int kNSR = ((kNS + kRing - 1) / kRing) * kRing;
    constexpr int NA = kNSR * TPR; // columns addressable through the ring
    // h is read in blocks of 16 slots (one LDS read per lane and block)
    constexpr int kNSB = ((kNS + 15) / 16) * 16;
    constexpr int NH = (kNSB > kNSR ? kNSB : kNSR) * TPR;
    static_assert(TPR == 1 || TPR == 2 || TPR == 4, "a 16-lane row must hold one column class");
    extern __shared__ double stage[]; // R x 34, epilogue only

    __shared__ double hv[NH];
    __shared__ double hrow[NA];
    __shared__ double tl[kMaxBlock];
    __shared__ int pl[kMaxBlock];
    __shared__ int posl[R];
    __shared__ PivotLds<NW> pv;


    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // With one_xcd = 1 + x the grid holds 8 workgroups per panel group and
    // only those whose id is x modulo 8 work: workgroup ids are dealt
    // round-robin to the 8 XCDs, so the working groups normally share XCD x;
    // the kernel checks that (XCC_ID) before it lets the exchange use plain
    // stores, so correctness does not depend on the placement, only the speed
    // does.
    int w = blockIdx.x;
    if (one_xcd) {
        if ((w & 7) != one_xcd - 1)
            return;
        w >>= 3;
    }
    const int base = k0 + 1;        // first trailing row
    // The TPR threads of a row are RL = 64 / TPR lanes apart, so each 16-lane
    // row of a wave holds one column class and h is broadcast inside it.
    constexpr int RL = 64 / TPR;
    const int lr = (tid >> 6) * RL + lane % RL; // register row of this thread
    const int sub = lane / RL;                  // column class of this thread
    const int phys = w * R + lr;    // its row in the mirror (fixed)
    const int orow = base + phys;   // its row of the panel-start matrix (fixed)
    const bool multi = (G > 1);

    // The matrix row a register row represents.  Exchanging rows r and p
    // relabels the two register rows instead of moving their data: the one
    // that held row r now holds row p and keeps its x, the one that held
    // row p becomes row r, which is final for this panel.
    int pos = orow;
    const bool exists = (orow < n);

    double Lreg[kNS];   // slots of flushed ring groups (slot q: column sub + TPR q)
    double Lnew[kRing]; // slots g kRing .. g kRing + kRing - 1 of the current group g
#pragma unroll
    for (int q = 0; q < kNS; ++q)
        Lreg[q] = 0.0;
#pragma unroll
    for (int i = 0; i < kRing; ++i)
        Lnew[i] = 0.0;
    // copy the ring into ring group g of Lreg and clear it (g uniform)
    auto flush_ring = [&](int g) {
#pragma unroll
        for (int q = 0; q < kNS; ++q)
            Lreg[q] = (q / kRing == g) ? Lnew[q % kRing] : Lreg[q];
#pragma unroll
        for (int i = 0; i < kRing; ++i)
            Lnew[i] = 0.0;
    };

    // ---- panel start: carried column (column 0 of the panel) and the first
    //      column of Y
    double ycol = 0.0;
    bool yneg = false; // ycol holds the negation of the entry (an upper one)
    for (int a = tid; a < NH; a += NT)
        hv[a] = 0.0;
    for (int a = tid; a < NA; a += NT)
        hrow[a] = 0.0;
    if (exists && sub == 0)
        Lnew[0] = (k0 == 0) ? 0.0 : lcar[pos];
    if (exists) // every thread of the row (one address)
        ycol = W[(size_t)k0 * ldw + orow];
    if (tid == 0) {
        pv.bc_fail = 0;
    }
    __syncthreads();
    // with one_xcd, whether the working groups did land on one XCD (then the
    // exchange uses plain stores)
    bool local = false;
    if (one_xcd) {
        int fl = 0;
        local = groups_share_xcd(slots, G, w, k0, fl);
        if (fl && tid == 0)
            pv.bc_fail = 1;
    }
    const SlotIO sio(slots, base, local);
    // the carried column's mirror entry
    if (multi && exists && sub == 0)
        st_xcd(&mirror[(size_t)phys * ldm], Lnew[0], local);
    const MirrorIO mio(mirror, (int)sizeof(double) * G * R * ldm, local);
    // nothing in flight when the steps begin (a load still pending from here
    // would make the compiler wait for every load at each step's start)
    wait_vm();

    for (int j = 0; j < nb; ++j) {
        const int c = k0 + j;
        const int r = c + 1;
        const int par = c & 1;
        const unsigned stamp = (unsigned)(c + 1);

        // 1. h[a] = sum_b T[a][b] L[c][b] over the panel columns a, b in 0..j,
        //    T tridiagonal with T[a+1][a] = t_a, T[a][a+1] = -t_a, L[c][j] = 1.
        //    Entries of h beyond j stay zero.  With several groups h is
        //    formed at the end of the previous step (no barrier here).
        if (!multi) {
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
        }

        // 2. x_i = Y[i, c] - sum_a L[i][a] h[a] over the filled columns:
        //    flushed ring groups from Lreg, the current group from the ring.
        const int gr = (j / TPR) / kRing; // ring group of column j (uniform)
        const bool cand = exists && (pos >= r);
        // h is read from LDS once per lane and block of 16 slots (lane i of
        //   a 16-lane row reads slot i of the block for the row's column
        //   class) and each slot's value is broadcast inside the row by DPP;
        //   all reads are issued before the products.  Slots of the
        //   unflushed group in Lreg are 0.
        const int hl = lane & 15;
        double hb[kNSB / 16];
#pragma unroll
        for (int k = 0; k < kNSB / 16; ++k)
            hb[k] = (16 * k < gr * kRing) ? hv[sub + TPR * (16 * k + hl)] : 0.0; // uniform
        const double hr = hv[sub + TPR * (gr * kRing + (lane & 7))];
        double sacc[4] = {0.0, 0.0, 0.0, 0.0};
        if (0 < gr * kRing)
            bcast_fma<0, 16, 0, kNS>(sacc, Lreg, hb[0]);
        if constexpr (kNSB > 16)
            if (16 < gr * kRing)
                bcast_fma<0, 16, 16, kNS>(sacc, Lreg, hb[1 % (kNSB / 16)]);
        if constexpr (kNSB > 32)
            if (32 < gr * kRing)
                bcast_fma<0, 16, 32, kNS>(sacc, Lreg, hb[2 % (kNSB / 16)]);
        if constexpr (kNSB > 48)
            if (48 < gr * kRing)
                bcast_fma<0, 16, 48, kNS>(sacc, Lreg, hb[3 % (kNSB / 16)]);
        if constexpr (kNSB > 64)
            if (64 < gr * kRing)
                bcast_fma<0, 16, 64, kNS>(sacc, Lreg, hb[4 % (kNSB / 16)]);
        static_assert(kNSB <= 80, "h blocks");
        bcast_fma<0, kRing, 0, kRing>(sacc, Lnew, hr);
        double s = (sacc[0] + sacc[1]) + (sacc[2] + sacc[3]);
        // the TPR partial sums of a row (lanes RL apart)
        if constexpr (RL <= 32)
            s = xor_add<32>(s);
        if constexpr (RL <= 16)
            s = xor_add<16>(s);
        const double xv = (yneg ? -ycol : ycol) - s;

        // 3-4. group argmax, then (several groups) the exchange of the
        //      groups' candidates: every group arrives at the same pivot.
        {
            double cv = 0.0;
            int ci = INT_MAX, cph = 0;
            if (cand && sub == 0) {
                cv = xv;
                ci = pos;
                cph = phys;
            }
            find_pivot<NT, RL>(pv, sio, multi, G, w, par, stamp, r, n, R, cv, ci, cph);
        }
        const int p = pv.bc_p;
        const double tau = pv.bc_fail ? __longlong_as_double(0x7ff8000000000000ll) : pv.bc_tau;
        const int physp = pv.bc_physp;

        // 5a. loads that depend on the pivot, all issued before any of them
        //     is used (a use in between makes each wait for the one before):
        //     - with several groups, entries a-1 and a+1 of the pivot row of
        //       L (row p before the exchange, the previous row for the next
        //       step's h) from the mirror, for thread a's h[a];
        //     - the next column: entry (label i, label r) of the exchanged
        //       matrix is Y0[orig(i), orig(r)], and orig(r) is the original
        //       row of the register row that held p; Y0 is kept as its lower
        //       triangle, so rows above orig(r) read the mirrored entry and
        //       negate it where it is used.  Every thread of a row loads it
        //       (one address); rows that are final or absent load a valid
        //       entry they do not use.  W is not written during the panel.
        //     Unused lanes read clamped addresses inside the same rows.
        const bool hthr = multi && tid <= j + 1 && j + 1 < nb;
        double mup = 0.0, mdn = 0.0;
        if (multi) {
            const double *mrow = mirror + (size_t)physp * ldm;
            mup = ld_dev(&mrow[hthr ? min(tid + 1, j + 1) : 0]);
            mdn = ld_dev(&mrow[(hthr && tid >= 1) ? tid - 1 : 0]);
        }
        bool yneg_next;
        const double ynext = W[skew_at(exists ? orow : base, base + physp, ldw, yneg_next)];

        // 5b. with one group the pivot row copies its L row to LDS (row p
        //     before the exchange); h is formed from it at the next step.
        if (!multi && exists && pos == p) {
#pragma unroll
            for (int q = 0; q < kNS; ++q)
                hrow[sub + TPR * q] = Lreg[q];
#pragma unroll
            for (int i = 0; i < kRing; ++i)
                hrow[sub + TPR * (gr * kRing + i)] = Lnew[i];
        }

        // 5c. relabel: the register row of r now holds p, the one of p holds r.
        if (exists) {
            if (pos == r)
                pos = p;
            else if (pos == p)
                pos = r;
        }

        // 5d. new column of L: l_i = x_i / tau for rows i > r (each register
        //     row keeps its own x); row r gets its unit diagonal.
        //     Column j+1 sits in ring group (j+1)/TPR/kRing; when that is a
        //     new group, the finished one is flushed first (every thread).
        //     Its mirror store is issued while the loads above are in
        //     flight, so it has completed sooner when the next step's
        //     publication waits for it; every thread issues it (see
        //     MirrorIO), so the next column's load stays in flight past the
        //     waits for the mirror loads and the barrier ending the step,
        //     until the next step's products are formed.
        const int a1 = j + 1;
        if (((a1 / TPR) / kRing) != gr)
            flush_ring(gr);
        const bool lrow_on = exists && pos >= r && sub == a1 % TPR;
        const double l = (pos == r) ? 1.0 : ((tau != 0.0) ? xv / tau : 0.0);
        if (lrow_on) {
            // select into the ring (keeps it in registers: an indexed
            // store would move the array to scratch memory)
            const int slot = (a1 / TPR) % kRing;
#pragma unroll
            for (int i = 0; i < kRing; ++i)
                Lnew[i] = (i == slot) ? l : Lnew[i];
        }
        mio.store(multi && lrow_on && pos > r, phys, ldm, a1, l);

        // 5e. with several groups, thread a forms h[a] of the next step from
        //     the mirror entries and t.
        double hn = 0.0;
        if (hthr) {
            const int a = tid;
            if (a + 1 <= j + 1) {
                const double up = (a + 1 < j + 1) ? mup : 1.0;
                hn -= ((a == j) ? tau : tl[a]) * up;
            }
            if (a >= 1)
                hn += ((a - 1 == j) ? tau : tl[a - 1]) * mdn;
        }
        ycol = ynext;
        yneg = yneg_next;
        if (multi && tid <= j + 1 && j + 1 < nb)
            hv[tid] = hn;
        if (tid == 0) {
            tl[j] = tau;
            pl[j] = p;
        }
        __syncthreads();
    }
    flush_ring((nb / TPR) / kRing); // the group of the last column

    // ---- panel end: pivots and t, L into A (shifted one column left), t on
    //      the subdiagonal, the carried column, and the skr2k operands.
    if (w == 0) {
        for (int a = tid; a < nb; a += NT) {
            t[k0 + a] = tl[a];
            ipiv[k0 + a + 1] = pl[a];
            A[(size_t)(k0 + a) * lda + (k0 + a + 1)] = tl[a];
        }
    }
    const int cp = k0 + nb;
    if (exists) {
#pragma unroll
        for (int q = 0; q < kNS; ++q) {
            const int a = sub + TPR * q;
            const int col = k0 + a;
            if (a <= nb && col >= 1 && pos >= col + 1)
                A[(size_t)(col - 1) * lda + pos] = Lreg[q];
            if (a == nb && pos >= cp + 1)
                lcar[pos] = Lreg[q];
        }
    }
    if (sub == 0) {
        posl[lr] = exists ? pos : -1;
        if (exists)
            perm[pos] = orow;
    }
    if (cp < n - 1) {
        // U_q = -t_2q L[:,2q] + t_2q+1 L[:,2q+2], V_q = L[:,2q+1] for the rows
        // >= cp, staged in LDS 32 columns at a time
        const int nq = (nb + 1) / 2;
        for (int c0 = 0; c0 < 2 * nq; c0 += 32) {
            if (exists) {
#pragma unroll
                for (int q = 0; q < kNS; ++q) {
                    const int a = sub + TPR * q;
                    if (a >= c0 && a <= c0 + 32)
                        stage[(size_t)lr * 34 + (a - c0)] = (a <= nb) ? Lreg[q] : 0.0;
                }
            }
            __syncthreads();
            const int qlo = c0 / 2, qhi = min(nq, qlo + 16);
            for (int e = tid; e < R * (qhi - qlo); e += NT) {
                const int rr = e % R;
                const int qq = qlo + e / R;
                const int row = posl[rr];
                if (row >= cp && row < n) {
                    const double *srow = stage + (size_t)rr * 34;
                    const double vq = srow[2 * qq + 1 - c0];
                    double uq = -tl[2 * qq] * srow[2 * qq - c0];
                    if (2 * qq + 2 <= nb)
                        uq += tl[2 * qq + 1] * srow[2 * qq + 2 - c0];
                    uv[(size_t)qq * n + row] = uq;
                    uv[(size_t)(nq + qq) * n + row] = vq;
                    uv[(size_t)(2 * nq + qq) * n + row] = -vq;
                    uv[(size_t)(3 * nq + qq) * n + row] = uq;
                    if (want32) {
                        uv32[(size_t)qq * n + row] = (float)uq;
                        uv32[(size_t)(nq + qq) * n + row] = (float)vq;
                        uv32[(size_t)(2 * nq + qq) * n + row] = -(float)vq;
                        uv32[(size_t)(3 * nq + qq) * n + row] = (float)uq;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Pfaffian-only panel (Wimmer's reduction: Sec. 3.5.2, Notes, and the
// accumulated rank-2k form of Sec. 3.6.5, Note).  Columns come in pairs
// (c, c+1), c even; only c is pivoted.  With M the panel's accumulated
// columns, M[:, 2i] = l_i (the pair's Gauss vector) and M[:, 2i+1] = c_i
// (its second column), the trailing matrix as of column step c is
// Y + sum_i (l_i c_i^T - c_i l_i^T) = Y - M h-products, so a column is
// x = Y[:, label] - M h with h[2i] = -c_i[label], h[2i+1] = l_i[label].
// Per pair:
//   1. x_c = Y[:, c] - M h_c over the earlier pairs; argmax over rows > c
//      and the slot exchange (as in the full panel) give the pivot p;
//   2. relabel r = c+1 <-> p; load the pivot row's M entries, the row that
//      now holds label c+2 (its M entries and two W entries), and the W
//      columns of labels r and c+2 (one round trip for all of them);
//   3. l_i = x_c / tau for rows > r; the pair's second column
//      x_r = Y[:, r] - M h_r over the earlier pairs only (the pair's own
//      update leaves it unchanged), c_i = x_r for rows > r;
//   4. h for column c+2 is formed by every group from the fetched row: its
//      l_i and c_i entries are recomputed there with the same formulas
//      (two dot products over the group), so no third exchange is needed.
// Two device round trips per pair instead of four for the two columns of
// the full panel.  Nothing is written to A; t and ipiv receive the pairs'
// tau and pivots (0 and no exchange at the odd positions); the skr2k
// operands are U = [c_i], V = [l_i].
template <int NT, int TPR, int kNS>
__global__ __launch_bounds__(NT) void panel_pair_kernel(
    const double *__restrict__ W, int ldw, int n, int k0, int nb, double *__restrict__ t,
    int *__restrict__ ipiv, int *__restrict__ perm, double *__restrict__ mirror, int ldm,
    double *__restrict__ uv, float *__restrict__ uv32, int want32, Slot *__restrict__ slots,
    int G, int one_xcd)
{
    constexpr int R = NT / TPR;
    constexpr int NW = NT / 64;
    constexpr int kRing = 4; // (8 spills registers here)
    constexpr int kNSR = ((kNS + kRing - 1) / kRing) * kRing;
    constexpr int NA = kNSR * TPR; // columns addressable through the ring
    static_assert(NA <= NT, "one thread per h entry");
    static_assert(kNS % 16 == 0 && NA >= kNS * TPR, "h is read in blocks of 16 slots");
    static_assert(TPR == 1 || TPR == 2 || TPR == 4, "a 16-lane row must hold one column class");
    extern __shared__ double stage[]; // R x 34, epilogue only

    __shared__ double hv[NA]; // h of the pair's first column
    __shared__ double ho[NA]; // h of its second column
    __shared__ double tl[kMaxBlock / 2];
    __shared__ int pl[kMaxBlock / 2];
    __shared__ int wphys[kMaxBlock]; // register row of each label base .. base+nb-1
    __shared__ int posl[R];
    __shared__ double dred[2][NW];
    __shared__ PivotLds<NW> pv;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int w = blockIdx.x; // one_xcd: as in panel_kernel
    if (one_xcd) {
        if ((w & 7) != one_xcd - 1)
            return;
        w >>= 3;
    }
    const int base = k0 + 1;
    // the TPR threads of a row are RL = 64 / TPR lanes apart, so each 16-lane
    // row of a wave holds one column class and h is broadcast inside it
    constexpr int RL = 64 / TPR;
    const int lr = wave * RL + lane % RL;
    const int sub = lane / RL;
    const int phys = w * R + lr;
    const int orow = base + phys;
    const bool multi = (G > 1);
    int pos = orow;
    const bool exists = (orow < n);

    double Lreg[kNS];
    double Lnew[kRing];
#pragma unroll
    for (int q = 0; q < kNS; ++q)
        Lreg[q] = 0.0;
#pragma unroll
    for (int i = 0; i < kRing; ++i)
        Lnew[i] = 0.0;
    auto flush_ring = [&](int g) {
#pragma unroll
        for (int q = 0; q < kNS; ++q)
            Lreg[q] = (q / kRing == g) ? Lnew[q % kRing] : Lreg[q];
#pragma unroll
        for (int i = 0; i < kRing; ++i)
            Lnew[i] = 0.0;
    };
    int grc = 0; // ring group held in Lnew (uniform)
    // column a of M for this row (thread a % TPR keeps it)
    auto insert = [&](int a, double v, bool mine) {
        const int g = (a / TPR) / kRing;
        if (g != grc) {
            flush_ring(grc);
            grc = g;
        }
        if (mine && sub == a % TPR) {
            const int slot = (a / TPR) % kRing;
#pragma unroll
            for (int i = 0; i < kRing; ++i)
                Lnew[i] = (i == slot) ? v : Lnew[i];
        }
    };
    // x = y - sum_a M[row][a] h[a] over the filled columns: one LDS read of h
    // per lane and block of 16 slots, each slot's value broadcast inside the
    // 16-lane row as the FMA's DPP operand (slots of the unflushed group in
    // Lreg are 0)
    // (y is the loaded entry, ny whether it stands for its negation: the
    // sign is applied here, where y is first used)
    auto gemv = [&](const double *h, double y, bool ny) {
        const int hl = lane & 15;
        double hb[kNS / 16];
#pragma unroll
        for (int k = 0; k < kNS / 16; ++k)
            hb[k] = (16 * k < grc * kRing) ? h[sub + TPR * (16 * k + hl)] : 0.0; // uniform
        const double hr = h[sub + TPR * (grc * kRing + (lane & (kRing - 1)))];
        double sacc[4] = {0.0, 0.0, 0.0, 0.0};
        if (0 < grc * kRing)
            bcast_fma<0, 16, 0, kNS>(sacc, Lreg, hb[0]);
        if constexpr (kNS > 16)
            if (16 < grc * kRing)
                bcast_fma<0, 16, 16, kNS>(sacc, Lreg, hb[1 % (kNS / 16)]);
        if constexpr (kNS > 32)
            if (32 < grc * kRing)
                bcast_fma<0, 16, 32, kNS>(sacc, Lreg, hb[2 % (kNS / 16)]);
        if constexpr (kNS > 48)
            if (48 < grc * kRing)
                bcast_fma<0, 16, 48, kNS>(sacc, Lreg, hb[3 % (kNS / 16)]);
        static_assert(kNS <= 64, "h blocks");
        bcast_fma<0, kRing, 0, kRing>(sacc, Lnew, hr);
        double sm = (sacc[0] + sacc[1]) + (sacc[2] + sacc[3]);
        // the TPR partial sums of a row (lanes RL apart)
        if constexpr (RL <= 32)
            sm = xor_add<32>(sm);
        if constexpr (RL <= 16)
            sm = xor_add<16>(sm);
        return (ny ? -y : y) - sm;
    };

    double ycol = 0.0;
    bool yneg = false; // ycol holds the negation of the entry (an upper one)
    for (int a = tid; a < NA; a += NT) {
        hv[a] = 0.0;
        ho[a] = 0.0;
    }
    for (int q = tid; q < nb; q += NT)
        wphys[q] = q;
    if (exists) // every thread of the row (one address)
        ycol = W[(size_t)k0 * ldw + orow];
    if (tid == 0) {
        pv.bc_fail = 0;
    }
    __syncthreads();
    // with one_xcd, whether the working groups did land on one XCD (then the
    // exchange uses plain stores)
    bool local = false;
    if (one_xcd) {
        int fl = 0;
        local = groups_share_xcd(slots, G, w, k0, fl);
        if (fl && tid == 0)
            pv.bc_fail = 1;
    }
    const SlotIO sio(slots, base, local);
    const MirrorIO mio(mirror, (int)sizeof(double) * G * R * ldm, local);
    const double qnan = __longlong_as_double(0x7ff8000000000000ll);
    // nothing in flight when the pairs begin
    wait_vm();

    const int npair = nb / 2;
    for (int i = 0; i < npair; ++i) {
        const int c = k0 + 2 * i; // the pair's pivoted column
        const int r = c + 1;
        const int pr = (c >> 1) & 1;
        const unsigned stamp = (unsigned)((c >> 1) + 1);
        // window labels: r = base + 2i, c+2 = base + 2i + 1, c = base + 2i - 1
        const int physR0 = wphys[2 * i];
        // label c+2 is n (no row) at the last pair of a panel that ends the
        // matrix: its loads then read an existing row and are discarded
        const int physE0 = (2 * i + 1 < nb && base + 2 * i + 1 < n) ? wphys[2 * i + 1] : 0;
        const int origC = (i == 0) ? k0 : base + wphys[2 * i - 1];

        // 1. x_c and the pivot
        const double xv = gemv(hv, ycol, yneg);
        // one group: its own mirror stores must be complete before the
        // barrier in the pivot search (several groups wait there anyway)
        if (!multi)
            wait_vm();
        {
            double cv = 0.0;
            int ci = INT_MAX, cph = 0;
            if (exists && pos >= r && sub == 0) {
                cv = xv;
                ci = pos;
                cph = phys;
            }
            find_pivot<NT, RL>(pv, sio, multi, G, w, pr, stamp, r, n, R, cv, ci, cph);
        }
        const int p = pv.bc_p;
        const double tau = pv.bc_fail ? qnan : pv.bc_tau;
        const int physp = pv.bc_physp;

        // 2. relabel, then one round of loads
        if (exists) {
            if (pos == r)
                pos = p;
            else if (pos == p)
                pos = r;
        }
        const bool nxt = (i + 1 < npair); // column c+2 belongs to this panel
        const int physE = (p == c + 2) ? physR0 : physE0; // row holding label c+2
        const int a = tid;
        const bool ha = (a < 2 * i);
        // Every thread issues every load of the pair, in the order of their
        // use, at addresses kept in range (rows and columns named by the
        // window exist, label n excepted: see physE0); what a thread does
        // not need is discarded where the value is used.  A load issued on
        // some paths only makes the compiler's waits for the earlier ones
        // also cover the later ones: the next column's HBM load then sat
        // before the pair's barriers.  Order: the pivot row's and the label-(c+2) row's mirror
        // entries (for h of the second column and the dot products), the
        // second column (every thread of a row loads, one address), entries
        // (label c+2, label r) or (label c+2, label c) of Y, and last the
        // next pair's first column.
        const int ac = ha ? a : 0;
        const double mp1 = ld_dev(&mirror[(size_t)physp * ldm + (ac ^ 1)]);
        const double me0 = ld_dev(&mirror[(size_t)physE * ldm + ac]);
        const double me1 = ld_dev(&mirror[(size_t)physE * ldm + (ac ^ 1)]);
        const int yrow = exists ? orow : base;
        // (Y0 is kept as its lower triangle: an upper entry is read at its
        // mirror and negated where it is used)
        bool yo_neg, wsc_neg, ye_neg;
        const double yo = W[skew_at(yrow, base + physp, ldw, yo_neg)];
        const double wsc =
            W[skew_at(base + physE, (a == 2 * i + 1) ? origC : base + physp, ldw, wsc_neg)];
        const double ye = W[skew_at(yrow, base + physE, ldw, ye_neg)];

        // 3a. l_i for the rows below r
        const bool below = exists && pos > r;
        const double lval = below ? ((tau != 0.0) ? xv / tau : 0.0) : 0.0;
        insert(2 * i, lval, below);
        mio.store(below && sub == (2 * i) % TPR, phys, ldm, 2 * i, lval);
        // h of the second column (pivot row entries) and the two dot
        // products of the label-(c+2) row with h_c and h_r
        const double hoa = ha ? ((a & 1) ? mp1 : -mp1) : 0.0;
        const double hea = (ha && nxt) ? ((a & 1) ? me1 : -me1) : 0.0;
        double dk = 0.0, dob = 0.0;
        if (a < NA) {
            ho[a] = hoa;
            if (ha && nxt) {
                dk = me0 * hv[a];
                dob = me0 * hoa;
            }
        }
        dk = wave_sum_f64(dk);
        dob = wave_sum_f64(dob);
        if (lane == 0) {
            dred[0][wave] = dk;
            dred[1][wave] = dob;
        }
        __syncthreads();

        // 3b. the pair's second column and c_i
        // (rows that are not below r load a value they do not use: their xo
        // is discarded)
        const double xo = gemv(ho, yo, yo_neg);
        insert(2 * i + 1, below ? xo : 0.0, below);
        mio.store(below && sub == (2 * i + 1) % TPR, phys, ldm, 2 * i + 1, xo);

        // 4. h of column c+2: earlier pairs from the fetched row; this
        //    pair's c_i and l_i at label c+2 recomputed from the same data
        if (nxt && a <= 2 * i + 1) {
            double hn = hea;
            if (a >= 2 * i) {
                double sk = 0.0, so = 0.0;
#pragma unroll
                for (int q = 0; q < NW; ++q) {
                    sk += dred[0][q];
                    so += dred[1][q];
                }
                if (a == 2 * i) // -c_i[c+2]
                    hn = -((wsc_neg ? -wsc : wsc) - so);
                else { // l_i[c+2]
                    const double xk = (wsc_neg ? -wsc : wsc) - sk;
                    hn = (tau != 0.0) ? xk / tau : 0.0;
                }
            }
            hv[a] = hn;
        }
        // the next pair's candidates all have labels above c+2, for which
        // ye is their entry; the other rows' x is never used
        ycol = ye;
        yneg = ye_neg;
        if (tid == 0) {
            tl[i] = tau;
            pl[i] = p;
            wphys[2 * i] = physp;
            if (p - base < nb && p != r)
                wphys[p - base] = physR0;
        }
        __syncthreads();
    }
    flush_ring(grc);

    // ---- panel end: tau and pivots of the pairs, the permutation, and the
    //      skr2k operands U_q = c_q, V_q = l_q for the rows >= cp
    if (w == 0) {
        for (int q = tid; q < npair; q += NT) {
            const int c = k0 + 2 * q;
            t[c] = tl[q];
            ipiv[c + 1] = pl[q];
            if (c + 1 < n - 1)
                t[c + 1] = 0.0;
            if (c + 2 < n)
                ipiv[c + 2] = c + 2;
        }
    }
    const int cp = k0 + nb;
    if (sub == 0) {
        posl[lr] = exists ? pos : -1;
        if (exists)
            perm[pos] = orow;
    }
    if (cp < n - 1) {
        const int nq = npair;
        for (int c0 = 0; c0 < nb; c0 += 32) {
            if (exists) {
#pragma unroll
                for (int q = 0; q < kNS; ++q) {
                    const int aa = sub + TPR * q;
                    if (aa >= c0 && aa < c0 + 32)
                        stage[(size_t)lr * 34 + (aa - c0)] = (aa < nb) ? Lreg[q] : 0.0;
                }
            }
            __syncthreads();
            const int qlo = c0 / 2, qhi = min(nq, qlo + 16);
            for (int e = tid; e < R * (qhi - qlo); e += NT) {
                const int rr = e % R;
                const int qq = qlo + e / R;
                const int row = posl[rr];
                if (row >= cp && row < n) {
                    const double *srow = stage + (size_t)rr * 34;
                    const double uq = srow[2 * qq + 1 - c0]; // c_q
                    const double vq = srow[2 * qq - c0];     // l_q
                    uv[(size_t)qq * n + row] = uq;
                    uv[(size_t)(nq + qq) * n + row] = vq;
                    uv[(size_t)(2 * nq + qq) * n + row] = -vq;
                    uv[(size_t)(3 * nq + qq) * n + row] = uq;
                    if (want32) {
                        uv32[(size_t)qq * n + row] = (float)uq;
                        uv32[(size_t)(nq + qq) * n + row] = (float)vq;
                        uv32[(size_t)(2 * nq + qq) * n + row] = -(float)vq;
                        uv32[(size_t)(3 * nq + qq) * n + row] = (float)uq;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Panel shapes: 512 threads per group, TPR threads per row, kNS register
// slots per thread holding b + 1 columns; R = 512 / TPR rows per group.
//   b <= 64:  TPR 1, 65 slots, 512 rows (n = 16384 needs 32 groups: one XCD)
//   b <= 128: TPR 2, 65 slots, 256 rows
//   b <= 256: TPR 4, 65 slots, 128 rows
constexpr int kNT = 512;
constexpr int kXcdCUs = 32; // CUs per XCD on MI355X

// XCD that runs the ordinary one-XCD panel grids launched on stream s: the
// first seven distinct streams seen get distinct XCDs among 1 .. 7 (later
// ones the table's order modulo 7); XCD 0 is left to the cooperative one-XCD
// grids.  Only a placement choice: the kernels check where their groups
// landed.
static int xcd_of_stream(hipStream_t s)
{
    constexpr int kTable = 64;
    static std::mutex mu;
    static hipStream_t seen[kTable];
    static int nseen = 0;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < nseen; ++i)
        if (seen[i] == s)
            return 1 + i % 7;
    if (nseen < kTable) {
        seen[nseen] = s;
        return 1 + (nseen++) % 7;
    }
    return 1 + (int)(((uintptr_t)s >> 8) % 7);
}

// Launch of a panel grid of G working groups.  The working groups wait for
// one another, so all of them must be resident together.
// * G <= kOrdinaryGroups: an ordinary launch, its groups on the stream's XCD.
//   The runtime serializes cooperative launches from all streams on one
//   queue, so factorizations on several streams would otherwise run their
//   panels one after another (measured on the serving mix: its n > 256
//   requests on four streams 3.95 s with cooperative launches, 1.23 s with
//   ordinary ones).  Residency holds by construction for up to seven
//   streams: a stream's panels run one at a time on its own XCD (1 .. 7), at
//   most 16 of its 32 CUs (one group per CU); a cooperative grid of up to 32
//   groups runs on XCD 0, and one of 33 .. 128 groups needs at most 16 CUs
//   of each XCD.  Beyond that (more streams, cooperative grids of more than
//   128 groups at the same time) a group may have to wait for CUs held by
//   waiting groups; the bounded waits then end the panel with a poisoned
//   result (NaN t) instead of a hang.
// * Larger grids: a cooperative launch (the runtime guarantees residency),
//   placed on XCD 0 up to kXcdCUs groups.
constexpr int kOrdinaryGroups = 16;
static hipError_t launch_grid(const void *fn, int G, void **args, int *one_xcd, size_t lds,
                              hipStream_t s)
{
    if (G == 1) { // no cross-group exchange
        *one_xcd = 0;
        return hipLaunchKernel(fn, dim3(1), dim3(kNT), args, (unsigned)lds, s);
    }
    if (G <= kOrdinaryGroups) {
        *one_xcd = 1 + xcd_of_stream(s);
        return hipLaunchKernel(fn, dim3(8 * G), dim3(kNT), args, (unsigned)lds, s);
    }
    *one_xcd = (G <= kXcdCUs) ? 1 : 0;
    const int grid = *one_xcd ? 8 * G : G;
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kNT), args, (unsigned)lds, s);
}

static int shape_id(int b)
{
    if (b + 1 <= 65)
        return 0;
    if (b + 1 <= 130)
        return 1;
    return 2;
}
static int rows_per_group(int b)
{
    const int id = shape_id(b);
    return id == 0 ? 512 : (id == 1 ? 256 : 128);
}

PanelShape panel_shape(int n, int k0, int b, int max_groups)
{
    PanelShape sh;
    const int m = n - k0 - 1;
    sh.R = rows_per_group(b);
    sh.G = (m + sh.R - 1) / sh.R;
    if (sh.G < 1)
        sh.G = 1;
    (void)max_groups;
    sh.lds = sizeof(double) * (size_t)sh.R * 34;
    return sh;
}

template <int TPR, int NS>
static hipError_t launch_t(double *A, int lda, const double *W, int n, int k0, int nb, int b,
                           double *t, int *ipiv, const FactorWs &ws, int want32,
                           const PanelShape &sh, hipStream_t s)
{
    int ldw = ws.ldw;
    int *perm = ws.perm;
    double *mirror = ws.mirror;
    int ldm = ws.ldm;
    double *lcar = ws.lcar;
    double *uv = ws.uv;
    float *uv32 = ws.uv32;
    Slot *slots = ws.slots;
    int G = sh.G;
    int one_xcd = 0; // set by launch_grid before the launch reads args
    void *args[] = {&A, &lda, &W, &ldw, &n, &k0, &nb, &b, &t, &ipiv, &perm, &mirror, &ldm,
                    &lcar, &uv, &uv32, &want32, &slots, &G, &one_xcd};
    return launch_grid((const void *)panel_kernel<kNT, TPR, NS>, G, args, &one_xcd, sh.lds, s);
}

hipError_t launch_panel(double *A, int lda, const double *W, int n, int k0, int nb, int b,
                        double *t, int *ipiv, const FactorWs &ws, int want32,
                        const PanelShape &sh, hipStream_t s)
{
    switch (shape_id(b)) {
    case 0: return launch_t<1, 65>(A, lda, W, n, k0, nb, b, t, ipiv, ws, want32, sh, s);
    case 1: return launch_t<2, 65>(A, lda, W, n, k0, nb, b, t, ipiv, ws, want32, sh, s);
    default: return launch_t<4, 65>(A, lda, W, n, k0, nb, b, t, ipiv, ws, want32, sh, s);
    }
}

template <int TPR, int NS>
static hipError_t launch_pair_t(const double *W, int n, int k0, int nb, double *t, int *ipiv,
                                const FactorWs &ws, int want32, const PanelShape &sh,
                                hipStream_t s)
{
    int ldw = ws.ldw;
    int *perm = ws.perm;
    double *mirror = ws.mirror;
    int ldm = ws.ldm;
    double *uv = ws.uv;
    float *uv32 = ws.uv32;
    Slot *slots = ws.slots;
    int G = sh.G;
    int one_xcd = 0; // set by launch_grid before the launch reads args
    void *args[] = {&W, &ldw, &n, &k0, &nb, &t, &ipiv, &perm, &mirror, &ldm,
                    &uv, &uv32, &want32, &slots, &G, &one_xcd};
    return launch_grid((const void *)panel_pair_kernel<kNT, TPR, NS>, G, args, &one_xcd, sh.lds,
                       s);
}

hipError_t launch_panel_pair(const double *W, int n, int k0, int nb, int b, double *t, int *ipiv,
                             const FactorWs &ws, int want32, const PanelShape &sh, hipStream_t s)
{
    switch (shape_id(b)) {
    case 0: return launch_pair_t<1, 64>(W, n, k0, nb, t, ipiv, ws, want32, sh, s);
    case 1: return launch_pair_t<2, 64>(W, n, k0, nb, t, ipiv, ws, want32, sh, s);
    default: return launch_pair_t<4, 64>(W, n, k0, nb, t, ipiv, ws, want32, sh, s);
    }
}

void panel_init_attrs()
{
    (void)hipFuncSetAttribute((const void *)panel_pair_kernel<kNT, 1, 64>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)panel_pair_kernel<kNT, 2, 64>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)panel_pair_kernel<kNT, 4, 64>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)panel_kernel<kNT, 1, 65>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)panel_kernel<kNT, 2, 65>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)panel_kernel<kNT, 4, 65>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

int panel_max_groups(size_t lds_bytes, bool pair)
{
    static int cached_cus = 0;
    if (!cached_cus)
        cached_cus = device_cu_count();
    int per_cu = 0, per_cu4 = 0;
    const void *f2 = pair ? (const void *)panel_pair_kernel<kNT, 2, 64>
                          : (const void *)panel_kernel<kNT, 2, 65>;
    const void *f4 = pair ? (const void *)panel_pair_kernel<kNT, 4, 64>
                          : (const void *)panel_kernel<kNT, 4, 65>;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f2, kNT, lds_bytes) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu4, f4, kNT, lds_bytes) != hipSuccess)
        return 0;
    per_cu = per_cu < per_cu4 ? per_cu : per_cu4;
    if (per_cu < 1)
        per_cu = 1;
    long g = (long)per_cu * cached_cus;
    if (g > kMaxPanelGroups)
        g = kMaxPanelGroups;
    return (int)g;
}

}  // namespace skl
