// Coarse-tail cycle: the complete gamma-cycle (Sec. 2, "Cycle and acceleration";
// eq. (2.4)) of every level from a threshold level down to the directly solved one, run
// by ONE workgroup of 1024 threads per right-hand-side column in ONE launch per visit to
// the threshold level. The columns are independent (each has its own energy correction
// and recombination coefficients), so workgroup w takes column w on its own, with
// descriptors of its own: with several columns the tail levels' vectors hold them column
// by column (column w from element w n), and the top level's iterate and right-hand side
// are copied into that layout around the launch; with one column it is the ordinary one.
//
// Coarse levels are small but are visited many times per cycle (the cycle index grows
// towards 2 where coarsening is aggressive), and every visit is a chain of dependent
// steps: Gauss-Seidel colour passes, residual, restriction, coarse recombination,
// energy correction, prolongation. As separate kernels each step costs a dispatch of a
// few microseconds; here each step is a loop over the level's rows followed by one
// workgroup barrier, so the cost of a step is the latency of its few dependent memory
// accesses. Everything is arranged to keep that latency short:
//  - the smallest levels (operators and vectors) are copied into LDS at the start of a
//    launch and addressed through LDS pointers (ds_* instructions), the others stay in
//    global memory (L2-resident);
//  - level descriptors are read with scalar loads, all control flow is wave-uniform, and
//    the recursion over levels is a state machine whose per-level state (phase, visit
//    index, visit count, Beatty counter) lives in one VGPR lane per level of every wave,
//    so no LDS traffic or barrier is spent on bookkeeping;
//  - on levels whose (row, column) pairs fit one per thread and whose rows are short, a
//    thread holds its row (column offsets, values, diagonal, right-hand side) in
//    registers for a whole smoothing call, so a colour pass is one gather, one store and
//    one barrier, and the residual after pre-smoothing reuses the same registers;
//  - a workgroup reduction is one barrier: waves write partial sums, and after the
//    barrier every thread forms its column's totals itself (in wave order, so all
//    threads agree bit for bit), so the dependent update needs no second pass;
//  - 32-bit indexing throughout (a tail level has at most a few thousand rows).
//
// The arithmetic per step is that of the multi-kernel path (cycle_kernels.hip).
#include <algorithm>
#include <type_traits>

#include "lamg_internal.h"

namespace lamg {

namespace {

constexpr int TB = 1024;  // threads of the tail workgroup
constexpr int TW = TB / 64;
constexpr int kFast = 16;  // longest row held in registers
template <class T>
constexpr int kGather = sizeof(T) == 4 ? 8 : 4;  // gathers in flight per group
constexpr int kRedQ = 2;   // quantities per tail reduction
constexpr int kSplitRow = 256;  // levels with longer rows share a long row between waves
constexpr int kMediumRow = 64;  // long rows up to this length are relaxed with the short ones

// Level descriptor. Array fields hold device pointers for levels in global memory and
// byte offsets into the launch's dynamic LDS for LDS-resident levels (Z always global).
template <class T>
struct TailLvl {
    int32_t n, ncolors, coarsest, nc;  // nc: rows of the next level
    int32_t n_rlong, maxlen, maxcol, ew;  // maxcol: rows of the largest colour; ew: ELL width
    int32_t maxrow;                       // longest off-diagonal row (long ones included)
    int32_t elim;                         // 1: elimination level (colour 0 = eliminated rows)
    double gamma;
    const int64_t *blk;  // 2*ncolors + 1 offsets (class 0 colours, class 1 colours)
    const int32_t *rp, *ci;
    const T *v, *d, *dinv;
    const int32_t *p0, *p1;  // P to the next level
    const T *w0, *w1;
    const int32_t *rrp, *rci, *rlong;  // P^T
    const T *rw;
    const double *Z;  // coarsest: pseudo-inverse
    T *x, *f, *r, *rho, *x1, *rho1;
    const int32_t *eci;  // ELL copy of the off-diagonals (0 if absent; always global)
    const T *ev;
};

// Global -> LDS copy performed at the start of every tail launch. Jobs that bring the top
// level's iterate (`top` 1) or right-hand side (`top` 2) copy the workgroup's column:
// `colb` bytes.
struct CopyJob {
    const void *src;
    uint32_t dst;    // byte offset in the dynamic LDS buffer (multiple of 16)
    uint32_t bytes;  // multiple of 4
    uint32_t top;    // 0: an operator array; 1: the top level's x; 2: its f
    uint32_t colb;   // top jobs: bytes per column (the level's rows x element size)
};

// One workgroup of a grouped launch (several requests' cycles in one launch): where its
// descriptors and copy jobs start in the launch's combined arrays, its visit counters and
// its plan (one column of one request).
struct TailWG {
    int64_t *visits;       // nlev visit counters of this workgroup
    int32_t desc_off;      // first of its nlev descriptors in the launch's descriptor array
    int32_t jobs_off;      // first of its njobs copy jobs in the launch's job array
    int32_t njobs, l0, nlev, l_lds, l_x, pad;
};

struct TailArgs {
    const CopyJob *jobs;  // njobs per workgroup, workgroup after workgroup
    int64_t *visits;      // per workgroup and level, persistent within a solve
    int32_t njobs, l0, nlev, l_lds, k, lkp;  // k, lkp: the columns of one workgroup (1, 0)
    uint32_t red_off;    // byte offset of the two reduction buffers in the dynamic LDS
    int32_t l_x;         // levels [l_x, l_lds) have their iterate alone in LDS (-1: none)
    uint32_t cpart_off;  // byte offset of the coarsest solve's part sums (TB doubles)
    uint32_t pad;
};

__device__ inline void bar() { __syncthreads(); }
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// a pointer read from memory by every lane, made wave-uniform (scalar registers)
template <class P>
__device__ inline P *uni_ptr(P *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return reinterpret_cast<P *>(((uint64_t)hi << 32) | lo);
}

template <bool LDS, class P>
__device__ inline P *at(char *smem, P *p) {
    if constexpr (LDS)
        return reinterpret_cast<P *>(smem + static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p)));
    else
        return p;
}

// Residency of a level's arrays: everything in global memory; only the iterate x in LDS
// (the level right above the LDS-resident ones, whose operator does not fit but whose
// randomly gathered iterate does); everything in LDS.
constexpr int kGlobal = 0, kXLds = 1, kAllLds = 2;

// The arrays of one level, rebased into LDS where they live there.
template <class T, int M>
struct Lv {
    static constexpr bool OL = M == kAllLds;  // operator, transfer and other vectors
    static constexpr bool XL = M != kGlobal;  // iterate
    int n, nc, ncol, nrl, maxlen, maxcol, ew, maxrow;
    bool split;  // long rows long enough to share them between waves
    bool elim;   // elimination level
    const int32_t *eci;
    const T *ev;
    const int64_t *blk;
    const int32_t *rp, *ci;
    const T *v, *d, *dinv;
    const int32_t *p0, *p1;
    const T *w0, *w1;
    const int32_t *rrp, *rci, *rlong;
    const T *rw;
    T *x, *f, *r, *rho, *x1, *rho1;
    __device__ Lv(const TailLvl<T> &D, char *s)
        : n(D.n), nc(D.nc), ncol(D.ncolors), nrl(D.n_rlong), maxlen(D.maxlen), maxcol(D.maxcol),
          ew(D.ew), maxrow(D.maxrow), split(D.maxrow > kSplitRow), elim(D.elim != 0), eci(D.eci), ev(D.ev),
          blk(at<OL>(s, D.blk)), rp(at<OL>(s, D.rp)), ci(at<OL>(s, D.ci)), v(at<OL>(s, D.v)),
          d(at<OL>(s, D.d)), dinv(at<OL>(s, D.dinv)), p0(at<OL>(s, D.p0)), p1(at<OL>(s, D.p1)),
          w0(at<OL>(s, D.w0)), w1(at<OL>(s, D.w1)), rrp(at<OL>(s, D.rrp)), rci(at<OL>(s, D.rci)),
          rlong(at<OL>(s, D.rlong)), rw(at<OL>(s, D.rw)), x(at<XL>(s, D.x)), f(at<OL>(s, D.f)),
          r(at<OL>(s, D.r)), rho(at<OL>(s, D.rho)), x1(at<OL>(s, D.x1)),
          rho1(at<OL>(s, D.rho1)) {}
};

// sum over [j0, e) step `stride` of v[j] * x[ci[j] * k + col], U entries in flight.
template <class T, int U>
__device__ inline T row_sum(const int32_t *ci, const T *v, const T *x, int j0, int e, int stride,
                            int k, int col) {
    T acc = T(0);
    for (int j = j0; j < e; j += U * stride) {
        int cc[U];
        T vv[U], xx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int jj = j + u * stride;
            const bool ok = jj < e;
            cc[u] = ok ? ci[jj] : -1;
            vv[u] = ok ? v[jj] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xx[u] = cc[u] >= 0 ? x[cc[u] * k + col] : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u) acc += vv[u] * xx[u];
    }
    return acc;
}

// Short rows [a, b) by groups of kp x lpr lanes: lpr (up to 2^max_llpr, as long as every
// row keeps at least two groups' worth of threads) lanes split a row's entries, and the
// partial sums are combined by shuffles inside the group. Used for the few short rows of a
// colour pass on the denser levels, whose rows run up to kLongRow entries.
template <class T, int OP>
__device__ __forceinline__ void csr_short_split(int a, int b, int skip_long,
                                                           const int32_t *rp, const int32_t *ci,
                                                           const T *v, const T *dd, const T *f,
                                                           const T *xin, T *out, int k, int lkp,
                                                           int max_llpr) {
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int nrow = b - a;
    int llpr = 0;
    while (llpr < max_llpr && lkp + llpr < 6 && (nrow << (lkp + llpr + 1)) <= TB) ++llpr;
    const int lg = lkp + llpr, G = 1 << lg, lpr = 1 << llpr;
    const int g = tid & (G - 1);
    const int c = g & (kp - 1), sub = g >> lkp;
    for (int row = a + (tid >> lg); row < b; row += (TB >> lg)) {
        const int e0 = rp[row], e1 = rp[row + 1];
        if (skip_long > 0 && e1 - e0 > skip_long) continue;
        T acc = T(0);
        if (c < k) acc = row_sum<T, 4>(ci, v, xin, e0 + sub, e1, lpr, k, c);
        for (int o = kp; o < G; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (sub == 0 && c < k) {
            const int o = row * k + c;
            if (OP == 0)
                out[o] = (f[o] - acc) * dd[row];
            else if (OP == 1)
                out[o] = f[o] - dd[row] * xin[o] - acc;
            else
                out[o] = acc;
        }
    }
}

// Rows [a, b) and [la, lb) of one pass as a single set, by groups of kp x lpr lanes (lpr up
// to 8, as long as the set still gives every lane a row): used when the level's long rows
// have at most kMediumRow entries, so that they need no second, wave-per-row phase after
// the short ones.
template <class T, int OP>
__device__ __forceinline__ void csr_medium_split(int a, int b, int la, int lb, const int32_t *rp,
                                                 const int32_t *ci, const T *v, const T *dd,
                                                 const T *f, const T *xin, T *out, int k, int lkp) {
    constexpr int U = 4;
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int ns = b - a, nrow = ns + (lb - la);
    int llpr = 0;
    while (llpr < 3 && lkp + llpr < 6 && (nrow << (lkp + llpr + 1)) <= TB) ++llpr;
    const int lg = lkp + llpr, G = 1 << lg, lpr = 1 << llpr;
    const int g = tid & (G - 1);
    const int c = g & (kp - 1), sub = g >> lkp;
    for (int t = tid >> lg; t < nrow; t += (TB >> lg)) {
        const int row = t < ns ? a + t : la + (t - ns);
        const int e0 = rp[row], e1 = rp[row + 1];
        T acc = T(0);
        if (c < k) acc = row_sum<T, U>(ci, v, xin, e0 + sub, e1, lpr, k, c);
        for (int o = kp; o < G; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (sub == 0 && c < k) {
            const int o = row * k + c;
            if (OP == 0)
                out[o] = (f[o] - acc) * dd[row];
            else
                out[o] = f[o] - dd[row] * xin[o] - acc;
        }
    }
}

// CSR pass over rows [a, b) (short rows) and [la, lb) (long rows, through `rows` if given):
//   OP 0: x[r] = (f[r] - sum_off) * dd[r]      (Gauss-Seidel colour pass, in place)
//   OP 1: out[r] = f[r] - dd[r] x[r] - sum_off  (residual)
//   OP 2: out[r] = sum_off                      (P^T r)
// Short rows: one thread per (row, column); rows longer than skip_long (> 0) are left to
// the long list. Long rows: one wave per row, the 64 lanes split as kp columns x (64/kp).
template <class T, int OP, bool SPLIT = false>
__device__ __forceinline__ void csr_rows(int a, int b, int la, int lb, const int32_t *rows, int skip_long,
                         const int32_t *rp, const int32_t *ci, const T *v, const T *dd, const T *f,
                         const T *xin, T *out, int k, int lkp, T *lpart, bool split,
                         int max_llpr, int maxrow = 0) {
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    // SPLIT levels whose long rows are medium (Gauss-Seidel and residual passes): one phase
    if (SPLIT && OP != 2 && !rows && maxrow <= kMediumRow) {
        csr_medium_split<T, OP>(a, b, la, lb, rp, ci, v, dd, f, xin, out, k, lkp);
        return;
    }
    // SPLIT (the denser levels) and few short rows: several lanes split each row; a separate
    // instantiation, so the other levels run the plain loop
    if (SPLIT && ((b - a) << (lkp + 2)) <= TB && lkp < 6) {
        csr_short_split<T, OP>(a, b, skip_long, rp, ci, v, dd, f, xin, out, k, lkp, max_llpr);
    } else {
        const int c = tid & (kp - 1);
        if (c < k) {
            for (int row = a + (tid >> lkp); row < b; row += (TB >> lkp)) {
                const int e0 = rp[row], e1 = rp[row + 1];
                if (skip_long > 0 && e1 - e0 > skip_long) continue;
                const T acc = row_sum<T, 8>(ci, v, xin, e0, e1, 1, k, c);
                const int o = row * k + c;
                if (OP == 0)
                    out[o] = (f[o] - acc) * dd[row];
                else if (OP == 1)
                    out[o] = f[o] - dd[row] * xin[o] - acc;
                else
                    out[o] = acc;
            }
        }
    }
    const int nl = lb - la;
    if (nl <= 0) return;
    // long rows: gw waves per row, as many as keep every wave busy when they are few (the
    // hubs of power-law graphs stay long on every coarse level); the waves' partial sums
    // are added in wave order after a barrier, through lpart (TW x kp values in LDS)
    int gw = 1;
    while (split && gw < TW && gw * 2 * nl <= TW) gw *= 2;
    const int wave = tid >> 6, lane = tid & 63;
    const int sub = lane >> lkp, col = lane & (kp - 1), nsub = 64 >> lkp;
    const int wr = wave / gw, wp = wave - wr * gw, slots = TW / gw;
    for (int i0 = la; i0 < lb; i0 += slots) {
        const int i = i0 + wr;
        int row = 0;
        T acc = T(0);
        if (i < lb) {
            row = rows ? rows[i] : i;
            const int e0 = rp[row], e1 = rp[row + 1];
            if (col < k) acc = row_sum<T, 4>(ci, v, xin, e0 + wp * nsub + sub, e1, nsub * gw, k, col);
        }
        for (int o = kp; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (gw > 1) {
            if (lane < kp) lpart[wave * kp + lane] = acc;
            bar();
            if (wp == 0) {
                acc = T(0);
                for (int q = 0; q < gw; ++q) acc += lpart[(wr * gw + q) * kp + col];
            }
        }
        if (i < lb && wp == 0 && sub == 0 && col < k) {
            const int o = row * k + col;
            if (OP == 0)
                out[o] = (f[o] - acc) * dd[row];
            else if (OP == 1)
                out[o] = f[o] - dd[row] * xin[o] - acc;
            else
                out[o] = acc;
        }
        if (gw > 1) bar();
    }
}

// out = f - L x over all rows of level L (the caller's barrier follows). Levels in global
// memory with an ELL copy read it coalesced: one thread per (row, column), entry u of all
// rows at consecutive addresses; the sum runs in entry order as in the CSR pass.
template <class T, int M>
__device__ __forceinline__ void residual(const Lv<T, M> &L, T *out, int k, int lkp, T *lp) {
    if (M != kAllLds && L.ew > 0 && L.maxlen > 0) {  // no long rows
        const int tid = threadIdx.x;
        const int kp = 1 << lkp;
        const int c = tid & (kp - 1);
        const int n = L.n, ew = L.ew;
        constexpr int G = kGather<T>;
        if (c < k)
            for (int row = tid >> lkp; row < n; row += TB >> lkp) {
                T acc = T(0);
                for (int u0 = 0; u0 < ew; u0 += G) {
                    int jj[G];
                    T vv[G], xx[G];
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const bool ok = u0 + u < ew;
                        jj[u] = ok ? L.eci[(u0 + u) * n + row] : row;
                        vv[u] = ok ? L.ev[(u0 + u) * n + row] : T(0);
                    }
#pragma unroll
                    for (int u = 0; u < G; ++u) xx[u] = L.x[jj[u] * k + c];
#pragma unroll
                    for (int u = 0; u < G; ++u) acc += vv[u] * xx[u];
                }
                const int o = row * k + c;
                out[o] = L.f[o] - L.d[row] * L.x[o] - acc;
            }
        return;
    }
    const int nc = L.ncol;
    if (L.maxrow > kLongRow)
        csr_rows<T, 1, true>(0, (int)L.blk[nc], (int)L.blk[nc], L.n, nullptr, 0, L.rp, L.ci, L.v,
                             L.d, L.f, L.x, out, k, lkp, lp, L.split, 3, L.maxrow);
    else
        csr_rows<T, 1>(0, (int)L.blk[nc], (int)L.blk[nc], L.n, nullptr, 0, L.rp, L.ci, L.v, L.d,
                       L.f, L.x, out, k, lkp, lp, L.split, 0);
}

// One Gauss-Seidel colour pass over rows [a, b) from the ELL copy (coalesced loads, entry
// order as in the CSR pass); for levels in global memory whose rows are too long for the
// pipelined register rows.
template <class T, int M>
__device__ __forceinline__ void ell_gs_pass(const Lv<T, M> &L, int a, int b, int k, int lkp) {
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int c = tid & (kp - 1);
    const int n = L.n, ew = L.ew;
    constexpr int G = kGather<T>;
    if (c >= k) return;
    for (int row = a + (tid >> lkp); row < b; row += TB >> lkp) {
        T acc = T(0);
        for (int u0 = 0; u0 < ew; u0 += G) {
            int jj[G];
            T vv[G], xx[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const bool ok = u0 + u < ew;
                jj[u] = ok ? L.eci[(u0 + u) * n + row] : row;
                vv[u] = ok ? L.ev[(u0 + u) * n + row] : T(0);
            }
#pragma unroll
            for (int u = 0; u < G; ++u) xx[u] = L.x[jj[u] * k + c];
#pragma unroll
            for (int u = 0; u < G; ++u) acc += vv[u] * xx[u];
        }
        const int o = row * k + c;
        L.x[o] = (L.f[o] - acc) * L.dinv[row];
    }
}

template <class T>
constexpr int kPipe = sizeof(T) == 4 ? 16 : 10;  // longest row of the pipelined path

// The colour block offsets of a level (2 ncolors + 1 values, each below 65536), the first
// 192 held in the lanes of three registers for a whole smoothing call and read with
// readlane, so that finding a pass's rows needs no memory access (the pipelined passes
// would otherwise wait for these loads before issuing the row loads of the pass ahead).
struct BlkRegs {
    int b0, b1, b2;
    const int64_t *blk;
    template <class T, int M>
    __device__ __forceinline__ void load(const Lv<T, M> &L) {
        const int lane = threadIdx.x & 63, nb = 2 * L.ncol + 1;
        blk = L.blk;
        b0 = lane < nb ? (int)L.blk[lane] : 0;
        b1 = lane + 64 < nb ? (int)L.blk[lane + 64] : 0;
        b2 = lane + 128 < nb ? (int)L.blk[lane + 128] : 0;
    }
    __device__ __forceinline__ int operator()(int i) const {  // i: wave-uniform
        if (i < 64) return __builtin_amdgcn_readlane(b0, i);
        if (i < 128) return __builtin_amdgcn_readlane(b1, i - 64);
        if (i < 192) return __builtin_amdgcn_readlane(b2, i - 128);
        return (int)blk[i];
    }
};

// One thread's row of one colour pass, loaded ahead of its update (stage 1: inverse
// diagonal and right-hand side; stage 2: column indices and values from the level's ELL
// copy). Padding entries point at the row itself with weight 0. The loaded values go into
// registers as they arrive and are first used by the pass that relaxes the row, so the
// loads stay in flight across the current pass and its barrier (packing two indices into
// one register as they were loaded made every stage wait for its loads: 1.5 us per pass).
template <class T, int W>
struct PipeRow {
    int32_t ci[W];
    T vv[W];
    T dinv, fv;
    int row;
    bool live;
    template <int M>
    __device__ __forceinline__ void stage1(const Lv<T, M> &L, const BlkRegs &bk, int cl, int k,
                                           int lkp) {
        const int tid = threadIdx.x;
        const int c = tid & ((1 << lkp) - 1);
        row = bk(cl) + (tid >> lkp);
        live = row < bk(cl + 1) && c < k;
        if (live) {
            dinv = L.dinv[row];
            fv = L.f[row * k + c];
        }
    }
    // the row's entries from the ELL copy: lane-consecutive rows are address-consecutive
    template <int M>
    __device__ __forceinline__ void stage2(const Lv<T, M> &L) {
        if (!live) return;
        const int n = L.n, ew = L.ew;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const int uu = u < ew ? u : 0;  // slots past the width re-read entry 0, weight 0
            ci[u] = L.eci[uu * n + row];
            vv[u] = L.ev[uu * n + row];
        }
    }
    __device__ __forceinline__ void relax(T *x, int k, int c, int ew) const {
        if (!live) return;
        constexpr int G = kGather<T>;
        T acc = T(0);
#pragma unroll
        for (int u0 = 0; u0 < W; u0 += G) {
            T xx[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (u0 + u < W) xx[u] = x[ci[u0 + u] * k + c];
            }
#pragma unroll
            for (int u = 0; u < G; ++u)
                if (u0 + u < W) acc = (u0 + u < ew) ? acc + vv[u0 + u] * xx[u] : acc;
        }
        x[row * k + c] = (fv - acc) * dinv;
    }
};

template <class T>
constexpr int kPipeSplit = sizeof(T) == 4 ? 10 : 8;  // entries per lane of a split row

// One row of one colour pass split over lpr = 2^llpr adjacent lane groups (rows of both
// classes of the colour: the short ones, then the long ones), loaded ahead of its update
// like PipeRow: lane s of the row holds entries s, s + lpr, ... (at most W) of the level's
// full-width ELL copy, and the lanes' partial sums are added by xor shuffles (every lane
// takes part in them, live or not).
template <class T, int W>
struct PipeRowS {
    int32_t ci[W];
    T vv[W];
    T dinv, fv;
    int row, sub;
    bool live;
    template <int M>
    __device__ __forceinline__ void stage1(const Lv<T, M> &L, const BlkRegs &bk, int cl, int k,
                                           int lkp, int llpr) {
        const int tid = threadIdx.x;
        const int c = tid & ((1 << lkp) - 1);
        sub = (tid >> lkp) & ((1 << llpr) - 1);
        const int t = tid >> (lkp + llpr);
        const int a = bk(cl), ns = bk(cl + 1) - a;
        const int la = bk(L.ncol + cl), nl = bk(L.ncol + cl + 1) - la;
        row = t < ns ? a + t : la + (t - ns);
        live = t < ns + nl && c < k;
        if (live) {
            dinv = L.dinv[row];
            fv = L.f[row * k + c];
        }
    }
    template <int M>
    __device__ __forceinline__ void stage2(const Lv<T, M> &L, int llpr) {
        if (!live) return;
        const int n = L.n, ew = L.ew;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const int e = (u << llpr) + sub;
            const int ee = e < ew ? e : sub;  // slots past the width re-read entry sub, dropped
            ci[u] = L.eci[ee * n + row];
            vv[u] = L.ev[ee * n + row];
        }
    }
    __device__ __forceinline__ void relax(T *x, int k, int c, int lkp, int llpr, int ew) const {
        constexpr int G = kGather<T>;
        T acc = T(0);
        if (live) {
#pragma unroll
            for (int u0 = 0; u0 < W; u0 += G) {
                T xx[G];
#pragma unroll
                for (int u = 0; u < G; ++u)
                    if (u0 + u < W) xx[u] = x[ci[u0 + u] * k + c];
#pragma unroll
                for (int u = 0; u < G; ++u)
                    if (u0 + u < W)
                        acc = (((u0 + u) << llpr) + sub < ew) ? acc + vv[u0 + u] * xx[u] : acc;
            }
        }
        for (int o = 1 << lkp; o < (1 << (lkp + llpr)); o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (live && sub == 0) x[row * k + c] = (fv - acc) * dinv;
    }
};

// Lanes per row (log2) of the split pipelined pass: the fewest that leave at most
// kPipeSplit entries per lane, if every colour then gives each lane group one row at most;
// 0 if none does.
template <class T, int M>
__device__ __forceinline__ int split_llpr(const Lv<T, M> &L, int lkp) {
    int llpr = 1;
    while ((kPipeSplit<T> << llpr) < L.ew) ++llpr;
    return (lkp + llpr <= 6 && (L.maxcol << (lkp + llpr)) <= TB) ? llpr : 0;
}

// `sweeps` Gauss-Seidel sweeps over the colours of level L, then (if `resid`) the residual
// r = f - L x. On a level whose (row, column) pairs fit one per thread and whose rows have
// at most kFast off-diagonals, each thread loads its row into registers once (column
// offsets, values, inverse diagonal, diagonal, right-hand side; padding entries point at
// the row's own value with weight 0, so every gather is unconditional), and every colour
// pass is one gather, one store and one barrier.
template <class T, int M>
__device__ __forceinline__ void smooth(const Lv<T, M> &L, int k, int lkp, int sweeps, bool resid,
                                       T *lp) {
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int nc = L.ncol;
    if (L.elim) {
        // elimination level: its eliminated rows (colour 0, independent, all short) are set
        // exactly from the kept ones, once, whatever the sweep count
        csr_rows<T, 0>((int)L.blk[0], (int)L.blk[1], (int)L.blk[nc], (int)L.blk[nc + 1], nullptr,
                       0, L.rp, L.ci, L.v, L.dinv, L.f, L.x, L.x, k, lkp, lp, L.split, 0);
        bar();
        if (resid) {
            residual<T, M>(L, L.r, k, lkp, lp);
            bar();
        }
        return;
    }
    const bool fast = L.maxlen > 0 && L.maxlen <= kFast && (L.n << lkp) <= TB;
    constexpr int kGroup = kGather<T>;
    if (fast) {
        const int row = tid >> lkp;
        const int c = tid & (kp - 1);
        const bool live = row < L.n && c < k;
        const int o = row * k + c;
        int cc[kFast];
        T vv[kFast];
        T dinv = T(0), dg = T(0), fv = T(0);
        int mycol = -1;
        if (live) {
            const int e0 = L.rp[row], len = L.rp[row + 1] - e0;
#pragma unroll
            for (int u = 0; u < kFast; ++u) {
                const bool ok = u < len;
                cc[u] = ok ? L.ci[e0 + u] * k + c : o;
                vv[u] = ok ? L.v[e0 + u] : T(0);
            }
            dinv = L.dinv[row];
            dg = L.d[row];
            fv = L.f[o];
            int lo = 0, hi = nc;  // colour: blk[lo] <= row < blk[lo + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if ((int)L.blk[mid] <= row)
                    lo = mid;
                else
                    hi = mid;
            }
            mycol = lo;
        }
        T *x = L.x;
        // loads in groups of kGroup, summed in entry order; groups past the level's longest
        // row (a uniform bound) hold only padding and are skipped
        const int mlen = L.maxlen;
        auto gather = [&]() {
            T acc = T(0);
#pragma unroll
            for (int u0 = 0; u0 < kFast; u0 += kGroup) {
                if (u0 >= mlen) break;
                T xx[kGroup];
#pragma unroll
                for (int u = 0; u < kGroup; ++u) xx[u] = x[cc[u0 + u]];
#pragma unroll
                for (int u = 0; u < kGroup; ++u) acc += vv[u0 + u] * xx[u];
            }
            return acc;
        };
        for (int sw = 0; sw < sweeps; ++sw)
            for (int cl = 0; cl < nc; ++cl) {
                if (live && mycol == cl) x[o] = (fv - gather()) * dinv;
                bar();
            }
        if (resid) {
            if (live) L.r[o] = fv - dg * x[o] - gather();
            bar();
        }
        return;
    }
    constexpr int W = kPipe<T>;
    if (L.ew > 0 && L.ew <= W && (L.maxcol << lkp) <= TB && L.n < 65536) {
        // every colour has at most one (row, column) pair per thread: the row of the next
        // colour pass (column offsets, values, inverse diagonal, right-hand side) is loaded
        // while the current pass computes and waits at its barrier, so a pass costs one
        // gather, one store and one barrier
        // pass q relaxes with the row data of stage 2 issued during pass q-1, whose
        // bounds came from stage 1 issued during pass q-2 (right after that pass's update)
        PipeRow<T, W> A, Bn;
        BlkRegs bk;
        bk.load(L);
        const int q_end = sweeps * nc;
        const int c = tid & (kp - 1);
        A.stage1(L, bk, 0, k, lkp);
        if (1 < q_end) Bn.stage1(L, bk, 1 % nc, k, lkp);
        A.stage2(L);
        for (int q = 0; q < q_end; q += 2) {
            A.relax(L.x, k, c, L.ew);
            if (q + 2 < q_end) A.stage1(L, bk, (q + 2) % nc, k, lkp);
            if (q + 1 < q_end) Bn.stage2(L);
            bar();
            if (q + 1 >= q_end) break;
            Bn.relax(L.x, k, c, L.ew);
            if (q + 3 < q_end) Bn.stage1(L, bk, (q + 3) % nc, k, lkp);
            if (q + 2 < q_end) A.stage2(L);
            bar();
        }
    } else if (M != kAllLds && L.ew > W && L.n < 65536 && split_llpr(L, lkp) > 0) {
        // rows longer than the pipelined registers hold: each split over lpr lanes (at most
        // kPipeSplit entries per lane), the next colour's rows loaded during the current pass
        // as above; the long rows of a colour are relaxed with its short ones
        constexpr int W2 = kPipeSplit<T>;
        const int llpr = split_llpr(L, lkp);
        PipeRowS<T, W2> A, Bn;
        BlkRegs bk;
        bk.load(L);
        const int q_end = sweeps * nc;
        const int c = tid & (kp - 1);
        A.stage1(L, bk, 0, k, lkp, llpr);
        if (1 < q_end) Bn.stage1(L, bk, 1 % nc, k, lkp, llpr);
        A.stage2(L, llpr);
        for (int q = 0; q < q_end; q += 2) {
            A.relax(L.x, k, c, lkp, llpr, L.ew);
            if (q + 2 < q_end) A.stage1(L, bk, (q + 2) % nc, k, lkp, llpr);
            if (q + 1 < q_end) Bn.stage2(L, llpr);
            bar();
            if (q + 1 >= q_end) break;
            Bn.relax(L.x, k, c, lkp, llpr, L.ew);
            if (q + 3 < q_end) Bn.stage1(L, bk, (q + 3) % nc, k, lkp, llpr);
            if (q + 2 < q_end) A.stage2(L, llpr);
            bar();
        }
    } else if (M != kAllLds && L.ew > 0 && L.maxlen > 0) {  // no long rows
        for (int sw = 0; sw < sweeps; ++sw)
            for (int cl = 0; cl < nc; ++cl) {
                ell_gs_pass<T, M>(L, (int)L.blk[cl], (int)L.blk[cl + 1], k, lkp);
                bar();
            }
    } else {
        for (int sw = 0; sw < sweeps; ++sw)
            for (int cl = 0; cl < nc; ++cl) {
                if (L.maxrow > kLongRow)
                    csr_rows<T, 0, true>((int)L.blk[cl], (int)L.blk[cl + 1], (int)L.blk[nc + cl],
                                         (int)L.blk[nc + cl + 1], nullptr, 0, L.rp, L.ci, L.v,
                                         L.dinv, L.f, L.x, L.x, k, lkp, lp, L.split, 3, L.maxrow);
                else
                    csr_rows<T, 0>((int)L.blk[cl], (int)L.blk[cl + 1], (int)L.blk[nc + cl],
                                   (int)L.blk[nc + cl + 1], nullptr, 0, L.rp, L.ci, L.v, L.dinv,
                                   L.f, L.x, L.x, k, lkp, lp, L.split, 0);
                bar();
            }
    }
    if (resid) {
        residual<T, M>(L, L.r, k, lkp, lp);
        bar();
    }
}

// Partial sums of Q quantities per column: xor-shuffle inside each wave over the lanes of
// one column, then one write per (wave, column). The caller's barrier follows.
template <int Q>
__device__ inline void wave_partials(double (&q)[Q], double *red, int kp) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        for (int o = kp; o < 64; o <<= 1) q[i] += __shfl_xor(q[i], o, 64);
    if (lane < kp)
#pragma unroll
        for (int i = 0; i < Q; ++i) red[(i * TW + wave) * kp + lane] = q[i];
}

// Column totals from the wave partials, added in wave order (same bits in every thread).
template <int Q>
__device__ inline void column_totals(const double *red, int kp, int c, double (&t)[Q]) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        double a = 0.0;
        for (int w = 0; w < TW; ++w) a += red[(i * TW + w) * kp + c];
        t[i] = a;
    }
}

// y = Z f on the directly solved level (FP64 pseudo-inverse in global memory, exactly
// symmetric). Column-oriented so that a wave's loads are contiguous: thread (i, c) adds
// Z[j][i] f[j][c] (= Z[i][j] f[j][c]) over its part of the j range, 16 loads in flight, with
// f[j][c] broadcast to the wave. The threads are split into P parts of the j range (P as
// large as the (row, column) units allow, at most 4); the parts' sums are added in part
// order through LDS (the reduction area, TB doubles), so the result is deterministic.
template <class T, int M>
__device__ __forceinline__ void coarsest(const double *Z, const Lv<T, M> &L, int k, int lkp,
                                         double *cpart) {
    constexpr int kZ = 16;
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int n = L.n;
    if (k == 1 && (n & 1) == 0 && (reinterpret_cast<uintptr_t>(Z) & 15) == 0) {
        // one column and an even order: a thread takes two adjacent rows (i, i + 1), whose
        // entries Z[j][i], Z[j][i + 1] are one 16-byte load, and the j range is split into
        // up to 8 parts; twice the bytes per load and twice the parts of the form below, so
        // about a third as many rounds of loads. The parts' sums are added in part order through
        // LDS, first for the rows i, then for the rows i + 1.
        constexpr int kZ2 = 12;  // 16-byte loads in flight per thread
        const int np = n >> 1;
        int P = 1;
        while (P < 8 && np * P * 2 <= TB) P *= 2;
        const int chunk = TB / P;
        const int part = tid / chunk, uidx = tid - part * chunk;
        const int jlen = (n + P - 1) / P;
        const int j0 = part * jlen, j1 = min(n, j0 + jlen);
        const T *f = L.f;
        T *y = L.x;
        for (int u0 = 0; u0 < np; u0 += chunk) {
            const int unit = u0 + uidx;
            const bool live = unit < np;
            const int i = 2 * unit;
            double a0 = 0.0, a1 = 0.0;
            if (live) {
                for (int j = j0; j < j1; j += kZ2) {
                    double2 zz[kZ2];
#pragma unroll
                    for (int w = 0; w < kZ2; ++w)
                        zz[w] = (j + w < j1)
                                    ? *reinterpret_cast<const double2 *>(Z + (int64_t)(j + w) * n + i)
                                    : make_double2(0.0, 0.0);
#pragma unroll
                    for (int w = 0; w < kZ2; ++w)
                        if (j + w < j1) {
                            const double fj = (double)f[j + w];
                            a0 += zz[w].x * fj;
                            a1 += zz[w].y * fj;
                        }
                }
            }
            cpart[tid] = a0;
            bar();
            if (part == 0 && live) {
                double sm = 0.0;
                for (int q = 0; q < P; ++q) sm += cpart[q * chunk + uidx];
                y[i] = (T)sm;
            }
            bar();
            cpart[tid] = a1;
            bar();
            if (part == 0 && live) {
                double sm = 0.0;
                for (int q = 0; q < P; ++q) sm += cpart[q * chunk + uidx];
                y[i + 1] = (T)sm;
            }
            bar();
        }
        return;
    }
    const int units = n << lkp;
    int P = 1;
    while (P < 4 && units * P * 2 <= TB) P *= 2;
    const int chunk = TB / P;
    const int part = tid / chunk, uidx = tid - part * chunk;
    const int jlen = (n + P - 1) / P;
    const int j0 = part * jlen, j1 = min(n, j0 + jlen);
    const T *f = L.f;
    T *y = L.x;
    for (int u0 = 0; u0 < units; u0 += chunk) {
        const int unit = u0 + uidx;
        const int i = unit >> lkp;
        const int c = unit & (kp - 1);
        const bool live = unit < units && c < k;
        double acc = 0.0;
        if (live) {
            for (int j = j0; j < j1; j += kZ) {
                double zz[kZ];
#pragma unroll
                for (int w = 0; w < kZ; ++w) zz[w] = (j + w < j1) ? Z[(int64_t)(j + w) * n + i] : 0.0;
#pragma unroll
                for (int w = 0; w < kZ; ++w)
                    if (j + w < j1) acc += zz[w] * (double)f[(j + w) * k + c];
            }
        }
        if (P > 1) {
            cpart[tid] = acc;
            bar();
            if (part == 0 && live) {
                double s = 0.0;
                for (int q = 0; q < P; ++q) s += cpart[q * chunk + uidx];
                y[i * k + c] = (T)s;
            }
            bar();
        } else if (live) {
            y[i * k + c] = (T)acc;
        }
    }
    bar();
}

// Per-wave level state, one level per lane (the same values in every wave).
struct WaveState {
    int st;   // phase | j << 1 | nvis << 9
    int cnt;  // Beatty visit counter
    __device__ int get_st(int l) const { return __builtin_amdgcn_readlane(st, l); }
    __device__ int get_cnt(int l) const { return __builtin_amdgcn_readlane(cnt, l); }
    __device__ void set_st(int l, int val) { st = ((int)(threadIdx.x & 63) == l) ? val : st; }
    __device__ void set_cnt(int l, int val) { cnt = ((int)(threadIdx.x & 63) == l) ? val : cnt; }
};

// One phase of level l (not the coarsest) with child level l+1; returns the next level.
//  phase 0: pre-smoothing, residual, restriction, zero coarse iterate; descend.
//  phase 1: back from visit j of the child: child residual, recombination of the last two
//           child iterates (j >= 2); then descend again, or energy correction,
//           prolongation and post-smoothing, and ascend.
template <class T, int ML, int MC>
__device__ __forceinline__ int visit(const TailArgs &A, const TailLvl<T> &DL, const TailLvl<T> &DC, int l,
                     char *smem, WaveState &ws, int &rbuf) {
    const int tid = threadIdx.x;
    const int k = A.k, lkp = A.lkp, kp = 1 << lkp;
    const Lv<T, ML> L(DL, smem);
    const Lv<T, MC> C(DC, smem);
    T *lp = reinterpret_cast<T *>(smem + A.red_off);  // long-row partials (reduction area)
    const int s = ws.get_st(l);
    if ((s & 1) == 0) {
        smooth<T, ML>(L, k, lkp, 1, true, lp);
        csr_rows<T, 2>(0, L.nc, 0, L.nrl, L.rlong, L.nrl ? kLongRow : 0, L.rrp, L.rci, L.rw,
                       nullptr, nullptr, L.r, C.f, k, lkp, lp, false, 0);
        for (int t = tid; t < C.n * k; t += TB) C.x[t] = T(0);
        bar();
        const int i = ws.get_cnt(l);
        ws.set_cnt(l, i + 1);
        const double g = DL.gamma;
        const int nvis = (int)(floor((double)(i + 1) * g) - floor((double)i * g));
        ws.set_st(l, 1 | (0 << 1) | (nvis << 9));
        ws.set_st(l + 1, 0);
        return l + 1;
    }
    const int j = ((s >> 1) & 255) + 1;
    const int nvis = s >> 9;
    const int c = tid & (kp - 1);
    if (DL.elim) {
        // elimination level (one visit): the kept rows take the coarse values (P has weight
        // 1 there and 0 on the eliminated rows), no recombination or energy correction;
        // the eliminated rows are then set exactly again
        if (c < k)
            for (int i = tid >> lkp; i < L.n; i += TB >> lkp)
                L.x[i * k + c] += L.w0[i] * C.x[L.p0[i] * k + c];
        bar();
        smooth<T, ML>(L, k, lkp, 1, false, lp);
        return l - 1;
    }
    // rho = f_c - L_c x_c
    residual<T, MC>(C, C.rho, k, lkp, lp);
    bar();
    const bool again = j < nvis;
    if (j >= 2) {  // two-iterate recombination across the visits
        double *red = reinterpret_cast<double *>(smem + A.red_off) + rbuf * (kRedQ * TW * kp);
        rbuf ^= 1;
        double q[2] = {0.0, 0.0};
        if (c < k)
            for (int i = tid >> lkp; i < C.n; i += TB >> lkp) {
                const double rv = (double)C.rho[i * k + c];
                const double g = rv - (double)C.rho1[i * k + c];
                q[0] += g * g;
                q[1] += g * rv;
            }
        wave_partials<2>(q, red, kp);
        bar();
        double t[2];
        column_totals<2>(red, kp, c, t);
        const T a = (T)(t[0] > 0.0 ? t[1] / t[0] : 0.0);
        if (c < k)
            for (int i = tid >> lkp; i < C.n; i += TB >> lkp) {
                const int o = i * k + c;
                const T ev = C.x[o], rv = C.rho[o];
                const T xn = ev + a * (C.x1[o] - ev);
                const T rn = rv - a * (rv - C.rho1[o]);
                C.x[o] = xn;
                C.rho[o] = rn;
                if (again) {
                    C.x1[o] = xn;
                    C.rho1[o] = rn;
                }
            }
        bar();
    } else if (again) {
        if (c < k)
            for (int i = tid >> lkp; i < C.n; i += TB >> lkp) {
                const int o = i * k + c;
                C.x1[o] = C.x[o];
                C.rho1[o] = C.rho[o];
            }
        bar();
    }
    if (again) {
        ws.set_st(l, 1 | (j << 1) | (nvis << 9));
        ws.set_st(l + 1, 0);
        return l + 1;
    }
    // energy correction mu = <e, f_c> / <e, f_c - rho>, prolongation, post-smoothing
    {
        double *red = reinterpret_cast<double *>(smem + A.red_off) + rbuf * (kRedQ * TW * kp);
        rbuf ^= 1;
        double q[2] = {0.0, 0.0};
        if (c < k)
            for (int i = tid >> lkp; i < C.n; i += TB >> lkp) {
                const double e = (double)C.x[i * k + c], fc = (double)C.f[i * k + c];
                q[0] += e * fc;
                q[1] += e * (fc - (double)C.rho[i * k + c]);
            }
        wave_partials<2>(q, red, kp);
        bar();
        double t[2];
        column_totals<2>(red, kp, c, t);
        double mu = t[0] / t[1];
        if (!(t[1] > 0.0) || !isfinite(mu)) mu = 1.0;
        if (c < k)
            for (int i = tid >> lkp; i < L.n; i += TB >> lkp) {
                T pe = L.w0[i] * C.x[L.p0[i] * k + c];
                const int q1 = L.p1[i];
                if (q1 >= 0) pe += L.w1[i] * C.x[q1 * k + c];
                L.x[i * k + c] += (T)mu * pe;
            }
        bar();
    }
    smooth<T, ML>(L, k, lkp, 2, false, lp);
    return l - 1;
}

template <class T, bool GROUP>
__global__ void __launch_bounds__(TB) k_tail(TailArgs A, const TailLvl<T> *__restrict__ G0,
                                             const TailWG *__restrict__ wgs) {
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // this workgroup's column: its descriptors, copy jobs and visit counters -- from its
    // record in a grouped launch, else column blockIdx.x of the launch's one request
    const TailLvl<T> *__restrict__ G;
    const CopyJob *jobs;
    int64_t *visits;
    int njobs, l0, nlev, l_lds, l_x;
    if constexpr (GROUP) {
        const TailWG &W = wgs[blockIdx.x];
        G = G0 + uni(W.desc_off);
        jobs = A.jobs + uni(W.jobs_off);
        visits = uni_ptr(W.visits);
        njobs = uni(W.njobs);
        l0 = uni(W.l0);
        nlev = uni(W.nlev);
        l_lds = uni(W.l_lds);
        l_x = uni(W.l_x);
    } else {
        const int col = (int)blockIdx.x;
        visits = A.visits + (int64_t)col * A.nlev;
        G = G0 + (int64_t)col * A.nlev;
        jobs = A.jobs + (int64_t)col * A.njobs;
        njobs = A.njobs;
        l0 = A.l0;
        nlev = A.nlev;
        l_lds = A.l_lds;
        l_x = A.l_x;
    }
    // bring the LDS-resident levels (and the top level's iterate and right-hand side)
    const void *top_x = nullptr;
    for (int jb = 0; jb < njobs; ++jb) {
        const CopyJob J = jobs[jb];
        const uint32_t bytes = J.top ? (uint32_t)A.k * J.colb : J.bytes;
        if (J.top == 1) top_x = J.src;
        const uint32_t n16 = bytes >> 4;
        const uint4 *s16 = static_cast<const uint4 *>(J.src);
        uint4 *d16 = reinterpret_cast<uint4 *>(smem + J.dst);
        for (uint32_t w = tid; w < n16; w += TB) d16[w] = s16[w];
        const uint32_t *s4 = static_cast<const uint32_t *>(J.src);
        uint32_t *d4 = reinterpret_cast<uint32_t *>(smem + J.dst);
        for (uint32_t w = 4 * n16 + tid; w < (bytes >> 2); w += TB) d4[w] = s4[w];
    }
    WaveState ws;
    ws.st = 0;
    ws.cnt = (lane >= l0 && lane < nlev) ? (int)visits[lane] : 0;
    int rbuf = 0;
    bar();
    int l = l0;
    while (l >= l0) {
        l = uni(l);
        const TailLvl<T> &D = G[l];
        if (D.coarsest) {
            double *cpart = reinterpret_cast<double *>(smem + A.cpart_off);
            if (l >= l_lds)
                coarsest<T, kAllLds>(D.Z, Lv<T, kAllLds>(D, smem), A.k, A.lkp, cpart);
            else
                coarsest<T, kGlobal>(D.Z, Lv<T, kGlobal>(D, smem), A.k, A.lkp, cpart);
            --l;
            continue;
        }
        if (l >= l_lds)
            l = visit<T, kAllLds, kAllLds>(A, D, G[l + 1], l, smem, ws, rbuf);
        else if (l_x >= 0 && l >= l_x && l + 1 >= l_lds)
            l = visit<T, kXLds, kAllLds>(A, D, G[l + 1], l, smem, ws, rbuf);
        else if (l_x >= 0 && l >= l_x)
            l = visit<T, kXLds, kXLds>(A, D, G[l + 1], l, smem, ws, rbuf);
        else if (l + 1 == l_x)
            l = visit<T, kGlobal, kXLds>(A, D, G[l + 1], l, smem, ws, rbuf);
        else if (l + 1 >= l_lds)
            l = visit<T, kGlobal, kAllLds>(A, D, G[l + 1], l, smem, ws, rbuf);
        else
            l = visit<T, kGlobal, kGlobal>(A, D, G[l + 1], l, smem, ws, rbuf);
    }
    if (l0 >= l_lds || (l_x >= 0 && l0 >= l_x)) {  // the top level's iterate is in LDS: write it back
        const TailLvl<T> &D = G[l0];
        const T *lx = at<true>(smem, D.x);
        T *gx = static_cast<T *>(const_cast<void *>(top_x));
        for (int t = tid; t < D.n * A.k; t += TB) gx[t] = lx[t];
    }
    if (tid < 64 && lane >= l0 && lane < nlev) visits[lane] = ws.cnt;
}

__global__ void k_fill_i64(int64_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

// Descriptors of every level for precision T, written into a host buffer of
// nlev * tail_desc_bytes<T>() bytes (uploaded by the caller).
template <class T>
size_t tail_desc_bytes() {
    return sizeof(TailLvl<T>);
}

template <class T>
void tail_fill_desc(void *host_buf, int l, const Level &L, const SolveOp &op, const int64_t *d_blk,
                    const T *v, const T *d, const T *dinv, const T *w0, const T *w1, const T *rw,
                    const T *ev, T *x, T *f, T *r, T *rho, T *x1, T *rho1) {
    TailLvl<T> &D = static_cast<TailLvl<T> *>(host_buf)[l];
    std::memset(&D, 0, sizeof(D));
    D.n = (int32_t)L.n;
    D.ncolors = op.ncolors;
    D.coarsest = L.coarsest ? 1 : 0;
    D.nc = (int32_t)op.nc;
    D.n_rlong = (int32_t)op.n_rlong;
    D.maxlen = op.max_short_len;
    D.maxrow = op.max_len;
    D.elim = L.elim ? 1 : 0;
    for (int c = 0; c < op.ncolors; ++c)  // rows of a colour, short and long
        D.maxcol = std::max(D.maxcol, (int32_t)(op.blk[c + 1] - op.blk[c] + op.blk[op.ncolors + c + 1] -
                                                op.blk[op.ncolors + c]));
    D.gamma = L.gamma;
    D.blk = d_blk;
    D.rp = op.rp.p;
    D.ci = op.ci.p;
    D.v = v;
    D.d = d;
    D.dinv = dinv;
    D.p0 = op.p0.p;
    D.p1 = op.p1.p;
    D.w0 = w0;
    D.w1 = w1;
    D.rrp = op.rrp.p;
    D.rci = op.rci.p;
    D.rlong = op.rlong.p;
    D.rw = rw;
    D.Z = L.Z.p;
    D.x = x;
    D.f = f;
    D.r = r;
    D.rho = rho;
    D.x1 = x1;
    D.rho1 = rho1;
    D.ew = ev ? op.ell_w : 0;
    D.eci = ev ? op.ell_ci.p : nullptr;
    D.ev = ev;
}

// Lays out the launch's dynamic LDS: the two reduction buffers, then the coarsest levels
// of the tail starting at l0 whose operators and vectors fit together in what is left,
// then, as far as they fit, the iterates of the levels right above them, from the bottom up
// (levels [l_x, l_lds); l_x = -1: none).
// Writes the launch's descriptor array (arrays in LDS carry offsets) and the copy jobs.
// Returns l_lds (nlev: no level in LDS) and the dynamic LDS bytes.
template <class T>
int tail_lds_plan(const std::vector<Level> &lev, int l0, int k, const void *host_desc,
                  std::vector<char> &lds_desc, std::vector<char> &jobs, size_t &lds_bytes,
                  int &l_x) {
    const int nlev = (int)lev.size();
    l_x = -1;
    const TailLvl<T> *G = static_cast<const TailLvl<T> *>(host_desc);
    lds_desc.assign(sizeof(TailLvl<T>) * nlev, 0);
    std::memcpy(lds_desc.data(), host_desc, sizeof(TailLvl<T>) * nlev);
    jobs.clear();
    lds_bytes = 0;
    if (l0 < 0 || l0 >= nlev) return nlev;
    int kp = 1;
    while (kp < k) kp <<= 1;
    auto al = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
    const int64_t red_bytes = 2 * (int64_t)kRedQ * TW * kp * 8;
    int dev = 0;
    LAMG_HIP(hipGetDevice(&dev));
    int max_lds = 0;
    LAMG_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    hipFuncAttributes fa;
    LAMG_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_tail<T, false>)));
    const int64_t budget = (int64_t)max_lds - (int64_t)fa.sharedSizeBytes - 256;
    auto level_bytes = [&](int l) {
        const Level &L = lev[l];
        const SolveOp &op = L.op;
        const int64_t n = L.n, s = sizeof(T);
        int64_t b = al(8 * (int64_t)op.blk.size()) + al(4 * (n + 1)) + al(4 * op.nnz_off) +
                    al(s * op.nnz_off) + 2 * al(s * n);
        int64_t nv = L.coarsest ? 3 : 5;  // x, f, r(=rho) [, x1, rho1]
        b += nv * al(s * n * k);
        if (!L.coarsest)
            b += 2 * al(4 * n) + 2 * al(s * n) + al(4 * (op.nc + 1)) + al(4 * op.nnz_r) +
                 al(s * op.nnz_r) + al(4 * op.n_rlong);
        return b;
    };
    const int64_t cpart_bytes = (int64_t)TB * 8;
    int l_lds = nlev;
    int64_t total = 16 + al(red_bytes) + cpart_bytes;  // offset 0 means "no array"
    for (int l = nlev - 1; l >= l0; --l) {
        int64_t b = level_bytes(l);
        if (total + b > budget) break;
        total += b;
        l_lds = l;
    }
    int64_t off = 16 + al(red_bytes) + cpart_bytes;
    std::vector<CopyJob> jv;
    TailLvl<T> *D = reinterpret_cast<TailLvl<T> *>(lds_desc.data());
    for (int l = l_lds; l < nlev; ++l) {
        const Level &L = lev[l];
        const SolveOp &op = L.op;
        const int64_t n = L.n, s = sizeof(T);
        TailLvl<T> &E = D[l];
        E = G[l];
        auto place = [&](auto &field, int64_t bytes, bool copy) {
            using P = std::remove_reference_t<decltype(field)>;
            const void *src = (const void *)field;
            if (bytes <= 0) {
                field = P(nullptr);
                return;
            }
            field = reinterpret_cast<P>((uintptr_t)off);
            if (copy && src) jv.push_back(CopyJob{src, (uint32_t)off, (uint32_t)bytes, 0u, 0u});
            off += al(bytes);
        };
        place(E.blk, 8 * (int64_t)op.blk.size(), true);
        place(E.rp, 4 * (n + 1), true);
        place(E.ci, 4 * op.nnz_off, true);
        place(E.v, s * op.nnz_off, true);
        place(E.d, s * n, true);
        place(E.dinv, s * n, true);
        if (!L.coarsest) {
            place(E.p0, 4 * n, true);
            place(E.p1, 4 * n, true);
            place(E.w0, s * n, true);
            place(E.w1, s * n, true);
            place(E.rrp, 4 * (op.nc + 1), true);
            place(E.rci, 4 * op.nnz_r, true);
            place(E.rw, s * op.nnz_r, true);
            place(E.rlong, 4 * op.n_rlong, true);
        } else {
            E.p0 = E.p1 = nullptr;
            E.w0 = E.w1 = nullptr;
            E.rrp = E.rci = E.rlong = nullptr;
            E.rw = nullptr;
        }
        const bool top = (l == l0);  // the top level's iterate and rhs come from global memory
        if (top) {
            jv.push_back(CopyJob{(const void *)E.x, (uint32_t)off, (uint32_t)(s * n * k), 1u,
                                 (uint32_t)(s * n)});
            E.x = reinterpret_cast<T *>((uintptr_t)off);
            off += al(s * n * k);
            jv.push_back(CopyJob{(const void *)E.f, (uint32_t)off, (uint32_t)(s * n * k), 2u,
                                 (uint32_t)(s * n)});
            E.f = reinterpret_cast<T *>((uintptr_t)off);
            off += al(s * n * k);
        } else {
            place(E.x, s * n * k, false);
            place(E.f, s * n * k, false);
        }
        place(E.r, s * n * k, false);
        E.rho = E.r;  // the residual of a level is dead before its coarse residual is formed
        if (!L.coarsest) {
            place(E.x1, s * n * k, false);
            place(E.rho1, s * n * k, false);
        } else {
            E.x1 = E.rho1 = nullptr;
        }
    }
    // the levels right above: their iterates alone (gathered by every colour pass, residual
    // and prolongation of the level), from the bottom up while they fit
    l_x = -1;
    for (int l = l_lds - 1; l >= l0 && l_lds < nlev; --l) {
        const int64_t xb = (int64_t)sizeof(T) * lev[l].n * k;
        if (off + al(xb) > budget) break;
        TailLvl<T> &E = D[l];
        E = G[l];
        const void *src = (const void *)E.x;
        E.x = reinterpret_cast<T *>((uintptr_t)off);
        if (l == l0)
            jv.push_back(CopyJob{src, (uint32_t)off, (uint32_t)xb, 1u,
                                 (uint32_t)(sizeof(T) * lev[l].n)});
        off += al(xb);
        l_x = l;
    }
    lds_bytes = (size_t)off;
    jobs.resize(jv.size() * sizeof(CopyJob));
    if (!jv.empty()) std::memcpy(jobs.data(), jv.data(), jobs.size());
    // the attribute is process-wide while plans of several handles coexist: always the whole
    // budget, so that no plan lowers it below what another handle's launches request
    for (const void *f : {reinterpret_cast<const void *>(&k_tail<T, false>),
                          reinterpret_cast<const void *>(&k_tail<T, true>)})
        LAMG_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)budget));
    return l_lds;
}

template <class T>
void run_tail(const TailPlan &tp, int l0, int nlev, int k, int64_t *d_visits, hipStream_t s) {
    const bool cols = k > 1;
    if (k < 1 || k > tp.kmax || k > kTailMaxCols || (cols && !tp.lds_desc_cols))
        throw Error(LAMG_INVALID_ARG, "coarse tail: unsupported column count");
    TailArgs A;
    std::memset(&A, 0, sizeof(A));
    A.jobs = static_cast<const CopyJob *>(cols ? tp.jobs_cols : tp.jobs);
    A.njobs = tp.njobs;
    A.visits = d_visits;
    A.l0 = l0;
    A.nlev = nlev;
    A.l_lds = tp.l_lds;
    A.k = 1;  // each workgroup takes one column
    A.lkp = 0;
    A.red_off = 16;
    A.l_x = tp.l_x;
    A.cpart_off = (uint32_t)(16 + ((2 * (int64_t)kRedQ * TW * 8 + 15) & ~(int64_t)15));
    const TailLvl<T> *G = static_cast<const TailLvl<T> *>(cols ? tp.lds_desc_cols : tp.lds_desc);
    launch_kernel(k_tail<T, false>, dim3((unsigned)k), dim3(TB), (uint32_t)tp.lds_bytes, s, A, G,
                  (const TailWG *)nullptr);
    LAMG_LAUNCH_CHECK();
}

size_t tail_wg_bytes() { return sizeof(TailWG); }

// The records of one request's k columns (its workspace's plan and visit counters) for a
// grouped launch: appended to `recs`, with that request's descriptors and copy jobs appended
// to the launch's combined arrays as (device source, bytes) pieces to be gathered into them.
template <class T>
void tail_wg_records(const TailPlan &tp, int l0, int nlev, int k, int64_t *d_visits,
                     std::vector<char> &recs, int64_t &ndesc, int64_t &njobs_total,
                     std::vector<std::pair<const void *, size_t>> &desc_src,
                     std::vector<std::pair<const void *, size_t>> &jobs_src) {
    if (k < 1 || k > tp.kmax || k > kTailMaxCols || (k > 1 && !tp.lds_desc_cols))
        throw Error(LAMG_INVALID_ARG, "coarse tail: unsupported column count");
    const size_t db = sizeof(TailLvl<T>) * (size_t)nlev, jb = sizeof(CopyJob) * (size_t)tp.njobs;
    for (int c = 0; c < k; ++c) {
        TailWG W;
        std::memset(&W, 0, sizeof(W));
        W.visits = d_visits + (int64_t)c * nlev;
        W.desc_off = (int32_t)ndesc;
        W.jobs_off = (int32_t)njobs_total;
        W.njobs = tp.njobs;
        W.l0 = l0;
        W.nlev = nlev;
        W.l_lds = tp.l_lds;
        W.l_x = tp.l_x;
        const char *b = reinterpret_cast<const char *>(&W);
        recs.insert(recs.end(), b, b + sizeof(W));
        const char *dsrc = static_cast<const char *>(k > 1 ? tp.lds_desc_cols : tp.lds_desc) +
                           (k > 1 ? (int64_t)c * db : 0);
        const char *jsrc = static_cast<const char *>(k > 1 ? tp.jobs_cols : tp.jobs) +
                           (k > 1 ? (int64_t)c * jb : 0);
        desc_src.emplace_back(dsrc, db);
        if (jb) jobs_src.emplace_back(jsrc, jb);
        ndesc += nlev;
        njobs_total += tp.njobs;
    }
}

// One launch running the workgroups of `nwg` records (device array `wgs`) with `lds_bytes`
// of dynamic LDS (the largest plan among them).
template <class T>
void run_tail_group(const void *wgs, const void *descs, const void *jobs, int nwg,
                    size_t lds_bytes, hipStream_t s) {
    if (nwg <= 0) return;
    TailArgs A;
    std::memset(&A, 0, sizeof(A));
    A.k = 1;
    A.lkp = 0;
    A.red_off = 16;
    A.cpart_off = (uint32_t)(16 + ((2 * (int64_t)kRedQ * TW * 8 + 15) & ~(int64_t)15));
    A.jobs = static_cast<const CopyJob *>(jobs);
    launch_kernel(k_tail<T, true>, dim3((unsigned)nwg), dim3(TB), (uint32_t)lds_bytes, s, A,
                  static_cast<const TailLvl<T> *>(descs), static_cast<const TailWG *>(wgs));
    LAMG_LAUNCH_CHECK();
}

// n x k row-interleaved (x, f) -> column by column (cx, cf): element (i, c) to c n + i.
template <class T>
__global__ void k_to_cols(int64_t n, int k, const T *__restrict__ x, const T *__restrict__ f,
                          T *__restrict__ cx, T *__restrict__ cf) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int64_t o = (t - i * k) * n + i;
    cx[o] = x[t];
    cf[o] = f[t];
}

template <class T>
__global__ void k_from_cols(int64_t n, int k, const T *__restrict__ cx, T *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    x[t] = cx[(t - i * k) * n + i];
}

template <class T>
void run_to_cols(int64_t n, int k, const T *x, const T *f, T *cx, T *cf, hipStream_t s) {
    if (n * k <= 0) return;
    launch_kernel(k_to_cols<T>, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, s, n, k, x, f, cx, cf);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_from_cols(int64_t n, int k, const T *cx, T *x, hipStream_t s) {
    if (n * k <= 0) return;
    launch_kernel(k_from_cols<T>, dim3((unsigned)((n * k + 255) / 256)), dim3(256), 0, s, n, k, cx, x);
    LAMG_LAUNCH_CHECK();
}

size_t tail_copy_job_bytes() { return sizeof(CopyJob); }

void run_zero_i64(int64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    launch_kernel(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    LAMG_LAUNCH_CHECK();
}

template size_t tail_desc_bytes<double>();
template size_t tail_desc_bytes<float>();
template void tail_fill_desc<double>(void *, int, const Level &, const SolveOp &, const int64_t *,
                                     const double *, const double *, const double *,
                                     const double *, const double *, const double *,
                                     const double *, double *, double *, double *, double *,
                                     double *, double *);
template void tail_fill_desc<float>(void *, int, const Level &, const SolveOp &, const int64_t *,
                                    const float *, const float *, const float *, const float *,
                                    const float *, const float *, const float *, float *, float *,
                                    float *, float *, float *, float *);
template void run_tail<double>(const TailPlan &, int, int, int, int64_t *, hipStream_t);
template void run_tail<float>(const TailPlan &, int, int, int, int64_t *, hipStream_t);
#define LAMG_TAIL_GROUP_INST(T)                                                              \
    template void tail_wg_records<T>(const TailPlan &, int, int, int, int64_t *,               \
                                     std::vector<char> &, int64_t &, int64_t &,                \
                                     std::vector<std::pair<const void *, size_t>> &,           \
                                     std::vector<std::pair<const void *, size_t>> &);          \
    template void run_tail_group<T>(const void *, const void *, const void *, int, size_t,     \
                                    hipStream_t);
LAMG_TAIL_GROUP_INST(double)
LAMG_TAIL_GROUP_INST(float)
template void run_to_cols<double>(int64_t, int, const double *, const double *, double *,
                                  double *, hipStream_t);
template void run_to_cols<float>(int64_t, int, const float *, const float *, float *, float *,
                                 hipStream_t);
template void run_from_cols<double>(int64_t, int, const double *, double *, hipStream_t);
template void run_from_cols<float>(int64_t, int, const float *, float *, hipStream_t);
template int tail_lds_plan<double>(const std::vector<Level> &, int, int, const void *,
                                   std::vector<char> &, std::vector<char> &, size_t &, int &);
template int tail_lds_plan<float>(const std::vector<Level> &, int, int, const void *,
                                  std::vector<char> &, std::vector<char> &, size_t &, int &);

}  // namespace lamg
