// Host orchestration of lamg_solve: the gamma-cycle recursion (Sec. 2, "Cycle and
// acceleration"; eq. (2.4)), finest-level recombination, convergence tests, column
// freezing, and the FP32-cycle / FP64-refinement driver. Every arithmetic step is a
// kernel in cycle_kernels.hip; the host only sequences launches on the handle's stream
// and reads one residual norm per column per cycle.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <type_traits>

#include "lamg_internal.h"

namespace lamg {

namespace {

template <class T>
struct Prec;
template <>
struct Prec<double> {
    static const double *v(const SolveOp &o) { return o.v64.p; }
    static const double *d(const SolveOp &o) { return o.d64.p; }
    static const double *dinv(const SolveOp &o) { return o.dinv64.p; }
    static const double *w0(const SolveOp &o) { return o.w0_64.p; }
    static const double *w1(const SolveOp &o) { return o.w1_64.p; }
    static const double *rw(const SolveOp &o) { return o.rw64.p; }
    static const double *ev(const SolveOp &o) { return o.ell_w ? o.ell_v64.p : nullptr; }
    static std::vector<LevelVecs<double>> &vecs(Workspace &w) { return w.lv64; }
};
template <>
struct Prec<float> {
    static const float *v(const SolveOp &o) { return o.v32.p; }
    static const float *d(const SolveOp &o) { return o.d32.p; }
    static const float *dinv(const SolveOp &o) { return o.dinv32.p; }
    static const float *w0(const SolveOp &o) { return o.w0_32.p; }
    static const float *w1(const SolveOp &o) { return o.w1_32.p; }
    static const float *rw(const SolveOp &o) { return o.rw32.p; }
    static const float *ev(const SolveOp &o) { return o.ell_w ? o.ell_v32.p : nullptr; }
    static std::vector<LevelVecs<float>> &vecs(Workspace &w) { return w.lv32; }
};

template <class T>
struct WsSel;
template <>
struct WsSel<double> {
    static std::vector<LevelVecs<double>> &lv(Workspace &w) { return w.lv64; }
    static int &k(Workspace &w) { return w.k64; }
    static DArr<char> &desc(Workspace &w) { return w.tail64; }
    static DArr<char> &lds(Workspace &w) { return w.tlds64; }
    static DArr<char> &jobs(Workspace &w) { return w.tjobs64; }
    static TailPlan &plan(Workspace &w) { return w.plan64; }
    static DArr<double> &cx(Workspace &w) { return w.tcx64; }
    static DArr<double> &cf(Workspace &w) { return w.tcf64; }
    static DArr<char> &lds_cols(Workspace &w) { return w.tldsc64; }
    static DArr<char> &jobs_cols(Workspace &w) { return w.tjobsc64; }
};
template <>
struct WsSel<float> {
    static std::vector<LevelVecs<float>> &lv(Workspace &w) { return w.lv32; }
    static int &k(Workspace &w) { return w.k32; }
    static DArr<char> &desc(Workspace &w) { return w.tail32; }
    static DArr<char> &lds(Workspace &w) { return w.tlds32; }
    static DArr<char> &jobs(Workspace &w) { return w.tjobs32; }
    static TailPlan &plan(Workspace &w) { return w.plan32; }
    static DArr<float> &cx(Workspace &w) { return w.tcx32; }
    static DArr<float> &cf(Workspace &w) { return w.tcf32; }
    static DArr<char> &lds_cols(Workspace &w) { return w.tldsc32; }
    static DArr<char> &jobs_cols(Workspace &w) { return w.tjobsc32; }
};

// Algorithmic (compulsory) bytes of one launch of a level's cycle kernels, s = value
// and vector element size: every matrix index and value, row pointer and diagonal once,
// every vector element the launch reads or writes once.
double bytes_gs_color(const SolveOp &op, int c, int k, double s) {
    const int nc = op.ncolors;
    double r = (double)(op.blk[c + 1] - op.blk[c] + op.blk[nc + c + 1] - op.blk[nc + c]);
    double e = (double)(op.blk_nnz[c + 1] - op.blk_nnz[c] + op.blk_nnz[nc + c + 1] -
                        op.blk_nnz[nc + c]);
    return e * (4.0 + s) + 4.0 * (r + 1.0) + r * s + 3.0 * k * r * s;
}
double bytes_residual(const SolveOp &op, int k, double s) {
    const double n = (double)op.n;
    return (double)op.nnz_off * (4.0 + s) + 4.0 * (n + 1) + n * s + 3.0 * k * n * s;
}
double bytes_restrict(const SolveOp &op, int k, double s) {
    return 4.0 * (op.nc + 1) + (double)op.nnz_r * (4.0 + s) + (double)k * op.n * s +
           (double)k * op.nc * s;
}
double bytes_prolong(const SolveOp &op, int k, double s) {
    const double n = (double)op.n;
    return n * (8.0 + 2.0 * s) + (double)k * op.nc * s + 2.0 * k * n * s;
}

double bytes_coarsest(int64_t n, int k, double s) {
    return 8.0 * (double)n * (double)n + 2.0 * k * (double)n * s;
}
// two-iterate recombination: partial sums over (rho, rho1), then e, rho updated from the
// saved pair (and the result saved again when another visit follows)
double bytes_rc2(int64_t n, int k, double s, bool keep) {
    return (2.0 + 6.0 + (keep ? 2.0 : 0.0)) * k * (double)n * s;
}
double bytes_sweep(const SolveOp &op, int k, double s) {
    double b = 0.0;
    for (int c = 0; c < op.ncolors; ++c) b += bytes_gs_color(op, c, k, s);
    return b;
}
// block-Jacobi Gauss-Seidel sweep after the residual: each in-block entry once (1-byte
// position and value), the two row arrays, the diagonal and its inverse, and per column the
// residual and x read and x written
double bytes_bjgs(const SolveOp &op, int k, double s) {
    const double n = (double)op.n;
    return (double)op.bj_ni * (1.0 + s) + 4.0 * (2.0 * n + 1.0) + 2.0 * n * s + 3.0 * k * n * s;
}

// One launch, or a short group of launches of one kernel kind: its algorithmic bytes go
// into the solve's total, and while the in-situ timer is on and the launch is in its scope
// (every launch after lamg_timing_start_all; else the `narrow` ones: the timed level's
// kernels, the coarse tail and the FP64 outer residual) a pair of the timer's events is
// attached to the kernels launched during the object's lifetime.
struct Timed {
    KTimer &t;
    int idx = -1;
    LaunchEvents le;
    LaunchEvents *prev = nullptr;
    Timed(lamg_handle *h, int kind, int prec, double bytes, bool narrow) : t(h->timer) {
        h->solve_bytes += bytes;
        if (!t.on || !(t.all || (narrow && kind <= LAMG_KERNEL_TAIL))) return;
        idx = t.open(kind, prec, bytes);
        if (idx < 0) return;
        le.start = t.ev[2 * idx];
        le.stop = t.ev[2 * idx + 1];
        prev = t_launch_events;
        t_launch_events = &le;
    }
    ~Timed() {
        if (idx < 0) return;
        t_launch_events = prev;
        if (!le.started) t.recs[idx].kind = -1;
    }
};

// Whether the timer takes a launch of this scope (then per-step launches are made one by one).
inline bool timing(const lamg_handle *h, bool narrow) {
    return h->timer.on && (h->timer.all || narrow);
}

template <class T>
constexpr int prec_id() {
    return sizeof(T) == 4 ? 1 : 0;
}

template <class T>
struct Cycle {
    lamg_handle *h;
    int k;
    hipStream_t s;
    std::vector<LevelVecs<T>> *v;
    std::vector<int64_t> visits;  // entries into each level's coarse-correction phase
    double *partial;
    int l0;                 // first level run by the coarse-tail kernel (-1: none)
    int lt;                 // level whose per-step kernels the in-situ timer records
    const TailPlan *plan;   // its descriptors and LDS layout
    int64_t *d_visits;      // its visit counters (per column)
    T *cx, *cf;             // column-by-column copies of the top level's x and f (k > 1)
    std::vector<int64_t> tvisits;  // host mirror of the tail's visit counters (byte counts)
};

// Algorithmic bytes of the visit to level l that a coarse-tail launch makes (and of every
// visit below it), advancing the host mirror of the tail's visit counters as the kernel
// advances its own: the same schedule, step by step, with the operators counted once per
// launch whatever the column count.
template <class T>
double tail_level_bytes(Cycle<T> &C, int l) {
    const lamg_handle *h = C.h;
    const Level &L = h->lev[l];
    const int k = C.k;
    const double sz = sizeof(T);
    if (L.coarsest) return bytes_coarsest(L.n, k, sz);
    const SolveOp &op = L.op;
    const Level &Lc = h->lev[l + 1];
    const double zero_c = (double)k * Lc.n * sz;
    if (L.elim) {
        C.tvisits[l]++;
        return 2.0 * bytes_gs_color(op, 0, k, sz) + bytes_gs_color(op, 1, k, sz) +
               bytes_restrict(op, k, sz) + zero_c + 4.0 * op.nc + 3.0 * k * op.nc * sz +
               tail_level_bytes(C, l + 1);
    }
    double b = 3.0 * bytes_sweep(op, k, sz) + bytes_residual(op, k, sz) +
               bytes_restrict(op, k, sz) + zero_c;
    const int64_t i = C.tvisits[l]++;
    const int nvis = (int)(std::floor((double)(i + 1) * L.gamma) - std::floor((double)i * L.gamma));
    for (int j = 1; j <= nvis; ++j) {
        b += tail_level_bytes(C, l + 1) + bytes_residual(Lc.op, k, sz);
        if (j >= 2)
            b += bytes_rc2(Lc.n, k, sz, j < nvis);
        else if (j < nvis)
            b += 4.0 * zero_c;  // the first visit's pair saved
    }
    return b + 3.0 * zero_c + bytes_prolong(op, k, sz);  // energy-correction sums, prolongation
}

// First level (below the finest) whose cycle runs in the coarse-tail kernel: the first
// level with at most tail_rows nodes, extended upwards over levels whose visit is clearly
// cheaper as dependent steps of one workgroup than as kernel launches. Such levels have
// many colours of few rows each (the dense and the chain-like coarse levels of power-law
// graphs): a visit costs about 3 sweeps x colours launches plus ~15 others, each ~4 us,
// against the same number of workgroup steps of ~0.5 us plus the rows of a colour pass
// gathered through one compute unit (~2000 entries per us). Levels with long (hub) rows
// stay with the per-step kernels, which give each such row a whole block.
// Every column of a solve gets a workgroup of its own (at most kTailMaxCols columns), so
// the tail costs the same per launch whatever the column count; one workgroup carrying
// all columns was slower than the per-step kernels from four columns on (anisotropic
// grid, 4 columns: 126 ms against 109 ms without the tail), one per column is faster at
// every width measured (4 columns: 69 ms; 32 columns: 117 against 154 ms).
// With `fp32` (the FP32 cycles of an FP32+IR solve), a finest level of at most
// opt.tail_finest nodes joins the tail as well when every level below it is in the tail:
// the whole cycle is then one launch (and the launches of several such solves can be one,
// see solve_group). FP64 cycles keep the finest level's per-step kernels, which work on
// the finest FP64 state directly.
int tail_level(const lamg_handle *h, int k, bool fp32) {
    if (h->opt.tail_rows <= 0 || k > kTailMaxCols) return -1;
    int l0 = -1;
    for (int l = 1; l < h->nlev; ++l)
        if (h->lev[l].n <= h->opt.tail_rows) {
            l0 = l;
            break;
        }
    if (l0 < 0) return -1;
    // levels smoothed by Chebyshev polynomials or block-Jacobi Gauss-Seidel stay with the
    // per-step kernels
    for (int l = h->nlev - 1; l >= 0; --l)
        if (h->lev[l].cheb || h->lev[l].bjgs) {
            if (l0 <= l) l0 = l + 1;
            break;
        }
    if (l0 >= h->nlev) return -1;
    while (l0 > 1) {
        if (h->lev[l0 - 1].cheb || h->lev[l0 - 1].bjgs) break;
        const Level &L = h->lev[l0 - 1];
        const SolveOp &op = L.op;
        if (L.coarsest || L.n >= 65536) break;
        const int nc = std::max(1, op.ncolors);
        const bool has_long = op.blk[2 * nc] > op.blk[nc];
        if (has_long) break;  // hub rows: a block each in the per-step kernels
        const double launches = 3.0 * nc + 15.0;
        const double steps = 3.0 * nc + 15.0;
        const double entries_per_pass = (double)op.nnz_off / nc;
        const double tail_us = steps * (0.5 + entries_per_pass / 2000.0);
        if (tail_us > 0.5 * launches * 4.0) break;
        --l0;
    }
    const Level &F = h->lev[0];
    if (fp32 && l0 == 1 && h->opt.tail_finest > 0 && F.n <= h->opt.tail_finest && F.n < 65536 &&
        !F.coarsest && !F.cheb && !F.bjgs)
        l0 = 0;
    return l0;
}

// Level whose per-step cycle kernels the in-situ timer records and whose kernels carry the
// separate "finest" symbols: the finest aggregation level (elimination levels run no full
// smoothing pass), or the finest level when that aggregation level runs in the coarse tail.
int timed_level(const lamg_handle *h, int k) {
    const int l0 = tail_level(h, k, false);
    for (int l = 0; l < h->nlev; ++l) {
        const Level &L = h->lev[l];
        if (L.coarsest) break;
        if (!L.elim) return (l0 < 0 || l < l0) ? l : 0;
    }
    return 0;
}

// One gamma-cycle at level l on (x, f): (1,2) multicolour Gauss-Seidel, coarse
// correction by `nvis` visits to level l+1 (Beatty counts of the fractional cycle index)
// with two-iterate recombination across the visits, energy correction
// mu = <e, fc> / <e, L_c e>, prolongation.
template <class T>
void cycle(Cycle<T> &C, int l, T *x, const T *f) {
    lamg_handle *h = C.h;
    const int k = C.k;
    hipStream_t s = C.s;
    Level &L = h->lev[l];
    using P = Prec<T>;
    constexpr int pid = prec_id<T>();
    const double sz = sizeof(T);
    if (l == C.l0) {
        const double tb = tail_level_bytes<T>(C, l);
        if (k == 1) {
            Timed tm(h, LAMG_KERNEL_TAIL, pid, tb, true);
            run_tail<T>(*C.plan, l, h->nlev, k, C.d_visits, s);
            return;
        }
        // a workgroup per column, on the top level's (x, f) copied column by column
        {
            Timed tm(h, LAMG_KERNEL_VECTOR, pid, 4.0 * k * L.n * sz, false);
            run_to_cols<T>(L.n, k, x, f, C.cx, C.cf, s);
        }
        {
            Timed tm(h, LAMG_KERNEL_TAIL, pid, tb, true);
            run_tail<T>(*C.plan, l, h->nlev, k, C.d_visits, s);
        }
        Timed tm(h, LAMG_KERNEL_VECTOR, pid, 2.0 * k * L.n * sz, false);
        run_from_cols<T>(L.n, k, C.cx, x, s);
        return;
    }
    const bool nar = l == C.lt;  // the timed level
    if (L.coarsest) {
        Timed tm(h, LAMG_KERNEL_VECTOR, pid, bytes_coarsest(L.n, k, sz), false);
        run_coarsest<T>(L.n, L.Z.p, f, x, k, s);
        return;
    }
    const SolveOp &op = L.op;
    Level &Lc = h->lev[l + 1];
    const SolveOp &cop = Lc.op;
    LevelVecs<T> &me = (*C.v)[l];
    LevelVecs<T> &cv = (*C.v)[l + 1];
    const double zero_c = (double)k * Lc.n * sz;
    if (L.elim) {
        // elimination level (eq. (2.1)), cycle index 1: the eliminated rows (colour 0) are
        // set exactly from the kept ones, the coarse right-hand side is the residual of the
        // kept rows (colour 1; it equals P^T r since the eliminated rows' residual is then
        // zero), one coarse visit, the kept rows take the coarse correction, and the
        // eliminated rows are set exactly again. No smoothing or energy correction: the
        // interpolation is exact.
        auto relax_f = [&]() {
            Timed tm(h, LAMG_KERNEL_GS_COLOR, pid, bytes_gs_color(op, 0, k, sz), nar);
            run_gs_color<T>(op, 0, P::v(op), P::dinv(op), f, x, k, s, l == C.lt);
        };
        relax_f();
        {
            Timed tm(h, LAMG_KERNEL_RESIDUAL, pid, bytes_gs_color(op, 1, k, sz), nar);
            run_residual_color<T>(op, 1, P::v(op), P::d(op), x, f, me.r.p, k, s, l == C.lt);
        }
        {
            Timed tm(h, LAMG_KERNEL_RESTRICT, pid, bytes_restrict(op, k, sz) + zero_c, nar);
            run_restrict<T>(op, P::rw(op), me.r.p, cv.f.p, k, s, cv.x.p);
        }
        C.visits[l]++;
        cycle<T>(C, l + 1, cv.x.p, cv.f.p);
        {
            Timed tm(h, LAMG_KERNEL_PROLONG, pid, 4.0 * op.nc + 3.0 * k * op.nc * sz, nar);
            run_inject_add<T>(op, cv.x.p, x, k, s);
        }
        relax_f();
        return;
    }
    auto smooth = [&](int sweeps) {
        if (L.cheb) {  // Chebyshev sweeps (smoother option 1), in me.r as work space
            for (int sw = 0; sw < sweeps; ++sw) {
                Timed tm(h, LAMG_KERNEL_CHEB, pid,
                         kChebDegree * (bytes_residual(op, k, sz) + 3.0 * k * op.n * sz), nar);
                run_cheb_sweep<T>(op, L.cheb_lmax, P::v(op), P::d(op), P::dinv(op), f, x, me.r.p,
                                  k, s, l == C.lt);
            }
            return;
        }
        if (L.bjgs) {  // block-Jacobi Gauss-Seidel sweeps (smoother option 2), in me.r as work space
            for (int sw = 0; sw < sweeps; ++sw) {
                Timed tm(h, LAMG_KERNEL_BJGS, pid, bytes_residual(op, k, sz) + bytes_bjgs(op, k, sz),
                         nar);
                run_bjgs_sweep<T>(op, P::v(op), P::d(op), P::dinv(op), f, x, me.r.p, k, s,
                                  l == C.lt);
            }
            return;
        }
        if (!timing(h, nar)) {
            h->solve_bytes += sweeps * bytes_sweep(op, k, sz);
            run_gs<T>(op, P::v(op), P::dinv(op), f, x, k, sweeps, s, l == C.lt);
            return;
        }
        for (int sw = 0; sw < sweeps; ++sw)
            for (int c = 0; c < op.ncolors; ++c) {
                Timed tm(h, LAMG_KERNEL_GS_COLOR, pid, bytes_gs_color(op, c, k, sz), nar);
                run_gs_color<T>(op, c, P::v(op), P::dinv(op), f, x, k, s, l == C.lt);
            }
    };
    smooth(1);
    {
        Timed tm(h, LAMG_KERNEL_RESIDUAL, pid, bytes_residual(op, k, sz), nar);
        run_residual<T>(op, P::v(op), P::d(op), x, f, me.r.p, k, s, l == C.lt);
    }
    {  // f_c = P^T r, and the coarse iterate starts from zero (same launch)
        Timed tm(h, LAMG_KERNEL_RESTRICT, pid, bytes_restrict(op, k, sz) + zero_c, nar);
        run_restrict<T>(op, P::rw(op), me.r.p, cv.f.p, k, s, cv.x.p);
    }
    int64_t i = C.visits[l]++;
    int nvis = (int)(std::floor((double)(i + 1) * L.gamma) - std::floor((double)i * L.gamma));
    for (int j = 1; j <= nvis; ++j) {
        cycle<T>(C, l + 1, cv.x.p, cv.f.p);
        const bool again = j < nvis;
        if (j >= 2) {  // recombine with the previous visit's pair, keep it if revisiting
            {
                Timed tm(h, LAMG_KERNEL_RESIDUAL, pid, bytes_residual(cop, k, sz), false);
                run_residual<T>(cop, P::v(cop), P::d(cop), cv.x.p, cv.f.p, cv.rho.p, k, s, false);
            }
            Timed tm(h, LAMG_KERNEL_REDUCE, pid, bytes_rc2(Lc.n, k, sz, again), false);
            run_rc2_keep<T>(Lc.n, cv.x.p, cv.rho.p, cv.x1.p, cv.rho1.p, k, C.partial, cv.alpha.p,
                            again, s);
        } else {  // first visit: the pair (x, rho) is saved by the residual launch
            Timed tm(h, LAMG_KERNEL_RESIDUAL, pid,
                     bytes_residual(cop, k, sz) + (again ? 2.0 * zero_c : 0.0), false);
            run_residual<T>(cop, P::v(cop), P::d(cop), cv.x.p, cv.f.p, cv.rho.p, k, s, false,
                            again ? cv.x1.p : nullptr, again ? cv.rho1.p : nullptr);
        }
    }
    {  // energy correction and prolongation
        Timed tm(h, LAMG_KERNEL_PROLONG, pid, 3.0 * zero_c + bytes_prolong(op, k, sz), nar);
        run_mu_prolong<T>(op, P::w0(op), P::w1(op), Lc.n, cv.x.p, cv.f.p, cv.rho.p, k, C.partial,
                          cv.mu.p, x, s);
    }
    smooth(2);
}

template <class T>
void ensure_level_vecs(lamg_handle *h, int k) {
    using P = Prec<T>;
    using W = WsSel<T>;
    Workspace &w = h->ws;
    std::vector<LevelVecs<T>> &lv = W::lv(w);
    if (W::k(w) >= k && (int)lv.size() == h->nlev) return;
    clear_graphs(w);  // their kernel arguments point into the vectors replaced here
    Pool &pool = w.arena ? *w.arena : *h->pool;
    lv.clear();
    lv.resize(h->nlev);
    for (int l = 0; l < h->nlev; ++l) {
        int64_t m = h->lev[l].n * k;
        lv[l].x.alloc(pool, m);
        lv[l].f.alloc(pool, m);
        lv[l].r.alloc(pool, m);
        lv[l].rho.alloc(pool, m);
        lv[l].x1.alloc(pool, m);
        lv[l].rho1.alloc(pool, m);
        lv[l].mu.alloc(pool, k);
        lv[l].alpha.alloc(pool, k);
    }
    // coarse-tail descriptors (pointers to this precision's operators and vectors) and the
    // layout of its LDS-resident levels
    size_t db = tail_desc_bytes<T>();
    std::vector<char> host(db * h->nlev);
    for (int l = 0; l < h->nlev; ++l) {
        const Level &L = h->lev[l];
        const SolveOp &op = L.op;
        tail_fill_desc<T>(host.data(), l, L, op, op.dblk.p, P::v(op), P::d(op), P::dinv(op),
                          P::w0(op), P::w1(op), P::rw(op), P::ev(op), lv[l].x.p, lv[l].f.p, lv[l].r.p,
                          lv[l].rho.p, lv[l].x1.p, lv[l].rho1.p);
    }
    DArr<char> &desc = W::desc(w);
    desc.alloc(pool, (int64_t)host.size());
    desc.upload(host.data(), (int64_t)host.size(), h->stream);
    TailPlan &tp = W::plan(w);
    tp = TailPlan();
    tp.desc = desc.p;
    tp.l_lds = h->nlev;
    std::vector<char> lds_desc, jobs;
    size_t lds_bytes = 0;
    // the plan serves every later solve that uses the tail (at most kTailMaxCols columns),
    // including narrower solves reusing vectors sized for a wider one, so it is built for
    // the tail level of such solves whatever k these vectors were sized for
    const int l0 = tail_level(h, 1, std::is_same<T, float>::value);
    int l_x = -1;  // one column per workgroup
    int l_lds = tail_lds_plan<T>(h->lev, l0, 1, host.data(), lds_desc, jobs, lds_bytes, l_x);
    if (l0 >= 0) {
        DArr<char> &dl = W::lds(w);
        DArr<char> &dj = W::jobs(w);
        dl.alloc(pool, (int64_t)lds_desc.size());
        dl.upload(lds_desc.data(), (int64_t)lds_desc.size(), h->stream);
        dj.alloc(pool, (int64_t)std::max<size_t>(jobs.size(), 1));
        if (!jobs.empty()) dj.upload(jobs.data(), (int64_t)jobs.size(), h->stream);
        tp.lds_desc = dl.p;
        tp.jobs = dj.p;
        tp.njobs = (int)(jobs.size() / tail_copy_job_bytes());
        tp.l_lds = l_lds;
        tp.l_x = l_x;
        tp.lds_bytes = lds_bytes;
        tp.kmax = k;
        if (k > 1) {
            // one descriptor set per column: vectors from element c n of each level's
            // arrays, the top level's x and f from the column copies
            const int ncols = std::min(k, kTailMaxCols);
            const int64_t n0 = h->lev[l0].n;
            W::cx(w).alloc(pool, n0 * k);
            W::cf(w).alloc(pool, n0 * k);
            std::vector<char> hp(db * h->nlev), all_desc, all_jobs;
            for (int c = 0; c < ncols; ++c) {
                for (int l = 0; l < h->nlev; ++l) {
                    const Level &L = h->lev[l];
                    const SolveOp &op = L.op;
                    const int64_t o = (int64_t)c * L.n;
                    T *xv = l == l0 ? W::cx(w).p + c * n0 : lv[l].x.p + o;
                    T *fv = l == l0 ? W::cf(w).p + c * n0 : lv[l].f.p + o;
                    tail_fill_desc<T>(hp.data(), l, L, op, op.dblk.p, P::v(op), P::d(op),
                                      P::dinv(op), P::w0(op), P::w1(op), P::rw(op), P::ev(op), xv,
                                      fv, lv[l].r.p + o, lv[l].rho.p + o, lv[l].x1.p + o,
                                      lv[l].rho1.p + o);
                }
                std::vector<char> pd, pj;
                size_t pb = 0;
                int px_l = -1;
                const int pl = tail_lds_plan<T>(h->lev, l0, 1, hp.data(), pd, pj, pb, px_l);
                if (pl != l_lds || px_l != l_x || pb != lds_bytes || pj.size() != jobs.size())
                    throw Error(LAMG_HIP_ERROR, "coarse tail: column plans differ");
                all_desc.insert(all_desc.end(), pd.begin(), pd.end());
                all_jobs.insert(all_jobs.end(), pj.begin(), pj.end());
            }
            DArr<char> &dlp = W::lds_cols(w);
            DArr<char> &djp = W::jobs_cols(w);
            dlp.alloc(pool, (int64_t)all_desc.size());
            dlp.upload(all_desc.data(), (int64_t)all_desc.size(), h->stream);
            djp.alloc(pool, (int64_t)std::max<size_t>(all_jobs.size(), 1));
            if (!all_jobs.empty()) djp.upload(all_jobs.data(), (int64_t)all_jobs.size(), h->stream);
            tp.lds_desc_cols = dlp.p;
            tp.jobs_cols = djp.p;
        }
    }
    LAMG_HIP(hipStreamSynchronize(h->stream));
    W::k(w) = k;
}

void ensure_fine(lamg_handle *h, int k) {
    Workspace &w = h->ws;
    if (w.kf >= k) return;
    clear_graphs(w);
    Pool &pool = w.arena ? *w.arena : *h->pool;
    int64_t m = h->lev[0].n * k;
    w.phi.alloc(pool, m);
    w.b.alloc(pool, m);
    w.r.alloc(pool, m);
    w.b0.alloc(pool, m);
    w.tmp.alloc(pool, m);
    w.hphi.alloc(pool, 4 * m);
    w.hr.alloc(pool, 4 * m);
    w.nb.alloc(pool, k);
    w.rel.alloc(pool, k);
    w.scale.alloc(pool, k);
    w.alpha_f.alloc(pool, 4 * k);
    w.mean.alloc(pool, k);
    w.partial.alloc(pool, (int64_t)kRedBlocksMax * kRedQMax * k);
    w.mask.alloc(pool, k);
    w.visits.alloc(pool, (int64_t)h->nlev * kTailMaxCols);
    if (w.arena) {  // no pinned allocation: pageable mirrors (each copy is waited for)
        w.h_rel_v.assign(k, 0.0);
        w.h_mask_v.assign(k, 0);
        w.h_rel = w.h_rel_v.data();
        w.h_mask = w.h_mask_v.data();
        w.kf = k;
        return;
    }
    if (w.h_rel) (void)hipHostFree(w.h_rel);
    if (w.h_mask) (void)hipHostFree(w.h_mask);
    w.h_rel = nullptr;
    w.h_mask = nullptr;
    LAMG_HIP(hipHostMalloc((void **)&w.h_rel, sizeof(double) * k));
    LAMG_HIP(hipHostMalloc((void **)&w.h_mask, sizeof(int32_t) * k));
    w.kf = k;
}

// The graph set of solves with this precision and column count, created (evicting the
// least recently used set beyond kGraphSets) if there is none, and moved to the back.
Workspace::GraphSet &graph_set(Workspace &w, int prec, int k) {
    auto it = std::find_if(w.gsets.begin(), w.gsets.end(),
                           [&](const Workspace::GraphSet &g) { return g.prec == prec && g.k == k; });
    Workspace::GraphSet g;
    if (it != w.gsets.end()) {
        g = std::move(*it);
        w.gsets.erase(it);
    } else {
        g.prec = prec;
        g.k = k;
        if ((int)w.gsets.size() >= kGraphSets) {
            for (Workspace::CycleGraph &c : w.gsets.front().cycles)
                if (c.exec) (void)hipGraphExecDestroy(c.exec);
            w.gsets.erase(w.gsets.begin());
        }
    }
    w.gsets.push_back(std::move(g));
    return w.gsets.back();
}

// Records the launches `body` makes on a capture stream of the handle into a graph,
// instantiates it and launches it on `s`. Returns nullptr, having launched nothing, if
// capture is not possible or the graph has more than kGraphMaxNodes nodes; the caller
// then runs `body` on `s` itself.
template <class F>
hipGraphExec_t capture_and_launch(lamg_handle *h, hipStream_t s, F &&body) {
    Workspace &w = h->ws;
    if (!w.cap_stream && hipStreamCreateWithFlags(&w.cap_stream, hipStreamNonBlocking) != hipSuccess) {
        w.cap_stream = nullptr;
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipStreamBeginCapture(w.cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    try {
        body(w.cap_stream);
    } catch (...) {
        hipGraph_t g = nullptr;
        if (hipStreamEndCapture(w.cap_stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(w.cap_stream, &graph);
    hipGraphExec_t exec = nullptr;
    size_t nodes = 0;
    if (e == hipSuccess && graph && hipGraphGetNodes(graph, nullptr, &nodes) == hipSuccess &&
        nodes <= (size_t)kGraphMaxNodes &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        (void)hipGraphDestroy(graph);
        LAMG_HIP(hipGraphLaunch(exec, s));
        return exec;
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return nullptr;
}

double acf_of(const std::vector<double> &hist) {
    int last = (int)hist.size() - 1;
    int cnt = std::min(last, 5);
    if (cnt <= 0 || !(hist[last - cnt] > 0.0) || !(hist[last] > 0.0)) return 0.0;
    return std::pow(hist[last] / hist[last - cnt], 1.0 / cnt);
}

// Projects (mean removal) the listed columns of phi and writes them to the caller's
// column-major output.
void emit_columns(lamg_handle *h, int k, const int32_t *d_mask, double *phi_out) {
    Workspace &w = h->ws;
    hipStream_t s = h->stream;
    const int64_t n = h->lev[0].n;
    const double nk8 = 8.0 * n * k;
    {
        Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8, false);
        run_copy<double>(w.tmp.p, w.phi.p, n * k, s);
    }
    {
        Timed tm(h, LAMG_KERNEL_REDUCE, 0, nk8, false);
        run_colsum(n, k, w.tmp.p, w.partial.p, w.mean.p, 1.0 / (double)n, s);
    }
    {
        Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8, false);
        run_sub_col(n, k, w.tmp.p, w.mean.p, s);
    }
    Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8 + 4.0 * n, false);
    run_scatter_cols(n, k, h->lev[0].op.io_perm.p, w.tmp.p, d_mask, phi_out, s);
}

// The state of one solve of at most 32 columns, advanced cycle by cycle: begin() prepares
// the right-hand sides and the first iterate, each cycle launches its work (pre, the cycle,
// post), the relative residuals come back once per cycle (host()), and finish() writes the
// statistics. solve_chunk runs one chunk by itself; solve_group runs several in lockstep,
// with the coarse-tail launches of all of them made as one.
struct Chunk {
    lamg_handle *h = nullptr;
    int k = 0;
    double tol = 0.0;
    int max_cycles = 0;
    bool fp32 = false;
    double *phi_out = nullptr;
    int64_t n = 0, nk = 0;
    double nk8 = 0.0;
    std::vector<double> nb;
    std::vector<int32_t> active, failed, cycles;
    std::vector<std::vector<double>> hist;
    int n_active = 0, hm = 0, hnext = 0, kappa = 0, cyc = 0;
    bool direct = false;
    std::unique_ptr<Cycle<double>> c64;
    std::unique_ptr<Cycle<float>> c32;

    void begin(lamg_handle *hh, const double *b_user, int kk, double t, int mc, bool f32,
               double *out) {
        h = hh;
        k = kk;
        tol = t;
        max_cycles = mc;
        fp32 = f32;
        phi_out = out;
        hipStream_t s = h->stream;
        Workspace &w = h->ws;
        Level &L0 = h->lev[0];
        const SolveOp &op0 = L0.op;
        n = L0.n;
        nk = n * k;
        ensure_fine(h, k);
        if (fp32)
            ensure_level_vecs<float>(h, k);
        else
            ensure_level_vecs<double>(h, k);
        nk8 = 8.0 * (double)nk;
        {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 8.0 * h->nlev * kTailMaxCols, false);
            run_zero_i64(w.visits.p, (int64_t)h->nlev * kTailMaxCols, s);
        }
        // b <- P b, projected to mean zero (eq. (1.1)); ||b|| per column
        {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8 + 4.0 * n, false);
            run_gather_cols(n, k, op0.io_perm.p, b_user, w.b.p, s);
        }
        {
            Timed tm(h, LAMG_KERNEL_REDUCE, 0, nk8, false);
            run_colsum(n, k, w.b.p, w.partial.p, w.mean.p, 1.0 / (double)n, s);
        }
        {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 4.0 * nk8, false);
            run_sub_col(n, k, w.b.p, w.mean.p, s);
            run_copy<double>(w.b0.p, w.b.p, nk, s);
        }
        {
            Timed tm(h, LAMG_KERNEL_REDUCE, 0, nk8, false);
            run_norm2(n, k, w.b.p, w.partial.p, w.nb.p, s);
        }
        nb.assign(k, 0.0);
        w.nb.download(nb.data(), k, s);
        LAMG_HIP(hipStreamSynchronize(s));
        // eq. (1.1) needs a finite b: a NaN or infinite entry makes the projected column's
        // norm NaN or infinite (so does a norm that overflows); nothing has been written yet
        for (int c = 0; c < k; ++c)
            if (!std::isfinite(nb[c]))
                throw Error(LAMG_INVALID_ARG, "right-hand side column is not finite");
        active.assign(k, 0);
        failed.assign(k, 0);
        cycles.assign(k, 0);
        hist.assign(k, std::vector<double>());
        n_active = 0;
        for (int c = 0; c < k; ++c) {
            active[c] = nb[c] > 0.0 ? 1 : 0;
            n_active += active[c];
            hist[c].push_back(1.0);
        }
        // zero columns: phi = 0; everything else starts from phi = 0, r = b
        {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 3.0 * nk8, false);
            run_fill<double>(w.phi.p, nk, 0.0, s);
            run_copy<double>(w.r.p, w.b.p, nk, s);
        }
        if (fp32) {  // the first cycle's scale
            Timed tm(h, LAMG_KERNEL_REDUCE, 0, nk8, false);
            run_maxabs(n, k, w.r.p, w.partial.p, w.scale.p, s);
        }
        direct = L0.coarsest;
        kappa = std::max(0, std::min(4, (int)h->opt.kappa));
        hm = hnext = 0;
        if (!direct && kappa > 0) {  // history starts with (0, b)
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 3.0 * nk8, false);
            run_fill<double>(w.hphi.p, nk, 0.0, s);
            run_copy<double>(w.hr.p, w.b.p, nk, s);
            hm = 1;
            hnext = 1;
        }
        if (n_active < k) {  // columns with b = 0 finish immediately with phi = 0
            for (int c = 0; c < k; ++c) w.h_mask[c] = active[c] ? 0 : 1;
            w.mask.upload(w.h_mask, k, s);
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8 + 4.0 * n, false);
            run_scatter_cols(n, k, op0.io_perm.p, w.phi.p, w.mask.p, phi_out, s);
        }
        const int lt = timed_level(h, k);
        c64.reset(new Cycle<double>{h, k, s, &w.lv64, std::vector<int64_t>(h->nlev, 0),
                                    w.partial.p, tail_level(h, k, false), lt, &w.plan64,
                                    w.visits.p, w.tcx64.p, w.tcf64.p,
                                    std::vector<int64_t>(h->nlev, 0)});
        c32.reset(new Cycle<float>{h, k, s, &w.lv32, std::vector<int64_t>(h->nlev, 0),
                                   w.partial.p, tail_level(h, k, true), lt, &w.plan32,
                                   w.visits.p, w.tcx32.p, w.tcf32.p,
                                   std::vector<int64_t>(h->nlev, 0)});
        cyc = 0;
    }

    bool running() const { return n_active > 0 && cyc < max_cycles; }

    // FP32 cycles: the residual equation scaled by max |r| (w.scale, formed with the previous
    // relative residuals, or before the first cycle) as the level-0 right-hand side
    void pre(hipStream_t st) {
        if (!fp32) return;
        Workspace &w = h->ws;
        LevelVecs<float> &v0 = w.lv32[0];
        Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8, false);
        run_to_f32_scaled(n, k, w.r.p, w.scale.p, v0.f.p, v0.x.p, st);
    }

    void cycle_launches(hipStream_t st) {
        Workspace &w = h->ws;
        if (!fp32) {
            c64->s = st;
            cycle<double>(*c64, 0, w.phi.p, w.b.p);
            c64->s = h->stream;
        } else {
            LevelVecs<float> &v0 = w.lv32[0];
            c32->s = st;
            cycle<float>(*c32, 0, v0.x.p, v0.f.p);
            c32->s = h->stream;
        }
    }

    // the FP64 update, the fine residual, recombination and the relative residuals
    void post(hipStream_t st) {
        Workspace &w = h->ws;
        const SolveOp &op0 = h->lev[0].op;
        if (fp32) {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.5 * nk8, false);
            run_add_scaled_f32(n, k, w.lv32[0].x.p, w.scale.p, w.phi.p, st);
        }
        {
            Timed tm(h, LAMG_KERNEL_RESIDUAL, 0, bytes_residual(op0, k, 8.0), true);
            run_residual<double>(op0, op0.v64.p, op0.d64.p, w.phi.p, w.b.p, w.r.p, k, st, true);
        }
        if (!direct && kappa > 0) {
            // recombination; the recombined pair goes into the next history slot (partial
            // sums over r and the m saved residuals; update reading phi, r and the m pairs,
            // writing phi, r and the slot)
            Timed tm(h, LAMG_KERNEL_REDUCE, 0,
                     hm > 0 ? (1.0 + hm + 2.0 + 2.0 * hm + 4.0) * nk8 : 4.0 * nk8, false);
            run_recombine_fine(n, k, hm, w.phi.p, w.r.p, w.hphi.p, w.hr.p, hnext % kappa,
                               w.partial.p, w.alpha_f.p, st);
        }
        Timed tm(h, LAMG_KERNEL_REDUCE, 0, nk8, false);
        run_relres_maxabs(n, k, w.r.p, w.nb.p, w.partial.p, w.rel.p, w.scale.p, st);
    }

    // after the cycle's launches: history bookkeeping and the residuals' read-back (the
    // caller synchronises the stream before host())
    void read_back() {
        if (!direct && kappa > 0) {
            ++hnext;
            if (hm < kappa) ++hm;
        }
        ++cyc;
        h->ws.rel.download(h->ws.h_rel, k, h->stream);
    }

    void host() {
        Workspace &w = h->ws;
        hipStream_t s = h->stream;
        bool any_new = false;
        for (int c = 0; c < k; ++c) {
            w.h_mask[c] = 0;
            if (!active[c]) continue;
            double rel = w.h_rel[c];
            hist[c].push_back(rel);
            cycles[c] = cyc;
            // a column stops when it meets the tolerance, or when its relative residual is
            // no longer a finite number (then it has failed: the solve reports it)
            if (rel <= tol || !std::isfinite(rel)) {
                if (!(rel <= tol)) failed[c] = 1;
                active[c] = 0;
                --n_active;
                w.h_mask[c] = 1;
                any_new = true;
            }
        }
        if (any_new) {
            // freeze: emit the converged columns, then zero their state so later cycles
            // leave them untouched (no later cycle once every column has converged, and a
            // solve re-initialises all of this state)
            w.mask.upload(w.h_mask, k, s);
            emit_columns(h, k, w.mask.p, phi_out);
        }
        if (any_new && n_active > 0) {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, (3.0 + 2.0 * hm) * nk8, false);
            run_zero_cols(n, k, w.mask.p, w.phi.p, s);
            run_zero_cols(n, k, w.mask.p, w.b.p, s);
            run_zero_cols(n, k, w.mask.p, w.r.p, s);
            for (int i = 0; i < hm; ++i) {
                run_zero_cols(n, k, w.mask.p, w.hphi.p + i * nk, s);
                run_zero_cols(n, k, w.mask.p, w.hr.p + i * nk, s);
            }
        }
    }

    lamg_status finish(std::vector<double> &relres, std::vector<double> &acf,
                       std::vector<double> &hist0) {
        Workspace &w = h->ws;
        hipStream_t s = h->stream;
        const SolveOp &op0 = h->lev[0].op;
        lamg_status st = LAMG_OK;
        for (int c = 0; c < k; ++c)
            if (failed[c]) st = LAMG_NOT_CONVERGED;
        if (n_active > 0) {
            for (int c = 0; c < k; ++c) w.h_mask[c] = active[c];
            w.mask.upload(w.h_mask, k, s);
            emit_columns(h, k, w.mask.p, phi_out);
            st = LAMG_NOT_CONVERGED;
        }
        // true residual of the returned phi
        {
            Timed tm(h, LAMG_KERNEL_VECTOR, 0, 2.0 * nk8 + 4.0 * n, false);
            run_gather_cols(n, k, op0.io_perm.p, phi_out, w.phi.p, s);
        }
        {
            Timed tm(h, LAMG_KERNEL_RESIDUAL, 0, bytes_residual(op0, k, 8.0), false);
            run_residual<double>(op0, op0.v64.p, op0.d64.p, w.phi.p, w.b0.p, w.r.p, k, s, true);
        }
        {
            Timed tm(h, LAMG_KERNEL_REDUCE, 0, nk8, false);
            run_relres(n, k, w.r.p, w.nb.p, w.partial.p, w.rel.p, s);
        }
        w.rel.download(w.h_rel, k, s);
        LAMG_HIP(hipStreamSynchronize(s));
        relres.assign(k, 0.0);
        acf.assign(k, 0.0);
        for (int c = 0; c < k; ++c) {
            relres[c] = nb[c] > 0.0 ? w.h_rel[c] : 0.0;
            acf[c] = acf_of(hist[c]);
        }
        hist0 = hist[0];
        return st;
    }
};

// One chunk of at most 32 columns.
lamg_status solve_chunk(lamg_handle *h, const double *b_user, int k, double tol, int max_cycles,
                        bool fp32, double *phi_out, std::vector<double> &relres,
                        std::vector<int32_t> &cycles, std::vector<double> &acf,
                        std::vector<double> &hist0, int &graph_cycles) {
    hipStream_t s = h->stream;
    Workspace &w = h->ws;
    Chunk ch;
    ch.begin(h, b_user, k, tol, max_cycles, fp32, phi_out);
    // One cycle with its fine-level residual, recombination and relative residuals: the
    // launches depend only on the cycle's index (through the Beatty visit counters and
    // the history slots), so from the second solve of this precision and column count
    // each index's launches are captured once and replayed as a graph.
    auto cycle_body = [&](hipStream_t st) {
        ch.pre(st);
        ch.cycle_launches(st);
        ch.post(st);
    };
    Workspace::GraphSet *gset = nullptr, *gs = nullptr;
    if (h->opt.graphs && !h->timer.on && !w.arena) {
        gset = &graph_set(w, fp32 ? 1 : 0, k);
        if (gset->solves > 0 && !gset->direct) gs = gset;  // the first solve runs directly
    }
    while (ch.running()) {
        std::vector<int64_t> &vis = fp32 ? ch.c32->visits : ch.c64->visits;
        std::vector<int64_t> &tvis = fp32 ? ch.c32->tvisits : ch.c64->tvisits;
        const int cyc = ch.cyc;
        if (cyc >= kGraphMaxCycles) gs = nullptr;
        if (gs && cyc < (int)gs->cycles.size()) {
            const Workspace::CycleGraph &cg = gs->cycles[cyc];
            LAMG_HIP(hipGraphLaunch(cg.exec, s));
            vis = cg.visits_after;
            tvis = cg.tvisits_after;
            h->solve_bytes += cg.bytes;
            ++graph_cycles;
        } else if (gs) {
            // the capture runs the cycle's host side (visit counters, byte counts) without
            // executing its kernels: if it fails, that state goes back to before it
            const double b0 = h->solve_bytes;
            const std::vector<int64_t> vis0 = vis, tvis0 = tvis;
            hipGraphExec_t ex = capture_and_launch(h, s, cycle_body);
            if (ex) {
                gs->cycles.push_back(
                    Workspace::CycleGraph{ex, vis, tvis, h->solve_bytes - b0});
                ++graph_cycles;
            } else {
                gs->direct = true;
                gs = nullptr;
                h->solve_bytes = b0;
                vis = vis0;
                tvis = tvis0;
                cycle_body(s);
            }
        } else {
            cycle_body(s);
        }
        ch.read_back();
        LAMG_HIP(hipStreamSynchronize(s));
        ch.host();
    }
    cycles = ch.cycles;
    lamg_status st = ch.finish(relres, acf, hist0);
    if (gset) ++gset->solves;
    return st;
}

// Several solves in lockstep, each an FP32+IR chunk whose whole cycle runs in the coarse
// tail (tail_level 0): per cycle, every running solve's pre-cycle launches, then ONE tail
// launch holding every running solve's workgroups (one per column, each with its own
// descriptors, copy jobs and visit counters), then every solve's post-cycle launches, one
// synchronisation, and the host bookkeeping of each. Each solve computes exactly what it
// computes alone. The launch's records, descriptors and copy jobs are gathered into
// buffers of the first solve's workspace whenever the set of running solves changes.
void solve_lockstep(std::vector<Chunk *> &chs, hipStream_t s) {
    if (chs.empty()) return;
    Workspace &g = chs[0]->h->ws;
    Pool &gpool = g.arena ? *g.arena : *chs[0]->h->pool;
    std::vector<int> running_prev;
    int nwg = 0;
    size_t lds = 0;
    while (true) {
        std::vector<int> running;
        for (int i = 0; i < (int)chs.size(); ++i)
            if (chs[i]->running()) running.push_back(i);
        if (running.empty()) break;
        if (running != running_prev) {
            std::vector<char> recs;
            int64_t ndesc = 0, njobs = 0;
            std::vector<std::pair<const void *, size_t>> dsrc, jsrc;
            nwg = 0;
            lds = 0;
            for (int i : running) {
                Chunk &c = *chs[i];
                Workspace &w = c.h->ws;
                tail_wg_records<float>(w.plan32, 0, c.h->nlev, c.k, w.visits.p, recs, ndesc,
                                       njobs, dsrc, jsrc);
                nwg += c.k;
                lds = std::max(lds, w.plan32.lds_bytes);
            }
            const int64_t db = (int64_t)ndesc * (int64_t)tail_desc_bytes<float>();
            const int64_t jb = std::max<int64_t>(1, njobs * (int64_t)tail_copy_job_bytes());
            if (g.grp_recs.n < (int64_t)recs.size()) g.grp_recs.alloc(gpool, (int64_t)recs.size());
            if (g.grp_desc.n < db) g.grp_desc.alloc(gpool, db);
            if (g.grp_jobs.n < jb) g.grp_jobs.alloc(gpool, jb);
            g.grp_recs.upload(recs.data(), (int64_t)recs.size(), s);
            auto gather = [&](std::vector<std::pair<const void *, size_t>> &src, char *dst) {
                size_t off = 0;
                for (size_t i = 0; i < src.size();) {  // contiguous pieces go as one copy
                    const char *a = static_cast<const char *>(src[i].first);
                    size_t len = src[i].second, j = i + 1;
                    while (j < src.size() && static_cast<const char *>(src[j].first) == a + len) {
                        len += src[j].second;
                        ++j;
                    }
                    LAMG_HIP(hipMemcpyAsync(dst + off, a, len, hipMemcpyDeviceToDevice, s));
                    off += len;
                    i = j;
                }
            };
            gather(dsrc, g.grp_desc.p);
            gather(jsrc, g.grp_jobs.p);
            running_prev = running;
        }
        for (int i : running) {
            Chunk &c = *chs[i];
            c.pre(s);
            Cycle<float> &C = *c.c32;
            const double sz = 4.0;
            c.h->solve_bytes += tail_level_bytes<float>(C, 0);  // the grouped launch's share
            if (c.k > 1) {
                LevelVecs<float> &v0 = c.h->ws.lv32[0];
                Timed tm(c.h, LAMG_KERNEL_VECTOR, 1, 4.0 * c.k * c.n * sz, false);
                run_to_cols<float>(c.n, c.k, v0.x.p, v0.f.p, C.cx, C.cf, s);
            }
        }
        run_tail_group<float>(g.grp_recs.p, g.grp_desc.p, g.grp_jobs.p, nwg, lds, s);
        for (int i : running) {
            Chunk &c = *chs[i];
            if (c.k > 1) {
                Timed tm(c.h, LAMG_KERNEL_VECTOR, 1, 2.0 * c.k * c.n * 4.0, false);
                run_from_cols<float>(c.n, c.k, c.c32->cx, c.h->ws.lv32[0].x.p, s);
            }
            c.post(s);
            c.read_back();
        }
        LAMG_HIP(hipStreamSynchronize(s));
        for (int i : running) chs[i]->host();
    }
}

template <class T>
void profile_impl(lamg_handle *h, int level, int kernel, int k, int reps, double *sec,
                  double *bytes) {
    using P = Prec<T>;
    hipStream_t s = h->stream;
    Workspace &w = h->ws;
    std::vector<LevelVecs<T>> &lv = P::vecs(w);
    ensure_level_vecs<T>(h, k);
    Level &L = h->lev[level];
    const SolveOp &op = L.op;
    const bool fine = level == timed_level(h, k);
    const int64_t n = L.n;
    LevelVecs<T> &me = lv[level];
    run_fill<T>(me.x.p, n * k, T(1), s);
    run_fill<T>(me.f.p, n * k, T(1), s);
    LevelVecs<T> *cv = level + 1 < h->nlev ? &lv[level + 1] : nullptr;
    if (cv) {
        run_fill<T>(cv->x.p, h->lev[level + 1].n * k, T(1), s);
        run_fill<double>(me.mu.p, k, 1.0, s);
    }
    auto launch = [&]() {
        switch (kernel) {
            case LAMG_KERNEL_GS_COLOR:
                run_gs_color<T>(op, 0, P::v(op), P::dinv(op), me.f.p, me.x.p, k, s, fine);
                break;
            case LAMG_KERNEL_RESIDUAL:
                run_residual<T>(op, P::v(op), P::d(op), me.x.p, me.f.p, me.r.p, k, s, fine);
                break;
            case LAMG_KERNEL_RESTRICT:
                run_restrict<T>(op, P::rw(op), me.r.p, cv->f.p, k, s);
                break;
            default:
                run_prolong<T>(op, P::w0(op), P::w1(op), cv->x.p, me.mu.p, me.x.p, k, s);
                break;
        }
    };
    launch();  // warm-up
    hipEvent_t e0, e1;
    LAMG_HIP(hipEventCreate(&e0));
    LAMG_HIP(hipEventCreate(&e1));
    LAMG_HIP(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) launch();
    LAMG_HIP(hipEventRecord(e1, s));
    LAMG_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LAMG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *sec = (double)ms * 1e-3 / reps;
    const double sz = sizeof(T);
    if (kernel == LAMG_KERNEL_GS_COLOR)
        *bytes = bytes_gs_color(op, 0, k, sz);
    else if (kernel == LAMG_KERNEL_RESIDUAL)
        *bytes = bytes_residual(op, k, sz);
    else if (kernel == LAMG_KERNEL_RESTRICT)
        *bytes = bytes_restrict(op, k, sz);
    else
        *bytes = bytes_prolong(op, k, sz);
}

}  // namespace

void clear_graphs(Workspace &w) {
    for (Workspace::GraphSet &g : w.gsets)
        for (Workspace::CycleGraph &c : g.cycles)
            if (c.exec) (void)hipGraphExecDestroy(c.exec);
    w.gsets.clear();
}

thread_local LaunchEvents *t_launch_events = nullptr;

int KTimer::open(int kind, int prec, double b) {
    if (!on || kind < 0 || 2 * (recs.size() + 1) > ev.size()) return -1;
    recs.push_back(Rec{kind, prec, b});
    return (int)recs.size() - 1;
}

void KTimer::start(int max_launches, bool every_launch) {
    release();
    all = every_launch;
    for (auto &c : cnt) c[0] = c[1] = 0;
    for (auto &c : sec) c[0] = c[1] = 0.0;
    for (auto &c : bytes) c[0] = c[1] = 0.0;
    ev.assign(2 * (size_t)max_launches, nullptr);
    for (auto &e : ev) LAMG_HIP(hipEventCreate(&e));
    recs.clear();
    recs.reserve(max_launches);
    on = true;
}

void KTimer::stop() {
    on = false;
    for (size_t i = recs.size(); i-- > 0;)
        if (recs[i].kind >= 0) {
            LAMG_HIP(hipEventSynchronize(ev[2 * i + 1]));
            break;
        }
    for (size_t i = 0; i < recs.size(); ++i) {
        const Rec &r = recs[i];
        if (r.kind < 0) continue;
        float ms = 0.f;
        LAMG_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
        cnt[r.kind][r.prec] += 1;
        sec[r.kind][r.prec] += 1e-3 * (double)ms;
        bytes[r.kind][r.prec] += r.bytes;
    }
    release();
}

void KTimer::release() {
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    ev.clear();
    recs.clear();
}

lamg_status run_profile(lamg_handle *h, int level, int kernel, lamg_precision prec, int k,
                        int reps, double *sec, double *bytes) {
    if (level < 0 || level >= h->nlev || k < 1 || k > 32 || reps < 1 || kernel < 0 || kernel > 3)
        throw Error(LAMG_INVALID_ARG, "profile arguments");
    if (h->lev[level].coarsest && kernel != LAMG_KERNEL_RESIDUAL)
        throw Error(LAMG_INVALID_ARG, "kernel not run on the directly solved level");
    if (prec == LAMG_FP32_IR) {
        if (!h->opt.build_fp32) throw Error(LAMG_INVALID_ARG, "FP32 copies were not built");
        profile_impl<float>(h, level, kernel, k, reps, sec, bytes);
    } else {
        profile_impl<double>(h, level, kernel, k, reps, sec, bytes);
    }
    return LAMG_OK;
}

lamg_status run_solve(lamg_handle *h, const double *b, int nrhs, double tol, int max_cycles,
                      lamg_precision prec, double *phi, lamg_solve_info *info) {
    auto t0 = std::chrono::steady_clock::now();
    h->solve_bytes = 0.0;
    const bool fp32 = prec == LAMG_FP32_IR;
    if (fp32 && !h->opt.build_fp32) throw Error(LAMG_INVALID_ARG, "FP32 copies were not built");
    if (max_cycles <= 0) max_cycles = 300;
    const int64_t n = h->lev[0].n;
    lamg_status st = LAMG_OK;
    int32_t cyc_max = 0;
    double rel_max = 0.0, acf_max = 0.0;
    std::vector<double> hist0;
    int graph_cycles = 0;
    if (nrhs > 32) {
        // the columns are solved in chunks of 32 and each chunk checks its own columns before
        // writing; with several chunks every column is checked first, so a non-finite entry
        // in a later chunk leaves phi untouched too
        ensure_fine(h, 32);
        double bad = 0.0;
        run_count_nonfinite((int64_t)n * nrhs, b, h->ws.partial.p, h->ws.rel.p, h->stream);
        h->ws.rel.download(&bad, 1, h->stream);
        LAMG_HIP(hipStreamSynchronize(h->stream));
        if (bad != 0.0) throw Error(LAMG_INVALID_ARG, "right-hand side is not finite");
    }
    for (int c0 = 0; c0 < nrhs; c0 += 32) {
        int k = std::min(32, nrhs - c0);
        std::vector<double> rel(k), acf(k), hist;
        std::vector<int32_t> cyc(k);
        lamg_status s2 = solve_chunk(h, b + (int64_t)c0 * n, k, tol, max_cycles, fp32,
                                     phi + (int64_t)c0 * n, rel, cyc, acf, hist, graph_cycles);
        if (s2 != LAMG_OK) st = s2;
        if (c0 == 0) hist0 = hist;
        for (int c = 0; c < k; ++c) {
            cyc_max = std::max(cyc_max, cyc[c]);
            rel_max = std::max(rel_max, rel[c]);
            acf_max = std::max(acf_max, acf[c]);
            if (info && info->relres) info->relres[c0 + c] = rel[c];
            if (info && info->col_cycles) info->col_cycles[c0 + c] = cyc[c];
        }
    }
    if (info) {
        info->cycles = cyc_max;
        info->relres_max = rel_max;
        info->acf_max = acf_max;
        info->history_len = (int32_t)std::min<size_t>(hist0.size(), (size_t)max_cycles + 1);
        if (info->history)
            for (int i = 0; i < info->history_len; ++i) info->history[i] = hist0[i];
        info->graph_cycles = graph_cycles;
        info->bytes = h->solve_bytes;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return st;
}

// Fills a request's lamg_solve_info from its chunk's results.
static void fill_info(lamg_solve_info *info, int k, const std::vector<double> &rel,
                      const std::vector<int32_t> &cyc, const std::vector<double> &acf,
                      const std::vector<double> &hist0, int max_cycles, double bytes,
                      double seconds) {
    if (!info) return;
    info->cycles = 0;
    info->relres_max = 0.0;
    info->acf_max = 0.0;
    for (int c = 0; c < k; ++c) {
        info->cycles = std::max(info->cycles, cyc[c]);
        info->relres_max = std::max(info->relres_max, rel[c]);
        info->acf_max = std::max(info->acf_max, acf[c]);
        if (info->relres) info->relres[c] = rel[c];
        if (info->col_cycles) info->col_cycles[c] = cyc[c];
    }
    info->history_len = (int32_t)std::min<size_t>(hist0.size(), (size_t)max_cycles + 1);
    if (info->history)
        for (int i = 0; i < info->history_len; ++i) info->history[i] = hist0[i];
    info->graph_cycles = 0;
    info->bytes = bytes;
    info->seconds = seconds;
}

template <class F>
static lamg_status status_of(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        return e.status;
    } catch (const std::bad_alloc &) {
        return LAMG_OOM;
    }
}

lamg_status run_solve_group(int count, lamg_handle *const *hs, const double *const *bs,
                            const int32_t *nrhs, double tol, int max_cycles, lamg_precision prec,
                            double *const *phis, lamg_solve_info *infos, lamg_status *statuses,
                            hipStream_t stream) {
    auto t0 = std::chrono::steady_clock::now();
    if (max_cycles <= 0) max_cycles = 300;
    const bool fp32 = prec == LAMG_FP32_IR;
    std::vector<int> grouped;
    for (int r = 0; r < count; ++r) {
        lamg_handle *h = hs[r];
        h->stream = stream;
        h->pool->set_stream(stream);
        statuses[r] = LAMG_OK;
        const bool can = fp32 && h->opt.build_fp32 && nrhs[r] <= kTailMaxCols &&
                         tail_level(h, nrhs[r], true) == 0;
        if (!can)  // solved on its own, in order, before the group
            statuses[r] = status_of([&] {
                return run_solve(h, bs[r], nrhs[r], tol, max_cycles, prec, phis[r],
                                 infos ? &infos[r] : nullptr);
            });
        else
            grouped.push_back(r);
    }
    std::vector<Chunk> ch(grouped.size());
    std::vector<Chunk *> live;
    for (size_t i = 0; i < grouped.size(); ++i) {
        const int r = grouped[i];
        hs[r]->solve_bytes = 0.0;
        statuses[r] = status_of([&] {
            ch[i].begin(hs[r], bs[r], nrhs[r], tol, max_cycles, true, phis[r]);
            return LAMG_OK;
        });
        if (statuses[r] == LAMG_OK) live.push_back(&ch[i]);
    }
    solve_lockstep(live, stream);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (size_t i = 0; i < grouped.size(); ++i) {
        const int r = grouped[i];
        if (statuses[r] != LAMG_OK) continue;
        std::vector<double> rel, acf, hist0;
        statuses[r] = ch[i].finish(rel, acf, hist0);
        fill_info(infos ? &infos[r] : nullptr, ch[i].k, rel, ch[i].cycles, acf, hist0,
                  max_cycles, hs[r]->solve_bytes, secs);
    }
    for (int r = 0; r < count; ++r)
        if (statuses[r] != LAMG_OK) return statuses[r];
    return LAMG_OK;
}

int plan_tail_level(const lamg_handle *h) { return tail_level(h, 1, true); }
int plan_timed_level(const lamg_handle *h) { return timed_level(h, 1); }

}  // namespace lamg
