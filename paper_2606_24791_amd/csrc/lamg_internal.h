// Internal declarations of liblamg: hierarchy and workspace layout, device-memory
// ownership, and the kernel launchers shared by the host-side setup and solve code.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "lamg.h"

namespace lamg {

constexpr int kTV = 4;              // test vectors per level (fixed K = 4, Sec. 3.3)
constexpr int kTVSweeps = 3;        // relaxation sweeps per test vector (Sec. 2)
constexpr double kGuardQ = 2.5;     // energy-ratio guard bound, eq. (2.3)
constexpr double kTauSoc = 0.05;    // strength-of-connection threshold, eq. (3.1)
constexpr double kSnap = 0.01;      // caliber-2 snapping band around 0 and 1
constexpr int kMaxLevels = LAMG_MAX_LEVELS;
constexpr int kStallDirectMax = 1024;  // a non-coarsening level up to this size is solved directly
constexpr int kLongRow = 32;        // rows with more off-diagonals go to the block-per-row bin
constexpr int kBlock = 256;         // threads per block of every kernel
constexpr int kRedBlocksMax = 256;  // partial-sum blocks of a reduction
constexpr int kRedQMax = 14;        // quantities per reduction (4x4 normal equations + rhs)
// Largest number of partial-sum reads (doubles, over all blocks) that an update launch
// may spend on forming its per-column scalars itself.
constexpr int64_t kFuseTotalsMax = 1 << 15;
constexpr int kTVShortRow = 64;     // test-vector rows longer than this get a wave each
constexpr int kEllMaxWidth = 64;    // longest row of a level that gets an ELL copy
constexpr int kTailMaxCols = 32;  // workgroups (one per column) of one coarse-tail launch
constexpr int kGraphMaxNodes = 20000;  // longer cycles are launched kernel by kernel
constexpr int kGraphSets = 2;          // (precision, columns) pairs with cached graphs
constexpr int kGraphMaxCycles = 64;    // later cycles of a solve are launched kernel by kernel
constexpr int kChebColors = 32;      // smoother 1: levels with more colours use Chebyshev
constexpr int kChebDegree = 3;       // residual evaluations per Chebyshev sweep
constexpr double kChebRatio = 5.0;   // smoothed interval [lmax / kChebRatio, lmax]
constexpr int kBjBlock = 64;         // smoother 2: rows per block-Jacobi Gauss-Seidel block
constexpr int kElimMaxDegree = 4;   // eliminated nodes have at most this many neighbours
constexpr double kElimMinFrac = 0.1;  // an elimination level removes at least this share

// Error carried from the point of failure to the C-ABI boundary.
struct Error : std::runtime_error {
    lamg_status status;
    Error(lamg_status s, const std::string &what) : std::runtime_error(what), status(s) {}
};

#define LAMG_HIP(call)                                                                \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::lamg::Error(e_ == hipErrorOutOfMemory ? LAMG_OOM : LAMG_HIP_ERROR, \
                                std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

#define LAMG_LAUNCH_CHECK() LAMG_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// Device memory through the (optional) allocator hook
// ---------------------------------------------------------------------------

struct Allocator {
    lamg_alloc_fn alloc = nullptr;  // nullptr: hipMalloc
    lamg_free_fn free = nullptr;
    void *ctx = nullptr;
};
Allocator current_allocator();

// Every device allocation of a handle goes through its Pool, which counts bytes and
// releases everything on destruction.
class Pool {
  public:
    explicit Pool(Allocator a, hipStream_t s) : a_(a), s_(s) {}
    // An arena over `cap` bytes of device memory at `base` that the pool does not own:
    // get() hands out consecutive 256-byte-aligned pieces and throws
    // Error(LAMG_SCRATCH_TOO_SMALL) past the end; put() and the destructor free nothing.
    Pool(void *base, size_t cap, hipStream_t s)
        : s_(s), base_(static_cast<char *>(base)), cap_(cap) {}
    ~Pool();
    Pool(const Pool &) = delete;
    Pool &operator=(const Pool &) = delete;
    void *get(size_t bytes);  // throws Error(LAMG_OOM)
    void put(void *p);
    int64_t bytes() const { return bytes_; }
    int64_t peak() const { return peak_; }  // high-water mark of bytes()
    hipStream_t stream() const { return s_; }
    void set_stream(hipStream_t s) { s_ = s; }

  private:
    struct Blk {
        void *p;
        size_t bytes;
    };
    Allocator a_;
    hipStream_t s_;
    std::vector<Blk> blks_;
    int64_t bytes_ = 0;
    int64_t peak_ = 0;
    char *base_ = nullptr;  // arena mode
    size_t cap_ = 0;
};

// Typed device array owned by a Pool.
template <class T>
struct DArr {
    T *p = nullptr;
    int64_t n = 0;
    Pool *pool = nullptr;
    DArr() = default;
    DArr(const DArr &) = delete;
    DArr &operator=(const DArr &) = delete;
    DArr(DArr &&o) noexcept { *this = std::move(o); }
    DArr &operator=(DArr &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            pool = o.pool;
            o.p = nullptr;
            o.n = 0;
            o.pool = nullptr;
        }
        return *this;
    }
    ~DArr() { release(); }
    void alloc(Pool &pl, int64_t count) {
        release();
        pool = &pl;
        n = count;
        p = static_cast<T *>(pl.get(sizeof(T) * (size_t)(count > 0 ? count : 1)));
    }
    void release() {
        if (p && pool) pool->put(p);
        p = nullptr;
        n = 0;
    }
    void upload(const T *h, int64_t count, hipStream_t s) {
        if (count) LAMG_HIP(hipMemcpyAsync(p, h, sizeof(T) * (size_t)count, hipMemcpyHostToDevice, s));
    }
    void download(T *h, int64_t count, hipStream_t s) const {
        if (count) LAMG_HIP(hipMemcpyAsync(h, p, sizeof(T) * (size_t)count, hipMemcpyDeviceToHost, s));
    }
};

// ---------------------------------------------------------------------------
// Hierarchy
// ---------------------------------------------------------------------------

// Rows of one level in solve order. The solve numbering permutes the canonical nodes
// by (row class, colour, canonical index): class 0 = rows with <= kLongRow
// off-diagonals, class 1 = longer rows. Each (class, colour) block is contiguous, so a
// Gauss-Seidel colour pass reads a contiguous slice of the matrix.
struct SolveOp {
    int64_t n = 0, nnz_off = 0;
    int ncolors = 0;
    std::vector<int64_t> blk;      // (2*ncolors + 1) offsets: class 0 colours, then class 1 colours
    std::vector<int64_t> blk_nnz;  // off-diagonal entries before each blk offset
    DArr<int64_t> dblk;            // device copy of blk
    int lpr_short = 1;         // lanes per row of the short-row bin (k = 1)
    int max_short_len = 0;     // longest off-diagonal row; 0 if any row is in the long bin
    int max_len = 0;           // longest off-diagonal row
    DArr<int32_t> perm;        // solve index -> canonical index
    DArr<int32_t> io_perm;     // level 0: solve index -> the caller's node index (perm, composed
                               // with the input's renumbering when there is one)
    DArr<int32_t> rp, ci;      // off-diagonal CSR in solve numbering
    DArr<double> v64, d64, dinv64;
    DArr<float> v32, d32, dinv32;
    // interpolation from the next level, in both levels' solve numbering
    DArr<int32_t> p0, p1;
    DArr<double> w0_64, w1_64;
    DArr<float> w0_32, w1_32;
    // restriction P^T: coarse row -> (fine row, weight)
    int64_t nc = 0, nnz_r = 0;
    DArr<int32_t> rrp, rci, rlong;
    int64_t n_rlong = 0;
    int lpr_r = 1;
    DArr<double> rw64;
    DArr<float> rw32;
    // ELL copy of the off-diagonals (entry u of row i at u * n + i, padding: own index and
    // weight 0) for levels below 65536 rows whose rows have at most kEllMaxWidth entries,
    // read coalesced by the single-workgroup coarse-level kernel
    int ell_w = 0;
    DArr<int32_t> ell_ci;
    DArr<double> ell_v64;
    DArr<float> ell_v32;
    // block-Jacobi Gauss-Seidel (smoother 2), in the level's natural row order (block b =
    // rows [b kBjBlock, (b + 1) kBjBlock)): each row's solve index and its off-diagonal
    // entries whose column lies in its block (column as the position in the block, CSR order)
    int64_t bj_ni = 0;  // in-block entries
    DArr<int32_t> bj_rows, bj_irp;
    DArr<uint8_t> bj_iloc;
    DArr<double> bj_iv64;
    DArr<float> bj_iv32;
};

struct Level {
    int64_t n = 0, nnz = 0;  // canonical Laplacian size (diagonal included)
    bool coarsest = false;
    bool elim = false;  // elimination level: h_agg = coarse id of kept nodes, -1 on F
    bool cheb = false;        // smoothed by Chebyshev polynomials (smoother option 1)
    bool bjgs = false;        // smoothed by block-Jacobi Gauss-Seidel (smoother option 2)
    double cheb_lmax = 0.0;   // Gershgorin bound of the spectrum of D^{-1} L
    std::vector<int32_t> h_rp, h_ci;  // canonical pattern on the host
    DArr<int32_t> rp, ci;             // canonical CSR on the device
    DArr<double> val;
    int ncolors = 0;
    std::vector<int32_t> h_color;
    DArr<int32_t> color;
    DArr<uint8_t> strong;
    DArr<double> X, aff, mom;
    std::vector<int32_t> h_seed, h_agg;
    DArr<int32_t> p0, p1;  // canonical interpolation (coarse ids canonical)
    DArr<double> w0, w1;
    int64_t nc = 0, n_cal2 = 0;
    double gamma = 1.0, tau = 0.0;
    SolveOp op;
    DArr<double> Z;  // coarsest: the pseudo-inverse L^+ = (L + 11^T/n)^{-1} - 11^T/n, n x n
};

// Per-level cycle vectors of one precision (n_l * k elements each).
template <class T>
struct LevelVecs {
    DArr<T> x, f, r, rho, x1, rho1;
    DArr<double> mu, alpha;  // k per level
};

// Device-side plan of a coarse tail for one precision and column count.
struct TailPlan {
    const void *desc = nullptr;      // level descriptors (global arrays)
    const void *lds_desc = nullptr;  // the launch's descriptors (LDS-resident levels: offsets)
    const void *jobs = nullptr;      // global -> LDS copy jobs
    // the same for one workgroup per column (solves of several columns; null unless the
    // workspace holds several)
    const void *lds_desc_cols = nullptr;
    const void *jobs_cols = nullptr;
    int kmax = 0;                    // columns the workspace vectors hold
    int njobs = 0;
    int l_lds = 0;         // first LDS-resident level (nlev: none)
    int l_x = -1;          // level whose iterate alone is LDS-resident (-1: none)
    size_t lds_bytes = 0;  // dynamic LDS of the launch
};
// Cached solve workspace (grown on demand, per precision).
struct Workspace {
    // Non-null: the workspace of one allocation-free solve, laid out in this arena (the
    // fixed scratch array); its host mirrors are then pageable and no HIP graph is made.
    Pool *arena = nullptr;
    std::vector<double> h_rel_v;
    std::vector<int32_t> h_mask_v;
    int kf = 0;  // columns of the finest FP64 state
    DArr<double> phi, b, r, b0, tmp, hphi, hr;  // n*k each; history holds 4 slots
    DArr<double> nb, rel, scale, alpha_f, mean;  // per column
    DArr<double> partial;                        // reduction scratch
    DArr<int32_t> mask;                          // per column
    double *h_rel = nullptr;                     // pinned host mirror (k)
    int32_t *h_mask = nullptr;
    int k64 = 0, k32 = 0;
    std::vector<LevelVecs<double>> lv64;
    std::vector<LevelVecs<float>> lv32;
    DArr<char> tail64, tail32;  // coarse-tail level descriptors per precision
    DArr<char> tlds64, tlds32, tjobs64, tjobs32;  // LDS-resident tail levels
    TailPlan plan64, plan32;
    // the tail's top-level iterate and right-hand side column by column (solves of several
    // columns; with one the layout is the ordinary one)
    DArr<double> tcx64, tcf64;
    DArr<float> tcx32, tcf32;
    DArr<char> tldsc64, tldsc32, tjobsc64, tjobsc32;  // the per-column workgroups' plans
    DArr<int64_t> visits;       // coarse-tail visit counters (per column and level)
    // HIP graphs of whole cycles, replayed in later solves with the same precision and column
    // count: the launch sequence of the i-th cycle of a solve depends only on i (the visit
    // counters start from zero in every solve; column freezing changes data, not launches)
    struct CycleGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<int64_t> visits_after;   // the host visit counters after the cycle
        std::vector<int64_t> tvisits_after;  // the host mirror of the tail's counters after it
        double bytes = 0.0;                  // algorithmic bytes of the cycle's launches
    };
    struct GraphSet {
        int prec = 0, k = 0;
        int solves = 0;          // completed solves with this precision and column count
        bool direct = false;     // a cycle exceeded kGraphMaxNodes or capture failed
        std::vector<CycleGraph> cycles;
    };
    std::vector<GraphSet> gsets;  // least recently used first
    hipStream_t cap_stream = nullptr;
    // grouped coarse-tail launches led by this workspace's solve: workgroup records and the
    // launch's combined descriptors and copy jobs
    DArr<char> grp_recs, grp_desc, grp_jobs;
};
// Destroys the cached cycle graphs (their kernel arguments point into the workspace).
void clear_graphs(Workspace &w);

// In-situ launch timer: a pair of HIP events per timed launch, recorded by the launch
// itself (hipExtLaunchKernel takes the dispatch's own start and end timestamps), so the
// elapsed time is the kernel's execution time without stream-marker overhead.
struct KTimer {
    static constexpr int kKinds = 9;
    bool on = false;
    bool all = false;  // every launch of every level (else the timed level, the tail and the
                       // FP64 outer residual)
    std::vector<hipEvent_t> ev;  // 2 per launch
    struct Rec {
        int kind, prec;  // prec 0: FP64, 1: FP32; kind -1: nothing was launched
        double bytes;
    };
    std::vector<Rec> recs;
    int64_t cnt[kKinds][2] = {};
    double sec[kKinds][2] = {}, bytes[kKinds][2] = {};
    // Reserves an event pair; returns its index or -1 (timer off or full).
    int open(int kind, int prec, double b);
    void start(int max_launches, bool every_launch);
    void stop();
    void release();
};

// Events that the launch helpers attach to the kernels they launch while set (the first
// launch records `start`, every launch records `stop`). Set by the solve on its own thread.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool started = false;
};
extern thread_local LaunchEvents *t_launch_events;

template <class... KArgs, class... Args>
inline void launch_kernel(void (*kern)(KArgs...), dim3 grid, dim3 block, uint32_t shmem,
                          hipStream_t s, Args... args) {
    LaunchEvents *le = t_launch_events;
    if (!le) {
        hipLaunchKernelGGL(kern, grid, block, shmem, s, args...);
        return;
    }
    hipEvent_t e0 = le->started ? nullptr : le->start;
    le->started = true;
    hipExtLaunchKernelGGL(kern, grid, block, shmem, s, e0, le->stop, 0u, args...);
}

}  // namespace lamg

struct lamg_handle {
    int device = 0;  // the HIP device the hierarchy lives on
    lamg::Allocator alloc;
    std::unique_ptr<lamg::Pool> pool;
    hipStream_t stream = nullptr;
    lamg_options opt{};
    int nlev = 0;
    std::vector<lamg::Level> lev;
    lamg::Workspace ws;
    lamg::KTimer timer;
    double solve_bytes = 0.0;  // algorithmic bytes of the current solve's launches
    double setup_seconds = 0.0;
    double setup_phase[LAMG_SETUP_PHASES] = {};  // seconds per lamg_setup_phase
    bool reordered = false;                      // the input was renumbered (option reorder)
    ~lamg_handle();
};

namespace lamg {

// ---------------------------------------------------------------------------
// Kernel launchers (setup_kernels.hip): canonical arithmetic, bit-reproducible
// ---------------------------------------------------------------------------
void launch_laplacian(int64_t n, const int32_t *arp, const int32_t *aci, const double *aw,
                      const int32_t *lrp, int32_t *lci, double *lv, hipStream_t s);
void launch_strong(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double tau,
                   int enable_veto, uint8_t *strong, hipStream_t s);
void launch_tv_init(int64_t n, uint64_t seed, int level, double *X, hipStream_t s);
void launch_tv_sweep_color(int64_t cnt, const int32_t *rows, const int32_t *rp, const int32_t *ci,
                           const double *v, double *X, hipStream_t s);
// the same relaxation for rows with more than kTVShortRow stored entries (one wave per row)
void launch_tv_sweep_long(int64_t cnt, const int32_t *rows, const int32_t *rp, const int32_t *ci,
                          const double *v, double *X, hipStream_t s);
void launch_affinity(int64_t n, const int32_t *rp, const int32_t *ci, const double *X,
                     double *sigma_tmp, double *aff, hipStream_t s);
void launch_moments(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    const double *X, double *mom, hipStream_t s);
void launch_interp(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
                   const double *X, const int32_t *seed, const int32_t *agg, const int32_t *aggseed,
                   int enable_caliber2, double snap, int32_t *p0, double *w0, int32_t *p1,
                   double *w1, hipStream_t s);
// Galerkin operator; allocates the coarse CSR in `pool`. Returns coarse nnz.
int64_t galerkin(Pool &pool, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                 const double *v, int64_t nc, const int32_t *p0, const double *w0,
                 const int32_t *p1, const double *w1, DArr<int32_t> &crp, DArr<int32_t> &cci,
                 DArr<double> &cv, hipStream_t s);
// Exact Schur complement onto the kept nodes of an elimination set (cid: coarse id or -1),
// canonical CSR, bit-reproducible (eq. (2.1)).
int64_t schur(Pool &pool, int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const int32_t *cid, int64_t nc, DArr<int32_t> &crp, DArr<int32_t> &cci,
              DArr<double> &cv, hipStream_t s);
// q[u] = (sum_j |L_uj|, CSR order from +0.0) / L_uu: the Gershgorin row bound of D^{-1} L
void launch_gershgorin_rows(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                            double *q, hipStream_t s);
// d[u] = the stored diagonal of row u
void launch_diag(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *d,
                 hipStream_t s);
// Z = L^+ = (L + 11^T/n)^{-1} - 11^T/n (Gauss-Jordan on the SPD matrix, no pivoting).
void coarsest_inverse(Pool &pool, int64_t n, const int32_t *rp, const int32_t *ci,
                      const double *v, double *Z, hipStream_t s);

// Solve-layout builders
void launch_permute_csr(int64_t n, const int32_t *perm, const int32_t *iperm, const int32_t *crp,
                        const int32_t *cci, const double *cv, const int32_t *srp, int32_t *sci,
                        double *sv64, float *sv32, double *d64, double *dinv64, float *d32,
                        float *dinv32, hipStream_t s);
void launch_cast_f32(int64_t n, const double *src, float *dst, hipStream_t s);
void launch_build_ell(int64_t n, int w, const int32_t *rp, const int32_t *ci, const double *v64,
                      const float *v32, int32_t *eci, double *ev64, float *ev32, hipStream_t s);

// ---------------------------------------------------------------------------
// Cycle launchers (cycle_kernels.hip), T = double or float
// ---------------------------------------------------------------------------
template <class T>
void run_gs(const SolveOp &op, const T *v, const T *dinv, const T *f, T *x, int k, int sweeps,
            hipStream_t s, bool fine);
template <class T>
void run_gs_color(const SolveOp &op, int c, const T *v, const T *dinv, const T *f, T *x, int k,
                  hipStream_t s, bool fine);
// With x_copy / r_copy: also x_copy = x and r_copy = r (same launch).
template <class T>
void run_residual(const SolveOp &op, const T *v, const T *d, const T *x, const T *f, T *r, int k,
                  hipStream_t s, bool fine, T *x_copy = nullptr, T *r_copy = nullptr);
// r = f - L x on the rows of colour c only (both row classes).
template <class T>
void run_residual_color(const SolveOp &op, int c, const T *v, const T *d, const T *x, const T *f,
                        T *r, int k, hipStream_t s, bool fine);
// One Chebyshev sweep (kChebDegree residual evaluations) on L x = f; dvec (n*k) is work space.
template <class T>
void run_cheb_sweep(const SolveOp &op, double lmax, const T *v, const T *d, const T *dinv,
                    const T *f, T *x, T *dvec, int k, hipStream_t s, bool fine);
// One block-Jacobi Gauss-Seidel sweep on L x = f (blocks of kBjBlock rows in the natural
// order); r (n*k) is work space, the residual at the sweep's start.
template <class T>
void run_bjgs_sweep(const SolveOp &op, const T *v, const T *d, const T *dinv, const T *f, T *x,
                    T *r, int k, hipStream_t s, bool fine);
// x += e_c on the kept rows of an elimination level (its one-entry-per-row P^T).
template <class T>
void run_inject_add(const SolveOp &op, const T *ec, T *x, int k, hipStream_t s);
// With zero_xc: also zero_xc = 0 on the coarse rows (same launch).
template <class T>
void run_restrict(const SolveOp &op, const T *rw, const T *r, T *fc, int k, hipStream_t s,
                  T *zero_xc = nullptr);
// mu = <e_c, f_c> / <e_c, f_c - rho> per column, then x += mu P e_c. Two launches when
// every block of the update can afford to add the partial sums itself, else three (the
// per-column scalars formed once into `scal`, k doubles); the arithmetic is the same.
template <class T>
void run_mu_prolong(const SolveOp &op, const T *w0, const T *w1, int64_t nc, const T *ec,
                    const T *fc, const T *rho, int k, double *partial, double *scal, T *x,
                    hipStream_t s);
// Two-iterate recombination (two or three launches, as above); with keep, (e1, rho1) = the
// recombined pair.
template <class T>
void run_rc2_keep(int64_t n, T *e, T *rho, T *e1, T *rho1, int k, double *partial,
                  double *scal, bool keep, hipStream_t s);
template <class T>
void run_prolong(const SolveOp &op, const T *w0, const T *w1, const T *ec, const double *mu,
                 T *x, int k, hipStream_t s);
template <class T>
void run_fill(T *x, int64_t count, T value, hipStream_t s);
template <class T>
void run_copy(T *dst, const T *src, int64_t count, hipStream_t s);
template <class T>
void run_mu(int64_t n, const T *e, const T *f, const T *rho, int k, double *partial, double *mu,
            hipStream_t s);
template <class T>
void run_rc2(int64_t n, T *e, T *rho, const T *e1, const T *rho1, int k, double *partial,
             double *alpha, hipStream_t s);
template <class T>
void run_coarsest(int64_t n, const double *Z, const T *f, T *y, int k, hipStream_t s);

// Coarse tail (tail_kernel.hip)
template <class T>
size_t tail_desc_bytes();
template <class T>
void tail_fill_desc(void *host_buf, int l, const Level &L, const SolveOp &op, const int64_t *d_blk,
                    const T *v, const T *d, const T *dinv, const T *w0, const T *w1, const T *rw,
                    const T *ev, T *x, T *f, T *r, T *rho, T *x1, T *rho1);
template <class T>
int tail_lds_plan(const std::vector<Level> &lev, int l0, int k, const void *host_desc,
                  std::vector<char> &lds_desc, std::vector<char> &jobs, size_t &lds_bytes,
                  int &l_x);
size_t tail_copy_job_bytes();
template <class T>
void run_tail(const TailPlan &tp, int l0, int nlev, int k, int64_t *d_visits, hipStream_t s);
// Grouped launches (several requests in one launch): per-workgroup records, with offsets
// into the launch's combined descriptor and copy-job arrays (tail_desc_bytes<T>() and
// tail_copy_job_bytes() per entry).
size_t tail_wg_bytes();
template <class T>
void tail_wg_records(const TailPlan &tp, int l0, int nlev, int k, int64_t *d_visits,
                     std::vector<char> &recs, int64_t &ndesc, int64_t &njobs_total,
                     std::vector<std::pair<const void *, size_t>> &desc_src,
                     std::vector<std::pair<const void *, size_t>> &jobs_src);
template <class T>
void run_tail_group(const void *wgs, const void *descs, const void *jobs, int nwg,
                    size_t lds_bytes, hipStream_t s);
// n x k row-interleaved (x, f) -> column by column (cx, cf), and back for x.
template <class T>
void run_to_cols(int64_t n, int k, const T *x, const T *f, T *cx, T *cf, hipStream_t s);
template <class T>
void run_from_cols(int64_t n, int k, const T *cx, T *x, hipStream_t s);
void run_zero_i64(int64_t *p, int64_t n, hipStream_t s);

// Finest-level FP64 helpers
void run_gather_cols(int64_t n, int k, const int32_t *perm, const double *src_colmajor,
                     double *dst, hipStream_t s);
void run_scatter_cols(int64_t n, int k, const int32_t *perm, const double *src, const int32_t *mask,
                      double *dst_colmajor, hipStream_t s);
void run_colsum(int64_t n, int k, const double *x, double *partial, double *out, double scale,
                hipStream_t s);  // out[c] = scale * sum_i x[i,c]
void run_sub_col(int64_t n, int k, double *x, const double *m, hipStream_t s);  // x[:,c] -= m[c]
void run_norm2(int64_t n, int k, const double *x, double *partial, double *out, hipStream_t s);
// out[0] = number of entries of x[0, n) that are NaN or infinite
void run_count_nonfinite(int64_t n, const double *x, double *partial, double *out, hipStream_t s);
void run_maxabs(int64_t n, int k, const double *x, double *partial, double *out, hipStream_t s);
void run_relres(int64_t n, int k, const double *r, const double *nb, double *partial, double *out,
                hipStream_t s);
// The relative residual of run_relres and, from the same pass, max |r| per column.
void run_relres_maxabs(int64_t n, int k, const double *r, const double *nb, double *partial,
                       double *rel, double *maxabs, hipStream_t s);
// Fine-level recombination over m history pairs (Sec. 2, "Cycle and acceleration"); the
// recombined (phi, r) is also saved in history slot `slot`.
void run_recombine_fine(int64_t n, int k, int m, double *phi, double *r, double *hphi, double *hr,
                        int slot, double *partial, double *alpha, hipStream_t s);
void run_to_f32_scaled(int64_t n, int k, const double *r, const double *scale, float *dst,
                       float *zero_x, hipStream_t s);  // dst = r / scale[c]; zero_x = 0
void run_add_scaled_f32(int64_t n, int k, const float *e, const double *scale, double *phi,
                        hipStream_t s);  // phi += scale[c] * e
void run_zero_cols(int64_t n, int k, const int32_t *zero_mask, double *x, hipStream_t s);

// Device address of the allocation-free entry point's scratch array on `device` (resolved
// once per device, that device current) and its size in bytes.
void *noalloc_scratch(int device);
size_t noalloc_scratch_bytes();

}  // namespace lamg
