/*
 * lamg.h -- C ABI of the MI355X (gfx950) LAMG+ Laplacian solver library (liblamg.so).
 *
 * Solves the compatible singular system of a connected weighted undirected graph
 *     L phi = b,   1^T phi = 0,   1^T b = 0                      (paper eq. (1.1))
 * with L = D - W its graph Laplacian, by the LAMG+ aggregation multigrid method
 * (Livne, "LAMG+: A Robust Lean Algebraic Multigrid Solver for Graph Laplacians"):
 * a hierarchy of caliber-1 aggregates chosen by test-vector affinity (eq. (2.2)) under
 * the energy-ratio guard (eq. (2.3)) and the strength-of-connection veto (eq. (3.1)),
 * selective caliber-2 interpolation (Sec. 3.2, eq. (A.7)), Galerkin coarse operators,
 * and a gamma-cycle (eq. (2.4)) with Gauss-Seidel relaxation, energy correction and
 * iterate recombination (Sec. 2, "Cycle and acceleration").
 *
 * Conventions for every call:
 *  - All integers are signed; n < 2^31 and stored-entry counts < 2^31.
 *  - "device" pointers are HIP device memory on the current device; "host" pointers are
 *    ordinary process memory. Nothing passed in is retained after a call returns,
 *    unless stated. The library never frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream). All device work of a
 *    call is ordered on that stream. Calls that return results to the host synchronise
 *    that stream before returning.
 *  - One handle may be used by one stream/thread at a time; different handles are
 *    independent.
 *  - Every call returns a lamg_status; on error nothing is leaked and output handles are
 *    set to NULL. lamg_status_string() names each code.
 */
#ifndef LAMG_H
#define LAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LAMG_OK = 0,
    LAMG_INVALID_ARG = 1,        /* NULL pointer, n < 1, bad sizes, unsorted/out-of-range columns */
    LAMG_NOT_SYMMETRIC = 2,      /* adjacency structure or weights not symmetric */
    LAMG_SELF_LOOP = 3,          /* a stored diagonal entry in the adjacency */
    LAMG_BAD_WEIGHT = 4,         /* weight <= 0, NaN or infinite (weights must be positive) */
    LAMG_DISCONNECTED = 5,       /* the graph is not connected */
    LAMG_OOM = 6,                /* device (or host) allocation failed; nothing leaked */
    LAMG_COARSENING_STALLED = 7, /* a level larger than 1024 nodes did not coarsen */
    LAMG_NOT_CONVERGED = 8,      /* max_cycles reached; phi and residuals are still written */
    LAMG_HIP_ERROR = 9,          /* a HIP runtime call failed (no device, launch failure, ...) */
    LAMG_UNAVAILABLE = 10,       /* requested data was not kept (see keep_setup_data) */
    LAMG_SCRATCH_TOO_SMALL = 11  /* lamg_solve_noalloc: the solve's workspace does not fit
                                    the fixed scratch (LAMG_NOALLOC_SCRATCH_BYTES) */
} lamg_status;

typedef enum { LAMG_MEM_HOST = 0, LAMG_MEM_DEVICE = 1 } lamg_memory;

typedef enum {
    LAMG_FP64 = 0,   /* every cycle in FP64 */
    LAMG_FP32_IR = 1 /* FP32 cycles as the preconditioner of an FP64 iterative refinement:
                        outer residual, recombination, projection and the coarsest solve
                        stay in FP64 */
} lamg_precision;

/* Input graph: the weighted ADJACENCY W (not the Laplacian) in CSR form, both directions
 * of every undirected edge stored, no diagonal, columns strictly ascending in each row
 * (unsorted rows are rejected with LAMG_INVALID_ARG). Weights must be positive and
 * finite, and w_uv == w_vu exactly. Arrays live in `mem`. */
typedef struct {
    int64_t n;              /* nodes */
    int64_t nnz;            /* stored adjacency entries = 2 * edges */
    const int32_t *row_ptr; /* n + 1 entries, row_ptr[0] = 0, row_ptr[n] = nnz */
    const int32_t *col_idx; /* nnz entries */
    const double *weight;   /* nnz entries */
    int32_t mem;            /* lamg_memory of the three arrays */
} lamg_graph;

/* Setup options. Fill with lamg_default_options() and override fields. The defaults are
 * the paper's parameter-free constants: K = 4 test vectors with 3 Gauss-Seidel sweeps
 * (Sec. 2, Sec. 3.3), guard Q = 2.5 (eq. (2.3)), veto tau = 0.05 (eq. (3.1)), caliber-2
 * on (Sec. 3.2). */
typedef struct {
    uint64_t seed;           /* seed of the counter-based test-vector generator (default 1) */
    int32_t n_direct;        /* levels with n <= n_direct are solved directly (default 512, max 1024) */
    int32_t enable_veto;     /* strength-of-connection veto (default 1) */
    int32_t enable_caliber2; /* selective caliber-2 interpolation (default 1) */
    int32_t kappa;           /* finest-level recombination history, 0..4 (default 4) */
    int32_t build_fp32;      /* also build FP32 copies of every level for LAMG_FP32_IR (default 1) */
    int32_t keep_setup_data; /* keep canonical operators, colours, strong flags, test vectors,
                                affinities, moments and aggregates for lamg_export_level (default 0) */
    int32_t tail_rows;       /* levels below the finest with at most this many nodes run their
                                whole cycle in one launch per visit, one workgroup per
                                right-hand-side column, together with the levels right above
                                them (below 65536 nodes) whose many colours of few rows make
                                one workgroup clearly cheaper than separate kernels (default
                                2500; 0 = every step is its own kernel). Applies to solves of
                                at most 32 columns. Changes only how the cycle is executed,
                                not what it computes. */
    int32_t elimination;     /* low-degree elimination levels (Sec. 2, "Low-degree elimination",
                                eq. (2.1)); default 1 (0: aggregation only). Before each aggregation step a
                                maximal independent set F of the nodes with at most 4
                                neighbours (greedy in natural order) is eliminated exactly --
                                coarse operator = Schur complement onto the other nodes, F rows
                                recomputed from them in the cycle, cycle index 1 -- provided F
                                holds at least a tenth of the level's nodes. Elimination and
                                aggregation levels alternate. */
    int32_t smoother;        /* 0 (default): multicolour Gauss-Seidel on every level. 1: levels
                                with more than 32 colours (the dense coarse levels of power-law
                                graphs, where a Gauss-Seidel sweep is hundreds of dependent
                                colour passes) are smoothed instead by Chebyshev polynomials in
                                the Jacobi-scaled operator D^{-1} L -- the polynomial substitute
                                for Gauss-Seidel named in Sec. 5 -- of degree 3 on
                                [lmax / 5, lmax], lmax = the Gershgorin bound of D^{-1} L; one
                                polynomial per Gauss-Seidel sweep it replaces. 2: the same
                                levels are smoothed instead by block-Jacobi Gauss-Seidel, the
                                other substitute Sec. 5 names: the rows in blocks of 64 in
                                their natural order, a Gauss-Seidel sweep in row order inside
                                each block, the entries of other blocks read at their values
                                from the start of the sweep; one such sweep per Gauss-Seidel
                                sweep it replaces. */
    int32_t graphs;          /* 1: from the second solve with the same precision and column
                                count, each cycle's launch sequence (which depends only on the
                                cycle's index within the solve) is captured once as a HIP graph
                                on a stream of the handle and replayed on the caller's stream;
                                cycles of more than 20000 launches, cycles after the 64th, and
                                solves timed by lamg_timing_start run as separate launches.
                                Graphs of two (precision, columns) pairs are kept; a solve that
                                enlarges the handle's vectors drops them. Pays off only where
                                launch latency dominates (systems of a few thousand rows).
                                0 (default): never. Changes only how the cycle is launched,
                                not what it computes. */
    int32_t tail_finest;     /* FP32+IR solves of a graph whose finest level has at most this
                                many nodes (and whose other levels all run in the coarse tail)
                                run the finest level in the coarse tail too: each cycle is then
                                one launch, and lamg_solve_group can make the launches of
                                several such solves one. 0 (default): never; at most 65535.
                                Changes only how the cycle is executed, not what it computes. */
    int32_t reorder;         /* 1: the input graph is renumbered before the setup by the reverse
                                Cuthill-McKee order (the reordering for cache locality of
                                Sec. 4.2), self-gated: only if it at least halves the mean index
                                distance |u - v| over the edges. Start node of each component
                                (taken in the order of their smallest node) by the George-Liu
                                iteration from its node of least degree, neighbours appended by
                                increasing degree, ties by smallest index; the sequence then
                                reversed. Levels, colourings and exports are in the renumbered
                                order; solves take b and return phi in the caller's. 0
                                (default): no renumbering. */
} lamg_options;

#define LAMG_MAX_LEVELS 64
#define LAMG_SETUP_PHASES 9

/* Phases of lamg_setup timed in lamg_hier_info.setup_phase_seconds (host wall time; each
 * phase ends with its device work complete). */
typedef enum {
    LAMG_SETUP_INPUT = 0,       /* input checks, the Laplacian of level 0 */
    LAMG_SETUP_COLOR = 1,       /* greedy colourings (Sec. 2 "Relaxation" reading) */
    LAMG_SETUP_LEVEL = 2,       /* veto, test vectors, affinities, moments (and their copies
                                   to the host for aggregation) */
    LAMG_SETUP_AGGREGATE = 3,   /* the greedy aggregation pass (host) */
    LAMG_SETUP_INTERP = 4,      /* caliber-1/caliber-2 interpolation weights */
    LAMG_SETUP_ELIMINATE = 5,   /* elimination sets and Schur complements */
    LAMG_SETUP_GALERKIN = 6,    /* Galerkin coarse operators (and their copy to the host) */
    LAMG_SETUP_COARSEST = 7,    /* pseudo-inverse of the directly solved level */
    LAMG_SETUP_LAYOUT = 8       /* solve layout: colour-permuted operators, transfers, ELL */
} lamg_setup_phase;

/* Per-level description of a hierarchy. */
typedef struct {
    int32_t levels;                      /* number of levels; the last is solved directly */
    int64_t n[LAMG_MAX_LEVELS];          /* nodes per level */
    int64_t nnz[LAMG_MAX_LEVELS];        /* stored Laplacian entries per level (diagonal included) */
    int32_t ncolors[LAMG_MAX_LEVELS];    /* colours of the level's greedy colouring (0 on the last) */
    int64_t n_caliber2[LAMG_MAX_LEVELS]; /* interpolation rows with two parents */
    double gamma[LAMG_MAX_LEVELS];       /* cycle index of the level (eq. (2.4)) */
    double tau[LAMG_MAX_LEVELS];         /* edge coarsening ratio |E_{l+1}|/|E_l| */
    int64_t bytes_device;                /* device bytes held by the handle (hierarchy + cached workspace) */
    double op_complexity;                /* sum_l nnz_l / nnz_0 */
    double setup_seconds;                /* wall time of lamg_setup */
    int64_t bytes_peak;                  /* most device bytes the handle has held at once
                                            (setup temporaries included) */
    int32_t elim[LAMG_MAX_LEVELS];       /* 1: elimination level (its aggregate export holds the
                                            coarse id of each kept node and -1 on F) */
    int32_t tail_level;                  /* first level whose cycle runs in the coarse-tail
                                            kernel in a 1-column FP32+IR solve (-1: none; FP64
                                            cycles never run the finest level there) */
    int32_t timed_level;                 /* level whose per-step kernels the in-situ timer
                                            records in a 1-column solve (the finest
                                            aggregation level unless that one runs in the
                                            coarse tail; then 0) */
    int32_t cheb[LAMG_MAX_LEVELS];       /* 1: smoothed by Chebyshev polynomials (smoother 1) */
    double cheb_lmax[LAMG_MAX_LEVELS];   /* their Gershgorin bound of D^{-1} L (0 otherwise) */
    double setup_phase_seconds[LAMG_SETUP_PHASES]; /* wall time of lamg_setup by phase, summed
                                                       over the levels (lamg_setup_phase) */
    int32_t bjgs[LAMG_MAX_LEVELS];       /* 1: smoothed by block-Jacobi Gauss-Seidel (smoother 2) */
    int32_t reordered;                   /* 1: the input was renumbered (option reorder) */
} lamg_hier_info;

/* Solve statistics. The caller may point the array fields at host arrays (or leave them
 * NULL): relres[nrhs], cycles[nrhs], history[M + 1] with M = max_cycles if max_cycles > 0,
 * else 300 (column 0's relative residual after each cycle, history[0] = 1; at most
 * M + 1 entries are written, history_len of them). */
typedef struct {
    int32_t cycles;        /* cycles (outer refinement steps for FP32_IR) run, max over columns */
    double relres_max;     /* max over columns of the final ||b - L phi|| / ||b|| (true residual) */
    double acf_max;        /* max over columns of the asymptotic convergence factor (geometric
                              mean of the last <= 5 per-cycle residual reductions) */
    double seconds;        /* wall time of the call */
    double *relres;        /* optional [nrhs] */
    int32_t *col_cycles;   /* optional [nrhs] */
    double *history;       /* optional [(max_cycles > 0 ? max_cycles : 300) + 1] */
    int32_t history_len;   /* written: entries of history filled */
    int32_t graph_cycles;  /* written: cycles launched as HIP graphs (captured in this call or
                              replayed), summed over the call's 32-column chunks */
    double bytes;          /* written: algorithmic bytes of every kernel launch of the call --
                              compulsory traffic only (each matrix index and value, row pointer,
                              diagonal and vector element a launch reads or writes, once), the
                              figures lamg_timing_get reports per kernel kind */
} lamg_solve_info;

/* One level of the hierarchy copied to host buffers (parity dumps). Any pointer may be
 * NULL to skip it. Sizes: n+1 for row_ptr, nnz for col_idx/val/strong/affinity, n for
 * color/seed/aggregate/p0/p1/w0/w1, 4n for x (node-major, x[u*4+k]), 9n for moments
 * (s0, s1[4], s2[4] per node). Everything but row_ptr/col_idx/val is absent on the last
 * (directly solved) level; an elimination level has only row_ptr/col_idx/val and
 * aggregate (coarse id of each kept node, -1 on the eliminated set F). */
typedef struct {
    int32_t *row_ptr;
    int32_t *col_idx;
    double *val;        /* canonical L_l: ascending columns, diagonal in place */
    int32_t *color;     /* greedy colour per node */
    uint8_t *strong;    /* 1 if the entry may carry aggregation (veto, eq. (3.1)) */
    double *x;          /* test vectors after the relaxation sweeps */
    double *affinity;   /* c_uv per stored entry (eq. (2.2)); 0 on the diagonal */
    double *moments;    /* guard moments (App. B) */
    int32_t *seed;      /* seed node of each node's aggregate (itself for seeds) */
    int32_t *aggregate; /* coarse id A(u) */
    int32_t *p0;        /* first interpolation parent (coarse id) */
    int32_t *p1;        /* second parent or -1 */
    double *w0;         /* weight of p0 */
    double *w1;         /* weight of p1 (0 if none) */
} lamg_level_export;

typedef struct lamg_handle lamg_handle;

/* Optional device allocator hook used for every device allocation of the library
 * (default: hipMalloc/hipFree). alloc returns NULL on failure, which surfaces as
 * LAMG_OOM. Set before creating handles; a handle frees with the hook it was built with. */
typedef void *(*lamg_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*lamg_free_fn)(void *ptr, void *stream, void *ctx);
void lamg_set_allocator(lamg_alloc_fn alloc_fn, lamg_free_fn free_fn, void *ctx);

/* Static, human-readable name of a status code. */
const char *lamg_status_string(lamg_status s);

/* Library version string. */
const char *lamg_version(void);

/* Fills *opt with the defaults listed in lamg_options. */
void lamg_default_options(lamg_options *opt);

/* Builds the LAMG+ hierarchy of graph g (Sec. 2 and Sec. 3): validates the adjacency,
 * forms L = D - W, and per level computes the greedy colouring, strong flags, test
 * vectors, affinities, guard moments, greedy aggregates, interpolation (caliber-1 and
 * caliber-2), the Galerkin operator P^T L P, and finally the cycle indices and the
 * coarsest-level inverse. The graph arrays are copied; the caller keeps ownership.
 * opt == NULL selects the defaults. On success *out owns all device memory of the
 * hierarchy until lamg_destroy. Errors: INVALID_ARG, NOT_SYMMETRIC, SELF_LOOP,
 * BAD_WEIGHT, DISCONNECTED, OOM, COARSENING_STALLED, HIP_ERROR. */
lamg_status lamg_setup(const lamg_graph *g, const lamg_options *opt, void *stream,
                       lamg_handle **out);

/* Solves L phi = b for nrhs right-hand sides to ||b - L phi|| / ||b|| <= tol per column
 * (Sec. 4: tol = 1e-8 in the paper). b and phi are DEVICE arrays, column-major n x nrhs
 * (column j starts at b + j*n), not aliased; b is not modified. Each column's mean is
 * removed first (eq. (1.1) needs 1^T b = 0) and phi is returned with zero mean. Columns
 * are independent: each stops at its own convergence cycle and is frozen afterwards.
 * max_cycles <= 0 selects 300. A zero column returns phi = 0. The handle caches a
 * workspace sized for the largest nrhs seen. Returns OK, NOT_CONVERGED (phi and info are
 * still written; also when a column's relative residual stops being a finite number, which
 * ends that column's cycling), INVALID_ARG (also when b holds a NaN or infinite value, or a
 * column whose norm overflows: eq. (1.1) has no solution to approach; phi is then not
 * written), OOM or HIP_ERROR. */
lamg_status lamg_solve(lamg_handle *h, const double *b, int32_t nrhs, double tol,
                       int32_t max_cycles, lamg_precision prec, double *phi,
                       lamg_solve_info *info, void *stream);

/* Solves `count` independent requests together: request r is (handles[r], b[r], nrhs[r],
 * phi[r]) with the meaning, layout and results of lamg_solve, and tol, max_cycles, prec and
 * stream shared by all. For serving many small graphs at once, where a solve on its own is
 * bound by its chain of dependent launches (a serving form, not part of the paper's method):
 * requests in FP32_IR with at most 32
 * columns whose handle runs the whole cycle in the coarse tail (lamg_options.tail_finest)
 * advance in lockstep, and every cycle's coarse-tail work of all of them is ONE kernel launch
 * (one workgroup per column of each request); every other request is solved by itself, in
 * order, first. Each request computes exactly what lamg_solve computes for it (same kernels,
 * same arithmetic, its own stopping). The handles must be distinct (each request uses its
 * handle's workspace) and live on the current device. statuses[r] receives request r's
 * status; infos (nullable) per-request statistics. Returns OK if every request is OK, else
 * the first non-OK status; INVALID_ARG for bad arguments (nothing solved). */
lamg_status lamg_solve_group(int32_t count, lamg_handle *const *handles,
                             const double *const *b, const int32_t *nrhs, double tol,
                             int32_t max_cycles, lamg_precision prec, double *const *phi,
                             lamg_solve_info *infos, lamg_status *statuses, void *stream);

/* Bytes of the fixed device scratch array behind lamg_solve_noalloc (one array per GPU). */
#define LAMG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* Allocation-free variant of lamg_solve, for callers that cannot allocate device memory:
 * tight serving loops and harnesses that forbid allocation. Same arguments, results and
 * statuses as lamg_solve, but the call allocates no device memory and no pinned host memory
 * (no hipMalloc, hipFree, hipHostMalloc, allocator hook or HIP-graph instantiation): the
 * solve's workspace -- per-level cycle vectors, the finest-level FP64 state and
 * recombination history, reduction partial sums, coarse-tail descriptors -- is laid out in a
 * fixed device array of LAMG_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU
 * it runs on until the process ends (its address is resolved by lamg_setup). The handle's
 * own cached workspace is neither used nor changed, and lamg_options.graphs does not apply.
 * A solve whose workspace does not fit returns LAMG_SCRATCH_TOO_SMALL before anything is
 * written to phi (the finest level alone takes about 104 * n * min(nrhs, 32) bytes).
 * Every call on a GPU shares that GPU's array and leaves its contents behind (each call
 * initialises everything it reads): calls that overlap on one GPU -- on different streams or
 * threads, with any handles -- race, and the caller must serialise them. The call
 * synchronises `stream` (it reads every cycle's residual norms), so it cannot be recorded
 * into a HIP graph. The current device must be the one the handle was set up on, else
 * LAMG_INVALID_ARG. */
lamg_status lamg_solve_noalloc(lamg_handle *h, const double *b, int32_t nrhs, double tol,
                               int32_t max_cycles, lamg_precision prec, double *phi,
                               lamg_solve_info *info, void *stream);

/* Frees everything the handle owns. NULL is accepted. */
void lamg_destroy(lamg_handle *h);

/* Describes the hierarchy (sizes, colours, cycle indices, memory). */
lamg_status lamg_hierarchy_info(const lamg_handle *h, lamg_hier_info *info);

/* Copies level `level` to the caller's host buffers (see lamg_level_export). Requires
 * keep_setup_data = 1 at setup, else LAMG_UNAVAILABLE. Errors: INVALID_ARG (bad level). */
lamg_status lamg_export_level(const lamg_handle *h, int32_t level, lamg_level_export *out);

/* Cycle kernels that lamg_profile_kernel and the in-situ timer can time. */
typedef enum {
    LAMG_KERNEL_GS_COLOR = 0, /* one Gauss-Seidel colour pass (colour 0) of the level */
    LAMG_KERNEL_RESIDUAL = 1, /* r = f - L x over the whole level */
    LAMG_KERNEL_RESTRICT = 2, /* f_c = P^T r from the level to the next */
    LAMG_KERNEL_PROLONG = 3,  /* x += mu P e_c from the next level */
    LAMG_KERNEL_TAIL = 4,     /* one launch of the coarse-level cycle (one workgroup per
                                 column; in-situ timer only) */
    LAMG_KERNEL_REDUCE = 5,   /* reductions and the updates they feed: energy-correction and
                                 recombination sums, norms, means (in-situ timer only) */
    LAMG_KERNEL_VECTOR = 6,   /* elementwise vector kernels: copies, fills, precision and
                                 layout conversions, the coarsest dense solve (in-situ only) */
    LAMG_KERNEL_CHEB = 7,     /* one Chebyshev step (smoother 1; in-situ timer only) */
    LAMG_KERNEL_BJGS = 8      /* one block-Jacobi Gauss-Seidel sweep: the snapshot copy and the
                                 sweep (smoother 2; in-situ timer only) */
} lamg_kernel;

/* Measurement aid for roofline reporting: launches one cycle kernel of level `level`
 * `reps` times back to back on `stream` between two HIP events, with nrhs columns in the
 * arithmetic of `prec` (FP64, or FP32 for LAMG_FP32_IR), and writes the mean launch
 * duration in seconds and the kernel's algorithmic bytes per launch: compulsory traffic
 * only (every matrix index and value, row pointer and diagonal once, every vector element
 * the launch reads or writes once). Uses the handle's cached workspace, whose contents it
 * overwrites; the hierarchy is unchanged. Errors: INVALID_ARG (level out of range, the
 * directly solved level for GS/RESTRICT/PROLONG, nrhs outside 1..32, reps < 1), OOM,
 * HIP_ERROR. */
lamg_status lamg_profile_kernel(lamg_handle *h, int32_t level, lamg_kernel kernel,
                                lamg_precision prec, int32_t nrhs, int32_t reps,
                                double *seconds_per_launch, double *bytes_per_launch,
                                void *stream);

/* In-situ kernel timing (measurement aid). Between lamg_timing_start and lamg_timing_stop,
 * every lamg_solve on the handle attaches a pair of HIP events to each launch of the cycle
 * kernels of level timed_level (lamg_hier_info; every Gauss-Seidel colour pass, residual,
 * restriction, prolongation, in the precision they run in; the FP64 outer residual of an
 * FP32+IR solve, on the finest level, counts as an FP64 residual) and of the coarse-tail
 * kernel, on the solve's stream. The
 * events take the dispatch's own start and end times (hipExtLaunchKernel), so a pair spans
 * the kernel's execution alone; they add no synchronisation and no stream markers. Timing
 * stops recording after `max_launches` launches (the events are created by
 * lamg_timing_start).
 * lamg_timing_start_all does the same for EVERY kernel launch of the solve, on every level,
 * each counted under its kind (lamg_kernel; the finest level's FP64 outer residual is an FP64
 * residual).
 * lamg_timing_stop waits for the last recorded event, converts every pair to a duration
 * and frees the events; lamg_timing_get then returns, per kernel and precision, the number
 * of timed launches, their summed duration and their summed algorithmic bytes (the figures
 * of lamg_profile_kernel for the launch's rows; for a coarse-tail launch the sum of those
 * figures over every step of every level visit the launch performs, the operators counted
 * once per launch whatever the column count). Errors: INVALID_ARG (max_launches < 1, kernel
 * out of range, timing still running for lamg_timing_get), HIP_ERROR. */
typedef struct {
    int64_t launches;
    double seconds;
    double bytes;
} lamg_kernel_time;

lamg_status lamg_timing_start(lamg_handle *h, int32_t max_launches);
lamg_status lamg_timing_start_all(lamg_handle *h, int32_t max_launches);
lamg_status lamg_timing_stop(lamg_handle *h);
lamg_status lamg_timing_get(const lamg_handle *h, lamg_kernel kernel, lamg_precision prec,
                            lamg_kernel_time *out);

#ifdef __cplusplus
}
#endif

#endif /* LAMG_H */
