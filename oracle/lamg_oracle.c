/*
 * LAMG+ reference oracle: TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the LAMG+ aggregation
 * hierarchy and gamma-cycle (Livne, "LAMG+: A Robust Lean Algebraic Multigrid Solver
 * for Graph Laplacians"). It exists only so that tests, the smoke check and the
 * benchmark's CPU baseline can compare the HIP library against an independent
 * implementation. It shares no source, header, table or helper with the HIP path.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * Contraction is off so that every product and sum below is rounded exactly as written.
 *
 * Canonical arithmetic (the contract every setup quantity follows, so that an
 * independent implementation can reproduce it bit for bit):
 *   - IEEE FP64, no fused multiply-add, correctly rounded division;
 *   - every sum runs left to right in the order stated, starting from +0.0;
 *   - CSR rows hold their columns in ascending order with the diagonal in place.
 *
 * Parity status of each function is recorded beside it ("pinned by ..."). The pins
 * live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_K 4 /* test vectors per level: LAMG+ fixes K = 4 (Sec. 3.3) */
#define ORC_MAX_LEVELS 64
#define ORC_BJ_BLOCK 64 /* rows per block of the block-Jacobi Gauss-Seidel smoother */

enum {
    ORC_OK = 0,
    ORC_ERR_ARG = 1,
    ORC_ERR_ALLOC = 2,
    ORC_ERR_STALLED = 3,
    ORC_NOT_CONVERGED = 4
};

/* ------------------------------------------------------------------------- */
/* Data                                                                       */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n;
    int nnz;
    int *rp; /* n+1 */
    int *ci; /* nnz, ascending per row, diagonal included */
    double *v;
} ocsr;

typedef struct {
    ocsr L;
    int coarsest;     /* 1 if this level is solved directly */
    int ncolors;
    int *color;       /* n */
    unsigned char *strong; /* nnz: 1 = may aggregate across this entry */
    double *X;        /* n*K, node-major: X[u*K+k] */
    double *aff;      /* nnz: affinity c_uv (0 on the diagonal) */
    double *mom;      /* n*9: s0, s1[K], s2[K] */
    int *seed;        /* n: seed node of u's aggregate (u itself for seeds) */
    int *agg;         /* n: coarse id A(u) */
    int *p0, *p1;     /* n: interpolation parents (p1 = -1 if none) */
    double *w0, *w1;  /* n: their weights */
    int elim;         /* 1: low-degree elimination level (agg = coarse id, -1 on F) */
    int cheb;         /* 1: smoothed by Chebyshev polynomials instead of Gauss-Seidel */
    double cheb_lmax; /* Gershgorin bound of the spectrum of D^{-1} L */
    int bjgs;         /* 1: smoothed by block-Jacobi Gauss-Seidel instead */
    int nc;           /* size of the next level */
    int n_cal2;       /* rows with two parents */
    double gamma, tau;
    double *chol;     /* coarsest only: Cholesky factor of L + 11^T/n (row-major, lower) */
} olevel;

typedef struct {
    int nlev;
    olevel lev[ORC_MAX_LEVELS];
    /* parameters */
    uint64_t seed;
    int n_direct;
    int enable_veto, enable_caliber2, enable_elim;
    int smoother;       /* 0: multicolour GS; 1: Chebyshev on levels with many colours;
                           2: block-Jacobi Gauss-Seidel on those levels */
    int cheb_colors;    /* ... more than this many colours */
    int bj_block;       /* rows per block of the block-Jacobi Gauss-Seidel sweep */
    int cheb_degree;    /* residual evaluations per Chebyshev sweep */
    double cheb_ratio;  /* smoothed interval [lmax / ratio, lmax] */
    double q_guard, tau_soc, snap, elim_min;
    int kappa;
} ohier;

static void csr_free(ocsr *A) {
    free(A->rp);
    free(A->ci);
    free(A->v);
    memset(A, 0, sizeof(*A));
}

static void level_free(olevel *l) {
    csr_free(&l->L);
    free(l->color);
    free(l->strong);
    free(l->X);
    free(l->aff);
    free(l->mom);
    free(l->seed);
    free(l->agg);
    free(l->p0);
    free(l->p1);
    free(l->w0);
    free(l->w1);
    free(l->chol);
    memset(l, 0, sizeof(*l));
}

/* ------------------------------------------------------------------------- */
/* Counter-based random numbers                                              */
/* ------------------------------------------------------------------------- */

/* Output i (i >= 0) of SplitMix64 seeded with `seed` (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014): the state
 * advances by the golden-ratio increment and is passed through the mix64 finaliser.
 * Pinned by published known-answer sequences. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Random start of test vector k at node u on level l (Sec. 2, "from a random start";
 * the distribution is not stated: U[-1,1) is used). Counter = level<<56 | k<<48 | u. */
double orc_tv_start(uint64_t seed, int level, int k, int64_t u) {
    uint64_t ctr = ((uint64_t)level << 56) | ((uint64_t)k << 48) | (uint64_t)u;
    uint64_t h = orc_splitmix64(seed, ctr);
    double unit = (double)(h >> 11) * 0x1.0p-53; /* exact: 53 significant bits */
    return 2.0 * unit - 1.0;                     /* exact */
}

/* ------------------------------------------------------------------------- */
/* S0: graph Laplacian L = D - W (Sec. 1, eq. (1.1) and the line above it)     */
/* ------------------------------------------------------------------------- */

/* Adjacency CSR (both directions, ascending columns, no diagonal) -> canonical
 * Laplacian CSR with the diagonal in its sorted position. L_uu is the sum of the
 * row's weights in column order. Pinned: L1 = 0 exactly for integer weights,
 * equals dense D - W. */
int orc_laplacian(int n, const int *rp, const int *ci, const double *w, int *Lrp, int *Lci,
                  double *Lv) {
    int pos = 0;
    Lrp[0] = 0;
    for (int u = 0; u < n; ++u) {
        double d = 0.0;
        for (int j = rp[u]; j < rp[u + 1]; ++j) d = d + w[j];
        int placed = 0;
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            if (!placed && ci[j] > u) {
                Lci[pos] = u;
                Lv[pos] = d;
                ++pos;
                placed = 1;
            }
            Lci[pos] = ci[j];
            Lv[pos] = -w[j];
            ++pos;
        }
        if (!placed) {
            Lci[pos] = u;
            Lv[pos] = d;
            ++pos;
        }
        Lrp[u + 1] = pos;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* S2: natural-order greedy colouring                                        */
/* ------------------------------------------------------------------------- */

/* Nodes in index order; colour(u) = smallest c >= 0 used by no neighbour v < u.
 * Every stored off-diagonal entry is a neighbour. Returns the number of colours.
 * Pinned: parity colouring (i+j[+k]) mod 2 on lexicographic grids; validity and a
 * brute-force re-run on random graphs. */
int orc_color(int n, const int *rp, const int *ci, int *color) {
    int maxdeg = 0;
    for (int u = 0; u < n; ++u)
        if (rp[u + 1] - rp[u] > maxdeg) maxdeg = rp[u + 1] - rp[u];
    int *mark = (int *)malloc(sizeof(int) * (size_t)(maxdeg + 2));
    if (!mark) return -1;
    for (int c = 0; c < maxdeg + 2; ++c) mark[c] = -1;
    int ncol = 0;
    for (int u = 0; u < n; ++u) {
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int v = ci[j];
            if (v < u && color[v] < maxdeg + 2) mark[color[v]] = u;
        }
        int c = 0;
        while (mark[c] == u) ++c;
        color[u] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(mark);
    return ncol;
}

/* ------------------------------------------------------------------------- */
/* S3: strength-of-connection veto (Sec. 3.1, eq. (3.1))                       */
/* ------------------------------------------------------------------------- */

/* strong[j] = 1 iff entry j = (u,v), v != u, is not vetoed from u's side:
 * !(|L_uv| < tau * max_{t != u} |L_ut|), and L_uv != 0 (an exactly-zero coupling
 * joins nothing). With the veto disabled only the nonzero test remains.
 * Pinned: every weak edge of a grid-aligned anisotropic grid is vetoed and every
 * strong one kept; brute force on random graphs. */
int orc_strong(int n, const int *rp, const int *ci, const double *v, double tau, int enable_veto,
               unsigned char *strong) {
    for (int u = 0; u < n; ++u) {
        double mx = 0.0;
        for (int j = rp[u]; j < rp[u + 1]; ++j)
            if (ci[j] != u && fabs(v[j]) > mx) mx = fabs(v[j]);
        double thr = tau * mx;
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int s = (ci[j] != u) && (v[j] != 0.0);
            if (s && enable_veto && fabs(v[j]) < thr) s = 0;
            strong[j] = (unsigned char)s;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* S4: test vectors = nu Gauss-Seidel sweeps on L x = 0 (Sec. 2, "Caliber-1     */
/* aggregation"; K = 4 fixed, Sec. 3.3)                                        */
/* ------------------------------------------------------------------------- */

/* One multicolour Gauss-Seidel sweep on L x = f for K vectors stored node-major
 * (f == NULL means f = 0). Colours are visited in ascending order; within a colour,
 * rows do not couple, so the visiting order inside a colour does not matter. Row
 * arithmetic: acc = sum over v != u in CSR order of L_uv * x_v; x_u = (f_u - acc)/L_uu.
 * Pinned: equals a forward Gauss-Seidel sweep (triangular solve) on the colour-sorted
 * matrix. */
int orc_gs_sweep_multi(int n, const int *rp, const int *ci, const double *v, const int *color,
                       int ncolors, int K, const double *f, double *X) {
    for (int c = 0; c < ncolors; ++c) {
        for (int u = 0; u < n; ++u) {
            if (color[u] != c) continue;
            for (int k = 0; k < K; ++k) {
                double acc = 0.0, d = 0.0;
                for (int j = rp[u]; j < rp[u + 1]; ++j) {
                    if (ci[j] == u)
                        d = v[j];
                    else
                        acc = acc + v[j] * X[(size_t)ci[j] * K + k];
                }
                double fu = f ? f[(size_t)u * K + k] : 0.0;
                X[(size_t)u * K + k] = (fu - acc) / d;
            }
        }
    }
    return ORC_OK;
}

/* Test vectors of level `level`: random start, then `sweeps` canonical sweeps. */
int orc_test_vectors(int n, const int *rp, const int *ci, const double *v, const int *color,
                     int ncolors, uint64_t seed, int level, int sweeps, double *X) {
    for (int u = 0; u < n; ++u)
        for (int k = 0; k < ORC_K; ++k) X[(size_t)u * ORC_K + k] = orc_tv_start(seed, level, k, u);
    for (int s = 0; s < sweeps; ++s)
        orc_gs_sweep_multi(n, rp, ci, v, color, ncolors, ORC_K, NULL, X);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* S5: affinity (Sec. 2, eq. (2.2))                                           */
/* ------------------------------------------------------------------------- */

/* aff[j] for entry (u,v): (sum_k x_u x_v)^2 / (sum_k x_u^2 * sum_k x_v^2); 0 on the
 * diagonal and where the denominator is 0. Sums run k = 0..K-1 from +0.0.
 * Pinned: squared cosine of the profile angle (1 for parallel, 0 for orthogonal,
 * cos^2 t for a rotation by t), symmetry, range [0,1]. */
int orc_affinity(int n, const int *rp, const int *ci, const double *X, double *aff) {
    for (int u = 0; u < n; ++u) {
        double su = 0.0;
        for (int k = 0; k < ORC_K; ++k) su = su + X[(size_t)u * ORC_K + k] * X[(size_t)u * ORC_K + k];
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int t = ci[j];
            if (t == u) {
                aff[j] = 0.0;
                continue;
            }
            double st = 0.0, p = 0.0;
            for (int k = 0; k < ORC_K; ++k) st = st + X[(size_t)t * ORC_K + k] * X[(size_t)t * ORC_K + k];
            for (int k = 0; k < ORC_K; ++k) p = p + X[(size_t)u * ORC_K + k] * X[(size_t)t * ORC_K + k];
            double den = su * st;
            aff[j] = (den == 0.0) ? 0.0 : (p * p) / den;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* S6: guard moments (App. B)                                                 */
/* ------------------------------------------------------------------------- */

/* Per node u, over v != u in CSR order with w = -L_uv:
 *   s0 = sum w, s1[k] = sum w x_v[k], s2[k] = sum w (x_v[k] x_v[k]).
 * Stored as mom[u*9 + 0] = s0, mom[u*9 + 1 + k] = s1[k], mom[u*9 + 5 + k] = s2[k].
 * Pinned: App. B closed forms against a brute-force minimisation of the nodal energy. */
int orc_moments(int n, const int *rp, const int *ci, const double *v, const double *X, double *mom) {
    for (int u = 0; u < n; ++u) {
        double s0 = 0.0, s1[ORC_K], s2[ORC_K];
        for (int k = 0; k < ORC_K; ++k) s1[k] = s2[k] = 0.0;
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int t = ci[j];
            if (t == u) continue;
            double w = -v[j];
            s0 = s0 + w;
            for (int k = 0; k < ORC_K; ++k) {
                double x = X[(size_t)t * ORC_K + k];
                s1[k] = s1[k] + w * x;
                s2[k] = s2[k] + w * (x * x);
            }
        }
        mom[(size_t)u * 9] = s0;
        for (int k = 0; k < ORC_K; ++k) {
            mom[(size_t)u * 9 + 1 + k] = s1[k];
            mom[(size_t)u * 9 + 5 + k] = s2[k];
        }
    }
    return ORC_OK;
}

/* Energy-ratio guard q_{u<-s} <= Q (Sec. 2, eq. (2.3)) via the App. B closed forms,
 * in multiplied-out form so that a zero relaxed energy is handled:
 *   2*Emin  = s2 - s1*s1/s0,  2*Eforce = (xs*xs*s0 - 2*xs*s1) + s2,
 *   admissible iff 2*Eforce <= Q * 2*Emin for every k.
 * If ef/em are non-NULL the per-k doubled energies are written there.
 * Pinned: brute-force nodal energy, the linear-chain value q = 2. */
int orc_guard(const double *mom_u, const double *xs, double Q, double *ef, double *em) {
    int ok = 1;
    double s0 = mom_u[0];
    for (int k = 0; k < ORC_K; ++k) {
        double s1 = mom_u[1 + k], s2 = mom_u[5 + k], x = xs[k];
        double m2 = s2 - (s1 * s1) / s0;
        double f2 = ((x * x) * s0 - (2.0 * x) * s1) + s2;
        if (ef) ef[k] = f2;
        if (em) em[k] = m2;
        if (!(f2 <= Q * m2)) ok = 0;
    }
    return ok;
}

/* ------------------------------------------------------------------------- */
/* S7: greedy aggregation (Sec. 2 "Caliber-1 aggregation"; Sec. 3.1)          */
/* ------------------------------------------------------------------------- */

enum { ST_UNDECIDED = 0, ST_SEED = 1, ST_MEMBER = 2 };

/* One pass over u = 0..n-1. An undecided u considers its strong neighbours v that are
 * undecided or seeds; v is admissible if the guard holds for u forced onto x_v.
 * u joins the admissible candidate of largest affinity (first in CSR order on a tie),
 * which becomes a seed; with no admissible candidate u becomes a singleton seed that
 * others may still join. No size cap. Coarse ids number the seeds in ascending order.
 * Writes seed[u] (u for seeds) and agg[u]; returns the number of aggregates.
 * Pinned (parity unpinned against the paper's own implementation): replay invariants
 * checked in tests -- every member's guard holds against its seed, no admissible
 * candidate available at its turn had a larger affinity, singleton seeds had none. */
int orc_aggregate(int n, const int *rp, const int *ci, const unsigned char *strong,
                  const double *aff, const double *X, const double *mom, double Q, int *seed,
                  int *agg) {
    unsigned char *state = (unsigned char *)calloc((size_t)n, 1);
    if (!state) return -1;
    for (int u = 0; u < n; ++u) seed[u] = -1;
    for (int u = 0; u < n; ++u) {
        if (state[u] != ST_UNDECIDED) continue;
        int best = -1;
        double bestc = -1.0;
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int v = ci[j];
            if (!strong[j]) continue;
            if (state[v] == ST_MEMBER) continue;
            if (!orc_guard(mom + (size_t)u * 9, X + (size_t)v * ORC_K, Q, NULL, NULL)) continue;
            if (aff[j] > bestc) {
                bestc = aff[j];
                best = v;
            }
        }
        if (best >= 0) {
            state[best] = ST_SEED;
            seed[best] = best;
            state[u] = ST_MEMBER;
            seed[u] = best;
        } else {
            state[u] = ST_SEED;
            seed[u] = u;
        }
    }
    int nc = 0;
    for (int u = 0; u < n; ++u)
        if (state[u] == ST_SEED) agg[u] = nc++;
    for (int u = 0; u < n; ++u)
        if (state[u] == ST_MEMBER) agg[u] = agg[seed[u]];
    free(state);
    return nc;
}

/* ------------------------------------------------------------------------- */
/* S8/S9: interpolation rows, caliber-1 and selective caliber-2 (Sec. 3.2,     */
/* App. A.2 eq. (A.7))                                                         */
/* ------------------------------------------------------------------------- */

/* Least-squares weight of x_u ~ w x_a + (1-w) x_b over the K test vectors:
 * w = sum d_k e_k / sum d_k^2 with d = x_a - x_b, e = x_u - x_b (eq. (A.7)).
 * Returns NAN if sum d_k^2 == 0. Pinned: midpoint gives 1/2, x_u = x_a gives 1,
 * optimality against a library least-squares solve. */
double orc_caliber2_weight(const double *xu, const double *xa, const double *xb) {
    double D = 0.0, N = 0.0;
    for (int k = 0; k < ORC_K; ++k) {
        double d = xa[k] - xb[k];
        double e = xu[k] - xb[k];
        D = D + d * d;
        N = N + d * e;
    }
    if (D == 0.0) return NAN;
    return N / D;
}

/* Interpolation rows. Seeds: P_u = e_{A(u)}. A member u is upgraded when its strong
 * entries reach exactly two aggregates {A(u), b}: with x_a, x_b the seeds' test
 * vectors, w from eq. (A.7); w in [-snap, snap] -> row e_b; w in (snap, 1-snap) ->
 * w e_a + (1-w) e_b; otherwise (near 1, or outside [0,1]) caliber-1 e_{A(u)}.
 * Returns the number of two-parent rows. */
int orc_interp(int n, const int *rp, const int *ci, const unsigned char *strong, const double *X,
               const int *seed, const int *agg, int nc, int enable_caliber2, double snap, int *p0,
               double *w0, int *p1, double *w1) {
    int *aggseed = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    if (!aggseed) return -1;
    for (int u = 0; u < n; ++u)
        if (seed[u] == u) aggseed[agg[u]] = u;
    int n2 = 0;
    for (int u = 0; u < n; ++u) {
        int a = agg[u];
        p0[u] = a;
        w0[u] = 1.0;
        p1[u] = -1;
        w1[u] = 0.0;
        if (!enable_caliber2 || seed[u] == u) continue;
        int b = -1, two = 1;
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            if (!strong[j]) continue;
            int t = agg[ci[j]];
            if (t == a) continue;
            if (b < 0)
                b = t;
            else if (t != b) {
                two = 0;
                break;
            }
        }
        if (!two || b < 0) continue;
        double w = orc_caliber2_weight(X + (size_t)u * ORC_K, X + (size_t)aggseed[a] * ORC_K,
                                       X + (size_t)aggseed[b] * ORC_K);
        if (isnan(w)) continue;
        if (w >= -snap && w <= snap) {
            p0[u] = b;
            w0[u] = 1.0;
        } else if (w > snap && w < 1.0 - snap) {
            p0[u] = a;
            w0[u] = w;
            p1[u] = b;
            w1[u] = 1.0 - w;
            ++n2;
        }
    }
    free(aggseed);
    return n2;
}

/* ------------------------------------------------------------------------- */
/* S10: Galerkin coarse operator L^c = P^T L P in edge form (Sec. 2,          */
/* "Multigrid in one paragraph")                                               */
/* ------------------------------------------------------------------------- */

/* L = sum over edges of w (e_u - e_v)(e_u - e_v)^T, hence P^T L P = sum w d d^T with
 * d = P_u - P_v (a sparse vector over coarse ids). The off-diagonal (a,b) is the sum,
 * over stored entries (u,v) with u < v in CSR order, of w * (d_a * d_b), w = -L_uv,
 * starting from +0.0; entries of d that are exactly 0 are dropped; every generated
 * pair is kept even if it sums to 0. The diagonal is minus the sum of its row's
 * off-diagonals in ascending column order, so rows sum to zero by construction.
 * Pinned: dense P^T L P (numpy); exact integers for caliber-1 with integer weights;
 * exact symmetry. */
typedef struct {
    int a, b;
    long long seq;
    double c;
} orc_contrib;

static int contrib_cmp(const void *x, const void *y) {
    const orc_contrib *p = (const orc_contrib *)x, *q = (const orc_contrib *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->seq != q->seq) return p->seq < q->seq ? -1 : 1;
    return 0;
}

/* Phase 1 (Crp == NULL): returns nnz of L^c (diagonal included). Phase 2: fills the
 * caller-allocated canonical CSR (Crp: nc+1, Cci/Cv: nnz). Returns -1 on failure. */
long long orc_galerkin(int n, const int *rp, const int *ci, const double *v, int nc, const int *p0,
                       const double *w0, const int *p1, const double *w1, int *Crp, int *Cci,
                       double *Cv) {
    long long cap = 0;
    for (int u = 0; u < n; ++u)
        for (int j = rp[u]; j < rp[u + 1]; ++j)
            if (ci[j] > u) cap += 12;
    orc_contrib *list = (orc_contrib *)malloc(sizeof(orc_contrib) * (size_t)(cap > 0 ? cap : 1));
    if (!list) return -1;
    long long cnt = 0, seq = 0;
    for (int u = 0; u < n; ++u) {
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int t = ci[j];
            if (t <= u) continue;
            double w = -v[j];
            /* d = P_u - P_t over the union of their supports */
            int id[4];
            double dv[4];
            int nd = 0;
            int ua[2] = {p0[u], p1[u]}, ta[2] = {p0[t], p1[t]};
            double uw[2] = {w0[u], w1[u]}, tw[2] = {w0[t], w1[t]};
            for (int s = 0; s < 2; ++s) {
                if (ua[s] < 0) continue;
                double other = 0.0;
                for (int r = 0; r < 2; ++r)
                    if (ta[r] == ua[s]) other = tw[r];
                id[nd] = ua[s];
                dv[nd] = uw[s] - other;
                ++nd;
            }
            for (int r = 0; r < 2; ++r) {
                if (ta[r] < 0) continue;
                int dup = 0;
                for (int s = 0; s < 2; ++s)
                    if (ua[s] == ta[r]) dup = 1;
                if (dup) continue;
                id[nd] = ta[r];
                dv[nd] = 0.0 - tw[r];
                ++nd;
            }
            for (int x = 0; x < nd; ++x) {
                if (dv[x] == 0.0) continue;
                for (int y = 0; y < nd; ++y) {
                    if (y == x || dv[y] == 0.0) continue;
                    list[cnt].a = id[x];
                    list[cnt].b = id[y];
                    list[cnt].seq = seq;
                    list[cnt].c = w * (dv[x] * dv[y]);
                    ++cnt;
                }
            }
            ++seq;
        }
    }
    qsort(list, (size_t)cnt, sizeof(orc_contrib), contrib_cmp);
    /* count distinct (a,b) plus one diagonal per row */
    long long nnz = nc;
    for (long long i = 0; i < cnt; ++i)
        if (i == 0 || list[i].a != list[i - 1].a || list[i].b != list[i - 1].b) ++nnz;
    if (!Crp) {
        free(list);
        return nnz;
    }
    /* fill row by row */
    long long i = 0, pos = 0;
    for (int a = 0; a < nc; ++a) {
        Crp[a] = (int)pos;
        long long rowstart = pos;
        int diag_at = -1;
        while (i < cnt && list[i].a == a) {
            int b = list[i].b;
            double s = 0.0;
            while (i < cnt && list[i].a == a && list[i].b == b) {
                s = s + list[i].c;
                ++i;
            }
            if (diag_at < 0 && b > a) {
                diag_at = (int)pos;
                Cci[pos] = a;
                Cv[pos] = 0.0;
                ++pos;
            }
            Cci[pos] = b;
            Cv[pos] = s;
            ++pos;
        }
        if (diag_at < 0) {
            diag_at = (int)pos;
            Cci[pos] = a;
            Cv[pos] = 0.0;
            ++pos;
        }
        double off = 0.0;
        for (long long q = rowstart; q < pos; ++q)
            if (Cci[q] != a) off = off + Cv[q];
        Cv[diag_at] = -off;
    }
    Crp[nc] = (int)pos;
    free(list);
    return nnz;
}


/* ------------------------------------------------------------------------- */
/* S11: low-degree elimination (Sec. 2, "Low-degree elimination", eq. (2.1))  */
/* ------------------------------------------------------------------------- */

static double diag_of(const int *rp, const int *ci, const double *v, int u) {
    for (int j = rp[u]; j < rp[u + 1]; ++j)
        if (ci[j] == u) return v[j];
    return 0.0;
}

static double entry_of(const int *rp, const int *ci, const double *v, int u, int t) {
    for (int j = rp[u]; j < rp[u + 1]; ++j)
        if (ci[j] == t) return v[j];
    return 0.0;
}

/* F: a maximal independent set among the nodes with at most dmax stored off-diagonals,
 * taken greedily in natural order (u joins F when it qualifies, its diagonal is positive
 * and none of its neighbours is in F yet). C = the other nodes, numbered by ascending
 * fine index: cid[u] = rank of u in C, or -1 for u in F. Returns |C|.
 * Pinned: independence and maximality by brute force; F empty when no node qualifies. */
int orc_elim_select(int n, const int *rp, const int *ci, const double *v, int dmax, int *cid) {
    for (int u = 0; u < n; ++u) cid[u] = 0;
    for (int u = 0; u < n; ++u) {
        int deg = rp[u + 1] - rp[u] - 1;
        if (deg > dmax || !(diag_of(rp, ci, v, u) > 0.0)) continue;
        int free_ = 1;
        for (int j = rp[u]; j < rp[u + 1]; ++j)
            if (ci[j] != u && cid[ci[j]] < 0) free_ = 0;
        if (free_) cid[u] = -1;
    }
    int nc = 0;
    for (int u = 0; u < n; ++u)
        if (cid[u] >= 0) cid[u] = nc++;
    return nc;
}

/* Exact Schur complement onto C, L^c = L_CC - L_CF L_FF^{-1} L_FC (eq. (2.1)); L_FF is
 * diagonal because F is independent. Off-diagonal (a, b) of coarse row a = cid[u]:
 * from +0.0, add L_ub if stored, then for every f in F adjacent to both u and b, in
 * ascending f, add -((L_fu * L_fb) / L_ff). Every pair reached is stored. The diagonal
 * is minus the sum of the row's off-diagonals in ascending column order (the Schur
 * complement of a Laplacian has zero row sums).
 * Pinned: dense L_CC - L_CF L_FF^{-1} L_FC (numpy); exact for integer weights whose
 * divisions are exact; exact symmetry; the solution of the eliminated system restricted
 * to C. Phase 1 (Crp == NULL) returns nnz of L^c; phase 2 fills the caller's CSR. */
long long orc_schur(int n, const int *rp, const int *ci, const double *v, const int *cid, int nc,
                    int *Crp, int *Cci, double *Cv) {
    int *slot = (int *)malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int cap = 64;
    int *col = (int *)malloc(sizeof(int) * (size_t)cap);
    double *acc = (double *)malloc(sizeof(double) * (size_t)cap);
    if (!slot || !col || !acc) {
        free(slot);
        free(col);
        free(acc);
        return -1;
    }
    for (int a = 0; a < nc; ++a) slot[a] = -1;
    long long nnz = 0;
    if (Crp) Crp[0] = 0;
    for (int u = 0; u < n; ++u) {
        if (cid[u] < 0) continue;
        int a = cid[u], cnt = 0;
        /* the entries this row reaches, in the order they are first reached */
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = rp[u]; j < rp[u + 1]; ++j) {
                int t = ci[j];
                if (t == u) continue;
                if (pass == 0 && cid[t] < 0) continue;
                if (pass == 1 && cid[t] >= 0) continue;
                /* pass 0: the C-C entry itself; pass 1: t = f in F, its other neighbours */
                int lo = pass == 0 ? j : rp[t], hi = pass == 0 ? j + 1 : rp[t + 1];
                double lff = pass == 0 ? 0.0 : diag_of(rp, ci, v, t);
                double lfu = pass == 0 ? 0.0 : entry_of(rp, ci, v, t, u);
                for (int jj = lo; jj < hi; ++jj) {
                    int bnode = ci[jj];
                    if (pass == 1 && (bnode == t || bnode == u)) continue;
                    double c = pass == 0 ? v[jj] : -((lfu * v[jj]) / lff);
                    int b = cid[bnode];
                    if (slot[b] < 0) {
                        if (cnt == cap) {
                            cap *= 2;
                            int *nc2 = (int *)realloc(col, sizeof(int) * (size_t)cap);
                            double *na = (double *)realloc(acc, sizeof(double) * (size_t)cap);
                            if (nc2) col = nc2;
                            if (na) acc = na;
                            if (!nc2 || !na) {
                                free(slot);
                                free(col);
                                free(acc);
                                return -1;
                            }
                        }
                        slot[b] = cnt;
                        col[cnt] = b;
                        acc[cnt] = 0.0;
                        ++cnt;
                    }
                    acc[slot[b]] = acc[slot[b]] + c;
                }
            }
        }
        for (int x = 0; x < cnt; ++x) slot[col[x]] = -1;
        /* ascending columns (insertion sort), diagonal in place */
        for (int x = 1; x < cnt; ++x) {
            int cc = col[x];
            double aa = acc[x];
            int y = x - 1;
            while (y >= 0 && col[y] > cc) {
                col[y + 1] = col[y];
                acc[y + 1] = acc[y];
                --y;
            }
            col[y + 1] = cc;
            acc[y + 1] = aa;
        }
        if (Crp) {
            double off = 0.0;
            for (int x = 0; x < cnt; ++x) off = off + acc[x];
            long long pos = Crp[a];
            int placed = 0;
            for (int x = 0; x < cnt; ++x) {
                if (!placed && col[x] > a) {
                    Cci[pos] = a;
                    Cv[pos] = -off;
                    ++pos;
                    placed = 1;
                }
                Cci[pos] = col[x];
                Cv[pos] = acc[x];
                ++pos;
            }
            if (!placed) {
                Cci[pos] = a;
                Cv[pos] = -off;
                ++pos;
            }
            Crp[a + 1] = (int)pos;
        }
        nnz += cnt + 1;
    }
    free(slot);
    free(col);
    free(acc);
    return nnz;
}

/* The F rows of an elimination level given the C values: phi_f = (f_f - sum_{c} L_fc
 * phi_c) / L_ff, the phi_F = P_F phi_C + L_FF^{-1} b_F of eq. (2.1). The rows of F are
 * independent, so the order does not matter. */
static void elim_relax_f(const olevel *lv, double *phi, const double *f) {
    const ocsr *A = &lv->L;
    for (int u = 0; u < A->n; ++u) {
        if (lv->agg[u] >= 0) continue;
        double s = 0.0, d = 0.0;
        for (int j = A->rp[u]; j < A->rp[u + 1]; ++j) {
            if (A->ci[j] == u)
                d = A->v[j];
            else
                s += A->v[j] * phi[A->ci[j]];
        }
        phi[u] = (f[u] - s) / d;
    }
}

/* ------------------------------------------------------------------------- */
/* S13: Chebyshev polynomial smoother, the parallel substitute for Gauss-Seidel  */
/* that Sec. 5 ("On the feasibility of a parallel LAMG+") names, after Adams,   */
/* Brezina, Hu and Tuminaro (2003)                                              */
/* ------------------------------------------------------------------------- */

/* Upper bound of the spectrum of D^{-1} L by Gershgorin's theorem: the largest
 * sum_j |L_uj| / L_uu over the rows (sum in CSR order from +0.0, diagonal included).
 * Pinned: >= the largest eigenvalue (dense eig), = 2 for a graph Laplacian with
 * non-negative weights. */
double orc_gershgorin(int n, const int *rp, const int *ci, const double *v) {
    double best = 0.0;
    for (int u = 0; u < n; ++u) {
        double s = 0.0, d = 0.0;
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            s = s + fabs(v[j]);
            if (ci[j] == u) d = v[j];
        }
        double q = s / d;
        if (q > best) best = q;
    }
    return best;
}

/* One Chebyshev sweep of `degree` residual evaluations on L x = f with the Jacobi
 * preconditioner D = diag(L), damping the eigencomponents of D^{-1} L in [a, b] =
 * [lmax / ratio, lmax]: the three-term Chebyshev semi-iteration (theta = (a+b)/2,
 * delta = (b-a)/2, sigma = theta/delta):
 *   rho_0 = 1/sigma, d = D^{-1} r / theta, x += d;
 *   then for each further step: r = f - L x, rho_1 = 1/(2 sigma - rho_0),
 *   d = rho_1 rho_0 d + (2 rho_1 / delta) D^{-1} r, x += d, rho_0 = rho_1.
 * Pinned: on an eigenvector of D^{-1} L the error is multiplied by the scaled
 * Chebyshev polynomial T_m((theta - lambda)/delta) / T_m(sigma). */
void orc_cheb_sweep(int n, const int *rp, const int *ci, const double *v, double lmax,
                    double ratio, int degree, const double *f, double *x, double *r, double *d) {
    const double b = lmax, a = lmax / ratio;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho0 = 1.0 / sigma;
    for (int step = 0; step < degree; ++step) {
        for (int u = 0; u < n; ++u) {
            double acc = 0.0, dg = 0.0;
            for (int j = rp[u]; j < rp[u + 1]; ++j) {
                acc += v[j] * x[ci[j]];
                if (ci[j] == u) dg = v[j];
            }
            r[u] = ((f ? f[u] : 0.0) - acc) / dg; /* D^{-1} r */
        }
        if (step == 0) {
            for (int u = 0; u < n; ++u) d[u] = r[u] / theta;
        } else {
            const double rho1 = 1.0 / (2.0 * sigma - rho0);
            for (int u = 0; u < n; ++u) d[u] = rho1 * rho0 * d[u] + (2.0 * rho1 / delta) * r[u];
            rho0 = rho1;
        }
        for (int u = 0; u < n; ++u) x[u] += d[u];
    }
}

/* ------------------------------------------------------------------------- */
/* S14: block-Jacobi Gauss-Seidel, the other parallel substitute for Gauss-Seidel  */
/* that Sec. 5 ("On the feasibility of a parallel LAMG+") names: the coupling     */
/* between blocks is frozen                                                       */
/* ------------------------------------------------------------------------- */

/* One sweep on L x = f (f may be NULL for f = 0). The rows are cut into consecutive
 * blocks of `bs` in their natural order; each block is relaxed by a Gauss-Seidel sweep in
 * row order, x_u = (f_u - sum_{j != u} L_uj x_j) / L_uu with the sum in CSR order from
 * +0.0, where x_j is the value just computed for j in u's block and the value at the
 * start of the sweep for j in any other block. x0: scratch of n.
 * Pinned: bs >= n is the natural-order forward Gauss-Seidel sweep (the lower-triangular
 * solve (D + L_lower) x' = f - L_upper x), bs = 1 a Jacobi sweep, and any bs the
 * triangular solve with the block-lower part of L. */
void orc_bjgs_sweep(int n, const int *rp, const int *ci, const double *v, int bs,
                    const double *f, double *x, double *x0) {
    for (int u = 0; u < n; ++u) x0[u] = x[u];
    for (int b0 = 0; b0 < n; b0 += bs) {
        const int b1 = n - b0 > bs ? b0 + bs : n;
        for (int u = b0; u < b1; ++u) {
            double acc = 0.0, dg = 0.0;
            for (int j = rp[u]; j < rp[u + 1]; ++j) {
                const int c = ci[j];
                if (c == u) {
                    dg = v[j];
                    continue;
                }
                acc = acc + v[j] * ((c >= b0 && c < b1) ? x[c] : x0[c]);
            }
            x[u] = ((f ? f[u] : 0.0) - acc) / dg;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* S15: self-gated reverse Cuthill-McKee renumbering of the input graph, the     */
/* reordering for cache locality that Sec. 4.2 lists among the implementation's  */
/* constant-lowering features                                                    */
/* ------------------------------------------------------------------------- */

/* Breadth-first search from r over r's component: order[0..*cnt) in visiting order, the
 * neighbours of each node taken in CSR order; level[u] = distance from r. Returns the
 * eccentricity of r (the last level). mark[] holds `stamp` for visited nodes. */
static int bfs_levels(const int *rp, const int *ci, int r, int *mark, int stamp, int *order,
                      int *level, int *cnt) {
    int head = 0, tail = 0;
    order[tail++] = r;
    mark[r] = stamp;
    level[r] = 0;
    while (head < tail) {
        int u = order[head++];
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            int v = ci[j];
            if (mark[v] == stamp) continue;
            mark[v] = stamp;
            level[v] = level[u] + 1;
            order[tail++] = v;
        }
    }
    *cnt = tail;
    return level[order[tail - 1]];
}

/* The reverse Cuthill-McKee order of a graph given as a CSR without self-loops
 * (perm[new] = old). Degree = number of stored neighbours. Components are taken in the
 * order of their smallest node. A component starts at a pseudo-peripheral node (the
 * George-Liu iteration): r = its node of least degree (ties: smallest index); breadth-first
 * levels from r; x = the node of least degree (ties: smallest index) in the last level; if
 * x's eccentricity exceeds r's, r = x and again, else r is the start. Cuthill-McKee from r:
 * breadth first, each node's not yet numbered neighbours appended in order of increasing
 * degree (ties: smallest index). The whole sequence is then reversed. Self-gate: the
 * renumbering is kept only if it at least halves the mean index distance |u - v| over the
 * entries (the sum, compared exactly in integers); returns 1 then, else 0 with perm the
 * identity. */
int orc_rcm(int n, const int *rp, const int *ci, int *perm) {
    int *mark = (int *)calloc((size_t)n, sizeof(int));
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    int *level = (int *)malloc(sizeof(int) * (size_t)n);
    int *done = (int *)calloc((size_t)n, sizeof(int));
    int *nb = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!mark || !order || !level || !done || !nb) {
        free(mark);
        free(order);
        free(level);
        free(done);
        free(nb);
        return -ORC_ERR_ALLOC;
    }
    int stamp = 0, pos = 0;
    for (int s0 = 0; s0 < n; ++s0) {
        if (done[s0]) continue;
        int cnt = 0;
        bfs_levels(rp, ci, s0, mark, ++stamp, order, level, &cnt);
        int r = order[0];
        for (int i = 1; i < cnt; ++i) {
            int u = order[i], du = rp[u + 1] - rp[u], dr = rp[r + 1] - rp[r];
            if (du < dr || (du == dr && u < r)) r = u;
        }
        int ecc = bfs_levels(rp, ci, r, mark, ++stamp, order, level, &cnt);
        for (;;) {
            int x = -1;
            for (int i = 0; i < cnt; ++i) {
                int u = order[i];
                if (level[u] != ecc) continue;
                if (x < 0) {
                    x = u;
                    continue;
                }
                int du = rp[u + 1] - rp[u], dx = rp[x + 1] - rp[x];
                if (du < dx || (du == dx && u < x)) x = u;
            }
            int ecc_x = bfs_levels(rp, ci, x, mark, ++stamp, order, level, &cnt);
            if (ecc_x > ecc) {
                r = x;
                ecc = ecc_x;
            } else {
                break;
            }
        }
        /* Cuthill-McKee from r */
        int head = pos;
        perm[pos++] = r;
        done[r] = 1;
        while (head < pos) {
            int u = perm[head++], m = 0;
            for (int j = rp[u]; j < rp[u + 1]; ++j)
                if (!done[ci[j]]) {
                    done[ci[j]] = 1;
                    nb[m++] = ci[j];
                }
            for (int a = 1; a < m; ++a) { /* insertion sort by (degree, index) */
                int v = nb[a], dv = rp[v + 1] - rp[v], b = a - 1;
                while (b >= 0) {
                    int w = nb[b], dw = rp[w + 1] - rp[w];
                    if (dw < dv || (dw == dv && w < v)) break;
                    nb[b + 1] = w;
                    --b;
                }
                nb[b + 1] = v;
            }
            for (int a = 0; a < m; ++a) perm[pos++] = nb[a];
        }
    }
    for (int i = 0; i < n / 2; ++i) {
        int t = perm[i];
        perm[i] = perm[n - 1 - i];
        perm[n - 1 - i] = t;
    }
    /* gate: summed index distance before and after (inverse of perm in `order`) */
    for (int i = 0; i < n; ++i) order[perm[i]] = i;
    long long sum0 = 0, sum1 = 0;
    for (int u = 0; u < n; ++u)
        for (int j = rp[u]; j < rp[u + 1]; ++j) {
            long long d0 = (long long)u - ci[j], d1 = (long long)order[u] - order[ci[j]];
            sum0 += d0 < 0 ? -d0 : d0;
            sum1 += d1 < 0 ? -d1 : d1;
        }
    int keep = 2 * sum1 <= sum0;
    if (!keep)
        for (int i = 0; i < n; ++i) perm[i] = i;
    free(mark);
    free(order);
    free(level);
    free(done);
    free(nb);
    return keep;
}

/* Block size of the block-Jacobi Gauss-Seidel smoother (smoother 2) of a hierarchy. */
int orc_set_bj_block(void *hp, int bs) {
    if (!hp || bs < 1) return ORC_ERR_ARG;
    ((ohier *)hp)->bj_block = bs;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* S12: coarsest level, dense solve of (L + 11^T/n) y = f                       */
/* ------------------------------------------------------------------------- */

static int coarsest_factor(olevel *l) {
    int n = l->L.n;
    double *A = (double *)calloc((size_t)n * n, sizeof(double));
    if (!A) return ORC_ERR_ALLOC;
    double one_n = 1.0 / (double)n;
    for (int u = 0; u < n; ++u) {
        for (int j = l->L.rp[u]; j < l->L.rp[u + 1]; ++j) A[(size_t)u * n + l->L.ci[j]] = l->L.v[j];
        for (int t = 0; t < n; ++t) A[(size_t)u * n + t] = A[(size_t)u * n + t] + one_n;
    }
    /* Cholesky A = R R^T, R lower triangular, stored in place */
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(s > 0.0)) {
            free(A);
            return ORC_ERR_STALLED;
        }
        double r = sqrt(s);
        A[(size_t)j * n + j] = r;
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = t / r;
        }
    }
    l->chol = A;
    return ORC_OK;
}

/* y = (L + 11^T/n)^{-1} (f - mean f), then y -= mean y. For a connected graph the
 * matrix is SPD and this is L^+ f (the solution of eq. (1.1)). */
static void coarsest_solve(const olevel *l, const double *f, double *y) {
    int n = l->L.n;
    if (n == 1) {
        y[0] = 0.0;
        return;
    }
    double mf = 0.0;
    for (int i = 0; i < n; ++i) mf += f[i];
    mf /= n;
    const double *R = l->chol;
    for (int i = 0; i < n; ++i) {
        double t = f[i] - mf;
        for (int k = 0; k < i; ++k) t -= R[(size_t)i * n + k] * y[k];
        y[i] = t / R[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < n; ++k) t -= R[(size_t)k * n + i] * y[k];
        y[i] = t / R[(size_t)i * n + i];
    }
    double my = 0.0;
    for (int i = 0; i < n; ++i) my += y[i];
    my /= n;
    for (int i = 0; i < n; ++i) y[i] -= my;
}

/* ------------------------------------------------------------------------- */
/* Setup: the whole hierarchy                                                  */
/* ------------------------------------------------------------------------- */

static int build_level_data(ohier *h, int l) {
    olevel *lv = &h->lev[l];
    int n = lv->L.n, nnz = lv->L.nnz;
    lv->color = (int *)malloc(sizeof(int) * (size_t)n);
    lv->strong = (unsigned char *)malloc((size_t)nnz);
    lv->X = (double *)malloc(sizeof(double) * (size_t)n * ORC_K);
    lv->aff = (double *)malloc(sizeof(double) * (size_t)nnz);
    lv->mom = (double *)malloc(sizeof(double) * (size_t)n * 9);
    lv->seed = (int *)malloc(sizeof(int) * (size_t)n);
    lv->agg = (int *)malloc(sizeof(int) * (size_t)n);
    lv->p0 = (int *)malloc(sizeof(int) * (size_t)n);
    lv->p1 = (int *)malloc(sizeof(int) * (size_t)n);
    lv->w0 = (double *)malloc(sizeof(double) * (size_t)n);
    lv->w1 = (double *)malloc(sizeof(double) * (size_t)n);
    if (!lv->color || !lv->strong || !lv->X || !lv->aff || !lv->mom || !lv->seed || !lv->agg ||
        !lv->p0 || !lv->p1 || !lv->w0 || !lv->w1)
        return ORC_ERR_ALLOC;
    const int *rp = lv->L.rp, *ci = lv->L.ci;
    const double *v = lv->L.v;
    lv->ncolors = orc_color(n, rp, ci, lv->color);
    if (lv->ncolors < 0) return ORC_ERR_ALLOC;
    orc_strong(n, rp, ci, v, h->tau_soc, h->enable_veto, lv->strong);
    orc_test_vectors(n, rp, ci, v, lv->color, lv->ncolors, h->seed, l, 3, lv->X);
    orc_affinity(n, rp, ci, lv->X, lv->aff);
    orc_moments(n, rp, ci, v, lv->X, lv->mom);
    int nc = orc_aggregate(n, rp, ci, lv->strong, lv->aff, lv->X, lv->mom, h->q_guard, lv->seed,
                           lv->agg);
    if (nc < 0) return ORC_ERR_ALLOC;
    lv->nc = nc;
    lv->n_cal2 = orc_interp(n, rp, ci, lv->strong, lv->X, lv->seed, lv->agg, nc,
                            h->enable_caliber2, h->snap, lv->p0, lv->w0, lv->p1, lv->w1);
    if (lv->n_cal2 < 0) return ORC_ERR_ALLOC;
    return ORC_OK;
}

/* Options: any value <= 0 (or NAN) selects the default. */
int orc_setup(int n, const int *rp, const int *ci, const double *w, uint64_t seed, int n_direct,
              int enable_veto, int enable_caliber2, int kappa, int enable_elim, int smoother,
              void **out) {
    *out = NULL;
    if (n < 1) return ORC_ERR_ARG;
    ohier *h = (ohier *)calloc(1, sizeof(ohier));
    if (!h) return ORC_ERR_ALLOC;
    h->seed = seed;
    h->n_direct = n_direct > 0 ? n_direct : 512;
    h->enable_veto = enable_veto;
    h->enable_caliber2 = enable_caliber2;
    h->q_guard = 2.5;   /* eq. (2.3) */
    h->tau_soc = 0.05;  /* eq. (3.1) */
    h->snap = 0.01;     /* snapping band of the caliber-2 weight (not stated in the paper) */
    h->kappa = (kappa > 0 && kappa <= 4) ? kappa : 4;
    h->enable_elim = enable_elim;
    h->elim_min = 0.1; /* an elimination level must remove at least this fraction of n */
    h->smoother = smoother;
    h->cheb_colors = 32;
    h->cheb_degree = 3;
    h->cheb_ratio = 5.0;
    h->bj_block = ORC_BJ_BLOCK;
    int rc = ORC_OK;
    /* level 0 */
    olevel *l0 = &h->lev[0];
    int nnz0 = rp[n] + n;
    l0->L.n = n;
    l0->L.nnz = nnz0;
    l0->L.rp = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    l0->L.ci = (int *)malloc(sizeof(int) * (size_t)nnz0);
    l0->L.v = (double *)malloc(sizeof(double) * (size_t)nnz0);
    if (!l0->L.rp || !l0->L.ci || !l0->L.v) {
        rc = ORC_ERR_ALLOC;
        goto fail;
    }
    orc_laplacian(n, rp, ci, w, l0->L.rp, l0->L.ci, l0->L.v);
    h->nlev = 1;
    for (int l = 0;; ++l) {
        olevel *lv = &h->lev[l];
        if (lv->L.n <= h->n_direct) {
            lv->coarsest = 1;
            break;
        }
        /* elimination and aggregation alternate: an elimination level (when it removes
         * enough nodes) comes before each aggregation step, never after another one */
        if (h->enable_elim && !(l > 0 && h->lev[l - 1].elim) && l + 1 < ORC_MAX_LEVELS) {
            int *cid = (int *)malloc(sizeof(int) * (size_t)lv->L.n);
            if (!cid) {
                rc = ORC_ERR_ALLOC;
                goto fail;
            }
            int nc = orc_elim_select(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, 4, cid);
            if ((double)(lv->L.n - nc) >= h->elim_min * (double)lv->L.n) {
                olevel *nx = &h->lev[l + 1];
                lv->elim = 1;
                lv->agg = cid;
                lv->nc = nc;
                long long cnnz =
                    orc_schur(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, cid, nc, NULL, NULL, NULL);
                if (cnnz < 0) {
                    rc = ORC_ERR_ALLOC;
                    goto fail;
                }
                nx->L.n = nc;
                nx->L.nnz = (int)cnnz;
                nx->L.rp = (int *)malloc(sizeof(int) * (size_t)(nc + 1));
                nx->L.ci = (int *)malloc(sizeof(int) * (size_t)cnnz);
                nx->L.v = (double *)malloc(sizeof(double) * (size_t)cnnz);
                if (!nx->L.rp || !nx->L.ci || !nx->L.v) {
                    rc = ORC_ERR_ALLOC;
                    goto fail;
                }
                orc_schur(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, cid, nc, nx->L.rp, nx->L.ci,
                          nx->L.v);
                h->nlev = l + 2;
                continue;
            }
            free(cid);
        }
        rc = build_level_data(h, l);
        if (rc) goto fail;
        if (h->smoother == 2 && lv->ncolors > h->cheb_colors) lv->bjgs = 1;
        if (h->smoother == 1 && lv->ncolors > h->cheb_colors) {
            lv->cheb = 1;
            lv->cheb_lmax = orc_gershgorin(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v);
        }
        if (lv->nc >= lv->L.n || l + 1 >= ORC_MAX_LEVELS) {
            /* no coarsening: a small level becomes the coarsest, a large one is an error */
            if (lv->L.n <= 1024) {
                lv->coarsest = 1;
                break;
            }
            rc = ORC_ERR_STALLED;
            goto fail;
        }
        olevel *nx = &h->lev[l + 1];
        long long cnnz = orc_galerkin(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, lv->nc, lv->p0, lv->w0,
                                      lv->p1, lv->w1, NULL, NULL, NULL);
        if (cnnz < 0) {
            rc = ORC_ERR_ALLOC;
            goto fail;
        }
        nx->L.n = lv->nc;
        nx->L.nnz = (int)cnnz;
        nx->L.rp = (int *)malloc(sizeof(int) * (size_t)(lv->nc + 1));
        nx->L.ci = (int *)malloc(sizeof(int) * (size_t)cnnz);
        nx->L.v = (double *)malloc(sizeof(double) * (size_t)cnnz);
        if (!nx->L.rp || !nx->L.ci || !nx->L.v) {
            rc = ORC_ERR_ALLOC;
            goto fail;
        }
        orc_galerkin(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, lv->nc, lv->p0, lv->w0, lv->p1, lv->w1,
                     nx->L.rp, nx->L.ci, nx->L.v);
        h->nlev = l + 2;
    }
    /* cycle index per level (eq. (2.4)); gamma = 1 above the directly solved level */
    {
        double m0 = 0.5 * (double)(h->lev[0].L.nnz - h->lev[0].L.n);
        for (int l = 0; l + 1 < h->nlev; ++l) {
            double ml = 0.5 * (double)(h->lev[l].L.nnz - h->lev[l].L.n);
            double mn = 0.5 * (double)(h->lev[l + 1].L.nnz - h->lev[l + 1].L.n);
            double tau = ml > 0.0 ? mn / ml : 1.0;
            double g;
            if (ml > 0.1 * m0)
                g = 1.5;
            else {
                g = tau > 0.0 ? 0.7 / tau : 2.0;
                if (g > 2.0) g = 2.0;
                if (g < 1.0) g = 1.0;
            }
            if (h->lev[l + 1].coarsest || h->lev[l].elim) g = 1.0;
            h->lev[l].gamma = g;
            h->lev[l].tau = tau;
        }
    }
    rc = coarsest_factor(&h->lev[h->nlev - 1]);
    if (rc) goto fail;
    *out = h;
    return ORC_OK;
fail:
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) level_free(&h->lev[l]);
    free(h);
    return rc;
}

void orc_free(void *hp) {
    ohier *h = (ohier *)hp;
    if (!h) return;
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) level_free(&h->lev[l]);
    free(h);
}

int orc_nlevels(const void *hp) { return ((const ohier *)hp)->nlev; }

/* sizes[0..8] = n, nnz, ncolors, nc, n_cal2, coarsest, elim, cheb, bjgs; sched = gamma,
 * tau, Chebyshev spectral bound */
int orc_level_info(const void *hp, int l, long long *sizes, double *sched) {
    const ohier *h = (const ohier *)hp;
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    const olevel *lv = &h->lev[l];
    sizes[0] = lv->L.n;
    sizes[1] = lv->L.nnz;
    sizes[2] = lv->ncolors;
    sizes[3] = lv->coarsest ? 0 : lv->nc;
    sizes[4] = lv->n_cal2;
    sizes[5] = lv->coarsest;
    sizes[6] = lv->elim;
    sizes[7] = lv->cheb;
    sizes[8] = lv->bjgs;
    sched[0] = lv->gamma;
    sched[1] = lv->tau;
    sched[2] = lv->cheb_lmax;
    return ORC_OK;
}

/* Copies level data into caller buffers (any pointer may be NULL; setup arrays are
 * absent on the coarsest level). */
int orc_export_level(const void *hp, int l, int *rp, int *ci, double *v, int *color,
                     unsigned char *strong, double *X, double *aff, double *mom, int *seed, int *agg,
                     int *p0, double *w0, int *p1, double *w1) {
    const ohier *h = (const ohier *)hp;
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    const olevel *lv = &h->lev[l];
    int n = lv->L.n, nnz = lv->L.nnz;
    if (rp) memcpy(rp, lv->L.rp, sizeof(int) * (size_t)(n + 1));
    if (ci) memcpy(ci, lv->L.ci, sizeof(int) * (size_t)nnz);
    if (v) memcpy(v, lv->L.v, sizeof(double) * (size_t)nnz);
    if (lv->coarsest) return ORC_OK;
    if (lv->elim) { /* only the coarse ids (-1 on F) */
        if (agg) memcpy(agg, lv->agg, sizeof(int) * (size_t)n);
        return ORC_OK;
    }
    if (color) memcpy(color, lv->color, sizeof(int) * (size_t)n);
    if (strong) memcpy(strong, lv->strong, (size_t)nnz);
    if (X) memcpy(X, lv->X, sizeof(double) * (size_t)n * ORC_K);
    if (aff) memcpy(aff, lv->aff, sizeof(double) * (size_t)nnz);
    if (mom) memcpy(mom, lv->mom, sizeof(double) * (size_t)n * 9);
    if (seed) memcpy(seed, lv->seed, sizeof(int) * (size_t)n);
    if (agg) memcpy(agg, lv->agg, sizeof(int) * (size_t)n);
    if (p0) memcpy(p0, lv->p0, sizeof(int) * (size_t)n);
    if (w0) memcpy(w0, lv->w0, sizeof(double) * (size_t)n);
    if (p1) memcpy(p1, lv->p1, sizeof(int) * (size_t)n);
    if (w1) memcpy(w1, lv->w1, sizeof(double) * (size_t)n);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Solve: gamma-cycle with (1,2) Gauss-Seidel, energy correction and iterate  */
/* recombination (Sec. 2, "Cycle and acceleration")                           */
/* ------------------------------------------------------------------------- */

typedef struct {
    const ohier *h;
    long long visits[ORC_MAX_LEVELS]; /* entries into each level's correction phase */
    double *r[ORC_MAX_LEVELS];        /* fine residual */
    double *fc[ORC_MAX_LEVELS];       /* restricted residual (lives on level l+1) */
    double *e[ORC_MAX_LEVELS];        /* coarse correction (level l+1) */
    double *rho[ORC_MAX_LEVELS];      /* coarse residual fc - L_{l+1} e */
    double *e1[ORC_MAX_LEVELS];       /* first coarse iterate of a visit */
    double *rho1[ORC_MAX_LEVELS];
    double *cr[ORC_MAX_LEVELS];       /* Chebyshev work vectors of level l */
    double *cd[ORC_MAX_LEVELS];
    double mu_last[ORC_MAX_LEVELS];
} osolver;

static void spmv_resid(const ocsr *A, const double *x, const double *f, double *r) {
    for (int u = 0; u < A->n; ++u) {
        double s = 0.0;
        for (int j = A->rp[u]; j < A->rp[u + 1]; ++j) s += A->v[j] * x[A->ci[j]];
        r[u] = f[u] - s;
    }
}

static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* One-step (two-iterate) minimal-residual recombination at a coarse level:
 * current (e, rho) and a saved (e1, rho1); E = e1 - e, G = rho - rho1 (= L E);
 * alpha = <G, rho>/<G, G>; e += alpha E; rho -= alpha G. */
static void recombine2(int n, double *e, double *rho, const double *e1, const double *rho1) {
    double gg = 0.0, gr = 0.0;
    for (int i = 0; i < n; ++i) {
        double g = rho[i] - rho1[i];
        gg += g * g;
        gr += g * rho[i];
    }
    if (!(gg > 0.0)) return;
    double a = gr / gg;
    for (int i = 0; i < n; ++i) {
        double g = rho[i] - rho1[i];
        e[i] += a * (e1[i] - e[i]);
        rho[i] -= a * g;
    }
}

/* One relaxation sweep of a level: multicolour Gauss-Seidel, or a Chebyshev or
 * block-Jacobi Gauss-Seidel sweep on the levels marked for it (work vectors r, d of the
 * level's size). */
static void smooth_level(const ohier *h, const olevel *lv, double *r, double *d, const double *f,
                         double *phi) {
    if (lv->cheb)
        orc_cheb_sweep(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, lv->cheb_lmax, h->cheb_ratio,
                       h->cheb_degree, f, phi, r, d);
    else if (lv->bjgs)
        orc_bjgs_sweep(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, h->bj_block, f, phi, r);
    else
        orc_gs_sweep_multi(lv->L.n, lv->L.rp, lv->L.ci, lv->L.v, lv->color, lv->ncolors, 1, f,
                           phi);
}

static void cycle(osolver *S, int l, double *phi, const double *f) {
    const ohier *h = S->h;
    const olevel *lv = &h->lev[l];
    int n = lv->L.n;
    if (lv->coarsest) {
        coarsest_solve(lv, f, phi);
        return;
    }
    const olevel *cl = &h->lev[l + 1];
    int nc = cl->L.n;
    double *r = S->r[l], *fc = S->fc[l], *e = S->e[l], *rho = S->rho[l];
    if (lv->elim) {
        /* elimination level (eq. (2.1)), gamma = 1: F rows exact given C; the coarse
         * right-hand side is then the residual on C (equal to P^T r with r_F = 0); one
         * visit; C takes the coarse correction; F rows exact again. No smoothing, no
         * energy correction: the interpolation is exact. */
        elim_relax_f(lv, phi, f);
        spmv_resid(&lv->L, phi, f, r);
        for (int u = 0; u < n; ++u)
            if (lv->agg[u] >= 0) fc[lv->agg[u]] = r[u];
        for (int a = 0; a < nc; ++a) e[a] = 0.0;
        S->visits[l]++;
        cycle(S, l + 1, e, fc);
        for (int u = 0; u < n; ++u)
            if (lv->agg[u] >= 0) phi[u] += e[lv->agg[u]];
        elim_relax_f(lv, phi, f);
        S->mu_last[l] = 1.0;
        return;
    }
    /* pre-relaxation: one sweep */
    smooth_level(h, lv, S->cr[l], S->cd[l], f, phi);
    spmv_resid(&lv->L, phi, f, r);
    for (int a = 0; a < nc; ++a) fc[a] = 0.0;
    for (int u = 0; u < n; ++u) {
        fc[lv->p0[u]] += lv->w0[u] * r[u];
        if (lv->p1[u] >= 0) fc[lv->p1[u]] += lv->w1[u] * r[u];
    }
    /* number of visits to level l+1: Beatty sequence of the (fractional) cycle index */
    long long i = S->visits[l]++;
    int nvis = (int)(floor((double)(i + 1) * lv->gamma) - floor((double)i * lv->gamma));
    for (int a = 0; a < nc; ++a) e[a] = 0.0;
    for (int j = 1; j <= nvis; ++j) {
        cycle(S, l + 1, e, fc);
        spmv_resid(&cl->L, e, fc, rho);
        if (j >= 2) recombine2(nc, e, rho, S->e1[l], S->rho1[l]);
        if (j < nvis) {
            memcpy(S->e1[l], e, sizeof(double) * (size_t)nc);
            memcpy(S->rho1[l], rho, sizeof(double) * (size_t)nc);
        }
    }
    /* energy correction: the L-energy-optimal multiple of the coarse correction,
     * mu = <e, fc> / <e, L_c e> with L_c e = fc - rho */
    double num = 0.0, den = 0.0;
    for (int a = 0; a < nc; ++a) {
        num += e[a] * fc[a];
        den += e[a] * (fc[a] - rho[a]);
    }
    double mu = num / den;
    if (!(den > 0.0) || !isfinite(mu)) mu = 1.0;
    S->mu_last[l] = mu;
    for (int u = 0; u < n; ++u) {
        double pe = lv->w0[u] * e[lv->p0[u]];
        if (lv->p1[u] >= 0) pe += lv->w1[u] * e[lv->p1[u]];
        phi[u] += mu * pe;
    }
    /* post-relaxation: two sweeps */
    smooth_level(h, lv, S->cr[l], S->cd[l], f, phi);
    smooth_level(h, lv, S->cr[l], S->cd[l], f, phi);
}

/* Minimal-residual recombination over up to kappa saved pairs (phi_i, r_i):
 * min || r - sum a_i G_i || with G_i = r - r_i = L (phi_i - phi). Jacobi-scaled normal
 * equations, Cholesky with pivots <= 1e-12 dropped (their a_i = 0). */
static void recombine_fine(int n, int m, double *phi, double *r, double **hphi, double **hr) {
    if (m == 0) return;
    double M[16], g[4], s[4], a[4];
    int keep[4];
    for (int i = 0; i < m; ++i) {
        g[i] = 0.0;
        for (int j = 0; j < m; ++j) M[i * 4 + j] = 0.0;
    }
    for (int x = 0; x < n; ++x) {
        double G[4];
        for (int i = 0; i < m; ++i) G[i] = r[x] - hr[i][x];
        for (int i = 0; i < m; ++i) {
            g[i] += G[i] * r[x];
            for (int j = 0; j < m; ++j) M[i * 4 + j] += G[i] * G[j];
        }
    }
    for (int i = 0; i < m; ++i) {
        s[i] = M[i * 4 + i] > 0.0 ? 1.0 / sqrt(M[i * 4 + i]) : 0.0;
        keep[i] = M[i * 4 + i] > 0.0;
    }
    double A[16], b[4];
    for (int i = 0; i < m; ++i) {
        b[i] = s[i] * g[i];
        for (int j = 0; j < m; ++j) A[i * 4 + j] = s[i] * M[i * 4 + j] * s[j];
    }
    /* Cholesky with pivot dropping */
    double R[16];
    memset(R, 0, sizeof(R));
    for (int j = 0; j < m; ++j) {
        if (!keep[j]) continue;
        double d = A[j * 4 + j];
        for (int k = 0; k < j; ++k)
            if (keep[k]) d -= R[j * 4 + k] * R[j * 4 + k];
        if (!(d > 1e-12)) {
            keep[j] = 0;
            continue;
        }
        R[j * 4 + j] = sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double t = A[i * 4 + j];
            for (int k = 0; k < j; ++k)
                if (keep[k]) t -= R[i * 4 + k] * R[j * 4 + k];
            R[i * 4 + j] = t / R[j * 4 + j];
        }
    }
    double y[4];
    for (int i = 0; i < m; ++i) {
        y[i] = 0.0;
        if (!keep[i]) continue;
        double t = b[i];
        for (int k = 0; k < i; ++k)
            if (keep[k]) t -= R[i * 4 + k] * y[k];
        y[i] = t / R[i * 4 + i];
    }
    for (int i = m - 1; i >= 0; --i) {
        a[i] = 0.0;
        if (!keep[i]) continue;
        double t = y[i];
        for (int k = i + 1; k < m; ++k)
            if (keep[k]) t -= R[k * 4 + i] * a[k];
        a[i] = t / R[i * 4 + i];
    }
    for (int i = 0; i < m; ++i) a[i] *= s[i];
    for (int x = 0; x < n; ++x) {
        double dp = 0.0, dr = 0.0;
        for (int i = 0; i < m; ++i) {
            dp += a[i] * (hphi[i][x] - phi[x]);
            dr += a[i] * (r[x] - hr[i][x]);
        }
        phi[x] += dp;
        r[x] -= dr;
    }
}

/* Asymptotic convergence factor (Sec. 4.1): the geometric mean of the last five
 * per-cycle reductions rels[i] / rels[i-1], i.e. (rels[last] / rels[last-5])^(1/5), or of all
 * of them when fewer than five cycles ran. rels[0] is the starting relative residual (1).
 * 0 when there is no reduction to average or an end point is not positive.
 * Pinned: geometric histories give their ratio; hand-built histories against the mean of
 * their printed ratios. */
double orc_acf(const double *rels, int nrels) {
    int last = nrels - 1, cnt = last < 5 ? last : 5;
    if (cnt <= 0 || !(rels[last - cnt] > 0.0) || !(rels[last] > 0.0)) return 0.0;
    return pow(rels[last] / rels[last - cnt], 1.0 / cnt);
}

/* Solve L phi = b (eq. (1.1)) for one right-hand side: b is projected to mean zero,
 * cycles run until ||r||/||b|| <= tol or max_cycles; phi is returned mean-zero.
 * hist (max_cycles+1 entries, may be NULL) receives relres after each cycle (hist[0]=1).
 * stats[0] = cycles, stats[1] = final true relres, stats[2] = ACF (geometric mean of
 * the last <= 5 per-cycle reductions), stats[3] = last finest-level mu.
 * Returns ORC_OK, ORC_NOT_CONVERGED (the tolerance was not met within max_cycles, or the
 * relative residual stopped being a finite number: cycling stops there), or ORC_ERR_ARG
 * when b holds a value that is not finite (its norm is then not finite either: eq. (1.1)
 * has no solution to approach; phi is set to 0). */
int orc_solve(const void *hp, const double *b_in, double tol, int max_cycles, double *phi,
              double *hist, double *stats) {
    const ohier *h = (const ohier *)hp;
    const olevel *l0 = &h->lev[0];
    int n = l0->L.n;
    osolver S;
    memset(&S, 0, sizeof(S));
    S.h = h;
    int rc = ORC_OK;
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    int kap = h->kappa;
    double *hphi[4], *hr[4];
    for (int i = 0; i < kap; ++i) {
        hphi[i] = (double *)malloc(sizeof(double) * (size_t)n);
        hr[i] = (double *)malloc(sizeof(double) * (size_t)n);
    }
    for (int l = 0; l + 1 < h->nlev; ++l) {
        int nf = h->lev[l].L.n, nc = h->lev[l + 1].L.n;
        S.r[l] = (double *)malloc(sizeof(double) * (size_t)nf);
        S.fc[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.e[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.rho[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.e1[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.rho1[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.cr[l] = (double *)malloc(sizeof(double) * (size_t)nf);
        S.cd[l] = (double *)malloc(sizeof(double) * (size_t)nf);
    }
    double mb = 0.0;
    for (int i = 0; i < n; ++i) mb += b_in[i];
    mb /= n;
    for (int i = 0; i < n; ++i) b[i] = b_in[i] - mb;
    double nb = sqrt(dot(n, b, b));
    for (int i = 0; i < n; ++i) phi[i] = 0.0;
    if (hist) hist[0] = 1.0;
    int cyc = 0;
    double rel = 1.0, acf = 0.0;
    if (!isfinite(nb)) {
        stats[0] = 0;
        stats[1] = NAN;
        stats[2] = 0.0;
        stats[3] = 1.0;
        rc = ORC_ERR_ARG;
        goto done;
    }
    if (nb == 0.0) {
        stats[0] = 0;
        stats[1] = 0.0;
        stats[2] = 0.0;
        stats[3] = 1.0;
        goto done;
    }
    /* history starts with the zero iterate and its residual b */
    int hm = 1, hnext = 1;
    for (int i = 0; i < n; ++i) {
        hphi[0][i] = 0.0;
        hr[0][i] = b[i];
    }
    double rels[1024];
    int nrels = 0;
    rels[nrels++] = 1.0;
    while (!(rel <= tol) && isfinite(rel) && cyc < max_cycles) {
        cycle(&S, 0, phi, b);
        spmv_resid(&l0->L, phi, b, r);
        if (!l0->coarsest) {
            recombine_fine(n, hm, phi, r, hphi, hr);
            int slot = hnext % kap;
            memcpy(hphi[slot], phi, sizeof(double) * (size_t)n);
            memcpy(hr[slot], r, sizeof(double) * (size_t)n);
            hnext++;
            if (hm < kap) hm++;
        }
        ++cyc;
        rel = sqrt(dot(n, r, r)) / nb;
        if (hist) hist[cyc] = rel;
        if (nrels < 1024) rels[nrels++] = rel;
    }
    acf = orc_acf(rels, nrels);
    {
        double mp = 0.0;
        for (int i = 0; i < n; ++i) mp += phi[i];
        mp /= n;
        for (int i = 0; i < n; ++i) phi[i] -= mp;
    }
    spmv_resid(&l0->L, phi, b, r);
    stats[0] = cyc;
    stats[1] = sqrt(dot(n, r, r)) / nb;
    stats[2] = acf;
    stats[3] = S.mu_last[0];
    if (!(rel <= tol)) rc = ORC_NOT_CONVERGED;
done:
    free(b);
    free(r);
    for (int i = 0; i < kap; ++i) {
        free(hphi[i]);
        free(hr[i]);
    }
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
        free(S.r[l]);
        free(S.fc[l]);
        free(S.e[l]);
        free(S.rho[l]);
        free(S.e1[l]);
        free(S.rho1[l]);
        free(S.cr[l]);
        free(S.cd[l]);
    }
    return rc;
}

/* Diagnostic: ncyc cycles from phi with f (visit counters persisting across them, as in
 * one solve), returning the finest-level energy correction factor mu of the last (used to
 * pin mu = 1 under an exact coarse solve); visits_out (nullable, nlev entries) receives
 * the entries into each level's correction phase (used to pin the cycle schedule). */
double orc_cycles(const void *hp, double *phi, const double *f, int ncyc, long long *visits_out) {
    const ohier *h = (const ohier *)hp;
    osolver S;
    memset(&S, 0, sizeof(S));
    S.h = h;
    for (int l = 0; l + 1 < h->nlev; ++l) {
        int nf = h->lev[l].L.n, nc = h->lev[l + 1].L.n;
        S.r[l] = (double *)malloc(sizeof(double) * (size_t)nf);
        S.fc[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.e[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.rho[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.e1[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.rho1[l] = (double *)malloc(sizeof(double) * (size_t)nc);
        S.cr[l] = (double *)malloc(sizeof(double) * (size_t)nf);
        S.cd[l] = (double *)malloc(sizeof(double) * (size_t)nf);
    }
    S.mu_last[0] = 1.0;
    for (int c = 0; c < ncyc; ++c) cycle(&S, 0, phi, f);
    double mu = S.mu_last[0];
    if (visits_out)
        for (int l = 0; l < h->nlev; ++l) visits_out[l] = S.visits[l];
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
        free(S.r[l]);
        free(S.fc[l]);
        free(S.e[l]);
        free(S.rho[l]);
        free(S.e1[l]);
        free(S.rho1[l]);
        free(S.cr[l]);
        free(S.cd[l]);
    }
    return mu;
}

double orc_cycle_once(const void *hp, double *phi, const double *f) {
    return orc_cycles(hp, phi, f, 1, NULL);
}

/* Exposed for the recombination pin: one coarse two-iterate recombination on caller data
 * (e, rho updated in place from the saved pair e1, rho1). */
void orc_recombine2(int n, double *e, double *rho, const double *e1, const double *rho1) {
    recombine2(n, e, rho, e1, rho1);
}

/* Exposed for the recombination pin: one fine-level recombination on caller data. */
void orc_recombine(int n, int m, double *phi, double *r, double *const *hphi, double *const *hr) {
    double *a[4], *b[4];
    for (int i = 0; i < m && i < 4; ++i) {
        a[i] = hphi[i];
        b[i] = hr[i];
    }
    recombine_fine(n, m < 4 ? m : 4, phi, r, a, b);
}
