// Host side of lamg_setup: input validation, the sequential greedy steps (colouring,
// aggregation), the cycle-index rule, and the colour-permuted solve layout. The
// data-parallel pieces (Laplacian, veto, test vectors, affinities, moments, caliber-2,
// Galerkin operator, coarsest inverse) run in setup_kernels.hip.
//
// Compiled with -ffp-contract=off: the guard comparison below must round exactly like
// the canonical arithmetic of the setup kernels.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <optional>
#include <cmath>
#include <cstdlib>
#include <system_error>
#include <thread>

#include "lamg_internal.h"

namespace lamg {

// ---------------------------------------------------------------------------
// Input validation (eq. (1.1) needs a connected graph with positive weights)
// ---------------------------------------------------------------------------
struct HostGraph {
    int64_t n = 0, nnz = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> w;
};

static HostGraph read_graph(const lamg_graph *g, hipStream_t s) {
    if (!g || g->n < 1 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && (!g->col_idx || !g->weight)))
        throw Error(LAMG_INVALID_ARG, "graph: null pointer or bad size");
    if (g->n >= (int64_t)INT32_MAX || g->nnz >= (int64_t)INT32_MAX - g->n)
        throw Error(LAMG_INVALID_ARG, "graph: too large for 32-bit indices");
    HostGraph h;
    h.n = g->n;
    h.nnz = g->nnz;
    h.rp.resize(h.n + 1);
    h.ci.resize(h.nnz);
    h.w.resize(h.nnz);
    if (g->mem == LAMG_MEM_DEVICE) {
        LAMG_HIP(hipMemcpyAsync(h.rp.data(), g->row_ptr, 4 * (h.n + 1), hipMemcpyDeviceToHost, s));
        if (h.nnz) {
            LAMG_HIP(hipMemcpyAsync(h.ci.data(), g->col_idx, 4 * h.nnz, hipMemcpyDeviceToHost, s));
            LAMG_HIP(hipMemcpyAsync(h.w.data(), g->weight, 8 * h.nnz, hipMemcpyDeviceToHost, s));
        }
        LAMG_HIP(hipStreamSynchronize(s));
    } else if (g->mem == LAMG_MEM_HOST) {
        std::memcpy(h.rp.data(), g->row_ptr, 4 * (h.n + 1));
        if (h.nnz) {
            std::memcpy(h.ci.data(), g->col_idx, 4 * h.nnz);
            std::memcpy(h.w.data(), g->weight, 8 * h.nnz);
        }
    } else {
        throw Error(LAMG_INVALID_ARG, "graph: unknown memory kind");
    }
    if (h.rp[0] != 0 || h.rp[h.n] != h.nnz) throw Error(LAMG_INVALID_ARG, "graph: row_ptr ends");
    for (int64_t u = 0; u < h.n; ++u) {
        if (h.rp[u + 1] < h.rp[u]) throw Error(LAMG_INVALID_ARG, "graph: row_ptr not monotone");
        for (int32_t j = h.rp[u]; j < h.rp[u + 1]; ++j) {
            int32_t c = h.ci[j];
            if (c < 0 || c >= h.n) throw Error(LAMG_INVALID_ARG, "graph: column out of range");
            if (j > h.rp[u] && c <= h.ci[j - 1])
                throw Error(LAMG_INVALID_ARG, "graph: columns not strictly ascending");
            if (c == u) throw Error(LAMG_SELF_LOOP, "graph: self loop");
            double w = h.w[j];
            if (!(w > 0.0) || !std::isfinite(w)) throw Error(LAMG_BAD_WEIGHT, "graph: weight");
        }
    }
    // symmetry: every stored (u, v, w) has its (v, u, w); the entries are split evenly over
    // up to 16 host threads (the binary searches into other rows are cache misses, so the
    // check is latency-bound and scales with threads)
    {
        const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::atomic<bool> sym{true};
        auto check = [&](int t) {
            const int64_t e0 = h.nnz * t / nt, e1 = h.nnz * (t + 1) / nt;
            int64_t u = std::upper_bound(h.rp.begin(), h.rp.end(), (int32_t)e0) - h.rp.begin() - 1;
            for (; u < h.n && h.rp[u] < e1; ++u) {
                if (!sym.load(std::memory_order_relaxed)) return;
                const int32_t ja = (int32_t)std::max<int64_t>(h.rp[u], e0);
                const int32_t jb = (int32_t)std::min<int64_t>(h.rp[u + 1], e1);
                for (int32_t j = ja; j < jb; ++j) {
                    const int32_t v = h.ci[j];
                    const int32_t *b = h.ci.data() + h.rp[v], *e = h.ci.data() + h.rp[v + 1];
                    const int32_t *it = std::lower_bound(b, e, (int32_t)u);
                    if (it == e || *it != u || h.w[it - h.ci.data()] != h.w[j]) {
                        sym.store(false, std::memory_order_relaxed);
                        return;
                    }
                }
            }
        };
        std::vector<std::thread> th;
        for (int t = 1; t < nt; ++t) {
            try {
                th.emplace_back(check, t);
            } catch (const std::system_error &) {
                check(t);  // no thread available: this share runs here
            }
        }
        check(0);
        for (std::thread &x : th) x.join();
        if (!sym.load()) throw Error(LAMG_NOT_SYMMETRIC, "graph: not symmetric");
    }
    // connectivity (breadth-first search from node 0)
    std::vector<uint8_t> seen(h.n, 0);
    std::vector<int32_t> q;
    q.reserve(h.n);
    q.push_back(0);
    seen[0] = 1;
    for (size_t i = 0; i < q.size(); ++i) {
        int32_t u = q[i];
        for (int32_t j = h.rp[u]; j < h.rp[u + 1]; ++j)
            if (!seen[h.ci[j]]) {
                seen[h.ci[j]] = 1;
                q.push_back(h.ci[j]);
            }
    }
    if ((int64_t)q.size() != h.n) throw Error(LAMG_DISCONNECTED, "graph: not connected");
    return h;
}

// Self-gated reverse Cuthill-McKee renumbering of the input (the reordering for cache
// locality that Sec. 4.2 lists among the implementation's constant-lowering features):
// order[new] = old. Components are taken in the order of their smallest node; each starts
// at a pseudo-peripheral node (George-Liu: from the component's node of least degree, ties
// to the smallest index, move to the least-degree node of the farthest breadth-first level
// while that lengthens the eccentricity); Cuthill-McKee numbers breadth first, each node's
// not yet numbered neighbours by increasing degree (ties: smallest index); the whole
// sequence is reversed. Kept only if it at least halves the summed index distance |u - v|
// over the entries; returns whether it is kept.
static bool rcm_order(const HostGraph &g, std::vector<int32_t> &order) {
    const int64_t n = g.n;
    auto deg = [&](int32_t u) { return g.rp[u + 1] - g.rp[u]; };
    auto less = [&](int32_t a, int32_t b) { return deg(a) < deg(b) || (deg(a) == deg(b) && a < b); };
    std::vector<int32_t> dist(n, -1), queue;
    queue.reserve(n);
    std::vector<char> numbered(n, 0);
    // breadth-first distances from r over its component (the component's nodes in queue);
    // returns r's eccentricity
    auto bfs = [&](int32_t r) {
        for (int32_t u : queue) dist[u] = -1;
        queue.clear();
        queue.push_back(r);
        dist[r] = 0;
        for (size_t q = 0; q < queue.size(); ++q) {
            const int32_t u = queue[q];
            for (int32_t j = g.rp[u]; j < g.rp[u + 1]; ++j) {
                const int32_t v = g.ci[j];
                if (dist[v] < 0) {
                    dist[v] = dist[u] + 1;
                    queue.push_back(v);
                }
            }
        }
        return dist[queue.back()];
    };
    order.clear();
    order.reserve(n);
    std::vector<int32_t> nb;
    for (int32_t s0 = 0; s0 < n; ++s0) {
        if (numbered[s0]) continue;
        bfs(s0);
        int32_t r = queue[0];
        for (int32_t u : queue)
            if (less(u, r)) r = u;
        int32_t ecc = bfs(r);
        for (;;) {
            int32_t x = -1;
            for (int32_t u : queue)
                if (dist[u] == ecc && (x < 0 || less(u, x))) x = u;
            const int32_t ex = bfs(x);
            if (ex <= ecc) break;
            r = x;
            ecc = ex;
        }
        size_t head = order.size();
        order.push_back(r);
        numbered[r] = 1;
        for (; head < order.size(); ++head) {
            const int32_t u = order[head];
            nb.clear();
            for (int32_t j = g.rp[u]; j < g.rp[u + 1]; ++j) {
                const int32_t v = g.ci[j];
                if (!numbered[v]) {
                    numbered[v] = 1;
                    nb.push_back(v);
                }
            }
            std::sort(nb.begin(), nb.end(), less);
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    std::vector<int32_t> inv(n);
    for (int64_t i = 0; i < n; ++i) inv[order[i]] = (int32_t)i;
    int64_t d0 = 0, d1 = 0;
    for (int64_t u = 0; u < n; ++u)
        for (int32_t j = g.rp[u]; j < g.rp[u + 1]; ++j) {
            d0 += std::llabs(u - (int64_t)g.ci[j]);
            d1 += std::llabs((int64_t)inv[u] - (int64_t)inv[g.ci[j]]);
        }
    return 2 * d1 <= d0;
}

// The graph with node order[p] renamed p, columns ascending again in every row.
static void renumber(HostGraph &g, const std::vector<int32_t> &order) {
    const int64_t n = g.n;
    std::vector<int32_t> inv(n), rp(n + 1, 0), ci(g.nnz);
    std::vector<double> w(g.nnz);
    for (int64_t i = 0; i < n; ++i) inv[order[i]] = (int32_t)i;
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t p = 0; p < n; ++p) {
        const int32_t u = order[p];
        row.clear();
        for (int32_t j = g.rp[u]; j < g.rp[u + 1]; ++j) row.emplace_back(inv[g.ci[j]], g.w[j]);
        std::sort(row.begin(), row.end(),
                  [](const auto &a, const auto &b) { return a.first < b.first; });
        rp[p + 1] = rp[p] + (int32_t)row.size();
        for (size_t e = 0; e < row.size(); ++e) {
            ci[rp[p] + e] = row[e].first;
            w[rp[p] + e] = row[e].second;
        }
    }
    g.rp.swap(rp);
    g.ci.swap(ci);
    g.w.swap(w);
}

// Adds the wall time of its scope to one of the handle's setup phases; each scope ends with
// its device work complete (the stream is synchronised before it closes).
struct PhaseClock {
    double &acc;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    PhaseClock(lamg_handle *h, lamg_setup_phase p) : acc(h->setup_phase[p]) {}
    ~PhaseClock() {
        acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// ---------------------------------------------------------------------------
// Natural-order greedy colouring: colour(u) = smallest colour unused by neighbours v < u.
// ---------------------------------------------------------------------------
static int greedy_color(int64_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                        std::vector<int32_t> &color) {
    color.assign(n, 0);
    std::vector<int64_t> used;
    int ncol = 0;
    for (int64_t u = 0; u < n; ++u) {
        int deg = rp[u + 1] - rp[u];
        if ((int)used.size() < deg + 2) used.resize(deg + 2, -1);
        for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
            int32_t v = ci[j];
            if (v < u && color[v] < (int)used.size()) used[color[v]] = u;
        }
        int c = 0;
        while (c < (int)used.size() && used[c] == u) ++c;
        color[u] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// ---------------------------------------------------------------------------
// Low-degree elimination set (Sec. 2, "Low-degree elimination"): one pass in index order;
// a node with at most kElimMaxDegree neighbours and a positive diagonal is eliminated
// unless a neighbour already is, which makes F a maximal independent set of those nodes.
// The kept nodes are numbered in index order (cid), eliminated ones get -1. Returns |C|.
// ---------------------------------------------------------------------------
static int64_t elimination_set(int64_t n, const std::vector<int32_t> &rp,
                               const std::vector<int32_t> &ci, const std::vector<double> &diag,
                               std::vector<int32_t> &cid) {
    std::vector<uint8_t> out(n, 0);
    for (int64_t u = 0; u < n; ++u) {
        if (rp[u + 1] - rp[u] - 1 > kElimMaxDegree || !(diag[u] > 0.0)) continue;
        bool free_ = true;
        for (int32_t j = rp[u]; j < rp[u + 1] && free_; ++j) free_ = !out[ci[j]];
        out[u] = free_ ? 1 : 0;
    }
    cid.resize(n);
    int64_t nc = 0;
    for (int64_t u = 0; u < n; ++u) cid[u] = out[u] ? -1 : (int32_t)nc++;
    return nc;
}

// Makes level l an elimination level with its Schur complement as level l + 1 when the
// elimination set holds at least kElimMinFrac of the nodes; returns whether it did.
static bool try_elimination(lamg_handle *h, int l) {
    Pool &pool = *h->pool;
    hipStream_t s = h->stream;
    Level &L = h->lev[l];
    const int64_t n = L.n;
    std::vector<double> diag(n);
    {
        DArr<double> d;
        d.alloc(pool, n);
        launch_diag(n, L.rp.p, L.ci.p, L.val.p, d.p, s);
        d.download(diag.data(), n, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }
    std::vector<int32_t> cid;
    const int64_t nc = elimination_set(n, L.h_rp, L.h_ci, diag, cid);
    if (!((double)(n - nc) >= kElimMinFrac * (double)n)) return false;
    L.elim = true;
    L.nc = nc;
    L.h_agg = std::move(cid);
    L.ncolors = 2;  // solve layout: eliminated rows first, then the kept ones
    L.h_color.resize(n);
    for (int64_t u = 0; u < n; ++u) L.h_color[u] = L.h_agg[u] < 0 ? 0 : 1;
    h->lev.emplace_back();
    Level &C = h->lev[l + 1];
    Level &F = h->lev[l];
    DArr<int32_t> d_cid;
    d_cid.alloc(pool, n);
    d_cid.upload(F.h_agg.data(), n, s);
    C.n = nc;
    C.nnz = schur(pool, n, F.rp.p, F.ci.p, F.val.p, d_cid.p, nc, C.rp, C.ci, C.val, s);
    C.h_rp.resize(C.n + 1);
    C.h_ci.resize(C.nnz);
    C.rp.download(C.h_rp.data(), C.n + 1, s);
    C.ci.download(C.h_ci.data(), C.nnz, s);
    LAMG_HIP(hipStreamSynchronize(s));
    return true;
}

// ---------------------------------------------------------------------------
// Greedy aggregation (Sec. 2 "Caliber-1 aggregation", Sec. 3.1): one pass in index
// order; an undecided node joins the admissible strong neighbour (undecided or seed)
// of largest affinity -- first in CSR order on ties -- which becomes a seed; with none
// it stays a singleton seed. Admissible: the energy-ratio guard eq. (2.3) evaluated by
// the App. B moments, multiplied out: (xs^2 s0 - 2 xs s1) + s2 <= Q (s2 - s1^2/s0) for all k.
// ---------------------------------------------------------------------------
static inline bool guard_ok(const double *m, const double *xs) {
    double s0 = m[0];
    for (int k = 0; k < kTV; ++k) {
        double s1 = m[1 + k], s2 = m[5 + k], x = xs[k];
        double m2 = s2 - (s1 * s1) / s0;
        double f2 = ((x * x) * s0 - (2.0 * x) * s1) + s2;
        if (!(f2 <= kGuardQ * m2)) return false;
    }
    return true;
}

static int64_t greedy_aggregate(int64_t n, const std::vector<int32_t> &rp,
                                const std::vector<int32_t> &ci, const std::vector<uint8_t> &strong,
                                const std::vector<double> &aff, const std::vector<double> &X,
                                const std::vector<double> &mom, std::vector<int32_t> &seed,
                                std::vector<int32_t> &agg) {
    enum : uint8_t { UND = 0, SEED = 1, MEMBER = 2 };
    std::vector<uint8_t> st(n, UND);
    seed.assign(n, -1);
    agg.assign(n, -1);
    for (int64_t u = 0; u < n; ++u) {
        if (st[u] != UND) continue;
        int32_t best = -1;
        double bestc = -1.0;
        const double *mu = mom.data() + 9 * u;
        for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
            if (!strong[j]) continue;
            int32_t v = ci[j];
            if (st[v] == MEMBER) continue;
            if (!guard_ok(mu, X.data() + (int64_t)kTV * v)) continue;
            if (aff[j] > bestc) {
                bestc = aff[j];
                best = v;
            }
        }
        if (best >= 0) {
            st[best] = SEED;
            seed[best] = best;
            st[u] = MEMBER;
            seed[u] = best;
        } else {
            st[u] = SEED;
            seed[u] = (int32_t)u;
        }
    }
    int64_t nc = 0;
    for (int64_t u = 0; u < n; ++u)
        if (st[u] == SEED) agg[u] = (int32_t)nc++;
    for (int64_t u = 0; u < n; ++u)
        if (st[u] == MEMBER) agg[u] = agg[seed[u]];
    return nc;
}

// ---------------------------------------------------------------------------
// One level's setup
// ---------------------------------------------------------------------------
static void setup_level(lamg_handle *h, int l) {
    Pool &pool = *h->pool;
    hipStream_t s = h->stream;
    Level &L = h->lev[l];
    const int64_t n = L.n, nnz = L.nnz;

    {
        PhaseClock pc(h, LAMG_SETUP_COLOR);
        L.ncolors = greedy_color(n, L.h_rp, L.h_ci, L.h_color);
    }
    std::optional<PhaseClock> pc_level(std::in_place, h, LAMG_SETUP_LEVEL);
    // rows of each colour: those with at most kTVShortRow stored entries ascending, then the
    // longer ones ascending (rows of one colour are independent, so the order only decides
    // which kernel relaxes them)
    std::vector<int64_t> coff(L.ncolors + 1, 0), clong(L.ncolors, 0);
    auto is_long = [&](int64_t u) { return L.h_rp[u + 1] - L.h_rp[u] > kTVShortRow; };
    for (int64_t u = 0; u < n; ++u) {
        coff[L.h_color[u] + 1]++;
        if (!is_long(u)) clong[L.h_color[u]]++;
    }
    for (int c = 0; c < L.ncolors; ++c) coff[c + 1] += coff[c];
    std::vector<int32_t> crow(n);
    {
        std::vector<int64_t> pos_s(coff.begin(), coff.end() - 1), pos_l(L.ncolors);
        for (int c = 0; c < L.ncolors; ++c) pos_l[c] = coff[c] + clong[c];
        for (int64_t u = 0; u < n; ++u) {
            const int c = L.h_color[u];
            crow[is_long(u) ? pos_l[c]++ : pos_s[c]++] = (int32_t)u;
        }
        for (int c = 0; c < L.ncolors; ++c) clong[c] += coff[c];  // start of the long rows
    }
    DArr<int32_t> d_crow;
    d_crow.alloc(pool, n);
    d_crow.upload(crow.data(), n, s);

    L.strong.alloc(pool, nnz);
    launch_strong(n, L.rp.p, L.ci.p, L.val.p, kTauSoc, h->opt.enable_veto, L.strong.p, s);
    L.X.alloc(pool, n * kTV);
    launch_tv_init(n, h->opt.seed, l, L.X.p, s);
    for (int sw = 0; sw < kTVSweeps; ++sw)
        for (int c = 0; c < L.ncolors; ++c) {
            launch_tv_sweep_color(clong[c] - coff[c], d_crow.p + coff[c], L.rp.p, L.ci.p, L.val.p,
                                  L.X.p, s);
            launch_tv_sweep_long(coff[c + 1] - clong[c], d_crow.p + clong[c], L.rp.p, L.ci.p,
                                 L.val.p, L.X.p, s);
        }
    L.aff.alloc(pool, nnz);
    {
        DArr<double> sig;
        sig.alloc(pool, n);
        launch_affinity(n, L.rp.p, L.ci.p, L.X.p, sig.p, L.aff.p, s);
        L.mom.alloc(pool, n * 9);
        launch_moments(n, L.rp.p, L.ci.p, L.val.p, L.X.p, L.mom.p, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }
    std::vector<uint8_t> hs(nnz);
    std::vector<double> ha(nnz), hx(n * kTV), hm(n * 9);
    L.strong.download(hs.data(), nnz, s);
    L.aff.download(ha.data(), nnz, s);
    L.X.download(hx.data(), n * kTV, s);
    L.mom.download(hm.data(), n * 9, s);
    LAMG_HIP(hipStreamSynchronize(s));
    pc_level.reset();

    {
        PhaseClock pc(h, LAMG_SETUP_AGGREGATE);
        L.nc = greedy_aggregate(n, L.h_rp, L.h_ci, hs, ha, hx, hm, L.h_seed, L.h_agg);
    }
    if (L.nc >= n || l + 1 >= kMaxLevels) return;  // caller decides (stall)
    PhaseClock pc_interp(h, LAMG_SETUP_INTERP);

    std::vector<int32_t> aggseed(L.nc);
    for (int64_t u = 0; u < n; ++u)
        if (L.h_seed[u] == u) aggseed[L.h_agg[u]] = (int32_t)u;
    DArr<int32_t> d_seed, d_agg, d_aggseed;
    d_seed.alloc(pool, n);
    d_agg.alloc(pool, n);
    d_aggseed.alloc(pool, L.nc);
    d_seed.upload(L.h_seed.data(), n, s);
    d_agg.upload(L.h_agg.data(), n, s);
    d_aggseed.upload(aggseed.data(), L.nc, s);
    L.p0.alloc(pool, n);
    L.p1.alloc(pool, n);
    L.w0.alloc(pool, n);
    L.w1.alloc(pool, n);
    launch_interp(n, L.rp.p, L.ci.p, L.strong.p, L.X.p, d_seed.p, d_agg.p, d_aggseed.p,
                  h->opt.enable_caliber2, kSnap, L.p0.p, L.w0.p, L.p1.p, L.w1.p, s);
    LAMG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Solve layout of a level: permutation to (class, colour, index), permuted off-diagonal
// CSR + diagonal, and (for non-coarsest levels) interpolation and restriction in the
// solve numbering of both levels.
// ---------------------------------------------------------------------------
static int pick_lpr(double mean_len) {
    if (mean_len <= 6.0) return 1;
    if (mean_len <= 12.0) return 2;
    if (mean_len <= 24.0) return 4;
    return 8;
}

static void compute_perm(Level &L, std::vector<int32_t> &perm, std::vector<int32_t> &iperm) {
    const int64_t n = L.n;
    const int nc = L.coarsest ? 1 : L.ncolors;
    auto color_of = [&](int64_t u) { return L.coarsest ? 0 : L.h_color[u]; };
    // the directly solved level keeps its canonical numbering (its inverse is stored in it)
    auto cls_of = [&](int64_t u) {
        return (!L.coarsest && (L.h_rp[u + 1] - L.h_rp[u] - 1) > kLongRow) ? 1 : 0;
    };
    std::vector<int64_t> cnt(2 * nc + 1, 0);
    for (int64_t u = 0; u < n; ++u) cnt[cls_of(u) * nc + color_of(u) + 1]++;
    for (int b = 0; b < 2 * nc; ++b) cnt[b + 1] += cnt[b];
    L.op.blk = cnt;
    L.op.ncolors = nc;
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    perm.resize(n);
    iperm.resize(n);
    for (int64_t u = 0; u < n; ++u) {
        int64_t i = pos[cls_of(u) * nc + color_of(u)]++;
        perm[i] = (int32_t)u;
        iperm[u] = (int32_t)i;
    }
}

static void build_solve_op(lamg_handle *h, int l, const std::vector<int32_t> &perm,
                           const std::vector<int32_t> &iperm, const std::vector<int32_t> *iperm_next) {
    Pool &pool = *h->pool;
    hipStream_t s = h->stream;
    Level &L = h->lev[l];
    SolveOp &op = L.op;
    const int64_t n = L.n;
    const bool f32 = h->opt.build_fp32 != 0;
    op.n = n;
    // permuted off-diagonal row pointers
    std::vector<int32_t> srp(n + 1, 0);
    double short_len = 0.0;
    int64_t nshort = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t u = perm[i];
        int32_t len = L.h_rp[u + 1] - L.h_rp[u] - 1;
        srp[i + 1] = srp[i] + len;
        if (len <= kLongRow) {
            short_len += len;
            ++nshort;
        }
    }
    op.nnz_off = srp[n];
    op.lpr_short = pick_lpr(nshort ? short_len / nshort : 1.0);
    op.max_short_len = 0;
    op.max_len = 0;
    for (int64_t i = 0; i < n; ++i) op.max_len = std::max(op.max_len, srp[i + 1] - srp[i]);
    if (nshort == n)
        for (int64_t i = 0; i < n; ++i) op.max_short_len = std::max(op.max_short_len, srp[i + 1] - srp[i]);
    op.blk_nnz.resize(op.blk.size());
    for (size_t b = 0; b < op.blk.size(); ++b) op.blk_nnz[b] = srp[op.blk[b]];
    op.dblk.alloc(pool, (int64_t)op.blk.size());
    op.dblk.upload(op.blk.data(), (int64_t)op.blk.size(), s);
    DArr<int32_t> d_iperm;
    op.perm.alloc(pool, n);
    d_iperm.alloc(pool, n);
    op.rp.alloc(pool, n + 1);
    op.ci.alloc(pool, op.nnz_off);
    op.v64.alloc(pool, op.nnz_off);
    op.d64.alloc(pool, n);
    op.dinv64.alloc(pool, n);
    if (f32) {
        op.v32.alloc(pool, op.nnz_off);
        op.d32.alloc(pool, n);
        op.dinv32.alloc(pool, n);
    }
    op.perm.upload(perm.data(), n, s);
    d_iperm.upload(iperm.data(), n, s);
    op.rp.upload(srp.data(), n + 1, s);
    launch_permute_csr(n, op.perm.p, d_iperm.p, L.rp.p, L.ci.p, L.val.p, op.rp.p, op.ci.p, op.v64.p,
                       f32 ? op.v32.p : nullptr, op.d64.p, op.dinv64.p, f32 ? op.d32.p : nullptr,
                       f32 ? op.dinv32.p : nullptr, s);
    if (L.bjgs) {
        // block-Jacobi Gauss-Seidel: rows in natural order and, per row, its entries inside
        // its block (canonical entry order kept)
        std::vector<double> hv((size_t)L.nnz);
        L.val.download(hv.data(), L.nnz, s);
        LAMG_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> irp(n + 1, 0);
        std::vector<uint8_t> iloc;
        std::vector<double> iv;
        for (int64_t u = 0; u < n; ++u) {
            const int64_t b0 = (u / kBjBlock) * kBjBlock;
            for (int32_t j = L.h_rp[u]; j < L.h_rp[u + 1]; ++j) {
                const int32_t c = L.h_ci[j];
                if (c != u && c >= b0 && c < b0 + kBjBlock) {
                    iloc.push_back((uint8_t)(c - b0));
                    iv.push_back(hv[j]);
                }
            }
            irp[u + 1] = (int32_t)iloc.size();
        }
        const int64_t ni = (int64_t)iloc.size();
        op.bj_ni = ni;
        op.bj_rows.alloc(pool, n);
        op.bj_irp.alloc(pool, n + 1);
        op.bj_iloc.alloc(pool, std::max<int64_t>(ni, 1));
        op.bj_iv64.alloc(pool, std::max<int64_t>(ni, 1));
        op.bj_rows.upload(iperm.data(), n, s);
        op.bj_irp.upload(irp.data(), n + 1, s);
        op.bj_iloc.upload(iloc.data(), ni, s);
        op.bj_iv64.upload(iv.data(), ni, s);
        std::vector<float> iv32;
        if (f32) {
            iv32.assign(iv.begin(), iv.end());
            op.bj_iv32.alloc(pool, std::max<int64_t>(ni, 1));
            op.bj_iv32.upload(iv32.data(), ni, s);
        }
        // the uploads read host vectors that end with this block
        LAMG_HIP(hipStreamSynchronize(s));
    }
    // ELL copy for the coarse tail: every row (long ones too) of levels below 65536 rows
    // whose longest row has at most kEllMaxWidth entries, when padding at most quadruples
    // the entries
    if (!L.coarsest && n < 65536 && op.max_len > 0 && op.max_len <= kEllMaxWidth &&
        (int64_t)op.max_len * n <= 4 * op.nnz_off) {
        op.ell_w = op.max_len;
        op.ell_ci.alloc(pool, n * op.ell_w);
        op.ell_v64.alloc(pool, n * op.ell_w);
        if (f32) op.ell_v32.alloc(pool, n * op.ell_w);
        launch_build_ell(n, op.ell_w, op.rp.p, op.ci.p, op.v64.p, f32 ? op.v32.p : nullptr,
                         op.ell_ci.p, op.ell_v64.p, f32 ? op.ell_v32.p : nullptr, s);
    }
    LAMG_HIP(hipStreamSynchronize(s));
    if (L.coarsest) return;

    // interpolation rows in solve numbering (coarse ids in the next level's numbering); an
    // elimination level injects the coarse values into its kept rows (weight 1) and gives
    // its eliminated rows no parent (entry 0 with weight 0: they are recomputed exactly)
    std::vector<int32_t> hp0(n), hp1(n);
    std::vector<double> hw0(n), hw1(n);
    if (L.elim) {
        for (int64_t u = 0; u < n; ++u) {
            const bool kept = L.h_agg[u] >= 0;
            hp0[u] = kept ? L.h_agg[u] : 0;
            hw0[u] = kept ? 1.0 : 0.0;
            hp1[u] = -1;
            hw1[u] = 0.0;
        }
    } else {
        L.p0.download(hp0.data(), n, s);
        L.p1.download(hp1.data(), n, s);
        L.w0.download(hw0.data(), n, s);
        L.w1.download(hw1.data(), n, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }
    const std::vector<int32_t> &ipn = *iperm_next;
    const int64_t nc = L.nc;
    std::vector<int32_t> sp0(n), sp1(n);
    std::vector<double> sw0(n), sw1(n);
    L.n_cal2 = 0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t u = perm[i];
        sp0[i] = ipn[hp0[u]];
        sp1[i] = hp1[u] >= 0 ? ipn[hp1[u]] : -1;
        sw0[i] = hw0[u];
        sw1[i] = hw1[u];
        if (hp1[u] >= 0) ++L.n_cal2;
    }
    op.p0.alloc(pool, n);
    op.p1.alloc(pool, n);
    op.w0_64.alloc(pool, n);
    op.w1_64.alloc(pool, n);
    op.p0.upload(sp0.data(), n, s);
    op.p1.upload(sp1.data(), n, s);
    op.w0_64.upload(sw0.data(), n, s);
    op.w1_64.upload(sw1.data(), n, s);
    if (f32) {
        op.w0_32.alloc(pool, n);
        op.w1_32.alloc(pool, n);
        launch_cast_f32(n, op.w0_64.p, op.w0_32.p, s);
        launch_cast_f32(n, op.w1_64.p, op.w1_32.p, s);
    }
    // restriction P^T (coarse row -> fine rows ascending)
    op.nc = nc;
    std::vector<int32_t> rrp(nc + 1, 0);
    // rows with a zero weight (the eliminated rows) stay out of P^T
    for (int64_t i = 0; i < n; ++i) {
        if (sw0[i] != 0.0) rrp[sp0[i] + 1]++;
        if (sp1[i] >= 0) rrp[sp1[i] + 1]++;
    }
    for (int64_t a = 0; a < nc; ++a) rrp[a + 1] += rrp[a];
    std::vector<int32_t> rci(rrp[nc]);
    std::vector<double> rw(rrp[nc]);
    {
        std::vector<int32_t> pos(rrp.begin(), rrp.end() - 1);
        for (int64_t i = 0; i < n; ++i) {
            int32_t a = sp0[i];
            if (sw0[i] != 0.0) {
                rci[pos[a]] = (int32_t)i;
                rw[pos[a]++] = sw0[i];
            }
            if (sp1[i] >= 0) {
                a = sp1[i];
                rci[pos[a]] = (int32_t)i;
                rw[pos[a]++] = sw1[i];
            }
        }
    }
    std::vector<int32_t> rlong;
    double rlen = 0.0;
    int64_t rshort = 0;
    for (int64_t a = 0; a < nc; ++a) {
        int32_t len = rrp[a + 1] - rrp[a];
        if (len > kLongRow)
            rlong.push_back((int32_t)a);
        else {
            rlen += len;
            ++rshort;
        }
    }
    op.lpr_r = pick_lpr(rshort ? rlen / rshort : 1.0);
    op.n_rlong = (int64_t)rlong.size();
    op.nnz_r = rrp[nc];
    op.rrp.alloc(pool, nc + 1);
    op.rci.alloc(pool, rrp[nc]);
    op.rw64.alloc(pool, rrp[nc]);
    op.rrp.upload(rrp.data(), nc + 1, s);
    op.rci.upload(rci.data(), rrp[nc], s);
    op.rw64.upload(rw.data(), rrp[nc], s);
    if (op.n_rlong) {
        op.rlong.alloc(pool, op.n_rlong);
        op.rlong.upload(rlong.data(), op.n_rlong, s);
    }
    if (f32) {
        op.rw32.alloc(pool, rrp[nc]);
        launch_cast_f32(rrp[nc], op.rw64.p, op.rw32.p, s);
    }
    LAMG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// The whole setup
// ---------------------------------------------------------------------------
void run_setup(lamg_handle *h, const lamg_graph *g) {
    auto t0 = std::chrono::steady_clock::now();
    for (double &t : h->setup_phase) t = 0.0;
    Pool &pool = *h->pool;
    hipStream_t s = h->stream;
    std::optional<PhaseClock> pc_input(std::in_place, h, LAMG_SETUP_INPUT);
    HostGraph hg = read_graph(g, s);
    const int64_t n = hg.n;
    std::vector<int32_t> rcm;  // order[new] = the caller's node, when renumbered
    h->reordered = false;
    if (h->opt.reorder && rcm_order(hg, rcm)) {
        renumber(hg, rcm);
        h->reordered = true;
    }

    // level 0: L = D - W
    h->lev.clear();
    h->lev.reserve(kMaxLevels);
    h->lev.emplace_back();
    {
        Level &L = h->lev[0];
        L.n = n;
        L.nnz = hg.nnz + n;
        L.h_rp.resize(n + 1);
        L.h_ci.resize(L.nnz);
        for (int64_t u = 0; u <= n; ++u) L.h_rp[u] = hg.rp[u] + (int32_t)u;
        for (int64_t u = 0; u < n; ++u) {
            int32_t pos = L.h_rp[u];
            bool placed = false;
            for (int32_t j = hg.rp[u]; j < hg.rp[u + 1]; ++j) {
                if (!placed && hg.ci[j] > u) {
                    L.h_ci[pos++] = (int32_t)u;
                    placed = true;
                }
                L.h_ci[pos++] = hg.ci[j];
            }
            if (!placed) L.h_ci[pos] = (int32_t)u;
        }
        DArr<int32_t> arp, aci;
        DArr<double> aw;
        arp.alloc(pool, n + 1);
        aci.alloc(pool, hg.nnz);
        aw.alloc(pool, hg.nnz);
        arp.upload(hg.rp.data(), n + 1, s);
        aci.upload(hg.ci.data(), hg.nnz, s);
        aw.upload(hg.w.data(), hg.nnz, s);
        L.rp.alloc(pool, n + 1);
        L.ci.alloc(pool, L.nnz);
        L.val.alloc(pool, L.nnz);
        L.rp.upload(L.h_rp.data(), n + 1, s);
        launch_laplacian(n, arp.p, aci.p, aw.p, L.rp.p, L.ci.p, L.val.p, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }
    pc_input.reset();
    const int64_t n_direct = h->opt.n_direct;
    for (int l = 0;; ++l) {
        Level &L = h->lev[l];
        if (L.n <= n_direct) {
            L.coarsest = true;
            break;
        }
        // elimination and aggregation alternate: an elimination level comes before each
        // aggregation step (when it removes enough nodes), never after another one
        bool eliminated = false;
        if (h->opt.elimination && !(l > 0 && h->lev[l - 1].elim) && l + 1 < kMaxLevels) {
            PhaseClock pc(h, LAMG_SETUP_ELIMINATE);
            eliminated = try_elimination(h, l);
        }
        if (eliminated) continue;
        setup_level(h, l);
        if (h->opt.smoother == 2 && L.ncolors > kChebColors) L.bjgs = true;
        if (h->opt.smoother == 1 && L.ncolors > kChebColors) {
            // Chebyshev smoothing on this dense level: the Gershgorin bound of D^{-1} L
            PhaseClock pc(h, LAMG_SETUP_LEVEL);
            std::vector<double> q(L.n);
            DArr<double> dq;
            dq.alloc(*h->pool, L.n);
            launch_gershgorin_rows(L.n, L.rp.p, L.ci.p, L.val.p, dq.p, h->stream);
            dq.download(q.data(), L.n, h->stream);
            LAMG_HIP(hipStreamSynchronize(h->stream));
            double lmax = 0.0;
            for (double x : q)
                if (x > lmax) lmax = x;
            L.cheb = true;
            L.cheb_lmax = lmax;
        }
        if (L.nc >= L.n || l + 1 >= kMaxLevels) {
            if (L.n <= kStallDirectMax) {
                L.coarsest = true;
                break;
            }
            throw Error(LAMG_COARSENING_STALLED, "coarsening stalled");
        }
        PhaseClock pc(h, LAMG_SETUP_GALERKIN);
        h->lev.emplace_back();
        Level &C = h->lev[l + 1];
        Level &F = h->lev[l];  // re-bind after emplace_back (reserve keeps it valid)
        C.n = F.nc;
        C.nnz = galerkin(pool, F.n, F.nnz, F.rp.p, F.ci.p, F.val.p, F.nc, F.p0.p, F.w0.p, F.p1.p,
                         F.w1.p, C.rp, C.ci, C.val, s);
        C.h_rp.resize(C.n + 1);
        C.h_ci.resize(C.nnz);
        C.rp.download(C.h_rp.data(), C.n + 1, s);
        C.ci.download(C.h_ci.data(), C.nnz, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }
    h->nlev = (int)h->lev.size();

    // cycle index per level, eq. (2.4): 1.5 while |E_l| > 0.1 |E_0|, else min(2, 0.7/tau)
    // floored at 1; gamma = 1 directly above the exactly solved level.
    {
        double m0 = 0.5 * (double)(h->lev[0].nnz - h->lev[0].n);
        for (int l = 0; l + 1 < h->nlev; ++l) {
            double ml = 0.5 * (double)(h->lev[l].nnz - h->lev[l].n);
            double mn = 0.5 * (double)(h->lev[l + 1].nnz - h->lev[l + 1].n);
            double tau = ml > 0.0 ? mn / ml : 1.0;
            double gmm;
            if (ml > 0.1 * m0) {
                gmm = 1.5;
            } else {
                gmm = tau > 0.0 ? 0.7 / tau : 2.0;
                if (gmm > 2.0) gmm = 2.0;
                if (gmm < 1.0) gmm = 1.0;
            }
            if (h->lev[l + 1].coarsest || h->lev[l].elim) gmm = 1.0;
            h->lev[l].gamma = gmm;
            h->lev[l].tau = tau;
        }
    }

    // coarsest inverse
    {
        Level &C = h->lev[h->nlev - 1];
        PhaseClock pc(h, LAMG_SETUP_COARSEST);
        C.Z.alloc(pool, C.n * C.n);
        coarsest_inverse(pool, C.n, C.rp.p, C.ci.p, C.val.p, C.Z.p, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }

    // solve layout, all levels
    {
        PhaseClock pc(h, LAMG_SETUP_LAYOUT);
        std::vector<std::vector<int32_t>> perm(h->nlev), iperm(h->nlev);
        for (int l = 0; l < h->nlev; ++l) compute_perm(h->lev[l], perm[l], iperm[l]);
        for (int l = 0; l < h->nlev; ++l)
            build_solve_op(h, l, perm[l], iperm[l], l + 1 < h->nlev ? &iperm[l + 1] : nullptr);
        // right-hand sides come in, and solutions go out, in the caller's numbering
        std::vector<int32_t> io(perm[0]);
        if (h->reordered)
            for (auto &u : io) u = rcm[u];
        SolveOp &op0 = h->lev[0].op;
        op0.io_perm.alloc(*h->pool, h->lev[0].n);
        op0.io_perm.upload(io.data(), h->lev[0].n, s);
        LAMG_HIP(hipStreamSynchronize(s));
    }

    if (!h->opt.keep_setup_data) {
        for (int l = 0; l < h->nlev; ++l) {
            Level &L = h->lev[l];
            L.rp.release();
            L.ci.release();
            L.val.release();
            L.strong.release();
            L.X.release();
            L.aff.release();
            L.mom.release();
            L.p0.release();
            L.p1.release();
            L.w0.release();
            L.w1.release();
            std::vector<int32_t>().swap(L.h_ci);
            std::vector<int32_t>().swap(L.h_seed);
            std::vector<int32_t>().swap(L.h_agg);
            std::vector<int32_t>().swap(L.h_color);
        }
    }
    h->setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace lamg
