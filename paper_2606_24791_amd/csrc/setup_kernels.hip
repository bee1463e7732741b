// Setup kernels of the LAMG+ hierarchy (Sec. 2 and Sec. 3 of the paper).
//
// This file is compiled with -ffp-contract=off: every product and sum below is rounded
// as written (no fused multiply-add), every sum runs left to right from +0.0 in
// canonical CSR order, and division is IEEE correctly rounded. Setup quantities feed
// discrete decisions (veto, guard, affinity argmax, caliber-2 gate) and the next level's
// operator, so the whole hierarchy is reproducible bit for bit by any implementation
// that follows the same arithmetic contract.
#include <hipcub/hipcub.hpp>

#include "lamg_internal.h"

namespace lamg {

namespace {

inline unsigned grid_for(int64_t work) {
    int64_t b = (work + kBlock - 1) / kBlock;
    return (unsigned)(b > 0 ? b : 1);
}

// ---------------------------------------------------------------------------
// L = D - W with the diagonal in its sorted position (Sec. 1). One thread per row; the
// row's weights are summed in column order.
// ---------------------------------------------------------------------------
__global__ void k_laplacian(int64_t n, const int32_t *__restrict__ arp,
                            const int32_t *__restrict__ aci, const double *__restrict__ aw,
                            const int32_t *__restrict__ lrp, int32_t *__restrict__ lci,
                            double *__restrict__ lv) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t b = arp[u], e = arp[u + 1];
    double d = 0.0;
    for (int32_t j = b; j < e; ++j) d = d + aw[j];
    int32_t pos = lrp[u];
    bool placed = false;
    for (int32_t j = b; j < e; ++j) {
        int32_t c = aci[j];
        if (!placed && c > (int32_t)u) {
            lci[pos] = (int32_t)u;
            lv[pos] = d;
            ++pos;
            placed = true;
        }
        lci[pos] = c;
        lv[pos] = -aw[j];
        ++pos;
    }
    if (!placed) {
        lci[pos] = (int32_t)u;
        lv[pos] = d;
    }
}

// ---------------------------------------------------------------------------
// Strength-of-connection veto, eq. (3.1): entry (u,v) may carry aggregation iff
// v != u, L_uv != 0 and not |L_uv| < tau * max_{t != u} |L_ut| (judged from u's side).
// ---------------------------------------------------------------------------
__global__ void k_strong(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, double tau, int enable_veto,
                         uint8_t *__restrict__ strong) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t b = rp[u], e = rp[u + 1];
    double mx = 0.0;
    for (int32_t j = b; j < e; ++j)
        if (ci[j] != (int32_t)u && fabs(v[j]) > mx) mx = fabs(v[j]);
    double thr = tau * mx;
    for (int32_t j = b; j < e; ++j) {
        bool s = (ci[j] != (int32_t)u) && (v[j] != 0.0);
        if (s && enable_veto && fabs(v[j]) < thr) s = false;
        strong[j] = s ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Test vectors (Sec. 2): U[-1,1) start from SplitMix64 (Steele, Lea & Flood 2014) on
// the counter level<<56 | k<<48 | u, then multicolour Gauss-Seidel sweeps on L x = 0.
// ---------------------------------------------------------------------------
__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_tv_init(int64_t n, uint64_t seed, int level, double *__restrict__ X) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * kTV) return;
    int64_t u = t / kTV;
    int k = (int)(t % kTV);
    uint64_t ctr = ((uint64_t)level << 56) | ((uint64_t)k << 48) | (uint64_t)u;
    uint64_t h = splitmix64_at(seed, ctr);
    double unit = (double)(h >> 11) * 0x1.0p-53;
    X[t] = 2.0 * unit - 1.0;
}

// One colour of a canonical sweep: for every listed row u and vector k,
// acc = sum_{v != u} L_uv x_v[k] in CSR order, x_u[k] = (0 - acc) / L_uu.
// Rows of one colour do not couple, so they run in parallel.
__global__ void k_tv_sweep_color(int64_t cnt, const int32_t *__restrict__ rows,
                                 const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, double *__restrict__ X) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int32_t u = rows[t];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, d = 0.0;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
        int32_t c = ci[j];
        double w = v[j];
        if (c == u) {
            d = w;
            continue;
        }
        const double *xc = X + (int64_t)c * kTV;
        a0 = a0 + w * xc[0];
        a1 = a1 + w * xc[1];
        a2 = a2 + w * xc[2];
        a3 = a3 + w * xc[3];
    }
    double *xu = X + (int64_t)u * kTV;
    xu[0] = (0.0 - a0) / d;
    xu[1] = (0.0 - a1) / d;
    xu[2] = (0.0 - a2) / d;
    xu[3] = (0.0 - a3) / d;
}

// The same update for long rows, one wave per row: the lanes load kTVChunk entries at a time
// (kTVChunk / 64 gathers in flight per lane) and form their products (each product rounded
// on its own, as in the per-row loop) into LDS, then lane 0 adds them to the four running
// sums in CSR order. The diagonal contributes +0.0, which leaves a sum that started at
// +0.0 unchanged, so every sum is the left-to-right sum of the per-row loop bit for bit.
constexpr int kTVLongRowsPerBlock = kBlock / 64;
constexpr int kTVChunk = 512;

__global__ void __launch_bounds__(kBlock)
    k_tv_sweep_long(int64_t cnt, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
                    const int32_t *__restrict__ ci, const double *__restrict__ v,
                    double *__restrict__ X) {
    extern __shared__ __align__(16) double tv_lds[];
    double(*prod)[kTV] = reinterpret_cast<double(*)[kTV]>(tv_lds);  // [rows per block][chunk]
    __shared__ double diag[kTVLongRowsPerBlock];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * kTVLongRowsPerBlock + wave;
    if (t >= cnt) return;  // uniform per wave; no block-wide barrier below
    double(*my)[kTV] = prod + (int64_t)wave * kTVChunk;
    const int32_t u = rows[t];
    const int32_t b = rp[u], e = rp[u + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int32_t j0 = b; j0 < e; j0 += kTVChunk) {
        const int m = (e - j0 < kTVChunk) ? (int)(e - j0) : kTVChunk;
#pragma unroll 8
        for (int q = lane; q < kTVChunk; q += 64) {
            double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
            if (q < m) {
                const int32_t j = j0 + q;
                const int32_t c = ci[j];
                const double w = v[j];
                if (c == u) {
                    diag[wave] = w;
                } else {
                    const double *xc = X + (int64_t)c * kTV;
                    p0 = w * xc[0];
                    p1 = w * xc[1];
                    p2 = w * xc[2];
                    p3 = w * xc[3];
                }
            }
            my[q][0] = p0;
            my[q][1] = p1;
            my[q][2] = p2;
            my[q][3] = p3;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane == 0) {
            for (int q = 0; q < m; ++q) {
                a0 = a0 + my[q][0];
                a1 = a1 + my[q][1];
                a2 = a2 + my[q][2];
                a3 = a3 + my[q][3];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (lane == 0) {
        const double d = diag[wave];
        double *xu = X + (int64_t)u * kTV;
        xu[0] = (0.0 - a0) / d;
        xu[1] = (0.0 - a1) / d;
        xu[2] = (0.0 - a2) / d;
        xu[3] = (0.0 - a3) / d;
    }
}

// ---------------------------------------------------------------------------
// Affinity, eq. (2.2): c_uv = (sum_k x_u x_v)^2 / (sum_k x_u^2 * sum_k x_v^2).
// ---------------------------------------------------------------------------
__global__ void k_sigma(int64_t n, const double *__restrict__ X, double *__restrict__ sig) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const double *x = X + u * kTV;
    double s = 0.0;
    s = s + x[0] * x[0];
    s = s + x[1] * x[1];
    s = s + x[2] * x[2];
    s = s + x[3] * x[3];
    sig[u] = s;
}

__global__ void k_affinity(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ X, const double *__restrict__ sig,
                           double *__restrict__ aff) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const double *xu = X + u * kTV;
    double su = sig[u];
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
        int32_t t = ci[j];
        if (t == (int32_t)u) {
            aff[j] = 0.0;
            continue;
        }
        const double *xt = X + (int64_t)t * kTV;
        double p = 0.0;
        p = p + xu[0] * xt[0];
        p = p + xu[1] * xt[1];
        p = p + xu[2] * xt[2];
        p = p + xu[3] * xt[3];
        double den = su * sig[t];
        aff[j] = (den == 0.0) ? 0.0 : (p * p) / den;
    }
}

// ---------------------------------------------------------------------------
// Guard moments (App. B): s0 = sum w, s1[k] = sum w x_v[k], s2[k] = sum w x_v[k]^2,
// w = -L_uv, over v != u in CSR order.
// ---------------------------------------------------------------------------
__global__ void k_moments(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const double *__restrict__ v, const double *__restrict__ X,
                          double *__restrict__ mom) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    double s0 = 0.0, s1[kTV], s2[kTV];
#pragma unroll
    for (int k = 0; k < kTV; ++k) s1[k] = s2[k] = 0.0;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
        int32_t t = ci[j];
        if (t == (int32_t)u) continue;
        double w = -v[j];
        s0 = s0 + w;
        const double *xt = X + (int64_t)t * kTV;
#pragma unroll
        for (int k = 0; k < kTV; ++k) {
            double x = xt[k];
            s1[k] = s1[k] + w * x;
            s2[k] = s2[k] + w * (x * x);
        }
    }
    double *m = mom + u * 9;
    m[0] = s0;
#pragma unroll
    for (int k = 0; k < kTV; ++k) {
        m[1 + k] = s1[k];
        m[5 + k] = s2[k];
    }
}

// ---------------------------------------------------------------------------
// Interpolation rows (Sec. 3.2, eq. (A.7)). Seeds: caliber-1 onto their own aggregate.
// A member whose strong entries reach exactly two aggregates {A(u), b} fits
// w = sum d e / sum d^2 with d = x_a - x_b, e = x_u - x_b (x_a, x_b the seeds' test
// vectors); w in [-snap, snap] -> e_b; w in (snap, 1-snap) -> w e_a + (1-w) e_b;
// otherwise caliber-1.
// ---------------------------------------------------------------------------
__global__ void k_interp(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const uint8_t *__restrict__ strong, const double *__restrict__ X,
                         const int32_t *__restrict__ seed, const int32_t *__restrict__ agg,
                         const int32_t *__restrict__ aggseed, int enable_caliber2, double snap,
                         int32_t *__restrict__ p0, double *__restrict__ w0, int32_t *__restrict__ p1,
                         double *__restrict__ w1) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    int32_t a = agg[u];
    int32_t o0 = a, o1 = -1;
    double ow0 = 1.0, ow1 = 0.0;
    if (enable_caliber2 && seed[u] != (int32_t)u) {
        int32_t b = -1;
        bool two = true;
        for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
            if (!strong[j]) continue;
            int32_t t = agg[ci[j]];
            if (t == a) continue;
            if (b < 0)
                b = t;
            else if (t != b) {
                two = false;
                break;
            }
        }
        if (two && b >= 0) {
            const double *xu = X + u * kTV;
            const double *xa = X + (int64_t)aggseed[a] * kTV;
            const double *xb = X + (int64_t)aggseed[b] * kTV;
            double D = 0.0, N = 0.0;
#pragma unroll
            for (int k = 0; k < kTV; ++k) {
                double d = xa[k] - xb[k];
                double e = xu[k] - xb[k];
                D = D + d * d;
                N = N + d * e;
            }
            if (D != 0.0) {
                double w = N / D;
                if (w >= -snap && w <= snap) {
                    o0 = b;
                } else if (w > snap && w < 1.0 - snap) {
                    o0 = a;
                    ow0 = w;
                    o1 = b;
                    ow1 = 1.0 - w;
                }
            }
        }
    }
    p0[u] = o0;
    w0[u] = ow0;
    p1[u] = o1;
    w1[u] = ow1;
}

// ---------------------------------------------------------------------------
// Galerkin operator P^T L P in edge form: for each stored (u,t), t > u, with w = -L_ut,
// d = P_u - P_t over the union of the rows' supports (exact zeros dropped) contributes
// w * (d_a * d_b) to every ordered pair a != b of supp(d). Contributions are generated in
// CSR order, stably sorted by (a,b), and each (a,b) is summed in generation order from
// +0.0. The diagonal is minus the row's off-diagonal sum in ascending column order.
// ---------------------------------------------------------------------------
struct Delta {
    int nd;
    int32_t id[4];
    double dv[4];
};

__device__ inline Delta make_delta(int32_t u, int32_t t, const int32_t *p0, const double *w0,
                                   const int32_t *p1, const double *w1) {
    Delta D;
    D.nd = 0;
    int32_t ua[2] = {p0[u], p1[u]}, ta[2] = {p0[t], p1[t]};
    double uw[2] = {w0[u], w1[u]}, tw[2] = {w0[t], w1[t]};
    for (int s = 0; s < 2; ++s) {
        if (ua[s] < 0) continue;
        double other = 0.0;
        for (int r = 0; r < 2; ++r)
            if (ta[r] == ua[s]) other = tw[r];
        D.id[D.nd] = ua[s];
        D.dv[D.nd] = uw[s] - other;
        ++D.nd;
    }
    for (int r = 0; r < 2; ++r) {
        if (ta[r] < 0) continue;
        bool dup = false;
        for (int s = 0; s < 2; ++s)
            if (ua[s] == ta[r]) dup = true;
        if (dup) continue;
        D.id[D.nd] = ta[r];
        D.dv[D.nd] = 0.0 - tw[r];
        ++D.nd;
    }
    return D;
}

__global__ void k_gal_count(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const int32_t *__restrict__ p0, const double *__restrict__ w0,
                            const int32_t *__restrict__ p1, const double *__restrict__ w1,
                            int64_t *__restrict__ cnt) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
        int32_t t = ci[j];
        if (t <= (int32_t)u) {
            cnt[j] = 0;
            continue;
        }
        Delta D = make_delta((int32_t)u, t, p0, w0, p1, w1);
        int nz = 0;
        for (int x = 0; x < D.nd; ++x) nz += (D.dv[x] != 0.0);
        cnt[j] = nz * (nz - 1);
    }
}

__global__ void k_gal_expand(int64_t n, int64_t nc, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, const double *__restrict__ v,
                             const int32_t *__restrict__ p0, const double *__restrict__ w0,
                             const int32_t *__restrict__ p1, const double *__restrict__ w1,
                             const int64_t *__restrict__ off, uint64_t *__restrict__ key,
                             double *__restrict__ val) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
        int32_t t = ci[j];
        if (t <= (int32_t)u) continue;
        double w = -v[j];
        Delta D = make_delta((int32_t)u, t, p0, w0, p1, w1);
        int64_t o = off[j];
        for (int x = 0; x < D.nd; ++x) {
            if (D.dv[x] == 0.0) continue;
            for (int y = 0; y < D.nd; ++y) {
                if (y == x || D.dv[y] == 0.0) continue;
                key[o] = (uint64_t)D.id[x] * (uint64_t)nc + (uint64_t)D.id[y];
                val[o] = w * (D.dv[x] * D.dv[y]);
                ++o;
            }
        }
    }
}

__global__ void k_seg_head(int64_t m, const uint64_t *__restrict__ key, int64_t *__restrict__ head) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_seg_start(int64_t m, const int64_t *__restrict__ head,
                            const int64_t *__restrict__ segid, int64_t *__restrict__ start) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (head[i]) start[segid[i] - 1] = i;
    if (i == m - 1) start[segid[i]] = m;
}

// Sequential sum of each (a,b) segment in generation order; counts entries per row.
__global__ void k_seg_sum(int64_t nseg, int64_t nc, const int64_t *__restrict__ start,
                          const uint64_t *__restrict__ key, const double *__restrict__ val,
                          int32_t *__restrict__ scol, double *__restrict__ sval,
                          int32_t *__restrict__ rowcnt) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    int64_t b = start[s], e = start[s + 1];
    double acc = 0.0;
    for (int64_t i = b; i < e; ++i) acc = acc + val[i];
    uint64_t k = key[b];
    scol[s] = (int32_t)(k % (uint64_t)nc);
    sval[s] = acc;
    atomicAdd(&rowcnt[(int64_t)(k / (uint64_t)nc)], 1);
}

__global__ void k_row_fill(int64_t nc, const int32_t *__restrict__ crp, const int32_t *__restrict__ scol,
                           const double *__restrict__ sval, int32_t *__restrict__ cci,
                           double *__restrict__ cv) {
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nc) return;
    int64_t pos = crp[a], end = crp[a + 1];
    int64_t s = pos - a;  // segments of earlier rows: crp[a] minus one diagonal per row
    int64_t diag = -1;
    double off = 0.0;
    while (pos < end) {
        if (diag < 0 && (s >= end - a - 1 || scol[s] > (int32_t)a)) {
            diag = pos;
            cci[pos] = (int32_t)a;
            cv[pos] = 0.0;
            ++pos;
            continue;
        }
        cci[pos] = scol[s];
        cv[pos] = sval[s];
        off = off + sval[s];
        ++pos;
        ++s;
    }
    cv[diag] = -off;
}

// ---------------------------------------------------------------------------
// Low-degree elimination (Sec. 2, eq. (2.1)): Schur complement onto the kept nodes C.
// Contributions in generation order: first every kept entry L_ab (fine rows ascending),
// then, for each eliminated node f ascending, -((L_fa * L_fb) / L_ff) for every ordered
// pair (a, b) of distinct neighbours of f. The stable sort by (a, b) and the in-order
// segment sums then add each coarse entry's terms in that order.
// ---------------------------------------------------------------------------
__global__ void k_gershgorin_rows(int64_t n, const int32_t *__restrict__ rp,
                                  const int32_t *__restrict__ ci, const double *__restrict__ v,
                                  double *__restrict__ q) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    double s = 0.0, d = 0.0;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) {
        s = s + fabs(v[j]);
        if (ci[j] == (int32_t)u) d = v[j];
    }
    q[u] = s / d;
}

__global__ void k_diag(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, double *__restrict__ d) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    double x = 0.0;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j)
        if (ci[j] == (int32_t)u) x = v[j];
    d[u] = x;
}

// cnt[u]: kept entries of a kept row; cnt[n + u]: fill pairs of an eliminated row
__global__ void k_schur_count(int64_t n, const int32_t *__restrict__ rp,
                              const int32_t *__restrict__ ci, const int32_t *__restrict__ cid,
                              int64_t *__restrict__ cnt) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int32_t b = rp[u], e = rp[u + 1];
    if (cid[u] >= 0) {
        int64_t c = 0;
        for (int32_t j = b; j < e; ++j) c += (ci[j] != (int32_t)u && cid[ci[j]] >= 0);
        cnt[u] = c;
        cnt[n + u] = 0;
    } else {
        const int64_t d = e - b - 1;
        cnt[u] = 0;
        cnt[n + u] = d * (d - 1);
    }
}

__global__ void k_schur_expand(int64_t n, int64_t nc, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, const double *__restrict__ v,
                               const int32_t *__restrict__ cid, const int64_t *__restrict__ off,
                               uint64_t *__restrict__ key, double *__restrict__ val) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    const int32_t b = rp[u], e = rp[u + 1];
    const int32_t a = cid[u];
    if (a >= 0) {
        int64_t o = off[u];
        for (int32_t j = b; j < e; ++j) {
            const int32_t t = ci[j];
            if (t == (int32_t)u || cid[t] < 0) continue;
            key[o] = (uint64_t)a * (uint64_t)nc + (uint64_t)cid[t];
            val[o] = v[j];
            ++o;
        }
        return;
    }
    // eliminated row: at most kElimMaxDegree neighbours, all kept
    int32_t nb[kElimMaxDegree];
    double w[kElimMaxDegree];
    double dg = 0.0;
    int d = 0;
    for (int32_t j = b; j < e; ++j) {
        if (ci[j] == (int32_t)u) {
            dg = v[j];
        } else if (d < kElimMaxDegree) {
            nb[d] = cid[ci[j]];
            w[d] = v[j];
            ++d;
        }
    }
    int64_t o = off[n + u];
    for (int x = 0; x < d; ++x)
        for (int y = 0; y < d; ++y) {
            if (y == x) continue;
            key[o] = (uint64_t)nb[x] * (uint64_t)nc + (uint64_t)nb[y];
            val[o] = -((w[x] * w[y]) / dg);
            ++o;
        }
}

// ---------------------------------------------------------------------------
// Coarsest level: (L + 11^T/n)^{-1} (SPD for a connected graph) by in-place Gauss-Jordan
// elimination without pivoting, then L^+ = that inverse - 11^T/n.
// ---------------------------------------------------------------------------
__global__ void k_dense_fill(int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, double *__restrict__ A) {
    int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    double one_n = 1.0 / (double)n;
    for (int64_t t = 0; t < n; ++t) A[u * n + t] = one_n;
    for (int32_t j = rp[u]; j < rp[u + 1]; ++j) A[u * n + ci[j]] = v[j] + one_n;
}

// Whole inversion in one workgroup (n <= 1024).
// Inverse of the SPD matrix A (n x n, row-major, in place) by blocked Gauss-Jordan
// elimination without pivoting: pivot blocks of kGJ rows, in order. With the pivot block D,
// the rest of its block row U, of its block column L and of the matrix E, one step sets
//     D <- D^-1,  U <- D^-1 U,  L <- -L D^-1,  E <- E - L D^-1 U,
// and after the last block A holds A^-1. Every pivot block is a Schur complement of an SPD
// matrix, hence SPD itself, so no pivoting is needed. Three launches per block: the pivot
// block inverted in LDS by one workgroup, the row panel D^-1 U (with a copy of the old column
// panel L), and the update of the whole matrix from those buffers.
constexpr int kGJ = 32;

// dinv = D^-1 for the pivot block [k0, k0 + b): scalar Gauss-Jordan in LDS, one thread per
// entry (kGJ x kGJ threads), two barriers per pivot.
__global__ void __launch_bounds__(kGJ * kGJ) k_bgj_diag(int64_t n, int64_t k0, int b,
                                                        const double *__restrict__ A,
                                                        double *__restrict__ dinv) {
    __shared__ double D[kGJ][kGJ + 1];
    const int i = threadIdx.x / kGJ, j = threadIdx.x % kGJ;
    const bool live = i < b && j < b;
    if (live) D[i][j] = A[(k0 + i) * n + k0 + j];
    __syncthreads();
    for (int p = 0; p < b; ++p) {
        double piv = 0.0, aip = 0.0, apj = 0.0, aij = 0.0;
        if (live) {
            piv = D[p][p];
            aip = D[i][p];
            apj = D[p][j];
            aij = D[i][j];
        }
        __syncthreads();
        if (live) {
            double v;
            if (i == p && j == p)
                v = 1.0 / piv;
            else if (i == p)
                v = apj / piv;
            else if (j == p)
                v = -aip / piv;
            else
                v = aij - aip * (apj / piv);
            D[i][j] = v;
        }
        __syncthreads();
    }
    if (live) dinv[i * kGJ + j] = D[i][j];
}

// R[t][j] = (D^-1 U)[t][j] for every column j outside the pivot block (R row-major, n wide),
// and Cp[i][t] = A[i][k0 + t], the old block column (n x kGJ).
__global__ void __launch_bounds__(kBlock) k_bgj_panels(int64_t n, int64_t k0, int b,
                                                       const double *__restrict__ A,
                                                       const double *__restrict__ dinv,
                                                       double *__restrict__ R,
                                                       double *__restrict__ Cp) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    for (int t = 0; t < b; ++t) Cp[j * kGJ + t] = A[j * n + k0 + t];
    if (j >= k0 && j < k0 + b) return;
    double u[kGJ];
    for (int t = 0; t < b; ++t) u[t] = A[(k0 + t) * n + j];
    for (int t = 0; t < b; ++t) {
        double acc = 0.0;
        for (int q = 0; q < b; ++q) acc += dinv[t * kGJ + q] * u[q];
        R[t * n + j] = acc;
    }
}

// The block step on every entry (i, j), from the buffers only (no entry reads another that
// this launch writes). Block (x, y): row i = y, columns j = x * blockDim + thread.
__global__ void __launch_bounds__(kBlock) k_bgj_update(int64_t n, int64_t k0, int b,
                                                       double *__restrict__ A,
                                                       const double *__restrict__ dinv,
                                                       const double *__restrict__ R,
                                                       const double *__restrict__ Cp) {
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const bool ri = i >= k0 && i < k0 + b, rj = j >= k0 && j < k0 + b;
    double v;
    if (ri && rj) {
        v = dinv[(i - k0) * kGJ + (j - k0)];
    } else if (ri) {
        v = R[(i - k0) * n + j];
    } else if (rj) {
        double acc = 0.0;
        for (int t = 0; t < b; ++t) acc += Cp[i * kGJ + t] * dinv[t * kGJ + (j - k0)];
        v = -acc;
    } else {
        double acc = 0.0;
        for (int t = 0; t < b; ++t) acc += Cp[i * kGJ + t] * R[t * n + j];
        v = A[i * n + j] - acc;
    }
    A[i * n + j] = v;
}

__global__ void k_minus_one_over_n(int64_t n, double *__restrict__ Z) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * n) Z[t] = Z[t] - 1.0 / (double)n;
}

// Makes the computed inverse exactly symmetric (it is symmetric up to rounding), so that
// its rows and columns are interchangeable in the coarsest solve.
__global__ void k_symmetrize(int64_t n, double *__restrict__ Z) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int64_t i = t / n, j = t - i * n;
    if (j <= i) return;
    const double a = 0.5 * (Z[i * n + j] + Z[j * n + i]);
    Z[i * n + j] = a;
    Z[j * n + i] = a;
}


// ---------------------------------------------------------------------------
// Solve layout: rows permuted to (class, colour, index) order; the diagonal is split off.
// ---------------------------------------------------------------------------
__global__ void k_permute_csr(int64_t n, const int32_t *__restrict__ perm,
                              const int32_t *__restrict__ iperm, const int32_t *__restrict__ crp,
                              const int32_t *__restrict__ cci, const double *__restrict__ cv,
                              const int32_t *__restrict__ srp, int32_t *__restrict__ sci,
                              double *__restrict__ sv64, float *__restrict__ sv32,
                              double *__restrict__ d64, double *__restrict__ dinv64,
                              float *__restrict__ d32, float *__restrict__ dinv32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t u = perm[i];
    int32_t pos = srp[i];
    double d = 0.0;
    for (int32_t j = crp[u]; j < crp[u + 1]; ++j) {
        int32_t c = cci[j];
        if (c == u) {
            d = cv[j];
            continue;
        }
        sci[pos] = iperm[c];
        sv64[pos] = cv[j];
        if (sv32) sv32[pos] = (float)cv[j];
        ++pos;
    }
    d64[i] = d;
    dinv64[i] = 1.0 / d;
    if (d32) {
        d32[i] = (float)d;
        dinv32[i] = (float)(1.0 / d);
    }
}

// ELL copy (entry u of row i at u * n + i) of an off-diagonal CSR whose rows have at most w
// entries; padding entries hold the row's own index and weight 0.
__global__ void k_build_ell(int64_t n, int w, const int32_t *__restrict__ rp,
                            const int32_t *__restrict__ ci, const double *__restrict__ v64,
                            const float *__restrict__ v32, int32_t *__restrict__ eci,
                            double *__restrict__ ev64, float *__restrict__ ev32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t e0 = rp[i], len = rp[i + 1] - e0;
    for (int u = 0; u < w; ++u) {
        const bool ok = u < len;
        eci[(int64_t)u * n + i] = ok ? ci[e0 + u] : (int32_t)i;
        ev64[(int64_t)u * n + i] = ok ? v64[e0 + u] : 0.0;
        if (ev32) ev32[(int64_t)u * n + i] = ok ? v32[e0 + u] : 0.0f;
    }
}

__global__ void k_cast_f32(int64_t n, const double *__restrict__ s, float *__restrict__ d) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_laplacian(int64_t n, const int32_t *arp, const int32_t *aci, const double *aw,
                      const int32_t *lrp, int32_t *lci, double *lv, hipStream_t s) {
    k_laplacian<<<grid_for(n), kBlock, 0, s>>>(n, arp, aci, aw, lrp, lci, lv);
    LAMG_LAUNCH_CHECK();
}

void launch_strong(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double tau,
                   int enable_veto, uint8_t *strong, hipStream_t s) {
    k_strong<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, tau, enable_veto, strong);
    LAMG_LAUNCH_CHECK();
}

void launch_tv_init(int64_t n, uint64_t seed, int level, double *X, hipStream_t s) {
    k_tv_init<<<grid_for(n * kTV), kBlock, 0, s>>>(n, seed, level, X);
    LAMG_LAUNCH_CHECK();
}

void launch_tv_sweep_color(int64_t cnt, const int32_t *rows, const int32_t *rp, const int32_t *ci,
                           const double *v, double *X, hipStream_t s) {
    if (cnt <= 0) return;
    k_tv_sweep_color<<<grid_for(cnt), kBlock, 0, s>>>(cnt, rows, rp, ci, v, X);
    LAMG_LAUNCH_CHECK();
}

void launch_tv_sweep_long(int64_t cnt, const int32_t *rows, const int32_t *rp, const int32_t *ci,
                          const double *v, double *X, hipStream_t s) {
    if (cnt <= 0) return;
    const unsigned blocks = (unsigned)((cnt + kTVLongRowsPerBlock - 1) / kTVLongRowsPerBlock);
    const size_t lds = sizeof(double) * kTV * kTVChunk * kTVLongRowsPerBlock;
    LAMG_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tv_sweep_long),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    k_tv_sweep_long<<<blocks, kBlock, lds, s>>>(cnt, rows, rp, ci, v, X);
    LAMG_LAUNCH_CHECK();
}

void launch_affinity(int64_t n, const int32_t *rp, const int32_t *ci, const double *X,
                     double *sigma_tmp, double *aff, hipStream_t s) {
    k_sigma<<<grid_for(n), kBlock, 0, s>>>(n, X, sigma_tmp);
    LAMG_LAUNCH_CHECK();
    k_affinity<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, X, sigma_tmp, aff);
    LAMG_LAUNCH_CHECK();
}

void launch_moments(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    const double *X, double *mom, hipStream_t s) {
    k_moments<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, X, mom);
    LAMG_LAUNCH_CHECK();
}

void launch_interp(int64_t n, const int32_t *rp, const int32_t *ci, const uint8_t *strong,
                   const double *X, const int32_t *seed, const int32_t *agg, const int32_t *aggseed,
                   int enable_caliber2, double snap, int32_t *p0, double *w0, int32_t *p1,
                   double *w1, hipStream_t s) {
    k_interp<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, strong, X, seed, agg, aggseed,
                                             enable_caliber2, snap, p0, w0, p1, w1);
    LAMG_LAUNCH_CHECK();
}

// Coarse CSR from m generated contributions (key = a * nc + b, value), consumed here:
// stable radix sort by key (equal keys keep generation order), in-order segment sums,
// canonical rows with the diagonal = minus the sum of the row's off-diagonals.
static int64_t assemble_coarse(Pool &pool, int64_t m, DArr<uint64_t> &key, DArr<double> &val,
                               int64_t nc, DArr<int32_t> &crp, DArr<int32_t> &cci,
                               DArr<double> &cv, hipStream_t s) {
    crp.alloc(pool, nc + 1);
    if (m == 0) {  // no coupling at all (only possible for nc == 1)
        std::vector<int32_t> hrp(nc + 1);
        for (int64_t a = 0; a <= nc; ++a) hrp[a] = (int32_t)a;
        cci.alloc(pool, nc);
        cv.alloc(pool, nc);
        std::vector<int32_t> hci(nc);
        std::vector<double> hv(nc, -0.0);  // minus an empty sum
        for (int64_t a = 0; a < nc; ++a) hci[a] = (int32_t)a;
        crp.upload(hrp.data(), nc + 1, s);
        cci.upload(hci.data(), nc, s);
        cv.upload(hv.data(), nc, s);
        LAMG_HIP(hipStreamSynchronize(s));
        key.release();
        val.release();
        return nc;
    }
    DArr<uint64_t> key2;
    DArr<double> val2;
    key2.alloc(pool, m);
    val2.alloc(pool, m);
    uint64_t maxkey = (uint64_t)nc * (uint64_t)nc;
    int end_bit = 1;
    while (end_bit < 64 && ((uint64_t)1 << end_bit) < maxkey) ++end_bit;
    size_t tmp_bytes = 0;
    LAMG_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key.p, key2.p, val.p, val2.p,
                                                (int)m, 0, end_bit, s));
    DArr<char> tmp;
    tmp.alloc(pool, (int64_t)tmp_bytes);
    LAMG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, key.p, key2.p, val.p, val2.p,
                                                (int)m, 0, end_bit, s));
    key.release();
    val.release();
    // segments
    DArr<int64_t> head, segid;
    head.alloc(pool, m);
    segid.alloc(pool, m);
    k_seg_head<<<grid_for(m), kBlock, 0, s>>>(m, key2.p, head.p);
    LAMG_LAUNCH_CHECK();
    tmp_bytes = 0;
    LAMG_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_bytes, head.p, segid.p, (int)m, s));
    tmp.alloc(pool, (int64_t)tmp_bytes);
    LAMG_HIP(hipcub::DeviceScan::InclusiveSum(tmp.p, tmp_bytes, head.p, segid.p, (int)m, s));
    int64_t nseg = 0;
    LAMG_HIP(hipMemcpyAsync(&nseg, segid.p + m - 1, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipStreamSynchronize(s));
    DArr<int64_t> start;
    start.alloc(pool, nseg + 1);
    k_seg_start<<<grid_for(m), kBlock, 0, s>>>(m, head.p, segid.p, start.p);
    LAMG_LAUNCH_CHECK();
    head.release();
    segid.release();
    DArr<int32_t> scol, rowcnt;
    DArr<double> sval;
    scol.alloc(pool, nseg);
    sval.alloc(pool, nseg);
    rowcnt.alloc(pool, nc + 1);
    {
        std::vector<int32_t> ones(nc + 1, 1);
        ones[nc] = 0;
        rowcnt.upload(ones.data(), nc + 1, s);
    }
    k_seg_sum<<<grid_for(nseg), kBlock, 0, s>>>(nseg, nc, start.p, key2.p, val2.p, scol.p, sval.p,
                                                 rowcnt.p);
    LAMG_LAUNCH_CHECK();
    key2.release();
    val2.release();
    start.release();
    // coarse CSR
    tmp_bytes = 0;
    LAMG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, rowcnt.p, crp.p, (int)(nc + 1), s));
    tmp.alloc(pool, (int64_t)tmp_bytes);
    LAMG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, rowcnt.p, crp.p, (int)(nc + 1), s));
    int64_t cnnz = nseg + nc;
    cci.alloc(pool, cnnz);
    cv.alloc(pool, cnnz);
    k_row_fill<<<grid_for(nc), kBlock, 0, s>>>(nc, crp.p, scol.p, sval.p, cci.p, cv.p);
    LAMG_LAUNCH_CHECK();
    LAMG_HIP(hipStreamSynchronize(s));
    return cnnz;
}

// Exclusive scan of `count` generation counts into offsets; returns the total.
static int64_t scan_counts(Pool &pool, DArr<int64_t> &cnt, int64_t count, DArr<int64_t> &off,
                           hipStream_t s) {
    off.alloc(pool, count + 1);
    LAMG_HIP(hipMemsetAsync(cnt.p + count, 0, sizeof(int64_t), s));
    size_t tmp_bytes = 0;
    LAMG_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, cnt.p, off.p, (int)(count + 1), s));
    DArr<char> tmp;
    tmp.alloc(pool, (int64_t)tmp_bytes);
    LAMG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp.p, tmp_bytes, cnt.p, off.p, (int)(count + 1), s));
    int64_t m = 0;
    LAMG_HIP(hipMemcpyAsync(&m, off.p + count, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LAMG_HIP(hipStreamSynchronize(s));
    return m;
}

int64_t galerkin(Pool &pool, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                 const double *v, int64_t nc, const int32_t *p0, const double *w0,
                 const int32_t *p1, const double *w1, DArr<int32_t> &crp, DArr<int32_t> &cci,
                 DArr<double> &cv, hipStream_t s) {
    // contributions per stored entry, exclusive scan -> generation-order offsets
    DArr<int64_t> cnt, off;
    cnt.alloc(pool, nnz + 1);
    k_gal_count<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, p0, w0, p1, w1, cnt.p);
    LAMG_LAUNCH_CHECK();
    const int64_t m = scan_counts(pool, cnt, nnz, off, s);
    cnt.release();
    DArr<uint64_t> key;
    DArr<double> val;
    if (m > 0) {
        key.alloc(pool, m);
        val.alloc(pool, m);
        k_gal_expand<<<grid_for(n), kBlock, 0, s>>>(n, nc, rp, ci, v, p0, w0, p1, w1, off.p,
                                                    key.p, val.p);
        LAMG_LAUNCH_CHECK();
    }
    off.release();
    return assemble_coarse(pool, m, key, val, nc, crp, cci, cv, s);
}

int64_t schur(Pool &pool, int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const int32_t *cid, int64_t nc, DArr<int32_t> &crp, DArr<int32_t> &cci,
              DArr<double> &cv, hipStream_t s) {
    DArr<int64_t> cnt, off;
    cnt.alloc(pool, 2 * n + 1);
    k_schur_count<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, cid, cnt.p);
    LAMG_LAUNCH_CHECK();
    const int64_t m = scan_counts(pool, cnt, 2 * n, off, s);
    cnt.release();
    DArr<uint64_t> key;
    DArr<double> val;
    if (m > 0) {
        key.alloc(pool, m);
        val.alloc(pool, m);
        k_schur_expand<<<grid_for(n), kBlock, 0, s>>>(n, nc, rp, ci, v, cid, off.p, key.p, val.p);
        LAMG_LAUNCH_CHECK();
    }
    off.release();
    return assemble_coarse(pool, m, key, val, nc, crp, cci, cv, s);
}

void launch_gershgorin_rows(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                            double *q, hipStream_t s) {
    k_gershgorin_rows<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, q);
    LAMG_LAUNCH_CHECK();
}

void launch_diag(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, double *d,
                 hipStream_t s) {
    k_diag<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, d);
    LAMG_LAUNCH_CHECK();
}

void coarsest_inverse(Pool &pool, int64_t n, const int32_t *rp, const int32_t *ci,
                      const double *v, double *Z, hipStream_t s) {
    k_dense_fill<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, Z);
    LAMG_LAUNCH_CHECK();
    DArr<double> dinv, R, Cp;
    dinv.alloc(pool, (int64_t)kGJ * kGJ);
    R.alloc(pool, (int64_t)kGJ * n);
    Cp.alloc(pool, n * kGJ);
    const dim3 ugrid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)n);
    for (int64_t k0 = 0; k0 < n; k0 += kGJ) {
        const int b = (int)std::min<int64_t>(kGJ, n - k0);
        k_bgj_diag<<<1, kGJ * kGJ, 0, s>>>(n, k0, b, Z, dinv.p);
        k_bgj_panels<<<grid_for(n), kBlock, 0, s>>>(n, k0, b, Z, dinv.p, R.p, Cp.p);
        k_bgj_update<<<ugrid, kBlock, 0, s>>>(n, k0, b, Z, dinv.p, R.p, Cp.p);
        LAMG_LAUNCH_CHECK();
    }
    k_minus_one_over_n<<<grid_for(n * n), kBlock, 0, s>>>(n, Z);
    LAMG_LAUNCH_CHECK();
    k_symmetrize<<<grid_for(n * n), kBlock, 0, s>>>(n, Z);
    LAMG_LAUNCH_CHECK();
    LAMG_HIP(hipStreamSynchronize(s));
}

void launch_permute_csr(int64_t n, const int32_t *perm, const int32_t *iperm, const int32_t *crp,
                        const int32_t *cci, const double *cv, const int32_t *srp, int32_t *sci,
                        double *sv64, float *sv32, double *d64, double *dinv64, float *d32,
                        float *dinv32, hipStream_t s) {
    k_permute_csr<<<grid_for(n), kBlock, 0, s>>>(n, perm, iperm, crp, cci, cv, srp, sci, sv64, sv32,
                                                  d64, dinv64, d32, dinv32);
    LAMG_LAUNCH_CHECK();
}

void launch_build_ell(int64_t n, int w, const int32_t *rp, const int32_t *ci, const double *v64,
                      const float *v32, int32_t *eci, double *ev64, float *ev32, hipStream_t s) {
    if (n <= 0 || w <= 0) return;
    k_build_ell<<<grid_for(n), kBlock, 0, s>>>(n, w, rp, ci, v64, v32, eci, ev64, ev32);
    LAMG_LAUNCH_CHECK();
}

void launch_cast_f32(int64_t n, const double *src, float *dst, hipStream_t s) {
    if (n <= 0) return;
    k_cast_f32<<<grid_for(n), kBlock, 0, s>>>(n, src, dst);
    LAMG_LAUNCH_CHECK();
}

}  // namespace lamg
