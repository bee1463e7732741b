// Coarse-tail cycle: the complete gamma-cycle (Sec. 2, "Cycle and acceleration";
// eq. (2.4)) of every level from a threshold level down to the directly solved one, run
// by ONE workgroup of 1024 threads in ONE launch per visit to the threshold level.
//
// Coarse levels are small but are visited many times per cycle (the cycle index grows
// towards 2 where coarsening is aggressive), and every visit is a chain of dependent
// steps: Gauss-Seidel colour passes, residual, restriction, coarse recombination,
// energy correction, prolongation. As separate kernels each step costs a dispatch of a
// few microseconds; here each step is a loop over the level's rows followed by a
// workgroup barrier, with the level data resident in L2. The recursion over levels is an
// explicit state machine; the per-level visit counters live in device memory so that the
// Beatty visit counts continue across launches within one solve.
//
// The arithmetic per step is that of the multi-kernel path (cycle_kernels.hip).
#include <type_traits>

#include "csr_device.h"
#include "lamg_internal.h"

namespace lamg {

namespace {

constexpr int TB = 1024;  // threads of the tail workgroup
constexpr int TW = TB / 64;

template <class T>
struct TailLvl {
    int64_t n;
    int ncolors, coarsest;
    const int64_t *blk;  // 2*ncolors + 1 offsets (class 0 colours, class 1 colours)
    const int32_t *rp, *ci;
    const T *v, *d, *dinv;
    const int32_t *p0, *p1;  // P to the next level
    const T *w0, *w1;
    int64_t nc;
    const int32_t *rrp, *rci, *rlong;  // P^T
    int64_t n_rlong;
    const T *rw;
    const double *Z;  // coarsest
    T *x, *f, *r, *rho, *x1, *rho1;
    double gamma;
    int maxlen;  // longest off-diagonal row; 0 if the level has long-class rows
};

constexpr int kTailMax = kTailMaxLevels;

// Global -> LDS copy performed at the start of every tail launch (4-byte words).
struct CopyJob {
    const void *src;
    uint32_t dst;    // byte offset in the dynamic LDS buffer
    uint32_t bytes;  // multiple of 4
};

template <class T>
struct TailArgs {
    const TailLvl<T> *lv;      // device descriptors of all levels (global-memory arrays)
    const TailLvl<T> *lds_lv;  // levels >= l_lds: pointer fields are LDS byte offsets (Z stays global)
    const CopyJob *jobs;
    int njobs;
    int l0, nlev, l_lds, k, lkp;
    int64_t *visits;  // per level, persistent within a solve
};

__device__ inline void bar() { __syncthreads(); }

// Sum over the sub-lanes of a group of G lanes (xor partners of stride kp).
template <class V>
__device__ inline V wave_sum_sub(V v, int kp, int G) {
    for (int o = kp; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// CSR pass over rows [a, b) (short rows) and [la, lb) (long rows):
//   OP 0: x[r] = (f[r] - sum_off) * dinv[r]      (Gauss-Seidel colour pass, in place)
//   OP 1: out[r] = f[r] - d[r] x[r] - sum_off     (residual)
//   OP 2: out[r] = sum_off                        (P^T r)
// Short rows: one thread per (row, column). Long rows: one wave per row, the 64 lanes
// split as kp columns x (64/kp) entry lanes.
template <class T, int OP>
__device__ void csr_pass(int64_t a, int64_t b, int64_t la, int64_t lb, const int32_t *rows,
                         int skip_long, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const T *__restrict__ v, const T *__restrict__ dd, const T *f, const T *xin,
                         T *out, int k, int lkp) {
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int c = tid & (kp - 1);
    if (c < k) {
        for (int64_t row = a + (tid >> lkp); row < b; row += (TB >> lkp)) {
            int32_t e0 = rp[row], e1 = rp[row + 1];
            if (skip_long > 0 && e1 - e0 > skip_long) continue;
            T acc = row_dot<T, 8>(ci, v, xin, e0, e1, 1, k, c);
            int64_t o = row * k + c;
            if (OP == 0)
                out[o] = (f[o] - acc) * dd[row];
            else if (OP == 1)
                out[o] = f[o] - dd[row] * xin[o] - acc;
            else
                out[o] = acc;
        }
    }
    const int wave = tid >> 6, lane = tid & 63;
    const int sub = lane >> lkp, col = lane & (kp - 1), nsub = 64 >> lkp;
    for (int64_t i = la + wave; i < lb; i += TW) {
        int64_t row = rows ? (int64_t)rows[i] : i;
        int32_t e0 = rp[row], e1 = rp[row + 1];
        T acc = T(0);
        if (col < k) acc = row_dot<T, 4>(ci, v, xin, e0 + sub, e1, nsub, k, col);
        acc = wave_sum_sub(acc, kp, 64);
        if (sub == 0 && col < k) {
            int64_t o = row * k + col;
            if (OP == 0)
                out[o] = (f[o] - acc) * dd[row];
            else if (OP == 1)
                out[o] = f[o] - dd[row] * xin[o] - acc;
            else
                out[o] = acc;
        }
    }
}

// Loop helper over (row, column) pairs of an n x k block with the kp mapping.
#define TAIL_ROWS(n, ...)                                                         \
    {                                                                              \
        const int c_ = tid & (kp - 1);                                             \
        if (c_ < k)                                                                \
            for (int64_t u_ = tid >> lkp; u_ < (n); u_ += (TB >> lkp)) {           \
                const int64_t t = u_ * k + c_;                                     \
                const int64_t u = u_;                                              \
                const int c = c_;                                                  \
                (void)u;                                                           \
                (void)c;                                                           \
                __VA_ARGS__                                                        \
            }                                                                      \
    }

// register-resident rows: at most this many off-diagonals (fewer in FP64 to stay in registers)
template <class T>
struct FastRow {
    static constexpr int N = sizeof(T) == 4 ? 16 : 12;
};

// `sweeps` Gauss-Seidel sweeps. On a level whose (row, column) pairs fit one per thread and
// whose rows are short, each thread loads its row (indices, values, inverse diagonal,
// right-hand side) into registers once per call; a colour pass is then one gather, one
// store and one barrier. Otherwise every colour pass is a full CSR pass.
template <class T>
__device__ void gs_sweeps(const TailLvl<T> &L, int k, int lkp, int sweeps) {
    const int nc = L.ncolors;
    const int tid = threadIdx.x;
    constexpr int kFastRow = FastRow<T>::N;
    if (L.maxlen > 0 && L.maxlen <= kFastRow && (L.n << lkp) <= TB) {
        const int64_t row = tid >> lkp;
        const int c = tid & ((1 << lkp) - 1);
        const bool live = row < L.n && c < k;
        int32_t cc[kFastRow];
        T vv[kFastRow];
        T dinv = T(0), fv = T(0);
        int mycol = -1;
        if (live) {
            const int32_t e0 = L.rp[row], len = L.rp[row + 1] - e0;
#pragma unroll
            for (int u = 0; u < kFastRow; ++u) {
                const bool ok = u < len;
                cc[u] = ok ? L.ci[e0 + u] : -1;
                vv[u] = ok ? L.v[e0 + u] : T(0);
            }
            dinv = L.dinv[row];
            fv = L.f[row * k + c];
            for (int cl = 0; cl < nc; ++cl)
                if (row >= L.blk[cl] && row < L.blk[cl + 1]) mycol = cl;
        }
        T *x = L.x;
        for (int sw = 0; sw < sweeps; ++sw) {
            for (int cl = 0; cl < nc; ++cl) {
                if (live && mycol == cl) {
                    T acc = T(0);
#pragma unroll
                    for (int u0 = 0; u0 < kFastRow; u0 += 4) {  // gathers in groups of four
                        T xx[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            xx[u] = (u0 + u < kFastRow && cc[u0 + u] >= 0)
                                        ? x[(int64_t)cc[u0 + u] * k + c]
                                        : T(0);
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (u0 + u < kFastRow) acc += vv[u0 + u] * xx[u];
                    }
                    x[row * k + c] = (fv - acc) * dinv;
                }
                bar();
            }
        }
        return;
    }
    for (int sw = 0; sw < sweeps; ++sw)
        for (int c = 0; c < nc; ++c) {
            csr_pass<T, 0>(L.blk[c], L.blk[c + 1], L.blk[nc + c], L.blk[nc + c + 1], nullptr, 0,
                           L.rp, L.ci, L.v, L.dinv, L.f, L.x, L.x, k, lkp);
            bar();
        }
}

template <class T>
__device__ void residual(const TailLvl<T> &L, const T *x, const T *f, T *r, int k, int lkp) {
    const int nc = L.ncolors;
    csr_pass<T, 1>(0, L.blk[nc], L.blk[nc], L.n, nullptr, 0, L.rp, L.ci, L.v, L.d, f, x, r, k, lkp);
    bar();
}

// Deterministic workgroup reduction of Q per-column sums. Thread (rloc, col), col = tid
// mod kp, holds partial sums over rows rloc, rloc + TB/kp, ...; a fixed xor-shuffle tree
// combines the lanes of one column inside each wave, then the first kp threads add the
// waves' totals in wave order. out[i*32 + col] receives sum i of column col.
template <int Q>
__device__ void block_sums(double (&q)[Q], double *sh, int kp, double *out /* Q*32 */) {
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    for (int i = 0; i < Q; ++i)
        for (int o = kp; o < 64; o <<= 1) q[i] += __shfl_xor(q[i], o, 64);
    if ((tid & 63) < kp)
        for (int i = 0; i < Q; ++i) sh[(wave * Q + i) * 32 + (tid & 63)] = q[i];
    bar();
    if (tid < kp)
        for (int i = 0; i < Q; ++i) {
            double acc = 0.0;
            for (int w = 0; w < TW; ++w) acc += sh[(w * Q + i) * 32 + tid];
            out[i * 32 + tid] = acc;
        }
    bar();
}

template <class T>
__device__ void coarsest_solve(const TailLvl<T> &L, const T *f, T *y, int k, int lkp) {
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int64_t n = L.n;
    const int64_t units = n << lkp;
    int lg = 0;
    while (lg < 6 && (units << (lg + 1)) <= TB) ++lg;
    const int G = 1 << lg;
    for (int64_t base = 0; base < (units << lg); base += TB) {
        const int64_t t = base + tid;
        const int64_t unit = t >> lg;
        const int p = (int)(t & (G - 1));
        const int64_t u = unit >> lkp;
        const int c = (int)(unit & (kp - 1));
        const bool live = unit < units && c < k;
        double acc = 0.0;
        if (live) {
            const double *zr = L.Z + u * n;
            for (int64_t j = p; j < n; j += 16 * G) {
                double zz[16], ff[16];
#pragma unroll
                for (int w = 0; w < 16; ++w) {
                    const int64_t jj = j + (int64_t)w * G;
                    const bool ok = jj < n;
                    zz[w] = ok ? zr[jj] : 0.0;
                    ff[w] = ok ? (double)f[jj * k + c] : 0.0;
                }
#pragma unroll
                for (int w = 0; w < 16; ++w) acc += zz[w] * ff[w];
            }
        }
        for (int o = 1; o < G; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (live && p == 0) y[u * k + c] = (T)acc;
    }
    bar();
}

template <class P>
__device__ inline P lds_ptr(char *base, P off) {
    return off ? reinterpret_cast<P>(base + reinterpret_cast<uintptr_t>(off)) : off;
}

template <class T>
__global__ void __launch_bounds__(TB) k_tail(TailArgs<T> A) {
    extern __shared__ __align__(16) char smem[];
    __shared__ double sh[TW * 2 * 32];
    __shared__ double tot[2 * 32];
    __shared__ double coef[32];
    __shared__ int s_phase[kMaxLevels], s_j[kMaxLevels], s_nvis[kMaxLevels];
    __shared__ TailLvl<T> dl[kTailMax];
    const int tid = threadIdx.x;
    const int k = A.k, lkp = A.lkp, kp = 1 << lkp;
    const int l0 = A.l0;
    // stage the descriptors of this tail's levels; LDS-resident levels point into smem
    if (tid < A.nlev - l0) {
        const int lv = l0 + tid;
        if (lv >= A.l_lds) {
            TailLvl<T> D = A.lds_lv[lv];
            D.blk = lds_ptr(smem, D.blk);
            D.rp = lds_ptr(smem, D.rp);
            D.ci = lds_ptr(smem, D.ci);
            D.v = lds_ptr(smem, D.v);
            D.d = lds_ptr(smem, D.d);
            D.dinv = lds_ptr(smem, D.dinv);
            D.p0 = lds_ptr(smem, D.p0);
            D.p1 = lds_ptr(smem, D.p1);
            D.w0 = lds_ptr(smem, D.w0);
            D.w1 = lds_ptr(smem, D.w1);
            D.rrp = lds_ptr(smem, D.rrp);
            D.rci = lds_ptr(smem, D.rci);
            D.rlong = lds_ptr(smem, D.rlong);
            D.rw = lds_ptr(smem, D.rw);
            D.x = lds_ptr(smem, D.x);
            D.f = lds_ptr(smem, D.f);
            D.r = lds_ptr(smem, D.r);
            D.rho = lds_ptr(smem, D.rho);
            D.x1 = lds_ptr(smem, D.x1);
            D.rho1 = lds_ptr(smem, D.rho1);
            dl[tid] = D;
        } else {
            dl[tid] = A.lv[lv];
        }
    }
    // bring the LDS-resident operators (and the top level's iterate and right-hand side)
    for (int jb = 0; jb < A.njobs; ++jb) {
        const uint32_t *src = static_cast<const uint32_t *>(A.jobs[jb].src);
        uint32_t *dst = reinterpret_cast<uint32_t *>(smem + A.jobs[jb].dst);
        const uint32_t words = A.jobs[jb].bytes >> 2;
        for (uint32_t w = tid; w < words; w += TB) dst[w] = src[w];
    }
    int l = l0;
    if (tid == 0) s_phase[l] = 0;
    bar();
    while (l >= l0) {
        const TailLvl<T> &L = dl[l - l0];
        if (L.coarsest) {
            coarsest_solve<T>(L, L.f, L.x, k, lkp);
            --l;
            continue;
        }
        const TailLvl<T> &C = dl[l + 1 - l0];
        if (s_phase[l] == 0) {
            // pre-relaxation, residual, restriction, zero coarse iterate
            gs_sweeps<T>(L, k, lkp, 1);
            residual<T>(L, L.x, L.f, L.r, k, lkp);
            csr_pass<T, 2>(0, L.nc, 0, L.n_rlong, L.rlong, L.n_rlong ? kLongRow : 0, L.rrp, L.rci,
                           L.rw, nullptr, nullptr, L.r, C.f, k, lkp);
            TAIL_ROWS(C.n, { C.x[t] = T(0); })
            if (tid == 0) {
                int64_t i = A.visits[l]++;
                s_nvis[l] = (int)(floor((double)(i + 1) * L.gamma) - floor((double)i * L.gamma));
                s_j[l] = 0;
                s_phase[l] = 1;
                s_phase[l + 1] = 0;
            }
            bar();
            ++l;
            continue;
        }
        // returned from one visit to level l+1
        residual<T>(C, C.x, C.f, C.rho, k, lkp);
        const int j = s_j[l] + 1;
        const int nvis = s_nvis[l];
        const int col = tid & (kp - 1);
        bar();  // every thread has read the level's loop state before thread 0 updates it
        if (j >= 2) {  // two-iterate recombination across the visits
            double q[2] = {0.0, 0.0};
            if (col < k)
                for (int64_t i = tid >> lkp; i < C.n; i += TB >> lkp) {
                    double rv = (double)C.rho[i * k + col], g = rv - (double)C.rho1[i * k + col];
                    q[0] += g * g;
                    q[1] += g * rv;
                }
            block_sums<2>(q, sh, kp, tot);
            if (tid < k) coef[tid] = tot[tid] > 0.0 ? tot[32 + tid] / tot[tid] : 0.0;
            bar();
            TAIL_ROWS(C.n, {
                T a = (T)coef[c];
                T ev = C.x[t], rv = C.rho[t];
                C.x[t] = ev + a * (C.x1[t] - ev);
                C.rho[t] = rv - a * (rv - C.rho1[t]);
            })
            bar();
        }
        if (j < nvis) {
            TAIL_ROWS(C.n, {
                C.x1[t] = C.x[t];
                C.rho1[t] = C.rho[t];
            })
            if (tid == 0) {
                s_j[l] = j;
                s_phase[l + 1] = 0;
            }
            bar();
            ++l;
            continue;
        }
        // energy correction mu = <e, fc> / <e, fc - rho>, prolongation, post-relaxation
        {
            double q[2] = {0.0, 0.0};
            if (col < k)
                for (int64_t i = tid >> lkp; i < C.n; i += TB >> lkp) {
                    double e = (double)C.x[i * k + col], fc = (double)C.f[i * k + col];
                    q[0] += e * fc;
                    q[1] += e * (fc - (double)C.rho[i * k + col]);
                }
            block_sums<2>(q, sh, kp, tot);
            if (tid < k) {
                double num = tot[tid], den = tot[32 + tid], mu = num / den;
                if (!(den > 0.0) || !isfinite(mu)) mu = 1.0;
                coef[tid] = mu;
            }
            bar();
            TAIL_ROWS(L.n, {
                T pe = L.w0[u] * C.x[(int64_t)L.p0[u] * k + c];
                int32_t q1 = L.p1[u];
                if (q1 >= 0) pe += L.w1[u] * C.x[(int64_t)q1 * k + c];
                L.x[t] += (T)coef[c] * pe;
            })
            bar();
        }
        gs_sweeps<T>(L, k, lkp, 2);
        --l;
    }
    if (l0 >= A.l_lds) {  // the top level's iterate lives in LDS: write it back
        T *gx = A.lv[l0].x;
        const T *lx = dl[0].x;
        TAIL_ROWS(dl[0].n, { gx[t] = lx[t]; })
    }
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
                    T *x, T *f, T *r, T *rho, T *x1, T *rho1) {
    TailLvl<T> &D = static_cast<TailLvl<T> *>(host_buf)[l];
    std::memset(&D, 0, sizeof(D));
    D.n = L.n;
    D.ncolors = op.ncolors;
    D.coarsest = L.coarsest ? 1 : 0;
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
    D.nc = op.nc;
    D.rrp = op.rrp.p;
    D.rci = op.rci.p;
    D.rlong = op.rlong.p;
    D.n_rlong = op.n_rlong;
    D.rw = rw;
    D.Z = L.Z.p;
    D.x = x;
    D.f = f;
    D.r = r;
    D.rho = rho;
    D.x1 = x1;
    D.rho1 = rho1;
    D.gamma = L.gamma;
    D.maxlen = op.max_short_len;
}

// Chooses the LDS-resident levels of a tail starting at l0 (the coarsest ones whose
// operators and vectors fit together in the LDS left beside the kernel's static use),
// and writes their offset descriptors and copy jobs. Returns l_lds (nlev: none) and the
// dynamic LDS bytes.
template <class T>
int tail_lds_plan(const std::vector<Level> &lev, int l0, int k, const void *host_desc,
                  std::vector<char> &lds_desc, std::vector<char> &jobs, size_t &lds_bytes) {
    const int nlev = (int)lev.size();
    lds_bytes = 0;
    lds_desc.assign(sizeof(TailLvl<T>) * nlev, 0);
    jobs.clear();
    if (l0 < 0 || nlev - l0 > kTailMax) return nlev;
    int dev = 0;
    LAMG_HIP(hipGetDevice(&dev));
    int max_lds = 0;
    LAMG_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    hipFuncAttributes fa;
    LAMG_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(&k_tail<T>)));
    const int64_t budget = (int64_t)max_lds - (int64_t)fa.sharedSizeBytes - 512;
    const TailLvl<T> *G = static_cast<const TailLvl<T> *>(host_desc);
    auto al = [](int64_t b) { return (b + 15) & ~(int64_t)15; };
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
    int l_lds = nlev;
    int64_t total = 16;  // offset 0 means "no array"
    for (int l = nlev - 1; l >= l0; --l) {
        int64_t b = level_bytes(l);
        if (total + b > budget) break;
        total += b;
        l_lds = l;
    }
    if (l_lds == nlev) return nlev;
    int64_t off = 16;
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
            if (copy && src) jv.push_back(CopyJob{src, (uint32_t)off, (uint32_t)bytes});
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
        place(E.x, s * n * k, top);
        place(E.f, s * n * k, top);
        place(E.r, s * n * k, false);
        E.rho = E.r;  // the residual of a level is dead before its coarse residual is formed
        if (!L.coarsest) {
            place(E.x1, s * n * k, false);
            place(E.rho1, s * n * k, false);
        } else {
            E.x1 = E.rho1 = nullptr;
        }
    }
    lds_bytes = (size_t)off;
    jobs.resize(jv.size() * sizeof(CopyJob));
    if (!jv.empty()) std::memcpy(jobs.data(), jv.data(), jobs.size());
    if (lds_bytes > 64 * 1024)
        LAMG_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tail<T>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    return l_lds;
}

template <class T>
void run_tail(const TailPlan &tp, int l0, int nlev, int k, int64_t *d_visits, hipStream_t s) {
    TailArgs<T> A;
    A.lv = static_cast<const TailLvl<T> *>(tp.desc);
    A.lds_lv = static_cast<const TailLvl<T> *>(tp.lds_desc);
    A.jobs = static_cast<const CopyJob *>(tp.jobs);
    A.njobs = tp.njobs;
    A.l0 = l0;
    A.nlev = nlev;
    A.l_lds = tp.l_lds;
    A.k = k;
    int lkp = 0;
    while ((1 << lkp) < k) ++lkp;
    A.lkp = lkp;
    A.visits = d_visits;
    launch_kernel(k_tail<T>, dim3(1), dim3(TB), (uint32_t)tp.lds_bytes, s, A);
    LAMG_LAUNCH_CHECK();
}

size_t tail_copy_job_bytes() { return sizeof(CopyJob); }

void run_zero_i64(int64_t *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_i64<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, n);
    LAMG_LAUNCH_CHECK();
}

template size_t tail_desc_bytes<double>();
template size_t tail_desc_bytes<float>();
template void tail_fill_desc<double>(void *, int, const Level &, const SolveOp &, const int64_t *,
                                     const double *, const double *, const double *,
                                     const double *, const double *, const double *, double *,
                                     double *, double *, double *, double *, double *);
template void tail_fill_desc<float>(void *, int, const Level &, const SolveOp &, const int64_t *,
                                    const float *, const float *, const float *, const float *,
                                    const float *, const float *, float *, float *, float *,
                                    float *, float *, float *);
template void run_tail<double>(const TailPlan &, int, int, int, int64_t *, hipStream_t);
template void run_tail<float>(const TailPlan &, int, int, int, int64_t *, hipStream_t);
template int tail_lds_plan<double>(const std::vector<Level> &, int, int, const void *,
                                   std::vector<char> &, std::vector<char> &, size_t &);
template int tail_lds_plan<float>(const std::vector<Level> &, int, int, const void *,
                                  std::vector<char> &, std::vector<char> &, size_t &);

}  // namespace lamg
