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
};

template <class T>
struct TailArgs {
    const TailLvl<T> *lv;  // device array of descriptors
    int l0, nlev, k, lkp;
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
                         T *out, int k, int kp) {
    const int tid = threadIdx.x;
    const int64_t ns = (b - a) * k;
    for (int64_t t = tid; t < ns; t += TB) {
        int64_t row = a + t / k;
        int c = (int)(t % k);
        int32_t e0 = rp[row], e1 = rp[row + 1];
        if (skip_long > 0 && e1 - e0 > skip_long) continue;
        T acc = T(0);
        for (int32_t j = e0; j < e1; ++j) acc += v[j] * xin[(int64_t)ci[j] * k + c];
        int64_t o = row * k + c;
        if (OP == 0)
            out[o] = (f[o] - acc) * dd[row];
        else if (OP == 1)
            out[o] = f[o] - dd[row] * xin[o] - acc;
        else
            out[o] = acc;
    }
    const int wave = tid >> 6, lane = tid & 63;
    const int sub = lane / kp, col = lane % kp, nsub = 64 / kp;
    for (int64_t i = la + wave; i < lb; i += TW) {
        int64_t row = rows ? (int64_t)rows[i] : i;
        int32_t e0 = rp[row], e1 = rp[row + 1];
        T acc = T(0);
        if (col < k)
            for (int32_t j = e0 + sub; j < e1; j += nsub) acc += v[j] * xin[(int64_t)ci[j] * k + col];
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

template <class T>
__device__ void gs_sweep(const TailLvl<T> &L, int k, int kp) {
    const int nc = L.ncolors;
    for (int c = 0; c < nc; ++c) {
        csr_pass<T, 0>(L.blk[c], L.blk[c + 1], L.blk[nc + c], L.blk[nc + c + 1], nullptr, 0, L.rp,
                       L.ci, L.v, L.dinv, L.f, L.x, L.x, k, kp);
        bar();
    }
}

template <class T>
__device__ void residual(const TailLvl<T> &L, const T *x, const T *f, T *r, int k, int kp) {
    const int nc = L.ncolors;
    csr_pass<T, 1>(0, L.blk[nc], L.blk[nc], L.n, nullptr, 0, L.rp, L.ci, L.v, L.d, f, x, r, k, kp);
    bar();
}

// Deterministic workgroup reduction of Q per-column sums: thread (rloc, col) with
// col = tid % kp accumulates rows rloc, rloc + TB/kp, ...; a fixed LDS tree combines them.
template <int Q>
__device__ void block_sums(double (&q)[Q], double *sh, int kp, double *out /* Q*32 */) {
    const int tid = threadIdx.x;
    for (int i = 0; i < Q; ++i) sh[i * TB + tid] = q[i];
    bar();
    for (int st = (TB / kp) >> 1; st > 0; st >>= 1) {
        if ((tid / kp) < st)
            for (int i = 0; i < Q; ++i) sh[i * TB + tid] += sh[i * TB + tid + st * kp];
        bar();
    }
    if (tid < kp)
        for (int i = 0; i < Q; ++i) out[i * 32 + tid] = sh[i * TB + tid];
    bar();
}

template <class T>
__device__ void coarsest_solve(const TailLvl<T> &L, const T *f, T *y, int k, int kp, double *sh,
                               double *tot) {
    const int tid = threadIdx.x;
    const int64_t n = L.n;
    const int col = tid % kp;
    double q[1] = {0.0};
    if (col < k)
        for (int64_t i = tid / kp; i < n; i += TB / kp) q[0] += (double)f[i * k + col];
    block_sums<1>(q, sh, kp, tot);  // tot[c] = sum f
    for (int64_t t = tid; t < n * k; t += TB) {
        int64_t i = t / k;
        int c = (int)(t % k);
        double mf = tot[c] / (double)n, acc = 0.0;
        for (int64_t j = 0; j < n; ++j) acc += L.Z[j * n + i] * ((double)f[j * k + c] - mf);
        y[t] = (T)acc;
    }
    bar();
    q[0] = 0.0;
    if (col < k)
        for (int64_t i = tid / kp; i < n; i += TB / kp) q[0] += (double)y[i * k + col];
    block_sums<1>(q, sh, kp, tot);
    for (int64_t t = tid; t < n * k; t += TB) {
        int c = (int)(t % k);
        y[t] = (T)((double)y[t] - tot[c] / (double)n);
    }
    bar();
}

template <class T>
__global__ void __launch_bounds__(TB) k_tail(TailArgs<T> A) {
    __shared__ double sh[2 * TB];
    __shared__ double tot[2 * 32];
    __shared__ double coef[32];
    __shared__ int s_phase[kMaxLevels], s_j[kMaxLevels], s_nvis[kMaxLevels];
    const int tid = threadIdx.x;
    const int k = A.k, kp = 1 << A.lkp;
    int l = A.l0;
    if (tid == 0) s_phase[l] = 0;
    bar();
    while (l >= A.l0) {
        const TailLvl<T> &L = A.lv[l];
        if (L.coarsest) {
            coarsest_solve<T>(L, L.f, L.x, k, kp, sh, tot);
            --l;
            continue;
        }
        const TailLvl<T> &C = A.lv[l + 1];
        if (s_phase[l] == 0) {
            // pre-relaxation, residual, restriction, zero coarse iterate
            gs_sweep<T>(L, k, kp);
            residual<T>(L, L.x, L.f, L.r, k, kp);
            csr_pass<T, 2>(0, L.nc, 0, L.n_rlong, L.rlong, L.n_rlong ? kLongRow : 0, L.rrp, L.rci,
                           L.rw, nullptr, nullptr, L.r, C.f, k, kp);
            for (int64_t t = tid; t < C.n * k; t += TB) C.x[t] = T(0);
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
        residual<T>(C, C.x, C.f, C.rho, k, kp);
        const int j = s_j[l] + 1;
        const int nvis = s_nvis[l];
        const int col = tid % kp;
        bar();  // every thread has read the level's loop state before thread 0 updates it
        if (j >= 2) {  // two-iterate recombination across the visits
            double q[2] = {0.0, 0.0};
            if (col < k)
                for (int64_t i = tid / kp; i < C.n; i += TB / kp) {
                    double rv = (double)C.rho[i * k + col], g = rv - (double)C.rho1[i * k + col];
                    q[0] += g * g;
                    q[1] += g * rv;
                }
            block_sums<2>(q, sh, kp, tot);
            if (tid < k) coef[tid] = tot[tid] > 0.0 ? tot[32 + tid] / tot[tid] : 0.0;
            bar();
            for (int64_t t = tid; t < C.n * k; t += TB) {
                T a = (T)coef[t % k];
                T ev = C.x[t], rv = C.rho[t];
                C.x[t] = ev + a * (C.x1[t] - ev);
                C.rho[t] = rv - a * (rv - C.rho1[t]);
            }
            bar();
        }
        if (j < nvis) {
            for (int64_t t = tid; t < C.n * k; t += TB) {
                C.x1[t] = C.x[t];
                C.rho1[t] = C.rho[t];
            }
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
                for (int64_t i = tid / kp; i < C.n; i += TB / kp) {
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
            for (int64_t t = tid; t < L.n * k; t += TB) {
                int64_t u = t / k;
                int c = (int)(t % k);
                T pe = L.w0[u] * C.x[(int64_t)L.p0[u] * k + c];
                int32_t q1 = L.p1[u];
                if (q1 >= 0) pe += L.w1[u] * C.x[(int64_t)q1 * k + c];
                L.x[t] += (T)coef[c] * pe;
            }
            bar();
        }
        gs_sweep<T>(L, k, kp);
        gs_sweep<T>(L, k, kp);
        --l;
    }
}

__global__ void k_fill_i64(int64_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

// Descriptors of levels l0..nlev-1 for precision T, written to `dst` (device memory of
// nlev * sizeof(TailLvl<T>) bytes) from the host copies.
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
}

template <class T>
void run_tail(const void *d_desc, int l0, int nlev, int k, int64_t *d_visits, hipStream_t s) {
    TailArgs<T> A;
    A.lv = static_cast<const TailLvl<T> *>(d_desc);
    A.l0 = l0;
    A.nlev = nlev;
    A.k = k;
    int lkp = 0;
    while ((1 << lkp) < k) ++lkp;
    A.lkp = lkp;
    A.visits = d_visits;
    k_tail<T><<<1, TB, 0, s>>>(A);
    LAMG_LAUNCH_CHECK();
}

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
template void run_tail<double>(const void *, int, int, int, int64_t *, hipStream_t);
template void run_tail<float>(const void *, int, int, int, int64_t *, hipStream_t);

}  // namespace lamg
