// Cycle kernels of the LAMG+ solve (Sec. 2, "Relaxation" and "Cycle and acceleration"):
// multicolour Gauss-Seidel, residual, restriction P^T r, prolongation with the energy
// correction, coarse and fine iterate recombination, the coarsest dense solve, and the
// finest-level FP64 vector work of the solve and of the FP32 iterative refinement.
//
// Vectors with k right-hand sides are stored row-interleaved: x[i*k + c]. A row is
// handled by a group of G = kp * lpr lanes (kp = k rounded up to a power of two,
// lpr = lanes splitting the row's entries); lane g of a group takes column g % kp and
// every lpr-th entry of the row, and the lpr partial sums are combined by cross-lane
// shuffles. Matrix indices and values are read once per group and broadcast across
// the kp column lanes. Rows of the long class get a whole block each (k_csr_long).
#include "csr_device.h"
#include "lamg_internal.h"

namespace lamg {

namespace {

inline unsigned blocks_for(int64_t work) {
    int64_t b = (work + kBlock - 1) / kBlock;
    return (unsigned)(b > 0 ? b : 1);
}

inline int ilog2(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

inline int kp_log2(int k) { return ilog2(k); }

// Reduction over the `sub` lanes of a group (xor partners kp, 2kp, ..., G/2).
template <class T>
__device__ inline T group_sum(T v, int lkp, int G) {
    for (int o = 1 << lkp; o < G; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

enum { OP_GS = 0, OP_RESID = 1, OP_SPMV = 2, OP_CHEB = 3 };

// Scalars of an OP_CHEB pass: out = c1 * out + c2 * (f - L x) / L_uu (out ignored when
// c1 == 0); the inverse diagonal comes in `dinv`.
template <class T>
struct ChebArgs {
    T c1 = T(0), c2 = T(0);
    const T *dinv = nullptr;
};

// One kernel body for the three CSR passes. Rows are r0 + (group index) or, with a row
// list, rows[group index]. `skip_long` > 0 skips rows longer than it (handled by a
// separate launch over a list).
// Side outputs (null: none): OP_RESID copies x to sx and the residual to sr (the pair the
// next two-iterate recombination starts from); OP_SPMV zeroes sx at the output row (the
// coarse iterate a visit starts from).
// Workgroups are dispatched to the eight XCDs round-robin (block b to XCD b mod 8), and each
// XCD has its own L2. Rows of neighbouring blocks share gathered x values, so a launch's
// blocks are renumbered such that each XCD takes one contiguous slice of the rows: XCD x
// gets the logical blocks [start(x), start(x) + count(x)) in dispatch order. A bijection
// of [0, nb): which block computes which row changes, not any row's arithmetic.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t q = nb / kXcds, r = nb % kXcds;
    const int64_t x = b % kXcds, s = b / kXcds;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// Short-row body: group `grp` of this launch handles one row.
template <class T, int OP>
__device__ __forceinline__ void csr_short_rows(int64_t grp, int64_t r0, int64_t nrows,
                                               const int32_t *__restrict__ rows, int skip_long,
                                               const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci,
                                               const T *__restrict__ v, const T *__restrict__ dd,
                                               const T *__restrict__ f, const T *xin, T *out,
                                               int k, int lkp, int llpr, T *sx, T *sr, ChebArgs<T> ch) {
    const int lg = lkp + llpr;
    const int G = 1 << lg;
    const int g = threadIdx.x & (G - 1);
    const int col = g & ((1 << lkp) - 1);
    const int sub = g >> lkp;
    const int lpr = 1 << llpr;
    bool live = grp < nrows;
    int64_t row = 0;
    int32_t b = 0, e = 0;
    if (live) {
        row = rows ? (int64_t)rows[grp] : r0 + grp;
        b = rp[row];
        e = rp[row + 1];
        if (skip_long > 0 && e - b > skip_long) live = false;
    }
    const int64_t o = row * k + col;
    // the row's own operands are loaded before its entries, so their latency overlaps the
    // gathers' instead of following them
    T acc = T(0), fo = T(0), dr = T(0), xo = T(0), di = T(0), oo = T(0);
    if (live && col < k) {
        if (OP != OP_SPMV) {
            fo = f[o];
            dr = dd[row];
        }
        if (OP == OP_RESID || OP == OP_CHEB) xo = xin[o];
        if (OP == OP_CHEB) {
            di = ch.dinv[row];
            if (ch.c1 != T(0)) oo = out[o];
        }
        acc = row_dot<T, 8>(ci, v, xin, b + sub, e, lpr, k, col);
    }
    if (G > (1 << lkp)) acc = group_sum(acc, lkp, G);
    if (!live || col >= k || sub != 0) return;
    if (OP == OP_GS) {
        out[o] = (fo - acc) * dr;
    } else if (OP == OP_CHEB) {
        const T res = (fo - dr * xo - acc) * di;
        out[o] = ch.c1 == T(0) ? ch.c2 * res : ch.c1 * oo + ch.c2 * res;
    } else if (OP == OP_RESID) {
        const T res = fo - dr * xo - acc;
        out[o] = res;
        if (sx) {
            sx[o] = xo;
            sr[o] = res;
        }
    } else {
        out[o] = acc;
        if (sx) sx[o] = T(0);
    }
}

// Vector of V consecutive columns of one row (16 bytes: 4 FP32 or 2 FP64 columns).
template <class T, int V>
struct alignas(16) ColVec {
    T c[V];
};

// Short-row body with V consecutive columns per lane (k a multiple of V, vectors 16-byte
// aligned): a group of (kp / V) column lanes x lpr entry lanes handles one row, every gather
// and every own-operand access a 16-byte load or store. A row's index/value loads are shared
// by a quarter (FP32) or half (FP64) as many lanes as in the one-column form, and each
// gather instruction moves four (two) times the bytes, so more of the row's neighbours are
// in flight per wave. Sums per column run in entry order per lane, then across the lpr
// lanes by the same xor tree as the one-column form.
template <class T, int OP, int V>
__device__ __forceinline__ void csr_short_rows_vec(int64_t grp, int64_t r0, int64_t nrows,
                                                   const int32_t *__restrict__ rows,
                                                   const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const T *__restrict__ v,
                                                   const T *__restrict__ dd,
                                                   const T *__restrict__ f, const T *xin, T *out,
                                                   int k, int lkv, int llpr, T *sx, T *sr,
                                                   ChebArgs<T> ch) {
    using CV = ColVec<T, V>;
    constexpr int U = 8;
    const int lg = lkv + llpr;
    const int G = 1 << lg;
    const int g = threadIdx.x & (G - 1);
    const int cv = g & ((1 << lkv) - 1);
    const int sub = g >> lkv;
    const int lpr = 1 << llpr;
    const int kv = k / V;
    const bool live = grp < nrows && cv < kv;
    int64_t row = 0;
    int32_t b = 0, e = 0;
    if (grp < nrows) {
        row = rows ? (int64_t)rows[grp] : r0 + grp;
        b = rp[row];
        e = rp[row + 1];
    }
    const int64_t o = row * k + (int64_t)cv * V;
    T acc[V];
#pragma unroll
    for (int q = 0; q < V; ++q) acc[q] = T(0);
    CV fo{}, xo{}, oo{};
    T dr = T(0), di = T(0);
    if (live) {
        if (OP != OP_SPMV) {
            fo = *reinterpret_cast<const CV *>(f + o);
            dr = dd[row];
        }
        if (OP == OP_RESID || OP == OP_CHEB) xo = *reinterpret_cast<const CV *>(xin + o);
        if (OP == OP_CHEB) {
            di = ch.dinv[row];
            if (ch.c1 != T(0)) oo = *reinterpret_cast<const CV *>(out + o);
        }
        for (int32_t j = b + sub; j < e; j += U * lpr) {
            int32_t cc[U];
            T vv[U];
            CV xx[U];
            // FP32: every slot loaded (past the end: the group's first entry, dropped by a
            // select), as in row_dot; FP64: slots past the end load nothing
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t jj = j + u * lpr;
                const bool ok = jj < e;
                if constexpr (sizeof(T) == 4) {
                    const int32_t js = ok ? jj : j;
                    cc[u] = ci[js];
                    vv[u] = v[js];
                } else {
                    cc[u] = ok ? ci[jj] : -1;
                    vv[u] = ok ? v[jj] : T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if constexpr (sizeof(T) == 4) {
                    xx[u] = *reinterpret_cast<const CV *>(xin + (int64_t)cc[u] * k + cv * V);
                } else if (cc[u] >= 0) {
                    xx[u] = *reinterpret_cast<const CV *>(xin + (int64_t)cc[u] * k + cv * V);
                } else {
#pragma unroll
                    for (int q = 0; q < V; ++q) xx[u].c[q] = T(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = j + u * lpr < e;
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    const T term = vv[u] * xx[u].c[q];
                    if constexpr (sizeof(T) == 4)
                        acc[q] = ok ? acc[q] + term : acc[q];
                    else
                        acc[q] += term;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < V; ++q)
        for (int sh = 1 << lkv; sh < G; sh <<= 1) acc[q] += __shfl_xor(acc[q], sh, 64);
    if (!live || sub != 0) return;
    CV res;
#pragma unroll
    for (int q = 0; q < V; ++q) {
        if (OP == OP_GS) {
            res.c[q] = (fo.c[q] - acc[q]) * dr;
        } else if (OP == OP_CHEB) {
            const T rr = (fo.c[q] - dr * xo.c[q] - acc[q]) * di;
            res.c[q] = ch.c1 == T(0) ? ch.c2 * rr : ch.c1 * oo.c[q] + ch.c2 * rr;
        } else if (OP == OP_RESID) {
            res.c[q] = fo.c[q] - dr * xo.c[q] - acc[q];
        } else {
            res.c[q] = acc[q];
        }
    }
    *reinterpret_cast<CV *>(out + o) = res;
    if (OP == OP_RESID && sx) {
        *reinterpret_cast<CV *>(sx + o) = xo;
        *reinterpret_cast<CV *>(sr + o) = res;
    }
    if (OP == OP_SPMV && sx) {
        CV z{};
        *reinterpret_cast<CV *>(sx + o) = z;
    }
}

// Long rows (more than kLongRow off-diagonals: the hubs of power-law graphs and of their
// dense coarse levels): one block of NT threads per row, kp column lanes times NT/kp entry
// lanes, each with 8 loads in flight; the entry lanes' partial sums are combined by a wave
// shuffle tree and then across the waves in wave order. NT = kBlock in general; launches
// of only a few long rows (the colours of dense levels that hold a handful of hubs, where
// the chip is idle but for those rows) use kLongWide threads per row, so that a row of
// thousands of entries spends a quarter of the steps in its chain of dependent loads.
constexpr int kLongWide = 1024;
constexpr int kLongWideRows = 64;  // launches of fewer long rows take the wide blocks

template <class T, int OP, int NT = kBlock>
__device__ __forceinline__ void csr_long_row(int64_t row, const int32_t *__restrict__ rp,
                                             const int32_t *__restrict__ ci,
                                             const T *__restrict__ v, const T *__restrict__ dd,
                                             const T *__restrict__ f, const T *xin, T *out, int k,
                                             int lkp, T *sx, T *sr, ChebArgs<T> ch) {
    constexpr int kWaves = NT / 64;
    __shared__ T part[kWaves][32];
    const int tid = threadIdx.x;
    const int kp = 1 << lkp;
    const int col = tid & (kp - 1);
    const int sub = tid >> lkp;
    const int32_t b = rp[row], e = rp[row + 1];
    const int64_t o = row * k + tid;
    T acc = T(0), fo = T(0), dr = T(0), xo = T(0), di = T(0), oo = T(0);
    if (tid < k) {  // the row's own operands, loaded before its entries
        if (OP != OP_SPMV) {
            fo = f[o];
            dr = dd[row];
        }
        if (OP == OP_RESID || OP == OP_CHEB) xo = xin[o];
        if (OP == OP_CHEB) {
            di = ch.dinv[row];
            if (ch.c1 != T(0)) oo = out[o];
        }
    }
    if (col < k) acc = row_dot<T, 8, false>(ci, v, xin, b + sub, e, NT >> lkp, k, col);
    for (int o2 = kp; o2 < 64; o2 <<= 1) acc += __shfl_xor(acc, o2, 64);
    const int wave = tid >> 6, lane = tid & 63;
    if (lane < kp) part[wave][lane] = acc;
    __syncthreads();
    if (tid >= k) return;
    T sum = T(0);
    for (int w = 0; w < kWaves; ++w) sum += part[w][tid];
    if (OP == OP_GS) {
        out[o] = (fo - sum) * dr;
    } else if (OP == OP_CHEB) {
        const T res = (fo - dr * xo - sum) * di;
        out[o] = ch.c1 == T(0) ? ch.c2 * res : ch.c1 * oo + ch.c2 * res;
    } else if (OP == OP_RESID) {
        const T res = fo - dr * xo - sum;
        out[o] = res;
        if (sx) {
            sx[o] = xo;
            sr[o] = res;
        }
    } else {
        out[o] = sum;
        if (sx) sx[o] = T(0);
    }
}

// One kernel body for the three CSR passes. Rows are r0 + (group index) or, with a row
// list, rows[group index]. `skip_long` > 0 skips rows longer than it (handled by a
// separate launch over a list).
// Side outputs (null: none): OP_RESID copies x to sx and the residual to sr (the pair the
// next two-iterate recombination starts from); OP_SPMV zeroes sx at the output row (the
// coarse iterate a visit starts from).
template <class T, int OP, int FINE>
__global__ void __launch_bounds__(kBlock)
    k_csr(int64_t r0, int64_t nrows, const int32_t *__restrict__ rows, int skip_long,
          const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, const T *__restrict__ v,
          const T *__restrict__ dd, const T *__restrict__ f, const T *xin, T *out, int k, int lkp,
          int llpr, T *sx, T *sr, ChebArgs<T> ch) {
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t grp = blk * (kBlock >> (lkp + llpr)) + (threadIdx.x >> (lkp + llpr));
    csr_short_rows<T, OP>(grp, r0, nrows, rows, skip_long, rp, ci, v, dd, f, xin, out, k, lkp,
                          llpr, sx, sr, ch);
}

template <class T, int OP, int FINE, int V>
__global__ void __launch_bounds__(kBlock)
    k_csr_vec(int64_t r0, int64_t nrows, const int32_t *__restrict__ rows,
              const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
              const T *__restrict__ v, const T *__restrict__ dd, const T *__restrict__ f,
              const T *xin, T *out, int k, int lkv, int llpr, T *sx, T *sr, ChebArgs<T> ch) {
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t grp = blk * (kBlock >> (lkv + llpr)) + (threadIdx.x >> (lkv + llpr));
    csr_short_rows_vec<T, OP, V>(grp, r0, nrows, rows, rp, ci, v, dd, f, xin, out, k, lkv, llpr,
                                 sx, sr, ch);
}

template <class T, int OP, int FINE, int NT>
__global__ void __launch_bounds__(NT)
    k_csr_long(int64_t r0, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp,
               const int32_t *__restrict__ ci, const T *__restrict__ v, const T *__restrict__ dd,
               const T *__restrict__ f, const T *xin, T *out, int k, int lkp, T *sx, T *sr, ChebArgs<T> ch) {
    const int64_t row = rows ? (int64_t)rows[blockIdx.x] : r0 + (int64_t)blockIdx.x;
    csr_long_row<T, OP, NT>(row, rp, ci, v, dd, f, xin, out, k, lkp, sx, sr, ch);
}

// Short and long rows of one pass in a single launch: the first `sblocks` blocks take the
// short rows as k_csr does, each further block one long row as k_csr_long does (the
// arithmetic of every row is that of the separate kernels). Dense coarse levels of
// power-law graphs have both kinds in every colour; one launch instead of two halves the
// dispatches of their many colour passes.
template <class T, int OP, int FINE>
__global__ void __launch_bounds__(kBlock)
    k_csr_mixed(int64_t sblocks, int64_t r0, int64_t nrows, const int32_t *__restrict__ rows,
                int skip_long, int64_t lr0, const int32_t *__restrict__ lrows,
                const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                const T *__restrict__ v, const T *__restrict__ dd, const T *__restrict__ f,
                const T *xin, T *out, int k, int lkp, int llpr, T *sx, T *sr, ChebArgs<T> ch) {
    const int64_t bid = blockIdx.x;
    if (bid < sblocks) {
        // the short-row blocks come first in dispatch order; renumber them among themselves
        const int64_t grp = xcd_block(bid, sblocks) * (kBlock >> (lkp + llpr)) +
                            (threadIdx.x >> (lkp + llpr));
        csr_short_rows<T, OP>(grp, r0, nrows, rows, skip_long, rp, ci, v, dd, f, xin, out, k,
                              lkp, llpr, sx, sr, ch);
    } else {
        const int64_t j = bid - sblocks;
        const int64_t row = lrows ? (int64_t)lrows[j] : lr0 + j;
        csr_long_row<T, OP>(row, rp, ci, v, dd, f, xin, out, k, lkp, sx, sr, ch);
    }
}

// k_csr_mixed with the short rows in the vector-column form (k_csr_vec's conditions).
template <class T, int OP, int FINE, int V>
__global__ void __launch_bounds__(kBlock)
    k_csr_mixed_vec(int64_t sblocks, int64_t r0, int64_t nrows, const int32_t *__restrict__ rows,
                    int64_t lr0, const int32_t *__restrict__ lrows,
                    const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                    const T *__restrict__ v, const T *__restrict__ dd, const T *__restrict__ f,
                    const T *xin, T *out, int k, int lkp, int lkv, int llv, T *sx, T *sr,
                    ChebArgs<T> ch) {
    const int64_t bid = blockIdx.x;
    if (bid < sblocks) {
        const int64_t grp = xcd_block(bid, sblocks) * (kBlock >> (lkv + llv)) +
                            (threadIdx.x >> (lkv + llv));
        csr_short_rows_vec<T, OP, V>(grp, r0, nrows, rows, rp, ci, v, dd, f, xin, out, k, lkv,
                                     llv, sx, sr, ch);
    } else {
        const int64_t j = bid - sblocks;
        const int64_t row = lrows ? (int64_t)lrows[j] : lr0 + j;
        csr_long_row<T, OP>(row, rp, ci, v, dd, f, xin, out, k, lkp, sx, sr, ch);
    }
}

// Lane split of a short-row launch: log2 of the lanes per row, at most a wave per row.
// With 16 or more columns a row's column lanes alone hold half a wave or more; when the
// launch has rows enough for at least 4096 such waves (rows x column lanes >= 2^18) they
// do not split the entries further: each lane then keeps its row's loads in flight on its
// own and no shuffle combines the parts (measured 1.3-1.8x faster per pass on levels of
// 50 K rows and more at k = 16 and 32; on smaller launches the split stays faster).
constexpr int64_t kNoSplitLanes = 1 << 18;
inline int short_llpr(int lkp, int lpr, int64_t nrows) {
    if (lkp >= 4 && (nrows << lkp) >= kNoSplitLanes) return 0;
    int llpr = ilog2(lpr);
    if (lkp + llpr > 6) llpr = 6 - lkp;
    if (llpr < 0) llpr = 0;
    return llpr;
}

// Whether every per-row vector of a launch is 16-byte aligned (the vector-column form).
inline bool vec_aligned(const void *a, const void *b, const void *c, const void *d,
                        const void *e) {
    for (const void *p : {a, b, c, d, e})
        if (p && (reinterpret_cast<uintptr_t>(p) & 15)) return false;
    return true;
}

// FINE = 1 marks launches on the timed level: the code is identical, the separate
// symbol lets a kernel trace attribute that level's time on its own.
template <class T, int OP, int FINE = 0>
void launch_csr(int64_t r0, int64_t nrows, const int32_t *rows, int skip_long, const int32_t *rp,
                const int32_t *ci, const T *v, const T *dd, const T *f, const T *xin, T *out, int k,
                int lpr, hipStream_t s, T *sx = nullptr, T *sr = nullptr,
                ChebArgs<T> ch = ChebArgs<T>()) {
    if (nrows <= 0) return;
    int lkp = kp_log2(k);
    int llpr = short_llpr(lkp, lpr, nrows);
    constexpr int V = 16 / sizeof(T);
    if (skip_long == 0 && k % V == 0 && k >= V && vec_aligned(f, xin, out, sx, sr)) {
        // V columns per lane on kp / V column lanes; the row's entries split over as many
        // lanes as the level asks for (none where the one-column form splits none)
        const int lkv = kp_log2(k / V);
        const int llv = llpr == 0 ? 0 : std::min(ilog2(lpr), 6 - lkv);
        const int64_t gpb = kBlock >> (lkv + llv);
        launch_kernel(k_csr_vec<T, OP, FINE, V>, dim3((unsigned)((nrows + gpb - 1) / gpb)),
                      dim3(kBlock), 0, s, r0, nrows, rows, rp, ci, v, dd, f, xin, out, k, lkv, llv,
                      sx, sr, ch);
        LAMG_LAUNCH_CHECK();
        return;
    }
    int lg = lkp + llpr;
    int64_t groups_per_block = kBlock >> lg;
    unsigned grid = (unsigned)((nrows + groups_per_block - 1) / groups_per_block);
    launch_kernel(k_csr<T, OP, FINE>, dim3(grid), dim3(kBlock), 0, s, r0, nrows, rows, skip_long,
                  rp, ci, v, dd, f, xin, out, k, lkp, llpr, sx, sr, ch);
    LAMG_LAUNCH_CHECK();
}

template <class T, int OP, int FINE = 0>
void launch_csr_long(int64_t r0, int64_t nrows, const int32_t *rows, const int32_t *rp,
                     const int32_t *ci, const T *v, const T *dd, const T *f, const T *xin, T *out,
                     int k, hipStream_t s, T *sx = nullptr, T *sr = nullptr,
                     ChebArgs<T> ch = ChebArgs<T>()) {
    if (nrows <= 0) return;
    if (nrows < kLongWideRows)
        launch_kernel(k_csr_long<T, OP, FINE, kLongWide>, dim3((unsigned)nrows), dim3(kLongWide),
                      0, s, r0, rows, rp, ci, v, dd, f, xin, out, k, kp_log2(k), sx, sr, ch);
    else
        launch_kernel(k_csr_long<T, OP, FINE, kBlock>, dim3((unsigned)nrows), dim3(kBlock), 0, s,
                      r0, rows, rp, ci, v, dd, f, xin, out, k, kp_log2(k), sx, sr, ch);
    LAMG_LAUNCH_CHECK();
}

// Short rows [r0, r0 + nrows) (or the list `rows`) and long rows [lr0, lr0 + nlong) (or the
// list `lrows`) of one pass: one launch when both are present, else the one that is.
template <class T, int OP, int FINE = 0>
void launch_csr_both(int64_t r0, int64_t nrows, const int32_t *rows, int skip_long, int64_t lr0,
                     int64_t nlong, const int32_t *lrows, const int32_t *rp, const int32_t *ci,
                     const T *v, const T *dd, const T *f, const T *xin, T *out, int k, int lpr,
                     hipStream_t s, T *sx = nullptr, T *sr = nullptr,
                     ChebArgs<T> ch = ChebArgs<T>()) {
    if (nrows <= 0) {
        launch_csr_long<T, OP, FINE>(lr0, nlong, lrows, rp, ci, v, dd, f, xin, out, k, s, sx, sr,
                                     ch);
        return;
    }
    if (nlong <= 0) {
        launch_csr<T, OP, FINE>(r0, nrows, rows, skip_long, rp, ci, v, dd, f, xin, out, k, lpr, s,
                                sx, sr, ch);
        return;
    }
    int lkp = kp_log2(k);
    int llpr = short_llpr(lkp, lpr, nrows);
    constexpr int V = 16 / sizeof(T);
    if (skip_long == 0 && k % V == 0 && k >= V && vec_aligned(f, xin, out, sx, sr)) {
        const int lkv = kp_log2(k / V);
        const int llv = llpr == 0 ? 0 : std::min(ilog2(lpr), 6 - lkv);
        const int64_t gpb = kBlock >> (lkv + llv);
        const int64_t sb = (nrows + gpb - 1) / gpb;
        launch_kernel(k_csr_mixed_vec<T, OP, FINE, V>, dim3((unsigned)(sb + nlong)), dim3(kBlock),
                      0, s, sb, r0, nrows, rows, lr0, lrows, rp, ci, v, dd, f, xin, out, k, lkp,
                      lkv, llv, sx, sr, ch);
        LAMG_LAUNCH_CHECK();
        return;
    }
    int64_t groups_per_block = kBlock >> (lkp + llpr);
    int64_t sblocks = (nrows + groups_per_block - 1) / groups_per_block;
    launch_kernel(k_csr_mixed<T, OP, FINE>, dim3((unsigned)(sblocks + nlong)), dim3(kBlock), 0, s,
                  sblocks, r0, nrows, rows, skip_long, lr0, lrows, rp, ci, v, dd, f, xin, out, k,
                  lkp, llpr, sx, sr, ch);
    LAMG_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Elementwise kernels
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T *x, int64_t n, T val) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = val;
}

template <class T>
__global__ void k_copy(T *__restrict__ d, const T *__restrict__ s, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// x[u] += mu_c * (w0 e[p0] + w1 e[p1])   (energy-corrected prolongation)
// Elementwise kernels over n rows x k columns use a (row, column) thread mapping with the
// column count rounded up to kp = 2^lkp, so that no integer division is needed.
#define ROWCOL(n, lkp)                                                         \
    const int64_t tt_ = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;        \
    const int64_t u = tt_ >> (lkp);                                            \
    const int c = (int)(tt_ & ((1 << (lkp)) - 1));                             \
    if (u >= (n) || c >= k) return;                                            \
    const int64_t t = u * k + c;

inline unsigned rc_blocks(int64_t n, int k) {
    int lkp = 0;
    while ((1 << lkp) < k) ++lkp;
    int64_t work = n << lkp;
    return (unsigned)((work + kBlock - 1) / kBlock > 0 ? (work + kBlock - 1) / kBlock : 1);
}

// (P e_c) at fine row u, column c: w0 e_c[p0] (+ w1 e_c[p1] when the row has a second
// parent). Both gathers are issued unconditionally (a row without a second parent re-reads
// its first) and the second term is dropped by a select, so neither load waits behind a
// branch.
template <class T>
__device__ __forceinline__ T interp(int64_t u, int k, int c, const int32_t *__restrict__ p0,
                                    const int32_t *__restrict__ p1, const T *__restrict__ w0,
                                    const T *__restrict__ w1, const T *__restrict__ ec) {
    const int32_t a = p0[u], q = p1[u];
    const T wa = w0[u], wb = w1[u];
    const T ea = ec[(int64_t)a * k + c];
    const T eb = ec[(int64_t)(q >= 0 ? q : a) * k + c];
    const T pe = wa * ea;
    const T pe2 = pe + wb * eb;
    return q >= 0 ? pe2 : pe;
}

template <class T>
__global__ void k_prolong(int64_t n, int k, int lkp, const int32_t *__restrict__ p0,
                          const int32_t *__restrict__ p1, const T *__restrict__ w0,
                          const T *__restrict__ w1, const T *__restrict__ ec,
                          const double *__restrict__ mu, T *__restrict__ x) {
    ROWCOL(n, lkp)
    x[t] += (T)mu[c] * interp(u, k, c, p0, p1, w0, w1, ec);
}

// x[rows[a]] += e[a] for the kept rows of an elimination level (their interpolation is
// the identity; the eliminated rows are recomputed afterwards)
template <class T>
__global__ void k_inject_add(int64_t nc, int k, int lkp, const int32_t *__restrict__ rows,
                             const T *__restrict__ ec, T *__restrict__ x) {
    ROWCOL(nc, lkp)
    x[(int64_t)rows[u] * k + c] += ec[t];
}

// ---------------------------------------------------------------------------
// Deterministic two-pass reductions: blocks write partial sums in a fixed order, one
// block combines them in block order and finishes the per-column scalar.
// Element mapping: block of 256 threads = (256/kp) rows x kp columns.
// ---------------------------------------------------------------------------
enum { R_MU = 0, R_RC2 = 1, R_NORM2 = 2, R_SUM = 3, R_MAXABS = 4, R_RCF = 5, R_RES2 = 6,
       R_NONFIN = 7 };

template <int R>
struct RedQ;
template <> struct RedQ<R_MU> { static constexpr int Q = 2; };
template <> struct RedQ<R_RC2> { static constexpr int Q = 2; };
template <> struct RedQ<R_NORM2> { static constexpr int Q = 1; };
template <> struct RedQ<R_SUM> { static constexpr int Q = 1; };
template <> struct RedQ<R_MAXABS> { static constexpr int Q = 1; };
template <> struct RedQ<R_RES2> { static constexpr int Q = 2; };  // ||r||^2 and max |r|
template <> struct RedQ<R_NONFIN> { static constexpr int Q = 1; };  // count of NaN / inf
// Quantities of a reduction combined by max instead of sum (bit i: quantity i).
template <int R>
constexpr int red_max_mask() {
    return R == R_MAXABS ? 1 : (R == R_RES2 ? 2 : 0);
}
template <> struct RedQ<R_RCF> { static constexpr int Q = 14; };

struct RedIn {
    const void *a, *b, *c, *d;  // operand vectors (meaning per reduction)
    int m;                      // RCF: history size
    int64_t hstride;            // RCF: elements between history slots
};

// One element's operands of a reduction (load) and its terms (add), kept apart so that
// several elements' loads can be in flight before their terms are added in order.
template <class T, int R>
struct RedElem {
    double a[5];
    __device__ inline void load(const RedIn &in, int64_t o) {
        if (R == R_MU) {  // a = e, b = fc, c = rho
            a[0] = (double)((const T *)in.a)[o];
            a[1] = (double)((const T *)in.b)[o];
            a[2] = (double)((const T *)in.c)[o];
        } else if (R == R_RC2) {  // a = rho, b = rho1
            a[0] = (double)((const T *)in.a)[o];
            a[1] = (double)((const T *)in.b)[o];
        } else if (R == R_NORM2 || R == R_SUM || R == R_MAXABS || R == R_RES2 || R == R_NONFIN) {
            a[0] = (double)((const T *)in.a)[o];
        } else {  // RCF: a = r, b = history residuals (m slots; slots past m reread m - 1)
            const double *hr = (const double *)in.b;
            a[0] = ((const double *)in.a)[o];
            for (int i = 0; i < 4; ++i) a[1 + i] = hr[(int64_t)min(i, in.m - 1) * in.hstride + o];
        }
    }
    __device__ inline void add(const RedIn &in, double *q) const {
        if (R == R_MU) {  // <e, fc>, <e, fc - rho>
            q[0] += a[0] * a[1];
            q[1] += a[0] * (a[1] - a[2]);
        } else if (R == R_RC2) {  // G = rho - rho1: <G, G>, <G, rho>
            const double g = a[0] - a[1];
            q[0] += g * g;
            q[1] += g * a[0];
        } else if (R == R_NORM2) {
            q[0] += a[0] * a[0];
        } else if (R == R_SUM) {
            q[0] += a[0];
        } else if (R == R_MAXABS) {
            q[0] = fmax(q[0], fabs(a[0]));
        } else if (R == R_RES2) {
            q[0] += a[0] * a[0];
            q[1] = fmax(q[1], fabs(a[0]));
        } else if (R == R_NONFIN) {
            q[0] += isfinite(a[0]) ? 0.0 : 1.0;
        } else {  // RCF: G_i = r - r_i (0 past m)
            const double rv = a[0];
            double G[4];
            for (int i = 0; i < 4; ++i) G[i] = (i < in.m) ? rv - a[1 + i] : 0.0;
            int t = 0;
            for (int i = 0; i < 4; ++i)
                for (int j = i; j < 4; ++j) q[t++] += G[i] * G[j];
            for (int i = 0; i < 4; ++i) q[10 + i] += G[i] * rv;
        }
    }
};

template <class T, int R>
__global__ void __launch_bounds__(kBlock)
    k_red_partial(int64_t n, int k, int lkp, RedIn in, double *__restrict__ partial) {
    constexpr int Q = RedQ<R>::Q;
    __shared__ double sh[Q][kBlock];
    const int kp = 1 << lkp;
    const int col = threadIdx.x & (kp - 1);
    const int rloc = threadIdx.x >> lkp;
    const int rows_blk = kBlock >> lkp;
    double q[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) q[i] = 0.0;
    if (col < k) {
        // four rows per step: their loads are issued together, their terms added in row order
        const int64_t step = (int64_t)gridDim.x * rows_blk;
        int64_t row = (int64_t)blockIdx.x * rows_blk + rloc;
        for (; row + 3 * step < n; row += 4 * step) {
            RedElem<T, R> el[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) el[u].load(in, (row + u * step) * k + col);
#pragma unroll
            for (int u = 0; u < 4; ++u) el[u].add(in, q);
        }
        for (; row < n; row += step) {
            RedElem<T, R> el;
            el.load(in, row * k + col);
            el.add(in, q);
        }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) sh[i][threadIdx.x] = q[i];
    __syncthreads();
    for (int st = rows_blk >> 1; st > 0; st >>= 1) {
        if (rloc < st) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if ((red_max_mask<R>() >> i) & 1)
                    sh[i][threadIdx.x] = fmax(sh[i][threadIdx.x], sh[i][threadIdx.x + (st << lkp)]);
                else
                    sh[i][threadIdx.x] += sh[i][threadIdx.x + (st << lkp)];
            }
        }
        __syncthreads();
    }
    if (rloc == 0 && col < k) {
#pragma unroll
        for (int i = 0; i < Q; ++i) partial[((int64_t)blockIdx.x * Q + i) * k + col] = sh[i][threadIdx.x];
    }
}

// Per-column finishers (one thread per column after the block totals are formed).
struct Fin {
    double *out;        // per-column result(s)
    const double *aux;  // per-column auxiliary input (e.g. ||b|| for relres)
    double scale;
    int m;
    double *out2 = nullptr;  // R_RES2: per-column max |r|
};

__device__ inline void solve_rcf(const double *q, int m, double *alpha) {
    // Jacobi-scaled normal equations of min ||r - sum a_i G_i||, Cholesky with pivots
    // <= 1e-12 dropped (their a_i = 0).
    double M[4][4], g[4], s[4], R[4][4], y[4], a[4];
    bool keep[4];
    int t = 0;
    for (int i = 0; i < 4; ++i)
        for (int j = i; j < 4; ++j) {
            M[i][j] = q[t];
            M[j][i] = q[t];
            ++t;
        }
    for (int i = 0; i < 4; ++i) g[i] = q[10 + i];
    for (int i = 0; i < m; ++i) {
        keep[i] = M[i][i] > 0.0;
        s[i] = keep[i] ? 1.0 / sqrt(M[i][i]) : 0.0;
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) R[i][j] = 0.0;
    for (int j = 0; j < m; ++j) {
        if (!keep[j]) continue;
        double d = s[j] * M[j][j] * s[j];
        for (int kk = 0; kk < j; ++kk)
            if (keep[kk]) d -= R[j][kk] * R[j][kk];
        if (!(d > 1e-12)) {
            keep[j] = false;
            continue;
        }
        R[j][j] = sqrt(d);
        for (int i = j + 1; i < m; ++i) {
            double v = s[i] * M[i][j] * s[j];
            for (int kk = 0; kk < j; ++kk)
                if (keep[kk]) v -= R[i][kk] * R[j][kk];
            R[i][j] = v / R[j][j];
        }
    }
    for (int i = 0; i < m; ++i) {
        y[i] = 0.0;
        if (!keep[i]) continue;
        double v = s[i] * g[i];
        for (int kk = 0; kk < i; ++kk)
            if (keep[kk]) v -= R[i][kk] * y[kk];
        y[i] = v / R[i][i];
    }
    for (int i = m - 1; i >= 0; --i) {
        a[i] = 0.0;
        if (!keep[i]) continue;
        double v = y[i];
        for (int kk = i + 1; kk < m; ++kk)
            if (keep[kk]) v -= R[kk][i] * a[kk];
        a[i] = v / R[i][i];
    }
    for (int i = 0; i < 4; ++i) alpha[i] = (i < m) ? a[i] * s[i] : 0.0;
}

// Totals over nblk block partials (partial[(b Q + i) k + c]) of Q x k quantities into
// tot[i * 32 + c] (then a barrier). A group of G lanes takes one quantity (G the largest
// power of two up to 64 with Q k G <= blockDim; groups loop over the quantities): lane g
// combines the partials b = g, g + G, ... in order and the group then combines its lanes
// by an xor butterfly, lane 0's value being the total. The order depends only on nblk, k
// and blockDim, so every launch of the same shape gives the same bits.
template <int Q, int MAXMASK>
__device__ inline void group_totals(int nblk, int k, const double *__restrict__ partial,
                                    double *tot) {
    const int nq = Q * k;
    int G = 64;
    while (G > 1 && nq * G > (int)blockDim.x) G >>= 1;
    const int groups = (int)blockDim.x / G;
    const int grp = (int)threadIdx.x / G, g = (int)threadIdx.x & (G - 1);
    for (int q0 = 0; q0 < nq; q0 += groups) {
        const int idx = q0 + grp;
        const bool live = idx < nq;
        const int i = live ? idx / k : 0, c = live ? idx - i * k : 0;
        const bool MAX = (MAXMASK >> i) & 1;  // uniform within the group
        double s = 0.0;
        if (live)
            for (int b0 = g; b0 < nblk; b0 += 8 * G) {  // 8 loads in flight, added in order
                double v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int b = b0 + u * G;
                    v[u] = b < nblk ? partial[((int64_t)b * Q + i) * k + c] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (b0 + u * G < nblk) s = MAX ? fmax(s, v[u]) : s + v[u];
            }
        for (int o = G >> 1; o > 0; o >>= 1) {
            const double t = __shfl_xor(s, o, 64);
            s = MAX ? fmax(s, t) : s + t;
        }
        if (live && g == 0) tot[i * 32 + c] = s;
    }
    __syncthreads();
}

template <int R>
__global__ void __launch_bounds__(kBlock)
    k_red_final(int nblk, int k, const double *__restrict__ partial, Fin fin) {
    constexpr int Q = RedQ<R>::Q;
    __shared__ double tot[Q * 32];
    group_totals<Q, red_max_mask<R>()>(nblk, k, partial, tot);
    int c = threadIdx.x;
    if (c >= k) return;
    if (R == R_MU) {
        double num = tot[c], den = tot[32 + c];
        double mu = num / den;
        if (!(den > 0.0) || !isfinite(mu)) mu = 1.0;
        fin.out[c] = mu;
    } else if (R == R_RC2) {
        double gg = tot[c], gr = tot[32 + c];
        fin.out[c] = (gg > 0.0) ? gr / gg : 0.0;
    } else if (R == R_NORM2) {
        double v = sqrt(tot[c]);
        fin.out[c] = fin.aux ? (fin.aux[c] > 0.0 ? v / fin.aux[c] : 0.0) : v;
    } else if (R == R_SUM || R == R_NONFIN) {
        fin.out[c] = fin.scale * tot[c];
    } else if (R == R_MAXABS) {
        fin.out[c] = tot[c];
    } else if (R == R_RES2) {  // relative residual (as R_NORM2 with aux) and max |r|
        double v = sqrt(tot[c]);
        fin.out[c] = fin.aux[c] > 0.0 ? v / fin.aux[c] : 0.0;
        fin.out2[c] = tot[32 + c];
    } else {
        double q[14];
        for (int i = 0; i < 14; ++i) q[i] = tot[i * 32 + c];
        solve_rcf(q, fin.m, fin.out + 4 * c);
    }
}

// Whether the blocks of an n x k update can each add the nblk partial sums of a
// two-quantity reduction themselves (the fused launch) instead of reading scalars formed
// once by one block: their extra reads, blocks x nblk x 2k doubles from L2, must stay small.
inline bool fuse_totals(int64_t n, int k, int nblk) {
    return (int64_t)rc_blocks(n, k) * nblk * 2 * k <= kFuseTotalsMax;
}

inline int red_blocks(int64_t n, int k) {
    int lkp = kp_log2(k);
    int64_t rows_blk = kBlock >> lkp;
    int64_t b = (n + rows_blk * 4 - 1) / (rows_blk * 4);
    if (b < 1) b = 1;
    if (b > kRedBlocksMax) b = kRedBlocksMax;
    return (int)b;
}

template <class T, int R>
void reduce(int64_t n, int k, RedIn in, double *partial, Fin fin, hipStream_t s) {
    int nblk = red_blocks(n, k);
    launch_kernel(k_red_partial<T, R>, dim3(nblk), dim3(kBlock), 0, s, n, k, kp_log2(k), in, partial);
    LAMG_LAUNCH_CHECK();
    launch_kernel(k_red_final<R>, dim3(1), dim3(kBlock), 0, s, nblk, k, partial, fin);
    LAMG_LAUNCH_CHECK();
}

// e += alpha (e1 - e); rho -= alpha (rho - rho1); with keep, (e1, rho1) = the result
template <class T>
__global__ void k_rc2_update(int64_t n, int k, int lkp, T *__restrict__ e, T *__restrict__ rho,
                             T *e1, T *rho1, const double *__restrict__ alpha, int keep) {
    ROWCOL(n, lkp)
    T a = (T)alpha[c];
    T ev = e[t], rv = rho[t];
    const T en = ev + a * (e1[t] - ev);
    const T rn = rv - a * (rv - rho1[t]);
    e[t] = en;
    rho[t] = rn;
    if (keep) {
        e1[t] = en;
        rho1[t] = rn;
    }
}

// Column totals of a two-quantity reduction from its block partials, in k_red_final's
// order (same block size), into tot[i][c] of the calling block (followed by a barrier).
__device__ inline void block_totals2(int nblk, int k, const double *__restrict__ partial,
                                     double (*tot)[32]) {
    group_totals<2, 0>(nblk, k, partial, &tot[0][0]);
}

// Energy correction and prolongation in one launch: every block forms mu per column from
// the partial sums of run_mu_partial (the arithmetic of k_red_final) and applies
// x += mu P e_c on its rows.
template <class T>
__global__ void __launch_bounds__(kBlock)
    k_prolong_mu(int64_t n, int k, int lkp, const int32_t *__restrict__ p0,
                 const int32_t *__restrict__ p1, const T *__restrict__ w0, const T *__restrict__ w1,
                 const T *__restrict__ ec, int nblk, const double *__restrict__ partial,
                 T *__restrict__ x) {
    __shared__ double tot[2][32];
    __shared__ double mu_s[32];
    // the element's operands are loaded first, so that their latency overlaps the totals'
    const int64_t tt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t u = tt >> lkp;
    const int c = (int)(tt & ((1 << lkp) - 1));
    const bool live = u < n && c < k;
    T pe = T(0), xv = T(0);
    if (live) {
        pe = interp(u, k, c, p0, p1, w0, w1, ec);
        xv = x[u * k + c];
    }
    block_totals2(nblk, k, partial, tot);
    if ((int)threadIdx.x < k) {
        const int cc = threadIdx.x;
        const double num = tot[0][cc], den = tot[1][cc];
        double mu = num / den;
        if (!(den > 0.0) || !isfinite(mu)) mu = 1.0;
        mu_s[cc] = mu;
    }
    __syncthreads();
    if (live) x[u * k + c] = xv + (T)mu_s[c] * pe;
}

// Two-iterate recombination update in one launch with its coefficient: every block forms
// alpha = <G, rho> / <G, G> per column from the partial sums, applies
// e += alpha (e1 - e), rho -= alpha (rho - rho1), and with `keep` saves the result as the
// next (e1, rho1).
template <class T>
__global__ void __launch_bounds__(kBlock)
    k_rc2_fused(int64_t n, int k, int lkp, T *__restrict__ e, T *__restrict__ rho, T *e1, T *rho1,
                int nblk, const double *__restrict__ partial, int keep) {
    __shared__ double tot[2][32];
    __shared__ double al_s[32];
    // the element's operands are loaded first, so that their latency overlaps the totals'
    const int64_t tt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t u = tt >> lkp;
    const int c = (int)(tt & ((1 << lkp) - 1));
    const bool live = u < n && c < k;
    const int64_t t = u * k + c;
    T ev = T(0), rv = T(0), e1v = T(0), r1v = T(0);
    if (live) {
        ev = e[t];
        rv = rho[t];
        e1v = e1[t];
        r1v = rho1[t];
    }
    block_totals2(nblk, k, partial, tot);
    if ((int)threadIdx.x < k) {
        const int cc = threadIdx.x;
        const double gg = tot[0][cc], gr = tot[1][cc];
        al_s[cc] = (gg > 0.0) ? gr / gg : 0.0;
    }
    __syncthreads();
    if (!live) return;
    T a = (T)al_s[c];
    const T en = ev + a * (e1v - ev);
    const T rn = rv - a * (rv - r1v);
    e[t] = en;
    rho[t] = rn;
    if (keep) {
        e1[t] = en;
        rho1[t] = rn;
    }
}

// Coarsest solve y = L^+ f (Z holds the pseudo-inverse, so y has zero mean), FP64. One
// wave per (row, column); its lanes split the row of the symmetric Z and add by shuffles.
template <class T>
__global__ void __launch_bounds__(kBlock)
    k_coarsest(int64_t n, const double *__restrict__ Z, const T *__restrict__ f, T *__restrict__ y,
               int k) {
    const int64_t unit = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t u = unit / k;
    const int c = (int)(unit - u * k);
    double acc = 0.0;
    if (u < n) {
        const double *zr = Z + u * n;
        for (int64_t j = lane; j < n; j += 64) acc += zr[j] * (double)f[j * k + c];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (u < n && lane == 0) y[u * k + c] = (T)acc;
}

// ---------------------------------------------------------------------------
// Finest-level FP64 vector kernels
// ---------------------------------------------------------------------------
__global__ void k_gather_cols(int64_t n, int k, const int32_t *__restrict__ perm,
                              const double *__restrict__ src, double *__restrict__ dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    int64_t i = t / k;
    int c = (int)(t - i * k);
    dst[t] = src[(int64_t)c * n + perm[i]];
}

__global__ void k_scatter_cols(int64_t n, int k, const int32_t *__restrict__ perm,
                               const double *__restrict__ src, const int32_t *__restrict__ mask,
                               double *__restrict__ dst) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    int64_t i = t / k;
    int c = (int)(t - i * k);
    if (mask && !mask[c]) return;
    dst[(int64_t)c * n + perm[i]] = src[t];
}

__global__ void k_sub_col(int64_t n, int k, int lkp, double *__restrict__ x,
                          const double *__restrict__ m) {
    ROWCOL(n, lkp)
    x[t] -= m[c];
}

// phi += sum_i a_i (phi_i - phi); r -= sum_i a_i (r - r_i)
// ... and the recombined pair is saved in history slot `slot` (the slot may be one of the
// m read: each thread reads its element of every slot before writing it)
__global__ void k_rcf_update(int64_t n, int k, int lkp, int m, double *__restrict__ phi,
                             double *__restrict__ r, double *hphi, double *hr, int64_t hstride,
                             const double *__restrict__ alpha, int slot) {
    ROWCOL(n, lkp)
    double p = phi[t], rv = r[t], dp = 0.0, dr = 0.0;
    for (int i = 0; i < m; ++i) {
        double a = alpha[4 * c + i];
        dp += a * (hphi[i * hstride + t] - p);
        dr += a * (rv - hr[i * hstride + t]);
    }
    const double pn = p + dp, rn = rv - dr;
    phi[t] = pn;
    r[t] = rn;
    hphi[slot * hstride + t] = pn;
    hr[slot * hstride + t] = rn;
}

// d = r / scale (per column) in FP32; zx (if given) = 0, the FP32 iterate a cycle starts from
__global__ void k_to_f32_scaled(int64_t n, int k, int lkp, const double *__restrict__ r,
                                const double *__restrict__ sc, float *__restrict__ d,
                                float *__restrict__ zx) {
    ROWCOL(n, lkp)
    double s = sc[c];
    d[t] = (float)(s > 0.0 ? r[t] / s : 0.0);
    if (zx) zx[t] = 0.0f;
}

__global__ void k_add_scaled_f32(int64_t n, int k, int lkp, const float *__restrict__ e,
                                 const double *__restrict__ sc, double *__restrict__ phi) {
    ROWCOL(n, lkp)
    phi[t] += sc[c] * (double)e[t];
}

__global__ void k_zero_cols(int64_t n, int k, int lkp, const int32_t *__restrict__ zmask,
                            double *__restrict__ x) {
    ROWCOL(n, lkp)
    if (zmask[c]) x[t] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// Cycle launchers
// ---------------------------------------------------------------------------

template <class T, int FINE>
static void gs_color(const SolveOp &op, int c, const T *v, const T *dinv, const T *f, T *x, int k,
                     hipStream_t s) {
    const int nc = op.ncolors;
    int64_t a = op.blk[c], b = op.blk[c + 1];              // short rows of colour c
    int64_t la = op.blk[nc + c], lb = op.blk[nc + c + 1];  // long rows of colour c
    launch_csr_both<T, OP_GS, FINE>(a, b - a, nullptr, 0, la, lb - la, nullptr, op.rp.p, op.ci.p,
                                    v, dinv, f, x, x, k, op.lpr_short, s);
}

template <class T>
void run_gs(const SolveOp &op, const T *v, const T *dinv, const T *f, T *x, int k, int sweeps,
            hipStream_t s, bool fine) {
    for (int sw = 0; sw < sweeps; ++sw)
        for (int c = 0; c < op.ncolors; ++c) {
            if (fine)
                gs_color<T, 1>(op, c, v, dinv, f, x, k, s);
            else
                gs_color<T, 0>(op, c, v, dinv, f, x, k, s);
        }
}

template <class T>
void run_gs_color(const SolveOp &op, int c, const T *v, const T *dinv, const T *f, T *x, int k,
                  hipStream_t s, bool fine) {
    if (fine)
        gs_color<T, 1>(op, c, v, dinv, f, x, k, s);
    else
        gs_color<T, 0>(op, c, v, dinv, f, x, k, s);
}

template <class T, int FINE>
static void residual_impl(const SolveOp &op, const T *v, const T *d, const T *x, const T *f, T *r,
                          int k, hipStream_t s, T *sx, T *sr) {
    const int nc = op.ncolors;
    int64_t nshort = op.blk[nc];
    launch_csr_both<T, OP_RESID, FINE>(0, nshort, nullptr, 0, nshort, op.n - nshort, nullptr,
                                       op.rp.p, op.ci.p, v, d, f, x, r, k, op.lpr_short, s, sx,
                                       sr);
}

template <class T>
void run_residual(const SolveOp &op, const T *v, const T *d, const T *x, const T *f, T *r, int k,
                  hipStream_t s, bool fine, T *x_copy, T *r_copy) {
    if (fine)
        residual_impl<T, 1>(op, v, d, x, f, r, k, s, x_copy, r_copy);
    else
        residual_impl<T, 0>(op, v, d, x, f, r, k, s, x_copy, r_copy);
}

template <class T>
void run_residual_color(const SolveOp &op, int c, const T *v, const T *d, const T *x, const T *f,
                        T *r, int k, hipStream_t s, bool fine) {
    const int nc = op.ncolors;
    int64_t a = op.blk[c], b = op.blk[c + 1], la = op.blk[nc + c], lb = op.blk[nc + c + 1];
    if (fine)
        launch_csr_both<T, OP_RESID, 1>(a, b - a, nullptr, 0, la, lb - la, nullptr, op.rp.p,
                                        op.ci.p, v, d, f, x, r, k, op.lpr_short, s);
    else
        launch_csr_both<T, OP_RESID, 0>(a, b - a, nullptr, 0, la, lb - la, nullptr, op.rp.p,
                                        op.ci.p, v, d, f, x, r, k, op.lpr_short, s);
}

template <class T>
__global__ void k_add_into(T *__restrict__ x, const T *__restrict__ d, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += d[i];
}

// Chebyshev semi-iteration on L x = f with the Jacobi preconditioner, damping the spectrum
// of D^{-1} L on [lmax / kChebRatio, lmax] (Adams, Brezina, Hu and Tuminaro 2003): step 0
// d = D^{-1} r / theta; step j > 0 d = rho_j rho_{j-1} d + (2 rho_j / delta) D^{-1} r with
// rho_0 = 1 / sigma, rho_j = 1 / (2 sigma - rho_{j-1}); x += d after each step. All rows of
// a step read the same x (one CSR pass into d, then the update), so any row order gives the
// same result.
template <class T>
void run_cheb_sweep(const SolveOp &op, double lmax, const T *v, const T *d, const T *dinv,
                    const T *f, T *x, T *dvec, int k, hipStream_t s, bool fine) {
    const double b = lmax, a = lmax / kChebRatio;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho0 = 1.0 / sigma;
    const int nc = op.ncolors;
    const int64_t nshort = op.blk[nc];
    const int64_t nk = op.n * k;
    for (int step = 0; step < kChebDegree; ++step) {
        ChebArgs<T> ch;
        ch.dinv = dinv;
        if (step == 0) {
            ch.c1 = T(0);
            ch.c2 = (T)(1.0 / theta);
        } else {
            const double rho1 = 1.0 / (2.0 * sigma - rho0);
            ch.c1 = (T)(rho1 * rho0);
            ch.c2 = (T)(2.0 * rho1 / delta);
            rho0 = rho1;
        }
        if (fine)
            launch_csr_both<T, OP_CHEB, 1>(0, nshort, nullptr, 0, nshort, op.n - nshort, nullptr,
                                           op.rp.p, op.ci.p, v, d, f, x, dvec, k, op.lpr_short, s,
                                           nullptr, nullptr, ch);
        else
            launch_csr_both<T, OP_CHEB, 0>(0, nshort, nullptr, 0, nshort, op.n - nshort, nullptr,
                                           op.rp.p, op.ci.p, v, d, f, x, dvec, k, op.lpr_short, s,
                                           nullptr, nullptr, ch);
        launch_kernel(k_add_into<T>, dim3(blocks_for(nk)), dim3(kBlock), 0, s, x, (const T *)dvec,
                      nk);
        LAMG_LAUNCH_CHECK();
    }
}

// Block-Jacobi Gauss-Seidel sweep (smoother 2) on L x = f, blocks of kBjBlock rows in their
// natural order, after r = f - L x at the sweep's start: a row's right-hand side minus its
// entries in other blocks is r + d x + (its in-block entries times x), all at the start
// values, so the cross-block sums -- the hub rows' thousands of entries among them -- come
// from the residual kernel, and this kernel keeps to one block per wave:
//  - the block's start values, diagonals and in-block entries (the first kBjStage of them;
//    blocks of hub rows read the rest from global memory) go to LDS, and every row's
//    right-hand side for the block's sweep is formed from them, rows side by side;
//  - then the rows in order (kp column lanes x 64/kp entry lanes per row) gather their
//    in-block entries from the LDS copy of the block's values, which holds the new value of
//    every row already relaxed and the start value of the others; the new value goes to
//    LDS and to x. The wave's LDS accesses complete in program order, so each row sees the
//    rows before it.
constexpr int kBjStage = 1024;

template <class T>
struct BjArgs {
    const int32_t *rows, *irp;
    const uint8_t *iloc;
    const T *iv, *d, *dinv, *r;
    T *x;
};

namespace {
template <class T>
__global__ void __launch_bounds__(64) k_bjgs(int64_t n, int k, int lkp, BjArgs<T> a) {
    extern __shared__ __align__(16) unsigned char bj_smem[];
    __shared__ T dv[kBjBlock], dg[kBjBlock], ivs[kBjStage];
    __shared__ int32_t rs[kBjBlock], ir[kBjBlock + 1];
    __shared__ uint8_t ils[kBjStage];
    const int kp = 1 << lkp;
    T *xs = reinterpret_cast<T *>(bj_smem);  // [kBjBlock][kp]: the block's current values
    T *fs = xs + kBjBlock * kp;              // [kBjBlock][kp]: right-hand sides of the block
    const int lane = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kBjBlock;
    const int nb = (int)min((int64_t)kBjBlock, n - b0);
    const int ib = a.irp[b0];
    for (int t = lane; t <= nb; t += 64) ir[t] = a.irp[b0 + t] - ib;
    const int ni = a.irp[b0 + nb] - ib;
    const int ns = min(ni, kBjStage);
    for (int e = lane; e < ns; e += 64) {
        ils[e] = a.iloc[ib + e];
        ivs[e] = a.iv[ib + e];
    }
    for (int t = lane; t < nb; t += 64) {
        const int i = a.rows[b0 + t];
        rs[t] = i;
        dv[t] = a.dinv[i];
        dg[t] = a.d[i];
    }
    __syncthreads();
    for (int q = lane; q < (nb << lkp); q += 64) {
        const int t = q >> lkp, c = q & (kp - 1);
        if (c < k) xs[q] = a.x[(int64_t)rs[t] * k + c];
    }
    __syncthreads();
    for (int q = lane; q < (nb << lkp); q += 64) {
        const int t = q >> lkp, c = q & (kp - 1);
        if (c >= k) continue;
        T s = a.r[(int64_t)rs[t] * k + c] + dg[t] * xs[q];
        for (int j = ir[t]; j < ir[t + 1]; ++j)
            s += (j < ns ? ivs[j] : a.iv[ib + j]) * xs[(j < ns ? ils[j] : a.iloc[ib + j]) * kp + c];
        fs[q] = s;
    }
    __syncthreads();
    const int c = lane & (kp - 1);
    const int s2 = lane >> lkp, g2 = 64 >> lkp;
    for (int t = 0; t < nb; ++t) {
        const int j1 = ir[t + 1];
        T acc = T(0);
        if (c < k)
            for (int j = ir[t] + s2; j < j1; j += g2) {
                int lc;
                T vv;
                if (j < ns) {
                    lc = ils[j];
                    vv = ivs[j];
                } else {
                    lc = a.iloc[ib + j];
                    vv = a.iv[ib + j];
                }
                acc += vv * xs[lc * kp + c];
            }
        for (int o = kp; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (s2 == 0 && c < k) {
            const T xn = (fs[t * kp + c] - acc) * dv[t];
            xs[t * kp + c] = xn;
            a.x[(int64_t)rs[t] * k + c] = xn;
        }
    }
}
}  // namespace

template <class T>
void run_bjgs_sweep(const SolveOp &op, const T *v, const T *d, const T *dinv, const T *f, T *x,
                    T *r, int k, hipStream_t s, bool fine) {
    if (op.n <= 0) return;
    if (k < 1 || k > 32) throw Error(LAMG_INVALID_ARG, "block-Jacobi sweep: column count");
    run_residual<T>(op, v, d, x, f, r, k, s, fine);
    const int lkp = kp_log2(k);
    BjArgs<T> a;
    a.rows = op.bj_rows.p;
    a.irp = op.bj_irp.p;
    a.iloc = op.bj_iloc.p;
    if constexpr (sizeof(T) == 8)
        a.iv = op.bj_iv64.p;
    else
        a.iv = op.bj_iv32.p;
    a.d = d;
    a.dinv = dinv;
    a.r = r;
    a.x = x;
    const uint32_t lds = (uint32_t)(2 * (size_t)kBjBlock * ((size_t)1 << lkp) * sizeof(T));
    launch_kernel(k_bjgs<T>, dim3((unsigned)((op.n + kBjBlock - 1) / kBjBlock)), dim3(64), lds, s,
                  op.n, k, lkp, a);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_inject_add(const SolveOp &op, const T *ec, T *x, int k, hipStream_t s) {
    if (op.nc <= 0) return;
    launch_kernel(k_inject_add<T>, dim3(rc_blocks(op.nc, k)), dim3(kBlock), 0, s, op.nc, k,
                  kp_log2(k), op.rci.p, ec, x);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_restrict(const SolveOp &op, const T *rw, const T *r, T *fc, int k, hipStream_t s,
                  T *zero_xc) {
    launch_csr_both<T, OP_SPMV>(0, op.nc, nullptr, op.n_rlong ? kLongRow : 0, 0, op.n_rlong,
                                op.rlong.p, op.rrp.p, op.rci.p, rw, nullptr, nullptr, r, fc, k,
                                op.lpr_r, s, zero_xc, nullptr);
}

template <class T>
void run_prolong(const SolveOp &op, const T *w0, const T *w1, const T *ec, const double *mu, T *x,
                 int k, hipStream_t s) {
    launch_kernel(k_prolong<T>, dim3(rc_blocks(op.n, k)), dim3(kBlock), 0, s, op.n, k, kp_log2(k),
                  op.p0.p, op.p1.p, w0, w1, ec, mu, x);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_fill(T *x, int64_t count, T value, hipStream_t s) {
    if (count <= 0) return;
    launch_kernel(k_fill<T>, dim3(blocks_for(count)), dim3(kBlock), 0, s, x, count, value);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_copy(T *dst, const T *src, int64_t count, hipStream_t s) {
    if (count <= 0) return;
    launch_kernel(k_copy<T>, dim3(blocks_for(count)), dim3(kBlock), 0, s, dst, src, count);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_mu(int64_t n, const T *e, const T *f, const T *rho, int k, double *partial, double *mu,
            hipStream_t s) {
    RedIn in{e, f, rho, nullptr, 0, 0};
    reduce<T, R_MU>(n, k, in, partial, Fin{mu, nullptr, 1.0, 0}, s);
}

template <class T>
void run_rc2(int64_t n, T *e, T *rho, const T *e1, const T *rho1, int k, double *partial,
             double *alpha, hipStream_t s) {
    RedIn in{rho, rho1, nullptr, nullptr, 0, 0};
    reduce<T, R_RC2>(n, k, in, partial, Fin{alpha, nullptr, 1.0, 0}, s);
    launch_kernel(k_rc2_update<T>, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), e, rho, const_cast<T *>(e1),
                                                       const_cast<T *>(rho1), alpha, 0);
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_mu_prolong(const SolveOp &op, const T *w0, const T *w1, int64_t nc, const T *ec,
                    const T *fc, const T *rho, int k, double *partial, double *scal, T *x,
                    hipStream_t s) {
    const int nblk = red_blocks(nc, k);
    RedIn in{ec, fc, rho, nullptr, 0, 0};
    launch_kernel(k_red_partial<T, R_MU>, dim3(nblk), dim3(kBlock), 0, s, nc, k, kp_log2(k), in, partial);
    LAMG_LAUNCH_CHECK();
    if (fuse_totals(op.n, k, nblk)) {
        launch_kernel(k_prolong_mu<T>, dim3(rc_blocks(op.n, k)), dim3(kBlock), 0, s, op.n, k,
                      kp_log2(k), op.p0.p, op.p1.p, w0, w1, ec, nblk, (const double *)partial, x);
    } else {
        launch_kernel(k_red_final<R_MU>, dim3(1), dim3(kBlock), 0, s, nblk, k, partial, Fin{scal, nullptr, 1.0, 0});
        launch_kernel(k_prolong<T>, dim3(rc_blocks(op.n, k)), dim3(kBlock), 0, s, op.n, k,
                      kp_log2(k), op.p0.p, op.p1.p, w0, w1, ec, (const double *)scal, x);
    }
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_rc2_keep(int64_t n, T *e, T *rho, T *e1, T *rho1, int k, double *partial,
                  double *scal, bool keep, hipStream_t s) {
    const int nblk = red_blocks(n, k);
    RedIn in{rho, rho1, nullptr, nullptr, 0, 0};
    launch_kernel(k_red_partial<T, R_RC2>, dim3(nblk), dim3(kBlock), 0, s, n, k, kp_log2(k), in, partial);
    LAMG_LAUNCH_CHECK();
    if (fuse_totals(n, k, nblk)) {
        launch_kernel(k_rc2_fused<T>, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), e, rho, e1, rho1, nblk,
                                                          partial, keep ? 1 : 0);
    } else {
        launch_kernel(k_red_final<R_RC2>, dim3(1), dim3(kBlock), 0, s, nblk, k, partial, Fin{scal, nullptr, 1.0, 0});
        launch_kernel(k_rc2_update<T>, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), e, rho, e1, rho1, scal,
                                                           keep ? 1 : 0);
    }
    LAMG_LAUNCH_CHECK();
}

template <class T>
void run_coarsest(int64_t n, const double *Z, const T *f, T *y, int k, hipStream_t s) {
    if (n > 1024) throw Error(LAMG_INVALID_ARG, "coarsest level larger than 1024");
    launch_kernel(k_coarsest<T>, dim3((unsigned)((n * k + 3) / 4)), dim3(kBlock), 0, s, n, Z, f, y, k);
    LAMG_LAUNCH_CHECK();
}

void run_gather_cols(int64_t n, int k, const int32_t *perm, const double *src, double *dst,
                     hipStream_t s) {
    launch_kernel(k_gather_cols, dim3(blocks_for(n * k)), dim3(kBlock), 0, s, n, k, perm, src, dst);
    LAMG_LAUNCH_CHECK();
}

void run_scatter_cols(int64_t n, int k, const int32_t *perm, const double *src, const int32_t *mask,
                      double *dst, hipStream_t s) {
    launch_kernel(k_scatter_cols, dim3(blocks_for(n * k)), dim3(kBlock), 0, s, n, k, perm, src, mask, dst);
    LAMG_LAUNCH_CHECK();
}

void run_colsum(int64_t n, int k, const double *x, double *partial, double *out, double scale,
                hipStream_t s) {
    RedIn in{x, nullptr, nullptr, nullptr, 0, 0};
    reduce<double, R_SUM>(n, k, in, partial, Fin{out, nullptr, scale, 0}, s);
}

void run_sub_col(int64_t n, int k, double *x, const double *m, hipStream_t s) {
    launch_kernel(k_sub_col, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), x, m);
    LAMG_LAUNCH_CHECK();
}

void run_norm2(int64_t n, int k, const double *x, double *partial, double *out, hipStream_t s) {
    RedIn in{x, nullptr, nullptr, nullptr, 0, 0};
    reduce<double, R_NORM2>(n, k, in, partial, Fin{out, nullptr, 1.0, 0}, s);
}

void run_count_nonfinite(int64_t n, const double *x, double *partial, double *out, hipStream_t s) {
    RedIn in{x, nullptr, nullptr, nullptr, 0, 0};
    reduce<double, R_NONFIN>(n, 1, in, partial, Fin{out, nullptr, 1.0, 0}, s);
}

void run_maxabs(int64_t n, int k, const double *x, double *partial, double *out, hipStream_t s) {
    RedIn in{x, nullptr, nullptr, nullptr, 0, 0};
    reduce<double, R_MAXABS>(n, k, in, partial, Fin{out, nullptr, 1.0, 0}, s);
}

void run_relres(int64_t n, int k, const double *r, const double *nb, double *partial, double *out,
                hipStream_t s) {
    RedIn in{r, nullptr, nullptr, nullptr, 0, 0};
    reduce<double, R_NORM2>(n, k, in, partial, Fin{out, nb, 1.0, 0}, s);
}

void run_relres_maxabs(int64_t n, int k, const double *r, const double *nb, double *partial,
                       double *rel, double *maxabs, hipStream_t s) {
    RedIn in{r, nullptr, nullptr, nullptr, 0, 0};
    Fin fin{rel, nb, 1.0, 0};
    fin.out2 = maxabs;
    reduce<double, R_RES2>(n, k, in, partial, fin, s);
}

void run_recombine_fine(int64_t n, int k, int m, double *phi, double *r, double *hphi, double *hr,
                        int slot, double *partial, double *alpha, hipStream_t s) {
    if (m <= 0) {  // nothing to recombine with: only save the pair
        run_copy<double>(hphi + (int64_t)slot * n * k, phi, n * k, s);
        run_copy<double>(hr + (int64_t)slot * n * k, r, n * k, s);
        return;
    }
    RedIn in{r, hr, nullptr, nullptr, m, n * k};
    reduce<double, R_RCF>(n, k, in, partial, Fin{alpha, nullptr, 1.0, m}, s);
    launch_kernel(k_rcf_update, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), m, phi, r, hphi, hr, n * k,
                                                     alpha, slot);
    LAMG_LAUNCH_CHECK();
}

void run_to_f32_scaled(int64_t n, int k, const double *r, const double *scale, float *dst,
                       float *zero_x, hipStream_t s) {
    launch_kernel(k_to_f32_scaled, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), r, scale, dst, zero_x);
    LAMG_LAUNCH_CHECK();
}

void run_add_scaled_f32(int64_t n, int k, const float *e, const double *scale, double *phi,
                        hipStream_t s) {
    launch_kernel(k_add_scaled_f32, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), e, scale, phi);
    LAMG_LAUNCH_CHECK();
}

void run_zero_cols(int64_t n, int k, const int32_t *zero_mask, double *x, hipStream_t s) {
    launch_kernel(k_zero_cols, dim3(rc_blocks(n, k)), dim3(kBlock), 0, s, n, k, kp_log2(k), zero_mask, x);
    LAMG_LAUNCH_CHECK();
}

#define LAMG_INST(T)                                                                              \
    template void run_gs<T>(const SolveOp &, const T *, const T *, const T *, T *, int, int,      \
                            hipStream_t, bool);                                                   \
    template void run_residual<T>(const SolveOp &, const T *, const T *, const T *, const T *,    \
                                  T *, int, hipStream_t, bool, T *, T *);                         \
    template void run_gs_color<T>(const SolveOp &, int, const T *, const T *, const T *, T *,     \
                                  int, hipStream_t, bool);                                        \
    template void run_restrict<T>(const SolveOp &, const T *, const T *, T *, int, hipStream_t,   \
                                  T *);                                                           \
    template void run_residual_color<T>(const SolveOp &, int, const T *, const T *, const T *,    \
                                        const T *, T *, int, hipStream_t, bool);                  \
    template void run_inject_add<T>(const SolveOp &, const T *, T *, int, hipStream_t);           \
    template void run_cheb_sweep<T>(const SolveOp &, double, const T *, const T *, const T *,     \
                                    const T *, T *, T *, int, hipStream_t, bool);                 \
    template void run_bjgs_sweep<T>(const SolveOp &, const T *, const T *, const T *, const T *,  \
                                    T *, T *, int, hipStream_t, bool);                            \
    template void run_mu_prolong<T>(const SolveOp &, const T *, const T *, int64_t, const T *,    \
                                    const T *, const T *, int, double *, double *, T *,           \
                                    hipStream_t);                                                 \
    template void run_rc2_keep<T>(int64_t, T *, T *, T *, T *, int, double *, double *, bool,     \
                                  hipStream_t);                                                   \
    template void run_prolong<T>(const SolveOp &, const T *, const T *, const T *,                \
                                 const double *, T *, int, hipStream_t);                          \
    template void run_fill<T>(T *, int64_t, T, hipStream_t);                                      \
    template void run_copy<T>(T *, const T *, int64_t, hipStream_t);                              \
    template void run_mu<T>(int64_t, const T *, const T *, const T *, int, double *, double *,    \
                            hipStream_t);                                                         \
    template void run_rc2<T>(int64_t, T *, T *, const T *, const T *, int, double *, double *,    \
                             hipStream_t);                                                        \
    template void run_coarsest<T>(int64_t, const double *, const T *, T *, int, hipStream_t);

LAMG_INST(double)
LAMG_INST(float)

}  // namespace lamg
