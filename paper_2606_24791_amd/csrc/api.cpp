// C ABI of liblamg (declared in include/lamg.h): argument checks, handle lifecycle,
// device-memory pool, hierarchy description and level export. Exceptions raised inside
// the library stop here and become status codes.
#include <algorithm>
#include <mutex>
#include <new>

#include "lamg_internal.h"

namespace lamg {
void run_setup(lamg_handle *h, const lamg_graph *g);
lamg_status run_solve(lamg_handle *h, const double *b, int nrhs, double tol, int max_cycles,
                      lamg_precision prec, double *phi, lamg_solve_info *info);
lamg_status run_profile(lamg_handle *h, int level, int kernel, lamg_precision prec, int k,
                        int reps, double *sec, double *bytes);
lamg_status run_solve_group(int count, lamg_handle *const *hs, const double *const *bs,
                            const int32_t *nrhs, double tol, int max_cycles, lamg_precision prec,
                            double *const *phis, lamg_solve_info *infos, lamg_status *statuses,
                            hipStream_t stream);
int plan_tail_level(const lamg_handle *h);
int plan_timed_level(const lamg_handle *h);

static std::mutex g_alloc_mu;
static Allocator g_alloc;

Allocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void *Pool::get(size_t bytes) {
    void *p = nullptr;
    if (base_) {
        const size_t off = ((size_t)bytes_ + 255) & ~(size_t)255;
        if (off > cap_ || bytes > cap_ - off)
            throw Error(LAMG_SCRATCH_TOO_SMALL,
                        "the solve needs more than the " + std::to_string(cap_) +
                            " bytes of the allocation-free scratch");
        bytes_ = (int64_t)(off + bytes);
        peak_ = std::max(peak_, bytes_);
        return base_ + off;
    }
    if (a_.alloc) {
        p = a_.alloc(bytes, (void *)s_, a_.ctx);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
        }
    }
    if (!p) throw Error(LAMG_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    blks_.push_back({p, bytes});
    bytes_ += (int64_t)bytes;
    peak_ = std::max(peak_, bytes_);
    return p;
}

void Pool::put(void *p) {
    if (base_) return;
    for (size_t i = blks_.size(); i-- > 0;) {
        if (blks_[i].p == p) {
            bytes_ -= (int64_t)blks_[i].bytes;
            blks_[i] = blks_.back();
            blks_.pop_back();
            if (a_.free)
                a_.free(p, (void *)s_, a_.ctx);
            else
                (void)hipFree(p);
            return;
        }
    }
}

Pool::~Pool() {
    if (base_) return;
    for (auto &b : blks_) {
        if (a_.free)
            a_.free(b.p, (void *)s_, a_.ctx);
        else
            (void)hipFree(b.p);
    }
}

template <class F>
static lamg_status guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        return e.status;
    } catch (const std::bad_alloc &) {
        return LAMG_OOM;
    } catch (...) {
        return LAMG_HIP_ERROR;
    }
}

}  // namespace lamg

lamg_handle::~lamg_handle() {
    timer.release();
    lamg::clear_graphs(ws);
    if (ws.cap_stream) (void)hipStreamDestroy(ws.cap_stream);
    ws.cap_stream = nullptr;
    // pinned host mirrors; device arrays are released by their owners before the pool
    if (ws.h_rel) (void)hipHostFree(ws.h_rel);
    if (ws.h_mask) (void)hipHostFree(ws.h_mask);
    ws.h_rel = nullptr;
    ws.h_mask = nullptr;
}

using namespace lamg;

extern "C" {

void lamg_set_allocator(lamg_alloc_fn alloc_fn, lamg_free_fn free_fn, void *ctx) {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    if (alloc_fn && free_fn) {
        g_alloc.alloc = alloc_fn;
        g_alloc.free = free_fn;
        g_alloc.ctx = ctx;
    } else {
        g_alloc = Allocator();
    }
}

const char *lamg_status_string(lamg_status s) {
    switch (s) {
        case LAMG_OK: return "ok";
        case LAMG_INVALID_ARG: return "invalid argument";
        case LAMG_NOT_SYMMETRIC: return "adjacency not symmetric";
        case LAMG_SELF_LOOP: return "self loop in adjacency";
        case LAMG_BAD_WEIGHT: return "non-positive or non-finite weight";
        case LAMG_DISCONNECTED: return "graph not connected";
        case LAMG_OOM: return "out of memory";
        case LAMG_COARSENING_STALLED: return "coarsening stalled";
        case LAMG_NOT_CONVERGED: return "not converged";
        case LAMG_HIP_ERROR: return "HIP runtime error";
        case LAMG_UNAVAILABLE: return "data not kept";
        case LAMG_SCRATCH_TOO_SMALL:
            return "solve larger than the fixed scratch of the allocation-free entry point";
    }
    return "unknown status";
}

const char *lamg_version(void) { return "lamg-mi355x 0.1 (gfx950)"; }

void lamg_default_options(lamg_options *opt) {
    if (!opt) return;
    opt->seed = 1;
    opt->n_direct = 512;
    opt->enable_veto = 1;
    opt->enable_caliber2 = 1;
    opt->kappa = 4;
    opt->build_fp32 = 1;
    opt->keep_setup_data = 0;
    opt->tail_rows = 2500;
    opt->elimination = 1;
    opt->smoother = 0;
    opt->graphs = 0;
    opt->tail_finest = 0;
    opt->reorder = 0;
}

lamg_status lamg_setup(const lamg_graph *g, const lamg_options *opt, void *stream,
                       lamg_handle **out) {
    if (!out) return LAMG_INVALID_ARG;
    *out = nullptr;
    if (!g) return LAMG_INVALID_ARG;
    lamg_options o;
    lamg_default_options(&o);
    if (opt) o = *opt;
    if (o.n_direct < 1 || o.n_direct > 1024 || o.kappa < 0 || o.kappa > 4 || o.tail_rows < 0 ||
        (o.elimination != 0 && o.elimination != 1) || (o.smoother < 0 || o.smoother > 2) || (o.reorder != 0 && o.reorder != 1) ||
        (o.graphs != 0 && o.graphs != 1) || o.tail_finest < 0 || o.tail_finest > 65535)
        return LAMG_INVALID_ARG;
    lamg_handle *h = nullptr;
    lamg_status st = guarded([&]() -> lamg_status {
        h = new lamg_handle();
        h->alloc = current_allocator();
        h->stream = (hipStream_t)stream;
        h->pool.reset(new Pool(h->alloc, h->stream));
        h->opt = o;
        run_setup(h, g);  // input errors surface before any device work
        LAMG_HIP(hipGetDevice(&h->device));
        // the allocation-free entry point's scratch on this device, resolved once per device
        (void)noalloc_scratch(h->device);
        return LAMG_OK;
    });
    if (st != LAMG_OK) {
        if (h) {
            // input errors are found on the host before any device work; only a failure
            // after device work began needs the stream drained before memory is returned
            if (h->pool && h->pool->bytes() > 0) (void)hipStreamSynchronize((hipStream_t)stream);
            delete h;
        }
        return st;
    }
    *out = h;
    return LAMG_OK;
}

lamg_status lamg_solve(lamg_handle *h, const double *b, int32_t nrhs, double tol,
                       int32_t max_cycles, lamg_precision prec, double *phi,
                       lamg_solve_info *info, void *stream) {
    if (!h || !b || !phi || nrhs < 1 || !(tol >= 0.0) || (prec != LAMG_FP64 && prec != LAMG_FP32_IR))
        return LAMG_INVALID_ARG;
    return guarded([&]() -> lamg_status {
        h->stream = (hipStream_t)stream;
        h->pool->set_stream(h->stream);
        return run_solve(h, b, nrhs, tol, max_cycles, prec, phi, info);
    });
}

lamg_status lamg_solve_group(int32_t count, lamg_handle *const *handles,
                             const double *const *b, const int32_t *nrhs, double tol,
                             int32_t max_cycles, lamg_precision prec, double *const *phi,
                             lamg_solve_info *infos, lamg_status *statuses, void *stream) {
    if (count < 1 || !handles || !b || !nrhs || !phi || !statuses || !(tol >= 0.0) ||
        (prec != LAMG_FP64 && prec != LAMG_FP32_IR))
        return LAMG_INVALID_ARG;
    for (int32_t r = 0; r < count; ++r) {
        if (!handles[r] || !b[r] || !phi[r] || nrhs[r] < 1) return LAMG_INVALID_ARG;
        for (int32_t q = 0; q < r; ++q)
            if (handles[q] == handles[r]) return LAMG_INVALID_ARG;  // one workspace each
    }
    return guarded([&]() -> lamg_status {
        return run_solve_group(count, handles, b, nrhs, tol, max_cycles, prec, phi, infos,
                               statuses, (hipStream_t)stream);
    });
}

lamg_status lamg_profile_kernel(lamg_handle *h, int32_t level, lamg_kernel kernel,
                                lamg_precision prec, int32_t nrhs, int32_t reps,
                                double *seconds_per_launch, double *bytes_per_launch,
                                void *stream) {
    if (!h || !seconds_per_launch || !bytes_per_launch) return LAMG_INVALID_ARG;
    return guarded([&]() -> lamg_status {
        h->stream = (hipStream_t)stream;
        h->pool->set_stream(h->stream);
        return run_profile(h, level, (int)kernel, prec, nrhs, reps, seconds_per_launch,
                           bytes_per_launch);
    });
}

lamg_status lamg_timing_start(lamg_handle *h, int32_t max_launches) {
    if (!h || max_launches < 1) return LAMG_INVALID_ARG;
    return guarded([&]() -> lamg_status {
        h->timer.start(max_launches, false);
        return LAMG_OK;
    });
}

lamg_status lamg_timing_start_all(lamg_handle *h, int32_t max_launches) {
    if (!h || max_launches < 1) return LAMG_INVALID_ARG;
    return guarded([&]() -> lamg_status {
        h->timer.start(max_launches, true);
        return LAMG_OK;
    });
}

lamg_status lamg_timing_stop(lamg_handle *h) {
    if (!h) return LAMG_INVALID_ARG;
    return guarded([&]() -> lamg_status {
        h->timer.stop();
        return LAMG_OK;
    });
}

lamg_status lamg_timing_get(const lamg_handle *h, lamg_kernel kernel, lamg_precision prec,
                            lamg_kernel_time *out) {
    if (!h || !out || (int)kernel < 0 || (int)kernel >= KTimer::kKinds || h->timer.on ||
        (prec != LAMG_FP64 && prec != LAMG_FP32_IR))
        return LAMG_INVALID_ARG;
    const int p = prec == LAMG_FP32_IR ? 1 : 0;
    out->launches = h->timer.cnt[kernel][p];
    out->seconds = h->timer.sec[kernel][p];
    out->bytes = h->timer.bytes[kernel][p];
    return LAMG_OK;
}

void lamg_destroy(lamg_handle *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    delete h;
}

lamg_status lamg_hierarchy_info(const lamg_handle *h, lamg_hier_info *info) {
    if (!h || !info) return LAMG_INVALID_ARG;
    std::memset(info, 0, sizeof(*info));
    info->levels = h->nlev;
    info->reordered = h->reordered ? 1 : 0;
    double nnz0 = (double)h->lev[0].nnz, tot = 0.0;
    for (int l = 0; l < h->nlev && l < LAMG_MAX_LEVELS; ++l) {
        const Level &L = h->lev[l];
        info->n[l] = L.n;
        info->nnz[l] = L.nnz;
        info->ncolors[l] = (L.coarsest || L.elim) ? 0 : L.ncolors;
        info->elim[l] = L.elim ? 1 : 0;
        info->cheb[l] = L.cheb ? 1 : 0;
        info->cheb_lmax[l] = L.cheb ? L.cheb_lmax : 0.0;
        info->bjgs[l] = L.bjgs ? 1 : 0;
        info->n_caliber2[l] = L.coarsest ? 0 : L.n_cal2;
        info->gamma[l] = L.coarsest ? 0.0 : L.gamma;
        info->tau[l] = L.coarsest ? 0.0 : L.tau;
        tot += (double)L.nnz;
    }
    info->bytes_device = h->pool->bytes();
    info->op_complexity = tot / nnz0;
    info->setup_seconds = h->setup_seconds;
    for (int i = 0; i < LAMG_SETUP_PHASES; ++i) info->setup_phase_seconds[i] = h->setup_phase[i];
    info->bytes_peak = h->pool->peak();
    info->tail_level = plan_tail_level(h);
    info->timed_level = plan_timed_level(h);
    return LAMG_OK;
}

lamg_status lamg_export_level(const lamg_handle *h, int32_t level, lamg_level_export *out) {
    if (!h || !out || level < 0 || level >= h->nlev) return LAMG_INVALID_ARG;
    if (!h->opt.keep_setup_data) return LAMG_UNAVAILABLE;
    return guarded([&]() -> lamg_status {
        const Level &L = h->lev[level];
        hipStream_t s = h->stream;
        const int64_t n = L.n, nnz = L.nnz;
        if (out->row_ptr) L.rp.download(out->row_ptr, n + 1, s);
        if (out->col_idx) L.ci.download(out->col_idx, nnz, s);
        if (out->val) L.val.download(out->val, nnz, s);
        if (L.elim) {
            if (out->aggregate) std::memcpy(out->aggregate, L.h_agg.data(), 4 * n);
        } else if (!L.coarsest) {
            if (out->color) std::memcpy(out->color, L.h_color.data(), 4 * n);
            if (out->strong) L.strong.download(out->strong, nnz, s);
            if (out->x) L.X.download(out->x, n * kTV, s);
            if (out->affinity) L.aff.download(out->affinity, nnz, s);
            if (out->moments) L.mom.download(out->moments, n * 9, s);
            if (out->seed) std::memcpy(out->seed, L.h_seed.data(), 4 * n);
            if (out->aggregate) std::memcpy(out->aggregate, L.h_agg.data(), 4 * n);
            if (out->p0) L.p0.download(out->p0, n, s);
            if (out->p1) L.p1.download(out->p1, n, s);
            if (out->w0) L.w0.download(out->w0, n, s);
            if (out->w1) L.w1.download(out->w1, n, s);
        }
        LAMG_HIP(hipStreamSynchronize(s));
        return LAMG_OK;
    });
}

}  // extern "C"
