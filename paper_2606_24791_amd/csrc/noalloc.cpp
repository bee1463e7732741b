// The allocation-free solve entry point (lamg_solve_noalloc, include/lamg.h) and the fixed
// device scratch array its workspace lives in.
//
// The array is a file-scope device variable of this translation unit. In host code its name
// is only a host-side stand-in: kernels must never receive it. Its real address is looked
// up once per device (hipGetSymbolAddress, with that device current) and every later use
// -- the arena that lays out the solve's workspace, and with it every kernel argument and
// copy -- goes through that address.
#include <mutex>

#include "lamg_internal.h"

namespace lamg {

namespace {

constexpr size_t kScratchBytes = LAMG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

}  // namespace

void *noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices)
        throw Error(LAMG_INVALID_ARG, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        int cur = -1;
        LAMG_HIP(hipGetDevice(&cur));
        if (cur != device) throw Error(LAMG_INVALID_ARG, "scratch resolved off its device");
        void *p = nullptr;
        LAMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(LAMG_HIP_ERROR, "no device address for the scratch array");
        g_scratch[device] = p;
    }
    return g_scratch[device];
}

size_t noalloc_scratch_bytes() { return kScratchBytes; }

lamg_status run_solve(lamg_handle *h, const double *b, int nrhs, double tol, int max_cycles,
                      lamg_precision prec, double *phi, lamg_solve_info *info);

namespace {

// The handle's cached workspace is set aside for the call and a fresh one, laid out in the
// scratch arena, takes its place; the destructor puts the handle's own back.
struct ArenaSwap {
    lamg_handle *h;
    Workspace &aside;
    ArenaSwap(lamg_handle *hh, Workspace &w) : h(hh), aside(w) { std::swap(aside, h->ws); }
    ~ArenaSwap() { std::swap(aside, h->ws); }
};

}  // namespace

}  // namespace lamg

extern "C" lamg_status lamg_solve_noalloc(lamg_handle *h, const double *b, int32_t nrhs,
                                          double tol, int32_t max_cycles, lamg_precision prec,
                                          double *phi, lamg_solve_info *info, void *stream) {
    using namespace lamg;
    if (!h || !b || !phi || nrhs < 1 || !(tol >= 0.0) || (prec != LAMG_FP64 && prec != LAMG_FP32_IR))
        return LAMG_INVALID_ARG;
    try {
        int cur = -1;
        LAMG_HIP(hipGetDevice(&cur));
        if (cur != h->device) return LAMG_INVALID_ARG;
        void *base = noalloc_scratch(h->device);
        hipStream_t s = (hipStream_t)stream;
        h->stream = s;
        h->pool->set_stream(s);
        // declared in this order: the arena outlives the workspace laid out in it, and the
        // swap back happens before that workspace's arrays are released (into the arena,
        // which frees nothing)
        Pool arena(base, kScratchBytes, s);
        Workspace ws;
        ws.arena = &arena;
        ArenaSwap swap(h, ws);
        return run_solve(h, b, nrhs, tol, max_cycles, prec, phi, info);
    } catch (const Error &e) {
        return e.status;
    } catch (const std::bad_alloc &) {
        return LAMG_OOM;
    } catch (...) {
        return LAMG_HIP_ERROR;
    }
}
