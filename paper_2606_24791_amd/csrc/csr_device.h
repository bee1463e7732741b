// Device helpers of the per-step cycle kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lamg {

// sum_{j in [j0, e), step `stride`} v[j] * x[ci[j] * k + col], with U entries in flight:
// the U index/value loads are issued together, then the U gathers, so a short row costs
// two memory latencies instead of two per entry.
//  - FP32: every load is unconditional (a slot past the row's end re-reads the group's
//    first entry, which exists when the loop runs) and such slots are dropped when the
//    terms are added in entry order. No load then sits behind a branch of its own, so the
//    compiler keeps all U gathers in flight at once (with a branch per slot it waited for
//    the first gather before issuing the others).
//  - FP64: slots past the end load nothing (index -1, value 0, term 0). The unconditional
//    form costs more than it saves here: on the Chung-Lu graph with 4 columns a plain FP64
//    solve took 1028 ms with it against 854 ms without, on the 128^3 grid with 32 columns
//    419 against 406 ms (the FP32 cycles of the same solves: 633 and 311 ms either way).
//  - Rows spread over many lanes (the long-row blocks) load predicated in both precisions:
//    there most lanes hold one or two entries, and unconditional slots would issue U loads
//    for each (Chung-Lu with one column: 463 against 386 ms).
template <class T, int U, bool UNCOND = (sizeof(T) == 4)>
__device__ inline T row_dot(const int32_t *__restrict__ ci, const T *__restrict__ v, const T *x,
                            int32_t j0, int32_t e, int32_t stride, int k, int col) {
    T acc = T(0);
    for (int32_t j = j0; j < e; j += U * stride) {
        int32_t cc[U];
        T vv[U], xx[U];
        if constexpr (UNCOND) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t jj = j + u * stride;
                const int32_t js = jj < e ? jj : j;
                cc[u] = ci[js];
                vv[u] = v[js];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xx[u] = x[(int64_t)cc[u] * k + col];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const T term = vv[u] * xx[u];
                acc = (j + u * stride < e) ? acc + term : acc;
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t jj = j + u * stride;
                const bool ok = jj < e;
                cc[u] = ok ? ci[jj] : -1;
                vv[u] = ok ? v[jj] : T(0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xx[u] = cc[u] >= 0 ? x[(int64_t)cc[u] * k + col] : T(0);
#pragma unroll
            for (int u = 0; u < U; ++u) acc += vv[u] * xx[u];
        }
    }
    return acc;
}

}  // namespace lamg
