// Device helpers shared by the cycle kernels and the coarse-tail kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lamg {

// sum_{j in [j0, e), step `stride`} v[j] * x[ci[j] * k + col], with U entries in flight:
// the U index/value loads are issued together, then the U gathers, so a short row costs
// two memory latencies instead of two per entry.
template <class T, int U>
__device__ inline T row_dot(const int32_t *__restrict__ ci, const T *__restrict__ v, const T *x,
                            int32_t j0, int32_t e, int32_t stride, int k, int col) {
    T acc = T(0);
    for (int32_t j = j0; j < e; j += U * stride) {
        int32_t cc[U];
        T vv[U], xx[U];
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
    return acc;
}

}  // namespace lamg
