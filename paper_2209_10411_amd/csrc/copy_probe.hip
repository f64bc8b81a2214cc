// Streaming-copy probe: the practical HBM ceiling of the stream-collide's
// access shape, measured on the same device and stream as the library's
// kernels.  The 19 populations of n nodes in the library's layout (runs of
// 1024 nodes, each run holding its populations one after another) are read
// and written (non-temporal stores), one node per lane, 512-thread blocks in
// node order, as the stream-collide does for a node, minus the neighbour
// shifts and the arithmetic.  Nothing of the method runs here.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/midelbm.h"

namespace {

constexpr int RUN_LOG2 = 10;  // the population layout's run of nodes

template <class T>
__global__ __launch_bounds__(512) void k_copy_soa(const T *__restrict__ src, T *__restrict__ dst, long long n) {
    const long long i = blockIdx.x * 512ll + threadIdx.x;
    if (i >= n) return;
    const long long base = (i >> RUN_LOG2) * (19ll << RUN_LOG2) + (i & ((1 << RUN_LOG2) - 1));
    T v[19];
#pragma unroll
    for (int a = 0; a < 19; ++a) v[a] = src[base + ((long long)a << RUN_LOG2)];
#pragma unroll
    for (int a = 0; a < 19; ++a) __builtin_nontemporal_store(v[a], dst + base + ((long long)a << RUN_LOG2));
}

}  // namespace

extern "C" lbm_status lbm_copy_probe(const void *dev_src, void *dev_dst, int64_t n, int64_t stride,
                                     int32_t elem_bytes, int32_t reps, void *hip_stream, double *ms) {
    if (!dev_src || !dev_dst || !ms || n <= 0 || stride < n || stride % (1 << RUN_LOG2) != 0 || reps < 1 ||
        (elem_bytes != 2 && elem_bytes != 4))
        return LBM_E_INVALID;
    hipStream_t s = (hipStream_t)hip_stream;
    const unsigned grid = (unsigned)((n + 511) / 512);
    auto launch = [&](const void *a, void *b) {
        if (elem_bytes == 4) k_copy_soa<float><<<grid, 512, 0, s>>>((const float *)a, (float *)b, n);
        else k_copy_soa<uint16_t><<<grid, 512, 0, s>>>((const uint16_t *)a, (uint16_t *)b, n);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return LBM_E_HIP;
    lbm_status st = LBM_OK;
    launch(dev_src, dev_dst);  // warm-up
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps; ++r) launch(dev_src, dev_dst);
    (void)hipEventRecord(e1, s);
    float t = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess ||
        hipGetLastError() != hipSuccess)
        st = LBM_E_HIP;
    *ms = (double)t / reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
