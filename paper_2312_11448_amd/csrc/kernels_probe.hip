// Read-bandwidth probe: the measurement utility behind the cache-level roofs
// the benchmark quotes (not part of the transport). One launch reads a
// buffer `passes` times over: each thread walks the same float4 positions in
// every pass (grid stride), so a buffer that fits a cache level is served
// from it after the first pass, and one launch's overhead is spread over all
// passes.
#include "common.hpp"

namespace mclya {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

__global__ __launch_bounds__(kProbeBlock) void probe_read_kernel(const float4 *__restrict__ p, uint64_t n4,
                                                                 int passes, float *__restrict__ sink)
{
    const uint64_t stride = (uint64_t)gridDim.x * kProbeBlock;
    const uint64_t t0 = (uint64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    float acc = 0.0f;
    for (int k = 0; k < passes; ++k) {
        uint64_t i = t0;
        // four independent loads in flight per thread
        for (; i + (kProbeUnroll - 1) * stride < n4; i += kProbeUnroll * stride) {
            float4 v[kProbeUnroll];
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) v[u] = p[i + u * stride];
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
        }
        for (; i < n4; i += stride) {
            const float4 v = p[i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    }
    // written only if the sum takes an impossible value for the buffers the
    // caller passes (finite data): the reads cannot be dropped, the writes
    // never happen
    if (acc != acc) sink[0] = acc;
}

}  // namespace

hipError_t launch_probe_read(const void *buf, uint64_t bytes, int passes, int grid, float *sink, hipStream_t s)
{
    hipLaunchKernelGGL(probe_read_kernel, dim3((unsigned)grid), dim3(kProbeBlock), 0, s,
                       static_cast<const float4 *>(buf), bytes / 16, passes, sink);
    return hipGetLastError();
}

}  // namespace mclya
