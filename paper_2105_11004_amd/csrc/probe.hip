// A plain streaming read of device memory: the measured ceiling the passes
// over A are compared with (each pass reads A once with 16-byte loads).
//
// 256 workgroups of 1024 threads (one per CU, four waves per SIMD), each
// lane with four independent 16-byte loads in flight per loop trip over a
// grid-stride walk; every loaded word enters a per-thread checksum that is
// stored, so no load can be dropped.  (Swept on gfx950 over 256..4096
// workgroups of 256..1024 threads and 4..16 loads per lane: this shape read
// fastest.)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lev.h"
#include "lev_internal.h"

namespace lev {
namespace {

constexpr int kProbeThreads = 1024;
constexpr int kProbeGroups = 256;
constexpr int kProbeU = 4;

__global__ __launch_bounds__(kProbeThreads) void stream_read_kernel(const uint4* __restrict__ p, int64_t nvec,
                                                                     uint32_t* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
  for (int64_t i = tid; i < nvec; i += stride * kProbeU) {
    uint4 v[kProbeU];
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) {
      const int64_t j = i + u * stride;
      v[u] = j < nvec ? p[j] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) acc ^= v[u].x + v[u].y + v[u].z + v[u].w;
  }
  sink[tid] = acc;
}

}  // namespace

static_assert(kProbeGroups * kProbeThreads == LEV_STREAM_READ_SINK, "sink length");

int64_t stream_read_sink_len() { return (int64_t)kProbeGroups * kProbeThreads; }

hipError_t launch_stream_read(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t s) {
  stream_read_kernel<<<kProbeGroups, kProbeThreads, 0, s>>>(static_cast<const uint4*>(buf), bytes / 16, sink);
  return hipGetLastError();
}

}  // namespace lev
