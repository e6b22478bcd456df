// The read ceiling the streaming pass is measured against: one pass over a
// device buffer with 16-byte nontemporal loads, one compare per 4-byte word
// and a single atomic per workgroup at the end (no other writes), on the same
// launch shape as the filter (workgroups of 256 threads striding over tiles of
// four loads per thread).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mitopk.h"
#include "tk_internal.hpp"

namespace tk {
namespace {

typedef uint32_t u32x4p __attribute__((ext_vector_type(4)));
constexpr int PROBE_NT = 256, PROBE_UNR = 4;

__global__ __launch_bounds__(PROBE_NT) void k_read_probe(const u32x4p* __restrict__ p, uint64_t n16,
                                                        uint32_t thr, uint32_t* sink) {
  uint32_t cnt = 0;
  constexpr uint64_t TILE = (uint64_t)PROBE_NT * PROBE_UNR;
  const uint64_t ntiles = n16 / TILE;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t b = t * TILE + threadIdx.x;
    u32x4p v[PROBE_UNR];
#pragma unroll
    for (int u = 0; u < PROBE_UNR; ++u) v[u] = __builtin_nontemporal_load(p + b + (uint64_t)u * PROBE_NT);
#pragma unroll
    for (int u = 0; u < PROBE_UNR; ++u)
      cnt += (v[u].x > thr) + (v[u].y > thr) + (v[u].z > thr) + (v[u].w > thr);
  }
  if (cnt) atomicAdd(sink, cnt);
}

}  // namespace
}  // namespace tk

extern "C" int tk_read_probe(const void* buf, uint64_t bytes, uint32_t wg_per_cu, void* sink,
                             void* stream) {
  if (!buf || !sink || wg_per_cu == 0 || wg_per_cu > 32 || ((uintptr_t)buf & 15u)) return TK_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TK_EHIP;
  const uint64_t n16 = bytes / 16;
  const int grid = (int)wg_per_cu * tk::device_cus(dev);
  hipLaunchKernelGGL(tk::k_read_probe, dim3(grid), dim3(tk::PROBE_NT), 0, (hipStream_t)stream,
                     static_cast<const tk::u32x4p*>(buf), n16, 0xFFFFFFFFu, static_cast<uint32_t*>(sink));
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}
