// Late materialization (paper sec. II-C): fetch payload rows at the row-ids a
// Top-K query returned.  The key-only path runs the host variant after the
// row-ids come back; the device variant serves the full-row comparison,
// where every payload column already sits in HBM.
#include <hip/hip_runtime.h>

#include "mitopk.h"

namespace {

// one thread per (column, output row); columns are rows of a [ncols][n] array
template <typename R>
__global__ __launch_bounds__(256) void k_gather_f64(const double* __restrict__ cols, uint32_t ncols,
                                                    uint64_t n, const R* __restrict__ rids,
                                                    uint64_t k, double* __restrict__ out,
                                                    unsigned int* __restrict__ bad) {
  const uint64_t total = (uint64_t)ncols * k;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t c = t / k, j = t - c * k;
    const uint64_t r = (uint64_t)rids[j];
    if (r < n) {
      out[t] = cols[c * n + r];
    } else {
      out[t] = 0.0;
      if (bad) atomicOr(bad, 1u);
    }
  }
}

}  // namespace

extern "C" int tk_gather_f64_device(const double* cols, uint32_t ncols, uint64_t n,
                                    const void* rowids, int rid_type, uint64_t k, double* out,
                                    void* stream) {
  if (rid_type != TK_RID_U32 && rid_type != TK_RID_U64) return TK_EINVAL;
  if (k == 0 || ncols == 0) return TK_OK;
  if (!cols || !rowids || !out) return TK_EINVAL;
  const uint64_t total = (uint64_t)ncols * k;
  uint64_t blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipStream_t st = (hipStream_t)stream;
  if (rid_type == TK_RID_U32)
    hipLaunchKernelGGL(k_gather_f64<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, st, cols,
                       ncols, n, static_cast<const uint32_t*>(rowids), k, out, nullptr);
  else
    hipLaunchKernelGGL(k_gather_f64<uint64_t>, dim3((unsigned)blocks), dim3(256), 0, st, cols,
                       ncols, n, static_cast<const uint64_t*>(rowids), k, out, nullptr);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}
