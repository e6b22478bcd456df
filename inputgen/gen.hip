// Seeded synthetic inputs for key-only Top-K: host (multi-threaded C++) and
// device (HIP) versions of the recipes in inputgen/__init__.py.  No Top-K
// arithmetic lives here; this library only fills buffers.
//
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), output i of stream `seed`:
//   z = seed + (i+1)*0x9E3779B97F4A7C15; z = (z^(z>>30))*0xBF58476D1CE4E5B9;
//   z = (z^(z>>27))*0x94D049BB133111EB; h = z^(z>>31).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <thread>
#include <vector>

namespace {

enum Kind {
  U_I32 = 0, U_I64 = 1, U_F32 = 2, ZIPF_I64 = 3, ZIPF_F32 = 4, SORTED_F32 = 5,
  SORTED_I64 = 6, IOTA_U32 = 7, IOTA_U64 = 8, PAYLOAD_F64 = 9, ZIPF_I32 = 10,
  JOIN_FK_I32 = 11, JOIN_FK_I64 = 12
};

__host__ __device__ inline uint64_t splitmix(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// rank = 1 + #{r : cdf[r] <= u}: the first index whose entry exceeds u
__host__ __device__ inline int64_t zipf_rank(const double* cdf, uint64_t m, double u) {
  uint64_t lo = 0, hi = m;  // answer in [lo, hi]
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (cdf[mid] <= u) lo = mid + 1; else hi = mid;
  }
  return (int64_t)lo + 1;
}

__host__ __device__ inline void gen_one(int kind, uint64_t seed, uint64_t i, uint64_t n_total,
                                        const double* cdf, uint64_t m, void* dst, uint64_t j) {
  switch (kind) {
    case U_I32: ((int32_t*)dst)[j] = (int32_t)(splitmix(seed, i) >> 33); break;
    case U_I64: ((int64_t*)dst)[j] = (int64_t)splitmix(seed, i); break;
    case U_F32: ((float*)dst)[j] = (float)(splitmix(seed, i) >> 40) * 0x1p-24f; break;
    case PAYLOAD_F64: ((double*)dst)[j] = (double)(splitmix(seed, i) >> 11) * 0x1p-53; break;
    case ZIPF_I64: case ZIPF_F32: case ZIPF_I32: {
      double u = (double)(splitmix(seed, i) >> 11) * 0x1p-53;
      int64_t r = zipf_rank(cdf, m, u);
      if (kind == ZIPF_I64) ((int64_t*)dst)[j] = r;
      else if (kind == ZIPF_I32) ((int32_t*)dst)[j] = (int32_t)r;
      else ((float*)dst)[j] = (float)r;
      break;
    }
    case SORTED_F32: ((float*)dst)[j] = (float)((i << 24) / n_total) * 0x1p-24f; break;
    case SORTED_I64: ((int64_t*)dst)[j] = (int64_t)((i << 24) / n_total) - (int64_t(1) << 23); break;
    case IOTA_U32: ((uint32_t*)dst)[j] = (uint32_t)i; break;
    case IOTA_U64: ((uint64_t*)dst)[j] = i; break;
    // a foreign key: the build recipe (uniform int32 / int64, same seed) at an
    // index drawn from the stream of seed + 1, modulo n_total
    case JOIN_FK_I32: ((int32_t*)dst)[j] = (int32_t)(splitmix(seed, splitmix(seed + 1, i) % n_total) >> 33); break;
    case JOIN_FK_I64: ((int64_t*)dst)[j] = (int64_t)splitmix(seed, splitmix(seed + 1, i) % n_total); break;
  }
}

__global__ void gen_kernel(int kind, uint64_t seed, uint64_t start, uint64_t n, uint64_t n_total,
                           const double* cdf, uint64_t m, void* dst) {
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride)
    gen_one(kind, seed, start + j, n_total, cdf, m, dst, j);
}

bool kind_ok(int kind) { return kind >= 0 && kind <= 12; }
bool needs_cdf(int kind) { return kind == ZIPF_I64 || kind == ZIPF_F32 || kind == ZIPF_I32; }

}  // namespace

extern "C" {

// Fills dst[0..n) on the host with elements start..start+n-1 of `kind`.
// Returns 0, or -1 on a bad argument.
int tkgen_host(int kind, uint64_t seed, uint64_t start, uint64_t n, uint64_t n_total,
               const double* cdf, uint64_t m, void* dst, int nthreads) {
  if (!kind_ok(kind) || (n && !dst) || (needs_cdf(kind) && (!cdf || !m))) return -1;
  if (nthreads < 1) nthreads = 1;
  if (n < (1u << 16)) nthreads = 1;
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) {
    uint64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
    th.emplace_back([=] {
      for (uint64_t j = lo; j < hi; ++j) gen_one(kind, seed, start + j, n_total, cdf, m, dst, j);
    });
  }
  for (auto& x : th) x.join();
  return 0;
}

// Same recipes on the device, enqueued on `stream`.  `cdf` is a device copy of
// the Zipf table (or null for the other kinds).  Returns 0, -1 on a bad
// argument, or the HIP error code.
int tkgen_device(int kind, uint64_t seed, uint64_t start, uint64_t n, uint64_t n_total,
                 const double* cdf, uint64_t m, void* dst, hipStream_t stream) {
  if (!kind_ok(kind) || (n && !dst) || (needs_cdf(kind) && (!cdf || !m))) return -1;
  if (n == 0) return 0;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(gen_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, kind, seed, start,
                     n, n_total, cdf, m, dst);
  return (int)hipGetLastError();
}

}  // extern "C"
