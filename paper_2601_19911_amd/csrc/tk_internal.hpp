// Declarations shared between the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "tk_device.hpp"
#include "tk_plan.hpp"

namespace tk {

// Start of every single-query workspace.  All counters are reset by the first
// kernel of each query, so the workspace needs no initialization by the caller.
// Per-query state of the sampled path: 64 bytes, so a batch can clear all of
// its queries' states with one small copy.
struct QHead {
  unsigned long long surv_count;  // keys that passed the sampled threshold
  unsigned long long thr_k;       // sampled threshold (key image)
  unsigned long long thr_f;       // sampled threshold (flipped row-id)
  uint32_t status;                // device failure bits (1: barrier timeout)
  uint32_t path;                  // path taken, see tk_info
  uint32_t tie_heavy;             // 1: most sample candidates share the threshold's key
  uint32_t pad[7];
};
static_assert(sizeof(QHead) == 64, "QHead is 64 bytes");

// A single query's workspace header.
struct Header {
  QHead q;
  unsigned long long sel_gt;      // exact select: writes of composites above the boundary
  unsigned long long sel_eq;      // exact select: writes of copies of the boundary
  GridSync gs;                    // grid barrier of the exact-select kernel
  uint32_t pad[2];
  unsigned long long hist[3][256];  // exact select: global digit histograms
};
static_assert(sizeof(Header) <= HEADER_BYTES, "header must fit its reserved bytes");

inline int device_cus(int dev) {
  static std::mutex mu;
  static std::vector<int> cache;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
      v = 1;
    cache[dev] = v;
  }
  return cache[dev];
}

Tuning current_tuning();
void profile_mark(hipStream_t st, bool begin);

template <int KT, int RT>
int run_sampled(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int order,
                void* out_keys, void* out_rids, void* ws, size_t ws_bytes, hipStream_t st,
                const Tuning& tun, const SamplePlan& p);

// Inputs below this size that the sample cannot serve are selected by one
// workgroup (path 8) instead of the cooperative grid.
constexpr uint64_t ONE_WG_INPUT_MAX = 1ull << 16;

// One workgroup's exact select + sort over the whole input (k_tail1 over the
// input), with the workspace regions of layout L for K beyond one LDS tile.
template <int KT, int RT>
int run_input_one_wg(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int order,
                     void* out_keys, void* out_rids, void* ws, hipStream_t st, const WsLayout& L);

// The Top-K of a query by its full sort (tk_sort.hip): the first k_eff pairs
// of the order go to the outputs; scratch holds sort_scratch_bytes(n, ...)
// bytes; h (or null) receives path 9.
int topk_by_sort(const void* keys, const void* rowids, uint64_t n, uint64_t k_eff, int key_type,
                 int rid_type, int order, void* out_keys, void* out_rowids, void* scratch,
                 QHead* h, hipStream_t st);

template <int KT, int RT>
int run_single(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int order,
               void* out_keys, void* out_rids, void* ws, size_t ws_bytes, hipStream_t st,
               const Tuning& tun);

}  // namespace tk
