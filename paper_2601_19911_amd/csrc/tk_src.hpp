// Device-side views of a query's data shared by the single-query kernels.
#pragma once

#include "tk_device.hpp"

namespace tk {

// Composites (key image, flipped row-id) of a query, by index.
template <int KT, int RT>
struct InputSrc {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  const typename Key<KT>::Raw* keys;
  const R* rids;
  U dmask;
  __device__ __forceinline__ U key(uint64_t i) const { return Key<KT>::enc(keys[i]) ^ dmask; }
  __device__ __forceinline__ R flip(uint64_t i) const { return ~(rids ? rids[i] : (R)i); }
};

template <typename U, typename R>
struct BufSrc {
  const U* k;
  const R* f;
  __device__ __forceinline__ U key(uint64_t i) const { return k[i]; }
  __device__ __forceinline__ R flip(uint64_t i) const { return f[i]; }
};

template <int KT, int RT>
struct alignas(16) LdsTile {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  static constexpr uint32_t CAP = (sizeof(U) + sizeof(R)) <= 8 ? 16384u : 8192u;
  U k[CAP];
  R f[CAP];
};

template <int KT, int RT>
__device__ __forceinline__ void write_out(uint64_t j, typename Key<KT>::U kk,
                                          typename Rid<RT>::R ff, typename Key<KT>::U dmask,
                                          void* out_keys, void* out_rids) {
  if (out_keys) static_cast<typename Key<KT>::Raw*>(out_keys)[j] = Key<KT>::dec(kk ^ dmask);
  if (out_rids) static_cast<typename Rid<RT>::R*>(out_rids)[j] = ~ff;
}

}  // namespace tk
