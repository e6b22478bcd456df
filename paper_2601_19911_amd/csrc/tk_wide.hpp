// The selection composite (key image above flipped row-id) read as one wide
// unsigned integer, and logarithmic buckets of a distance between two
// composites.  Used by the tails over the survivors (tk_rank.hpp,
// tk_bucket.hpp).
#pragma once

#include "tk_device.hpp"

namespace tk {

template <typename U, typename R>
struct Wide {
  using T = __uint128_t;
  static constexpr int W = 8 * (int)(sizeof(U) + sizeof(R));
};
template <>
struct Wide<uint32_t, uint32_t> {
  using T = uint64_t;
  static constexpr int W = 64;
};

template <typename U, typename R>
__device__ __forceinline__ typename Wide<U, R>::T wide(U u, R f) {
  using T = typename Wide<U, R>::T;
  return ((T)u << (8 * sizeof(R))) | (T)f;
}

__device__ __forceinline__ int wbitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }
__device__ __forceinline__ int wbitlen(__uint128_t x) {
  const uint64_t hi = (uint64_t)(x >> 64);
  return hi ? 64 + wbitlen(hi) : wbitlen((uint64_t)x);
}

// Logarithmic bucket with 2^SUB buckets per octave (the SUB bits under the
// leading one), D itself below 2^(SUB+1).  Non-decreasing in D; a W-bit D
// gives 2^SUB (W - SUB + 1) buckets.
template <int SUB, typename T>
__device__ __forceinline__ uint32_t log_bucket_s(T d) {
  const int L = wbitlen(d);
  if (L <= SUB + 1) return (uint32_t)d;
  return (2u << SUB) + (uint32_t)(L - SUB - 2) * (1u << SUB) +
         ((uint32_t)(d >> (L - SUB - 1)) & ((1u << SUB) - 1u));
}

// The G bits of d right under the ones log_bucket_s<SUB> keeps (zero-padded
// when fewer remain; 0 for the exact buckets): with the bucket, a finer key
// that is still non-decreasing in d.
template <int SUB, typename T>
__device__ __forceinline__ uint32_t log_subdigit(T d, int G) {
  const int L = wbitlen(d);
  if (L <= SUB + 1) return 0u;
  const int rem = L - SUB - 1;  // bits under the bucket's
  const uint32_t mask = (1u << G) - 1u;
  if (rem >= G) return (uint32_t)(d >> (rem - G)) & mask;
  return ((uint32_t)d << (G - rem)) & mask;
}

// Buckets of the large-K tail: 256 per octave for 8-byte composites, else 128.
template <typename U_, typename R_>
struct BTU {
  using U = U_;
  using R = R_;
  using T = typename Wide<U, R>::T;
  static constexpr int W = Wide<U, R>::W;
  static constexpr int SUB = W == 64 ? 8 : 7;
  static constexpr uint32_t NB = (1u << SUB) * (uint32_t)(W - SUB + 1);
  static __device__ __forceinline__ uint32_t bucket(U u, R f, T base) {
    return log_bucket_s<SUB, T>(wide(u, f) - base);
  }
  static __device__ __forceinline__ uint32_t subdigit(U u, R f, T base, int G) {
    return log_subdigit<SUB, T>(wide(u, f) - base, G);
  }
};
template <int KT, int RT>
using BT = BTU<typename Key<KT>::U, typename Rid<RT>::R>;

}  // namespace tk
