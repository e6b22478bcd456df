// Device building blocks for key-only Top-K on gfx950 (wave64).
//
// Selection works on an order-preserving unsigned image of every key (the
// "radix-based selection" of the ordering primitive, paper sec. III-A):
//   int32   u = x ^ 0x80000000
//   int64   u = x ^ 2^63
//   float32 u = bits ^ (sign ? 0xFFFFFFFF : 0x80000000)   (IEEE totalOrder)
// Ascending queries use ~u, so every query becomes "largest u first".  Ties are
// broken by ascending row-id, so the full selection key is the composite
// (u, f) with f = ~rowid, compared lexicographically, larger = better.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tk {

constexpr int KEY_I32 = 0, KEY_I64 = 1, KEY_F32 = 2, KEY_F64 = 3;
// bytes of a key of each type
__host__ __device__ constexpr uint32_t key_bytes(int kt) { return kt == KEY_I64 || kt == KEY_F64 ? 8u : 4u; }
constexpr int RID_U32 = 0, RID_U64 = 1;

template <int KT> struct Key;
template <> struct Key<KEY_I32> {
  using Raw = uint32_t;
  using U = uint32_t;
  static __host__ __device__ __forceinline__ U enc(Raw x) { return x ^ 0x80000000u; }
  static __host__ __device__ __forceinline__ Raw dec(U u) { return u ^ 0x80000000u; }
};
template <> struct Key<KEY_F32> {
  using Raw = uint32_t;
  using U = uint32_t;
  static __host__ __device__ __forceinline__ U enc(Raw x) {
    return x ^ ((uint32_t)((int32_t)x >> 31) | 0x80000000u);
  }
  static __host__ __device__ __forceinline__ Raw dec(U u) {
    return u ^ (((u >> 31) - 1u) | 0x80000000u);
  }
};
template <> struct Key<KEY_I64> {
  using Raw = uint64_t;
  using U = uint64_t;
  static __host__ __device__ __forceinline__ U enc(Raw x) { return x ^ 0x8000000000000000ull; }
  static __host__ __device__ __forceinline__ Raw dec(U u) { return u ^ 0x8000000000000000ull; }
};
// float64: as float32, on 64-bit patterns (negative: all bits flipped;
// non-negative: sign bit set), so that unsigned order is totalOrder
template <> struct Key<KEY_F64> {
  using Raw = uint64_t;
  using U = uint64_t;
  static __host__ __device__ __forceinline__ U enc(Raw x) {
    return x ^ ((uint64_t)((int64_t)x >> 63) | 0x8000000000000000ull);
  }
  static __host__ __device__ __forceinline__ Raw dec(U u) {
    return u ^ (((u >> 63) - 1ull) | 0x8000000000000000ull);
  }
};

template <int RT> struct Rid;
template <> struct Rid<RID_U32> { using R = uint32_t; };
template <> struct Rid<RID_U64> { using R = uint64_t; };

// composite comparisons: (ka, fa) >= / > (kb, fb)
template <typename U, typename R>
__device__ __forceinline__ bool cge(U ka, R fa, U kb, R fb) {
  return ka > kb || (ka == kb && fa >= fb);
}
template <typename U, typename R>
__device__ __forceinline__ bool cgt(U ka, R fa, U kb, R fb) {
  return ka > kb || (ka == kb && fa > fb);
}

// ---- wave64 primitives ------------------------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// A DPP lane move within the wave (a few cycles, where a shuffle goes
// through the LDS crossbar): lanes of the rows in ROWS take v from the lane
// CTRL names; other lanes, and lanes whose source is outside their row, take
// `old`.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_move(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xF, false);
}

// Inclusive prefix sum over the wave: shifts right by 1, 2, 4 and 8 inside
// each row of 16 lanes, then the last lane of row 0 into row 1 and of row 2
// into row 3 (row_bcast:15), and the last lane of row 1 into rows 2 and 3
// (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += dpp_move<0x111, 0xF>(0u, x);  // row_shr:1
  x += dpp_move<0x112, 0xF>(0u, x);  // row_shr:2
  x += dpp_move<0x114, 0xF>(0u, x);  // row_shr:4
  x += dpp_move<0x118, 0xF>(0u, x);  // row_shr:8
  x += dpp_move<0x142, 0xA>(0u, x);  // row_bcast:15
  x += dpp_move<0x143, 0xC>(0u, x);  // row_bcast:31
  return x;
}

// Sum of v over the lanes at and above this one.
__device__ __forceinline__ uint32_t wave_suffix_sum(uint32_t v) {
  const uint32_t incl = wave_incl_scan(v);
  const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
  return total - incl + v;
}

// ---- block primitives (NT threads, NT a multiple of 64) -----------------------------------

// Sum over the block.  `red` is LDS of 2 * NT/64 words; `parity` alternates so
// that back-to-back calls need one barrier each.
template <int NT>
__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t* red, int& parity) {
  constexpr int NW = NT / 64;
  v = wave_sum64(v);
  uint64_t* slot = red + parity * NW;
  parity ^= 1;
  if (lane_id() == 0) slot[threadIdx.x >> 6] = v;
  __syncthreads();
  uint64_t s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += slot[i];
  return s;
}

// Exclusive prefix sum over the block; `ws` is LDS of NT/64 words.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* ws, uint32_t& total) {
  constexpr int NW = NT / 64;
  const uint32_t x = wave_incl_scan(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) ws[w] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t t = ws[i];
    off += (i < w) ? t : 0u;
    tot += t;
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// Block bisection select.  Each thread holds E composites (k[e], f[e]) of
// which the first `nv` are valid.  Finds the largest T = (Tk, Tf) with
// #{valid c >= T} >= target, two bits per round from the most significant
// bit of k down to the last bit of f, and stops as soon as that count equals
// `target` (then T may have trailing zero bits, and exactly `target` elements
// are >= T).  Returns the count of elements >= T.  Needs target <= #valid and
// #valid < 2^21.
template <typename U, typename R, int E, int NT>
__device__ uint32_t block_select(const U (&k)[E], const R (&f)[E], int nv, uint32_t target,
                                 U& Tk, R& Tf, uint64_t* red, int& parity) {
  Tk = 0;
  Tf = 0;
  uint32_t cnt = (uint32_t)block_sum64<NT>((uint64_t)nv, red, parity);
  if (cnt <= target) return cnt;
  constexpr int WU = (int)sizeof(U) * 8, WR = (int)sizeof(R) * 8;
  for (int s = WU - 2; s >= 0; s -= 2) {
    const U c1 = Tk | ((U)1 << s), c2 = Tk | ((U)2 << s), c3 = Tk | ((U)3 << s);
    uint64_t p = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e < nv) {
        p += (uint64_t)(k[e] >= c1) + ((uint64_t)(k[e] >= c2) << 21) + ((uint64_t)(k[e] >= c3) << 42);
      }
    }
    p = block_sum64<NT>(p, red, parity);
    const uint32_t n1 = (uint32_t)(p & 0x1FFFFFu), n2 = (uint32_t)((p >> 21) & 0x1FFFFFu),
                   n3 = (uint32_t)(p >> 42);
    if (n3 >= target) { Tk = c3; cnt = n3; }
    else if (n2 >= target) { Tk = c2; cnt = n2; }
    else if (n1 >= target) { Tk = c1; cnt = n1; }
    if (cnt == target) return cnt;
  }
  for (int s = WR - 2; s >= 0; s -= 2) {
    const R c1 = Tf | ((R)1 << s), c2 = Tf | ((R)2 << s), c3 = Tf | ((R)3 << s);
    uint64_t p = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (e < nv) {
        const bool gt = k[e] > Tk, eq = k[e] == Tk;
        p += (uint64_t)(gt | (eq & (f[e] >= c1))) + ((uint64_t)(gt | (eq & (f[e] >= c2))) << 21) +
             ((uint64_t)(gt | (eq & (f[e] >= c3))) << 42);
      }
    }
    p = block_sum64<NT>(p, red, parity);
    const uint32_t n1 = (uint32_t)(p & 0x1FFFFFu), n2 = (uint32_t)((p >> 21) & 0x1FFFFFu),
                   n3 = (uint32_t)(p >> 42);
    if (n3 >= target) { Tf = c3; cnt = n3; }
    else if (n2 >= target) { Tf = c2; cnt = n2; }
    else if (n1 >= target) { Tf = c1; cnt = n1; }
    if (cnt == target) return cnt;
  }
  return cnt;
}

// Writes the best `target` of the block's composites (T, cnt from
// block_select) to dk/df[0..target): every element > T, then copies of T to
// fill.  Positions follow a block prefix sum, so the output is unsorted.
template <typename U, typename R, int E, int NT, typename KPtr, typename FPtr>
__device__ void block_emit_top(const U (&k)[E], const R (&f)[E], int nv, uint32_t target, U Tk,
                               R Tf, KPtr dk, FPtr df, uint32_t* ws) {
  uint32_t ngt = 0, neq = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < nv) {
      ngt += cgt(k[e], f[e], Tk, Tf);
      neq += (k[e] == Tk && f[e] == Tf);
    }
  }
  uint32_t tgt, teq;
  uint32_t pgt = block_excl_scan<NT>(ngt, ws, tgt);
  uint32_t peq = block_excl_scan<NT>(neq, ws, teq);
  (void)teq;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (e < nv) {
      if (cgt(k[e], f[e], Tk, Tf)) {
        dk[pgt] = k[e];
        df[pgt] = f[e];
        ++pgt;
      } else if (k[e] == Tk && f[e] == Tf) {
        const uint32_t pos = tgt + peq;
        if (pos < target) {
          dk[pos] = k[e];
          df[pos] = f[e];
        }
        ++peq;
      }
    }
  }
}

// In-place bitonic sort of P (a power of two) composites in LDS, best first.
template <typename U, typename R, int NT>
__device__ void bitonic_desc(U* sk, R* sf, uint32_t P) {
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (uint32_t t = threadIdx.x; t < (P >> 1); t += NT) {
        const uint32_t i = 2 * t - (t & (stride - 1));
        const uint32_t j = i + stride;
        const bool desc = (i & size) == 0;
        const U ki = sk[i], kj = sk[j];
        const R fi = sf[i], fj = sf[j];
        if (cgt(kj, fj, ki, fi) == desc) {
          sk[i] = kj;
          sk[j] = ki;
          sf[i] = fj;
          sf[j] = fi;
        }
      }
    }
  }
  __syncthreads();
}

// ---- grid barrier for co-resident (cooperative) grids ---------------------------------------
//
// Sense counter + generation word.  Every thread fences at agent scope before
// arriving and after leaving, so writes made before the barrier by any block
// are visible to every block after it, across the XCDs' separate L2s.  The wait
// is bounded: after `spin_limit` sleeps the barrier reports failure (the
// caller then exits and flags an error) instead of hanging.
struct GridSync {
  uint32_t count;
  uint32_t gen;
};

__device__ __forceinline__ bool grid_sync(GridSync* gs, uint32_t nblocks, uint32_t* err_flag,
                                          int* s_flag, uint64_t spin_limit = (1ull << 25)) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint32_t g = __hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived =
        __hip_atomic_fetch_add(&gs->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&gs->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&gs->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint64_t spins = 0;
      while (__hip_atomic_load(&gs->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins > spin_limit) {
          ok = 0;
          __hip_atomic_store(err_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    *s_flag = ok;
  }
  __syncthreads();
  const bool ok = *s_flag != 0;
  __threadfence();
  __syncthreads();
  return ok;
}

}  // namespace tk
