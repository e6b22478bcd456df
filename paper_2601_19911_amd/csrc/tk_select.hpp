// One-workgroup radix select and sort building blocks of the engine.
//
// block_radix_select finds the boundary of the best `target` composites
// among the elements a visitor presents (registers of the workgroup, or an
// array in global memory).  Digits are 8 bits of d = u - base, starting at
// the most significant set bit of max(d): the range of the candidates, not of
// the key type, sets the first digit, so keys that share their high bits
// (floats in [0, 1), survivors above a threshold) still split in the first
// round.  Each round builds an LDS histogram of the digit over the
// candidates that match the prefix so far and picks the bucket holding rank
// `need` with a wave-wide suffix scan.  When the key image is exhausted and
// the boundary bucket still holds more elements than needed, the flipped
// row-id is digitized the same way.
#pragma once

#include "tk_device.hpp"

namespace tk {

enum SelKind { SEL_KEY = 0, SEL_RID = 1, SEL_DUP = 2 };

template <typename U, typename R>
struct Sel {
  U base;      // every candidate has u >= base
  U P;         // resolved digits of d = u - base
  R Pf;        // resolved digits of the flipped row-id (SEL_RID / SEL_DUP)
  int kind;    // SelKind
  uint64_t need;  // SEL_DUP: copies of the exact boundary composite to take
};

// u in the selection iff its composite is at or above the boundary
template <typename U, typename R>
__device__ __forceinline__ bool sel_take(const Sel<U, R>& s, U u, R f) {
  if (u < s.base) return false;
  const U d = u - s.base;
  if (s.kind == SEL_KEY) return d >= s.P;
  if (s.kind == SEL_RID) return d > s.P || (d == s.P && f >= s.Pf);
  return d > s.P || (d == s.P && f > s.Pf);
}
template <typename U, typename R>
__device__ __forceinline__ bool sel_is_boundary_copy(const Sel<U, R>& s, U u, R f) {
  return s.kind == SEL_DUP && u >= s.base && u - s.base == s.P && f == s.Pf;
}
// whether u might be selected (so f has to be read)
template <typename U, typename R>
__device__ __forceinline__ bool sel_maybe(const Sel<U, R>& s, U u) {
  return u >= s.base && u - s.base >= s.P;
}

struct SelScratch {
  uint32_t hist[256];
  unsigned long long red[16];
  unsigned long long red2[16];
  uint32_t res[4];
  uint32_t cnt[2];
};

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T w = __shfl_xor(v, o, 64);
    v = w > v ? w : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const T w = __shfl_xor(v, o, 64);
    v = w < v ? w : v;
  }
  return v;
}

template <int NT, typename T>
__device__ __forceinline__ T block_max(T v, SelScratch& sc) {
  v = wave_max(v);
  __syncthreads();
  if (lane_id() == 0) sc.red[threadIdx.x >> 6] = (unsigned long long)v;
  __syncthreads();
  T m = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const T w = (T)sc.red[i];
    m = w > m ? w : m;
  }
  return m;
}
template <int NT, typename T>
__device__ __forceinline__ T block_min(T v, SelScratch& sc) {
  v = wave_min(v);
  __syncthreads();
  if (lane_id() == 0) sc.red[threadIdx.x >> 6] = (unsigned long long)v;
  __syncthreads();
  T m = (T)~(T)0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const T w = (T)sc.red[i];
    m = w < m ? w : m;
  }
  return m;
}

// Smallest composite (k, f) over the block, lexicographic; threads with
// nothing to offer pass (~0, ~0).  NT <= 1024.
template <int NT, typename U, typename R>
__device__ __forceinline__ void block_min_comp(U& k, R& f, SelScratch& sc) {
  const U wk = wave_min(k);
  R wf = wave_min(k == wk ? f : (R)~(R)0);
  __syncthreads();
  if (lane_id() == 0) {
    sc.red[threadIdx.x >> 6] = (unsigned long long)wk;
    sc.red2[threadIdx.x >> 6] = (unsigned long long)wf;
  }
  __syncthreads();
  U mk = (U)~(U)0;
  R mf = (R)~(R)0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const U ck = (U)sc.red[i];
    const R cf = (R)sc.red2[i];
    if (ck < mk || (ck == mk && cf < mf)) {
      mk = ck;
      mf = cf;
    }
  }
  k = mk;
  f = mf;
}

// After the histogram is complete: finds digit b with (sum of bins above b) <
// need <= (that sum + hist[b]).  Wave 0 scans; everyone reads the result.
template <int NT>
__device__ __forceinline__ void find_bucket(SelScratch& sc, uint64_t need, uint32_t& digit,
                                            uint64_t& above, uint64_t& cnt) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t L = threadIdx.x;
    const uint32_t h0 = sc.hist[4 * L], h1 = sc.hist[4 * L + 1], h2 = sc.hist[4 * L + 2],
                   h3 = sc.hist[4 * L + 3];
    const uint64_t s = (uint64_t)h0 + h1 + h2 + h3;
    uint64_t x = s;  // sum over lanes L..63
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint64_t y = __shfl_down(x, o, 64);
      if (L + o < 64) x += y;
    }
    const uint64_t excl = x - s;
    if (excl < need && need <= x) {
      uint64_t c = excl;
      uint32_t d = 4 * L;
      uint32_t hb = h0;
      if (c + h3 >= need) { d = 4 * L + 3; hb = h3; }
      else if ((c += h3) + h2 >= need) { d = 4 * L + 2; hb = h2; }
      else if ((c += h2) + h1 >= need) { d = 4 * L + 1; hb = h1; }
      else { c += h1; d = 4 * L; hb = h0; }
      sc.res[0] = d;
      sc.res[1] = (uint32_t)c;
      sc.res[2] = (uint32_t)(c >> 32);
      sc.res[3] = hb;
    }
  }
  __syncthreads();
  digit = sc.res[0];
  above = (uint64_t)sc.res[1] | ((uint64_t)sc.res[2] << 32);
  cnt = sc.res[3];
}

template <int NT>
__device__ __forceinline__ void hist_clear(SelScratch& sc) {
  for (uint32_t i = threadIdx.x; i < 256; i += NT) sc.hist[i] = 0;
  __syncthreads();
}

// Visitors present each thread's share of the candidates.
// Registers: E composites per thread, the first nv valid.
template <typename U, typename R, int E>
struct RegElems {
  U (&k)[E];
  R (&f)[E];
  int nv;
  template <typename Fn>
  __device__ __forceinline__ void each(Fn&& fn) const {
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e < nv) fn(k[e], [&]() { return f[e]; });
  }
};

// A global array seen through a source (key image and flipped row-id by
// index).  Keys are read four at a time so that each thread has several loads
// in flight.
template <int NT, typename Src>
struct GlobElems {
  const Src& src;
  uint64_t n;
  template <typename Fn>
  __device__ __forceinline__ void each(Fn&& fn) const {
    using U = decltype(src.key(0));
    uint64_t i = threadIdx.x;
    for (; i + 3 * NT < n; i += 4 * NT) {
      const U k0 = src.key(i), k1 = src.key(i + NT), k2 = src.key(i + 2 * NT),
              k3 = src.key(i + 3 * NT);
      const uint64_t i0 = i;
      fn(k0, [&]() { return src.flip(i0); });
      fn(k1, [&]() { return src.flip(i0 + NT); });
      fn(k2, [&]() { return src.flip(i0 + 2 * NT); });
      fn(k3, [&]() { return src.flip(i0 + 3 * NT); });
    }
    for (; i < n; i += NT) fn(src.key(i), [&]() { return src.flip(i); });
  }
};

template <typename U>
__device__ __forceinline__ int bitlen(U x) {
  if (x == 0) return 0;
  if constexpr (sizeof(U) == 8) return 64 - __builtin_clzll((unsigned long long)x);
  else return 32 - __builtin_clz((unsigned)x);
}

// Boundary of the best `target` candidates (every candidate has u >= base and
// there are at least `target` of them).
template <int NT, typename U, typename R, typename Elems>
__device__ __forceinline__ Sel<U, R> block_radix_select(const Elems& el, uint64_t target, U base, SelScratch& sc) {
  Sel<U, R> s;
  s.base = base;
  s.P = 0;
  s.Pf = 0;
  s.kind = SEL_KEY;
  U lmax = 0;
  el.each([&](U u, auto) {
    if (u >= base && u - base > lmax) lmax = u - base;
  });
  const U dmax = block_max<NT, U>(lmax, sc);
  const int hb = bitlen(dmax);
  uint64_t need = target;
  U M = 0;
  for (int sh = hb - 8;; sh -= 8) {
    const int s0 = sh < 0 ? 0 : sh;
    hist_clear<NT>(sc);
    el.each([&](U u, auto) {
      if (u >= base) {
        const U d = u - base;
        if ((d & M) == s.P) atomicAdd(&sc.hist[(uint32_t)(d >> s0) & 0xFFu], 1u);
      }
    });
    uint32_t dig;
    uint64_t above, cnt;
    find_bucket<NT>(sc, need, dig, above, cnt);
    need -= above;
    s.P |= (U)dig << s0;
    M |= (U)0xFF << s0;
    if (cnt == need) {
      s.need = need;
      return s;
    }
    if (s0 == 0) break;
  }
  // the key image is resolved; order the boundary key's copies by row-id
  s.kind = SEL_RID;
  R Mf = 0;
  constexpr int WR = (int)sizeof(R) * 8;
  for (int s0 = WR - 8; s0 >= 0; s0 -= 8) {
    hist_clear<NT>(sc);
    el.each([&](U u, auto getf) {
      if (u >= base && u - base == s.P) {
        const R f = getf();
        if ((f & Mf) == s.Pf) atomicAdd(&sc.hist[(uint32_t)(f >> s0) & 0xFFu], 1u);
      }
    });
    uint32_t dig;
    uint64_t above, cnt;
    find_bucket<NT>(sc, need, dig, above, cnt);
    need -= above;
    s.Pf |= (R)dig << s0;
    Mf |= (R)0xFF << s0;
    if (cnt == need) {
      s.need = need;
      return s;
    }
  }
  s.kind = SEL_DUP;
  s.need = need;
  return s;
}

// Writes the selected composites to (dk, df): the ones above the boundary in
// any order at [0, target - need) and, for SEL_DUP, `need` boundary copies
// after them.  Every thread must call these (their loops are
// workgroup-uniform).
template <int NT, typename U, typename R, int E, typename KOut, typename FOut>
__device__ __forceinline__ void block_compact_regs(const RegElems<U, R, E>& el, const Sel<U, R>& s,
                                   uint64_t target, KOut dk, FOut df, SelScratch& sc) {
  if (threadIdx.x == 0) { sc.cnt[0] = 0; sc.cnt[1] = 0; }
  __syncthreads();
  const uint64_t n_gt = s.kind == SEL_DUP ? target - s.need : target;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const bool valid = e < el.nv;
    const U u = valid ? el.k[e] : (U)0;
    const R f = valid ? el.f[e] : (R)0;
    const bool take = valid && sel_take(s, u, f);
    const bool eq = valid && sel_is_boundary_copy(s, u, f);
    const uint64_t mt = ballot(take), me = ballot(eq);
    if (mt) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(mt);
      uint32_t b = 0;
      if (lane_id() == leader) b = atomicAdd(&sc.cnt[0], (uint32_t)__popcll(mt));
      b = __shfl(b, (int)leader, 64);
      if (take) {
        const uint64_t pos = b + lanes_below(mt);
        if (pos < n_gt) { dk[pos] = u; df[pos] = f; }
      }
    }
    if (me) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(me);
      uint32_t b = 0;
      if (lane_id() == leader) b = atomicAdd(&sc.cnt[1], (uint32_t)__popcll(me));
      b = __shfl(b, (int)leader, 64);
      if (eq) {
        const uint64_t pos = n_gt + b + lanes_below(me);
        if (pos < target) { dk[pos] = u; df[pos] = f; }
      }
    }
  }
  __syncthreads();
}

template <int NT, typename U, typename R, typename Src, typename KOut, typename FOut>
__device__ __forceinline__ void block_compact_glob(const Src& src, uint64_t n, const Sel<U, R>& s, uint64_t target,
                                   KOut dk, FOut df, SelScratch& sc) {
  if (threadIdx.x == 0) { sc.cnt[0] = 0; sc.cnt[1] = 0; }
  __syncthreads();
  const uint64_t n_gt = s.kind == SEL_DUP ? target - s.need : target;
  for (uint64_t i0 = 0; i0 < n; i0 += NT) {
    const uint64_t i = i0 + threadIdx.x;
    bool take = false, eq = false;
    U u = 0;
    R f = 0;
    if (i < n) {
      u = src.key(i);
      if (sel_maybe(s, u)) {
        f = src.flip(i);
        take = sel_take(s, u, f);
        eq = sel_is_boundary_copy(s, u, f);
      }
    }
    const uint64_t mt = ballot(take), me = ballot(eq);
    if (mt) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(mt);
      uint32_t b = 0;
      if (lane_id() == leader) b = atomicAdd(&sc.cnt[0], (uint32_t)__popcll(mt));
      b = __shfl(b, (int)leader, 64);
      if (take) {
        const uint64_t pos = b + lanes_below(mt);
        if (pos < n_gt) { dk[pos] = u; df[pos] = f; }
      }
    }
    if (me) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(me);
      uint32_t b = 0;
      if (lane_id() == leader) b = atomicAdd(&sc.cnt[1], (uint32_t)__popcll(me));
      b = __shfl(b, (int)leader, 64);
      if (eq) {
        const uint64_t pos = n_gt + b + lanes_below(me);
        if (pos < target) { dk[pos] = u; df[pos] = f; }
      }
    }
  }
  __syncthreads();
}

// merge-path split: number of elements of A among the first d outputs of
// merge(A, B), best first, ties taken from A
template <typename U, typename R>
__device__ __forceinline__ uint64_t merge_split(const U* ak, const R* af, uint64_t na, const U* bk,
                                                const R* bf, uint64_t nb, uint64_t d) {
  uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) / 2;
    if (cge(ak[mid], af[mid], bk[d - 1 - mid], bf[d - 1 - mid])) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Bitonic sort, best first, of P <= NT composites held one per thread
// (thread t holds element t; P a power of two).  Strides below the wave
// width exchange through lane shuffles; wider strides through LDS, ping-
// ponging between two halves of (bk, bf) (2P slots) so each such stage takes
// one barrier.  On return thread t holds the element of rank t.
template <int NT, typename U, typename R>
__device__ __forceinline__ void bitonic_regs_desc(U& k, R& f, uint32_t P, U* bk, R* bf) {
  const uint32_t t = threadIdx.x;
  uint32_t buf = 0;
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      U ok;
      R of;
      if (stride >= 64) {
        U* xk = bk + buf * P;
        R* xf = bf + buf * P;
        if (t < P) {
          xk[t] = k;
          xf[t] = f;
        }
        __syncthreads();
        ok = t < P ? xk[t ^ stride] : k;
        of = t < P ? xf[t ^ stride] : f;
        buf ^= 1u;
      } else {
        ok = __shfl_xor(k, (int)stride, 64);
        of = __shfl_xor(f, (int)stride, 64);
      }
      const bool keep_max = ((t & stride) == 0) == ((t & size) == 0);
      const bool take = keep_max ? cgt(ok, of, k, f) : cgt(k, f, ok, of);
      if (take) {
        k = ok;
        f = of;
      }
    }
  }
}

// Bitonic sort, best first, of P <= NT * E composites held E per thread:
// element i sits in thread i / E, slot i % E (P a power of two, threads whose
// slots lie beyond P hold anything and take part in the exchanges).  Strides
// below E compare registers of one thread; strides up to 32 E exchange with
// lane shuffles; wider strides go through LDS, ping-ponging between two
// halves of (bk, bf) (2P slots), one barrier per stage.  On return element i
// is the composite of rank i.
template <int NT, int E, typename U, typename R>
__device__ __forceinline__ void bitonic_regs_desc_e(U (&k)[E], R (&f)[E], uint32_t P, U* bk,
                                                    R* bf) {
  const uint32_t t = threadIdx.x;
  const uint32_t i0 = t * E;
  uint32_t buf = 0;
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride >= (uint32_t)E; stride >>= 1) {
      const uint32_t ts = stride / E;
      U* xk = bk + buf * P;
      R* xf = bf + buf * P;
      if (ts >= 64) {
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (i0 + e < P) {
            xk[i0 + e] = k[e];
            xf[i0 + e] = f[e];
          }
        __syncthreads();
        buf ^= 1u;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        U ok;
        R of;
        if (ts >= 64) {
          const uint32_t j = (t ^ ts) * E + e;
          ok = j < P ? xk[j] : k[e];
          of = j < P ? xf[j] : f[e];
        } else {
          ok = __shfl_xor(k[e], (int)ts, 64);
          of = __shfl_xor(f[e], (int)ts, 64);
        }
        const uint32_t i = i0 + e;
        const bool keep_max = ((i & stride) == 0) == ((i & size) == 0);
        const bool take = keep_max ? cgt(ok, of, k[e], f[e]) : cgt(k[e], f[e], ok, of);
        if (take) {
          k[e] = ok;
          f[e] = of;
        }
      }
    }
#pragma unroll
    for (int s2 = E / 2; s2 >= 1; s2 >>= 1) {
      if ((uint32_t)s2 >= size) continue;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (e & s2) continue;
        const int e2 = e | s2;
        const uint32_t i = i0 + e;
        const bool desc = (i & size) == 0;
        const bool swap = desc ? cgt(k[e2], f[e2], k[e], f[e]) : cgt(k[e], f[e], k[e2], f[e2]);
        if (swap) {
          const U tk_ = k[e];
          const R tf_ = f[e];
          k[e] = k[e2];
          f[e] = f[e2];
          k[e2] = tk_;
          f[e2] = tf_;
        }
      }
    }
  }
}

// Bitonic sort, best first, of m <= NT composites of 4-byte key image and
// 4-byte flipped row-id, packed as (key << 32 | flipped row-id) so that one
// 64-bit compare orders them and each stage is a compare and two selects:
// strides below the wave width exchange through lane shuffles, wider ones
// through LDS (two halves of 8 P bytes each, one barrier per stage).  Thread t
// emits the composite of rank t.
template <int NT, typename U, typename R, typename Emit>
__device__ __forceinline__ void sort_emit_packed(uint32_t m, U* lk, R* lf, Emit&& emit) {
  static_assert(sizeof(U) == 4 && sizeof(R) == 4, "packed sort: 4-byte key image and row-id");
  const uint32_t t = threadIdx.x;
  uint32_t P = 1;
  while (P < m) P <<= 1;
  uint64_t v = t < m ? ((uint64_t)lk[t] << 32) | (uint64_t)lf[t] : 0ull;
  __syncthreads();  // the tile is reused as the exchange buffer
  uint64_t* xb = reinterpret_cast<uint64_t*>(lk);
  const int lane4 = (int)(lane_id() << 2);
  uint32_t buf = 0;
  for (uint32_t size = 2; size <= P; size <<= 1) {
    const bool up = (t & size) == 0;  // this run ends up descending
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t o;
      if (stride >= 64) {
        uint64_t* x = xb + buf * P;
        if (t < P) x[t] = v;
        __syncthreads();
        o = t < P ? x[t ^ stride] : v;
        buf ^= 1u;
      } else {
        const int addr = lane4 ^ (int)(stride << 2);
        const uint32_t olo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v);
        const uint32_t ohi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v >> 32));
        o = ((uint64_t)ohi << 32) | olo;
      }
      // the lower position of a descending pair (or the upper of an
      // ascending one) keeps the larger composite
      const bool keep_max = ((t & stride) == 0) == up;
      v = ((o > v) == keep_max) ? o : v;
    }
  }
  if (t < m) emit((uint64_t)t, (U)(v >> 32), (R)(uint32_t)v);
  __syncthreads();
}

// The packed bitonic sort with 4 composites per thread on the first 256
// threads (m <= 1024): composite i sits in thread i / 4, slot i % 4, so the
// strides 1 and 2 are compare-exchanges in registers, strides 4 to 128 are
// lane permutes of 4 values, and only strides 256 and 512 go through LDS.
// Fewer dependent exchange steps than one composite per thread.
template <int NT, typename U, typename R, typename Emit>
__device__ __forceinline__ void sort_emit_packed4(uint32_t m, U* lk, R* lf, Emit&& emit) {
  static_assert(sizeof(U) == 4 && sizeof(R) == 4, "packed sort: 4-byte key image and row-id");
  static_assert(NT >= 256 && NT % 64 == 0, "at least 256 threads");
  constexpr uint32_t W = 256;
  const uint32_t t = threadIdx.x;
  const bool act = t < W;  // whole waves
  const uint32_t i0 = 4 * t;
  uint32_t P = 4;
  while (P < m) P <<= 1;
  uint64_t v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e)
    v[e] = (act && i0 + e < m) ? ((uint64_t)lk[i0 + e] << 32) | (uint64_t)lf[i0 + e] : 0ull;
  __syncthreads();  // the tile is reused as the exchange buffer
  uint64_t* xb = reinterpret_cast<uint64_t*>(lk);
  const int lane4 = (int)(lane_id() << 2);
  uint32_t buf = 0;
  for (uint32_t size = 2; size <= P; size <<= 1) {
    for (uint32_t stride = size >> 1; stride >= 4; stride >>= 1) {
      const uint32_t ts = stride >> 2;
      uint64_t o[4];
      if (ts >= 64) {
        uint64_t* x = xb + buf * P;
        if (act && i0 < P) {
#pragma unroll
          for (int e = 0; e < 4; ++e) x[i0 + e] = v[e];
        }
        __syncthreads();
        if (act && i0 < P) {
          const uint32_t j0 = 4 * (t ^ ts);
#pragma unroll
          for (int e = 0; e < 4; ++e) o[e] = x[j0 + e];
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e) o[e] = v[e];
        }
        buf ^= 1u;
      } else if (act) {
        const int addr = lane4 ^ (int)(ts << 2);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t olo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)v[e]);
          const uint32_t ohi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(v[e] >> 32));
          o[e] = ((uint64_t)ohi << 32) | olo;
        }
      }
      if (act) {
        // same direction for the 4 slots: i0 is a multiple of 4 and stride >= 4
        const bool keep_max = ((i0 & stride) == 0) == ((i0 & size) == 0);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = ((o[e] > v[e]) == keep_max) ? o[e] : v[e];
      }
    }
    if (act) {
      const bool desc = (i0 & size) == 0;  // size >= 4 here shares i0's bit; size 2 uses slot bit
#pragma unroll
      for (int s2 = 2; s2 >= 1; s2 >>= 1) {
        if ((uint32_t)s2 >= size) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (e & s2) continue;
          const int e2 = e | s2;
          const bool d = size >= 4 ? desc : (((i0 + e) & size) == 0);
          const bool sw = d ? (v[e2] > v[e]) : (v[e] > v[e2]);
          const uint64_t a = v[e], b = v[e2];
          v[e] = sw ? b : a;
          v[e2] = sw ? a : b;
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i0 + e < m) emit((uint64_t)(i0 + e), (U)(v[e] >> 32), (R)(uint32_t)v[e]);
  }
  __syncthreads();
}

// Sorts m <= NT * E composites sitting at the start of the LDS tile (lk, lf)
// (2P <= CAP) in registers and emits them.
template <int NT, int E, typename U, typename R, typename Emit>
__device__ __forceinline__ void sort_emit_regs(uint32_t m, U* lk, R* lf, Emit&& emit) {
  uint32_t P = 1;
  while (P < m) P <<= 1;
  const uint32_t i0 = threadIdx.x * E;
  U k[E];
  R f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    k[e] = i0 + e < m ? lk[i0 + e] : (U)0;
    f[e] = i0 + e < m ? lf[i0 + e] : (R)0;
  }
  __syncthreads();  // the tile is reused as the exchange buffer
  bitonic_regs_desc_e<NT, E, U, R>(k, f, P, lk, lf);
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (i0 + e < m) emit((uint64_t)(i0 + e), k[e], f[e]);
  __syncthreads();
}

// The general sort of block_sort_emit: composites in LDS are sorted in
// registers (up to 16 per thread) or by an LDS bitonic network; composites in
// global memory (ck, cf) are bitonic-sorted in LDS tiles of CAP, then merged
// pairwise through (tk, tf) with merge-path splits.
template <int NT, typename U, typename R, typename Emit>
__device__ __noinline__ void block_sort_emit_general(uint64_t m, bool in_lds, U* lk, R* lf, uint32_t CAP, U* ck, R* cf,
                                U* tk, R* tf, Emit emit) {
  if (in_lds) {
    // registers: up to 4 (or 16) composites per thread, exchange buffer 2P <= CAP
    uint32_t P = 1;
    while (P < m) P <<= 1;
    if (m <= NT && 2 * P <= CAP) {
      sort_emit_regs<NT, 1, U, R>((uint32_t)m, lk, lf, emit);
      return;
    }
    if (m <= 4 * NT && 2 * P <= CAP) {
      sort_emit_regs<NT, 4, U, R>((uint32_t)m, lk, lf, emit);
      return;
    }
    if (m <= 16 * NT && 2 * P <= CAP) {
      sort_emit_regs<NT, 16, U, R>((uint32_t)m, lk, lf, emit);
      return;
    }
  }
  if (in_lds) {
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t i = (uint32_t)m + threadIdx.x; i < P; i += NT) {
      lk[i] = 0;
      lf[i] = 0;
    }
    bitonic_desc<U, R, NT>(lk, lf, P);
    for (uint32_t j = threadIdx.x; j < m; j += NT) emit((uint64_t)j, lk[j], lf[j]);
    __syncthreads();
    return;
  }
  for (uint64_t base = 0; base < m; base += CAP) {
    const uint64_t len = m - base < CAP ? m - base : CAP;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < CAP; i += NT) {
      lk[i] = i < len ? ck[base + i] : (U)0;
      lf[i] = i < len ? cf[base + i] : (R)0;
    }
    bitonic_desc<U, R, NT>(lk, lf, CAP);
    for (uint32_t i = threadIdx.x; i < len; i += NT) {
      ck[base + i] = lk[i];
      cf[base + i] = lf[i];
    }
  }
  __syncthreads();
  U* sk = ck;
  R* sf = cf;
  U* dk = tk;
  R* df = tf;
  constexpr uint64_t ITEMS = 8;
  for (uint64_t run = CAP; run < m; run <<= 1) {
    for (uint64_t s = 0; s < m; s += 2 * run) {
      const uint64_t amid = s + run < m ? s + run : m;
      const uint64_t aend = s + 2 * run < m ? s + 2 * run : m;
      const uint64_t na = amid - s, nb = aend - amid;
      for (uint64_t o0 = (uint64_t)threadIdx.x * ITEMS; o0 < na + nb; o0 += (uint64_t)NT * ITEMS) {
        uint64_t i = merge_split<U, R>(sk + s, sf + s, na, sk + amid, sf + amid, nb, o0);
        uint64_t j = o0 - i;
        const uint64_t cnt = na + nb - o0 < ITEMS ? na + nb - o0 : ITEMS;
        for (uint64_t q = 0; q < cnt; ++q) {
          bool from_a;
          if (i >= na) from_a = false;
          else if (j >= nb) from_a = true;
          else from_a = cge(sk[s + i], sf[s + i], sk[amid + j], sf[amid + j]);
          if (from_a) {
            dk[s + o0 + q] = sk[s + i];
            df[s + o0 + q] = sf[s + i];
            ++i;
          } else {
            dk[s + o0 + q] = sk[amid + j];
            df[s + o0 + q] = sf[amid + j];
            ++j;
          }
        }
      }
    }
    __syncthreads();
    U* xk = sk; sk = dk; dk = xk;
    R* xf = sf; sf = df; df = xf;
  }
  for (uint64_t j = threadIdx.x; j < m; j += NT) emit(j, sk[j], sf[j]);
  __syncthreads();
}


// One workgroup sorts m selected composites best first and hands each to
// emit(j, u, f).  in_lds: the composites sit at the start of the LDS tile
// (lk, lf) of CAP elements and m <= CAP.  The common case (m <= NT composites
// of 8 bytes) is sorted inline; the others go to block_sort_emit_general.
template <int NT, typename U, typename R, typename Emit>
__device__ __forceinline__ void block_sort_emit(uint64_t m, bool in_lds, U* lk, R* lf, uint32_t CAP,
                                                U* ck, R* cf, U* tk, R* tf, Emit&& emit) {
  if constexpr (sizeof(U) == 4 && sizeof(R) == 4) {
    // exchange buffer: 2P 8-byte words in the tile's 8 CAP bytes
    if constexpr (NT >= 256) {
      if (in_lds && m <= 1024 && 2048 <= CAP) {
        sort_emit_packed4<NT, U, R>((uint32_t)m, lk, lf, emit);
        return;
      }
    }
    if (in_lds && m <= NT && 2 * (uint64_t)NT <= CAP) {
      sort_emit_packed<NT, U, R>((uint32_t)m, lk, lf, emit);
      return;
    }
  }
  block_sort_emit_general<NT, U, R>(m, in_lds, lk, lf, CAP, ck, cf, tk, tf, emit);
}

}  // namespace tk
