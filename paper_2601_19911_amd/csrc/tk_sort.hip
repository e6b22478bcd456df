// Full sort of (key, row-id) pairs: ORDER BY key without LIMIT (the query
// template of paper sec. V-B with K = N), the same order as every Top-K entry
// point: key descending or ascending (int32/int64 numeric, float32/float64
// IEEE totalOrder), equal keys by ascending row-id.
//
// Least-significant-digit radix sort over 8-bit digits of the order image
// s = enc(key) (ascending) or ~enc(key) (descending), sorted ascending by
// (s, row-id).  With implicit row-ids the input order is the row-id order, so a
// stable pass per key digit suffices (4 passes for 32-bit keys, 8 for 64-bit);
// with explicit row-ids the row-id digits are sorted first.  Each pass is three
// launches with no inter-workgroup waiting:
//   k_sup    one workgroup per tile (8192 pairs of 8 bytes, 4096 wider ones):
//            the tile's digit counts
//   k_sscan  one workgroup per digit: exclusive scan of that digit's counts
//            over the tiles, and the digit's total
//   k_sdown  one workgroup per tile: stable rank of every pair inside the tile
//            (per wave, peers of equal digit found by 8 ballots), pairs staged
//            in LDS in digit order, then written as runs of consecutive
//            addresses at the digit's global offset
// The first pass reads the caller's keys (encoding them) and row-ids (or
// position), the last writes the caller's outputs (decoding the keys); the
// passes between ping-pong through the workspace.  A Top-K query that the
// sample cannot serve runs the same passes with the last one writing only the
// first K positions (topk_by_sort).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_internal.hpp"

namespace {

#ifndef TK_SORT_NT
#define TK_SORT_NT 512
#endif
#ifndef TK_SORT_ITEMS_SMALL
#define TK_SORT_ITEMS_SMALL 16
#endif
#ifndef TK_SORT_ITEMS_WIDE
#define TK_SORT_ITEMS_WIDE 8
#endif
constexpr int SORT_NT = TK_SORT_NT;    // threads per workgroup of k_sup and k_sdown
constexpr int SORT_WAVES = SORT_NT / 64;
constexpr int SCAN_NT = 256;           // threads per workgroup of k_sscan
constexpr int RADIX = 256;             // 8-bit digits
static_assert(SORT_NT >= RADIX, "a thread per digit");

// Pairs per thread and per tile: a tile is staged in LDS by k_sdown, and the
// longer a tile, the longer the run each digit writes.  Measured on MI355X at
// 2^24 pairs: 512 threads with 8192-pair tiles (8-byte pairs; 4096 for wider
// ones, 64 KiB of LDS, two workgroups per CU) beat 256 threads with 4096 pairs
// by 9-12 %, and one workgroup per CU with longer tiles by 15-40 %.
constexpr int items_for(uint32_t pair_bytes) {
  return pair_bytes <= 8 ? TK_SORT_ITEMS_SMALL : TK_SORT_ITEMS_WIDE;
}
constexpr uint32_t tile_for(uint32_t pair_bytes) { return SORT_NT * items_for(pair_bytes); }
static_assert(tile_for(8) >= 4096 && tile_for(16) >= 4096,
              "the scratch bound of the sort route counts 4096-pair tiles");

// Where a pass reads and writes.  Input keys are raw (encoded when first is
// set); keys in the workspace hold the order image; the last pass decodes.
template <typename U, typename R>
struct PassArgs {
  const void* in_keys;
  const R* in_rids;     // null (first pass only): row-id = position
  U* out_keys;          // null: keys not written (last pass without out_keys)
  R* out_rids;
  uint64_t n;
  uint32_t ntiles;
  uint32_t shift;       // digit position in bits
  uint32_t rid_digit;   // 1: the digit comes from the row-id
  uint32_t first, last;
  uint32_t desc;
  uint32_t* counts;     // [RADIX][ntiles], scanned in place by k_sscan
  uint32_t* totals;     // [RADIX]
  uint64_t limit;       // the last pass writes only positions below it (a Top-K of K = limit)
  tk::QHead* h;         // a Top-K query's header (path recorded by the first pass), or null
};

template <int KT>
__device__ __forceinline__ typename tk::Key<KT>::U image(typename tk::Key<KT>::Raw raw, uint32_t desc) {
  const auto u = tk::Key<KT>::enc(raw);
  return desc ? ~u : u;
}

template <int KT>
__device__ __forceinline__ typename tk::Key<KT>::Raw unimage(typename tk::Key<KT>::U s, uint32_t desc) {
  return tk::Key<KT>::dec(desc ? ~s : s);
}

template <int KT, typename R>
__device__ __forceinline__ void load_pair(const PassArgs<typename tk::Key<KT>::U, R>& a, uint64_t i,
                                          typename tk::Key<KT>::U& s, R& r) {
  using U = typename tk::Key<KT>::U;
  if (a.first) {
    s = image<KT>(static_cast<const typename tk::Key<KT>::Raw*>(a.in_keys)[i], a.desc);
    r = a.in_rids ? a.in_rids[i] : (R)i;
  } else {
    s = static_cast<const U*>(a.in_keys)[i];
    r = a.in_rids[i];
  }
}

template <typename U, typename R>
__device__ __forceinline__ uint32_t digit_of(U s, R r, uint32_t shift, uint32_t rid_digit) {
  return rid_digit ? (uint32_t)((uint64_t)r >> shift) & (RADIX - 1)
                   : (uint32_t)((uint64_t)s >> shift) & (RADIX - 1);
}

template <int KT, typename R>
__global__ __launch_bounds__(SORT_NT) void k_sup(PassArgs<typename tk::Key<KT>::U, R> a) {
  using U = typename tk::Key<KT>::U;
  constexpr int SORT_ITEMS = items_for(sizeof(U) + sizeof(R));
  constexpr uint32_t TILE = tile_for(sizeof(U) + sizeof(R));
  __shared__ uint32_t h[SORT_WAVES][RADIX];
  const uint32_t w = threadIdx.x >> 6;
  if (a.first && a.h && blockIdx.x == 0 && threadIdx.x == 0) {
    a.h->path = 9u;
    a.h->status = 0u;
  }
  // every load of the thread in flight at once, then the counts
  const uint64_t base = (uint64_t)blockIdx.x * TILE;
  U s[SORT_ITEMS];
  R r[SORT_ITEMS];
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const uint64_t i = base + (uint64_t)it * SORT_NT + threadIdx.x;
    if (i < a.n) load_pair<KT, R>(a, i, s[it], r[it]);
  }
  for (uint32_t i = threadIdx.x; i < SORT_WAVES * RADIX; i += SORT_NT) (&h[0][0])[i] = 0;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const uint64_t i = base + (uint64_t)it * SORT_NT + threadIdx.x;
    if (i < a.n) atomicAdd(&h[w][digit_of(s[it], r[it], a.shift, a.rid_digit)], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < RADIX; d += SORT_NT) {
    uint32_t c = 0;
#pragma unroll
    for (int x = 0; x < SORT_WAVES; ++x) c += h[x][d];
    a.counts[(uint64_t)d * a.ntiles + blockIdx.x] = c;
  }
}

// One workgroup per digit: exclusive scan of counts[d][0..ntiles) in place.
__global__ __launch_bounds__(SCAN_NT) void k_sscan(uint32_t* counts, uint32_t ntiles, uint32_t* totals) {
  __shared__ uint32_t ws[SCAN_NT / 64];
  uint32_t* row = counts + (uint64_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < ntiles; base += SCAN_NT * 4) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t t = base + threadIdx.x * 4 + q;
      v[q] = t < ntiles ? row[t] : 0u;
      sum += v[q];
    }
    uint32_t total = 0;
    const uint32_t off = tk::block_excl_scan<SCAN_NT>(sum, ws, total);
    uint32_t run = carry + off;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t t = base + threadIdx.x * 4 + q;
      if (t < ntiles) row[t] = run;
      run += v[q];
    }
    carry += total;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

template <int KT, typename R>
__global__ __launch_bounds__(SORT_NT) void k_sdown(PassArgs<typename tk::Key<KT>::U, R> a) {
  using U = typename tk::Key<KT>::U;
  using Raw = typename tk::Key<KT>::Raw;
  constexpr int SORT_ITEMS = items_for(sizeof(U) + sizeof(R));
  constexpr uint32_t TILE = tile_for(sizeof(U) + sizeof(R));
  constexpr uint32_t WAVE_CHUNK = 64 * SORT_ITEMS;  // a wave's contiguous share of a tile
  __shared__ uint32_t wcnt[SORT_WAVES][RADIX];  // per wave counts, then offsets
  __shared__ uint32_t dstart[RADIX];            // first local position of each digit
  __shared__ uint64_t gbase[RADIX];             // global position of each digit's run
  __shared__ uint32_t ws[SORT_WAVES];
  __shared__ U sk[TILE];
  __shared__ R sr[TILE];
  const uint32_t w = threadIdx.x >> 6, ln = tk::lane_id();
  const uint64_t tbase = (uint64_t)blockIdx.x * TILE;
  const uint32_t nt = (uint32_t)((a.n - tbase) < TILE ? (a.n - tbase) : TILE);

  // the tile's pairs, the digit totals and this tile's prefixes: every load in
  // flight at once
  U s[SORT_ITEMS];
  R r[SORT_ITEMS];
  uint32_t rk[SORT_ITEMS];
  const uint32_t wbase = w * WAVE_CHUNK;
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const uint32_t li = wbase + it * 64 + ln;
    if (li < nt) load_pair<KT, R>(a, tbase + li, s[it], r[it]);
  }
  // global start of every digit: scan of the digit totals + this tile's prefix
  // (thread d < RADIX holds digit d)
  {
    const uint32_t d = threadIdx.x;
    const bool dig = d < (uint32_t)RADIX;
    const uint32_t tot_d = dig ? a.totals[d] : 0u;
    const uint32_t pre_d = dig ? a.counts[(uint64_t)d * a.ntiles + blockIdx.x] : 0u;
    uint32_t total = 0;
    const uint32_t before = tk::block_excl_scan<SORT_NT>(tot_d, ws, total);
    if (dig) gbase[d] = (uint64_t)before + pre_d;
    for (uint32_t i = threadIdx.x; i < SORT_WAVES * RADIX; i += SORT_NT) (&wcnt[0][0])[i] = 0;
  }
  __syncthreads();

  // stable rank inside the wave: position order is (wave, round, lane)
  const uint64_t below = (1ull << ln) - 1ull;
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const uint32_t li = wbase + it * 64 + ln;
    const bool valid = li < nt;
    const uint32_t d = valid ? digit_of(s[it], r[it], a.shift, a.rid_digit) : 0u;
    uint64_t peers = tk::ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t m = tk::ballot(((d >> b) & 1u) != 0u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    uint32_t prior = 0;
    if (valid) prior = wcnt[w][d];
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      rk[it] = prior + (uint32_t)__popcll(peers & below);
      // the lowest lane of each peer group advances the wave's count
      if ((peers & below) == 0) wcnt[w][d] = prior + (uint32_t)__popcll(peers);
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: offsets of the waves inside the digit's run, and the run's start
  {
    const uint32_t d = threadIdx.x;
    const bool dig = d < (uint32_t)RADIX;
    uint32_t run = 0;
    if (dig) {
#pragma unroll
      for (int x = 0; x < SORT_WAVES; ++x) {
        const uint32_t c = wcnt[x][d];
        wcnt[x][d] = run;
        run += c;
      }
    }
    uint32_t total = 0;
    const uint32_t st = tk::block_excl_scan<SORT_NT>(run, ws, total);
    if (dig) dstart[d] = st;
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const uint32_t li = wbase + it * 64 + ln;
    if (li < nt) {
      const uint32_t d = digit_of(s[it], r[it], a.shift, a.rid_digit);
      const uint32_t p = dstart[d] + wcnt[w][d] + rk[it];
      sk[p] = s[it];
      sr[p] = r[it];
    }
  }
  __syncthreads();
  // write out in digit order: consecutive local positions of one digit go to
  // consecutive global positions
  for (uint32_t p = threadIdx.x; p < nt; p += SORT_NT) {
    const U sv = sk[p];
    const R rv = sr[p];
    const uint32_t d = digit_of(sv, rv, a.shift, a.rid_digit);
    const uint64_t g = gbase[d] + (p - dstart[d]);
    if (a.last) {
      if (g < a.limit) {
        if (a.out_keys) reinterpret_cast<Raw*>(a.out_keys)[g] = unimage<KT>(sv, a.desc);
        if (a.out_rids) a.out_rids[g] = rv;
      }
    } else {
      a.out_keys[g] = sv;
      a.out_rids[g] = rv;
    }
  }
}

uint64_t align256(uint64_t b) { return (b + 255) & ~255ull; }

struct SortLayout {
  uint64_t ntiles, keys_a, rids_a, keys_b, rids_b, counts, totals, bytes;
};

SortLayout layout(uint64_t n, int key_type, int rid_type) {
  const uint64_t kb = tk::key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  const uint64_t tile = tile_for((uint32_t)(kb + rb));
  SortLayout L;
  L.ntiles = (n + tile - 1) / tile;
  if (L.ntiles == 0) L.ntiles = 1;
  uint64_t o = 0;
  L.keys_a = o; o += align256(n * kb);
  L.rids_a = o; o += align256(n * rb);
  L.keys_b = o; o += align256(n * kb);
  L.rids_b = o; o += align256(n * rb);
  L.counts = o; o += align256(L.ntiles * RADIX * 4);
  L.totals = o; o += align256(RADIX * 4);
  L.bytes = o;
  return L;
}

template <int KT, typename R>
int sort_t(const void* keys, const void* rids, uint64_t n, int order, void* out_keys, void* out_rids,
           void* ws, hipStream_t st, int rid_type, uint64_t limit, tk::QHead* hq) {
  using U = typename tk::Key<KT>::U;
  const SortLayout L = layout(n, KT, rid_type);
  char* w = static_cast<char*>(ws);
  const uint32_t kbits = 8 * sizeof(U), rbits = 8 * sizeof(R);
  // digit passes, least significant first: row-id digits (explicit row-ids only), then key digits
  struct P { uint32_t shift, rid_digit; };
  P passes[16];
  int np = 0;
  if (rids)
    for (uint32_t b = 0; b < rbits; b += 8) passes[np++] = {b, 1};
  for (uint32_t b = 0; b < kbits; b += 8) passes[np++] = {b, 0};
  U* kbuf[2] = {reinterpret_cast<U*>(w + L.keys_a), reinterpret_cast<U*>(w + L.keys_b)};
  R* rbuf[2] = {reinterpret_cast<R*>(w + L.rids_a), reinterpret_cast<R*>(w + L.rids_b)};
  PassArgs<U, R> a;
  a.n = n;
  a.ntiles = (uint32_t)L.ntiles;
  a.desc = order == TK_DESC ? 1u : 0u;
  a.counts = reinterpret_cast<uint32_t*>(w + L.counts);
  a.totals = reinterpret_cast<uint32_t*>(w + L.totals);
  a.limit = limit;
  a.h = hq;
  for (int p = 0; p < np; ++p) {
    a.first = p == 0;
    a.last = p == np - 1;
    a.shift = passes[p].shift;
    a.rid_digit = passes[p].rid_digit;
    a.in_keys = a.first ? keys : static_cast<const void*>(kbuf[(p - 1) & 1]);
    a.in_rids = a.first ? static_cast<const R*>(rids) : rbuf[(p - 1) & 1];
    a.out_keys = a.last ? static_cast<U*>(out_keys) : kbuf[p & 1];
    a.out_rids = a.last ? static_cast<R*>(out_rids) : rbuf[p & 1];
    hipLaunchKernelGGL((k_sup<KT, R>), dim3(a.ntiles), dim3(SORT_NT), 0, st, a);
    hipLaunchKernelGGL(k_sscan, dim3(RADIX), dim3(SCAN_NT), 0, st, a.counts, a.ntiles, a.totals);
    hipLaunchKernelGGL((k_sdown<KT, R>), dim3(a.ntiles), dim3(SORT_NT), 0, st, a);
  }
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}

template <int KT>
int sort_rid(const void* keys, const void* rids, uint64_t n, int rid_type, int order, void* ok,
             void* orr, void* ws, hipStream_t st, uint64_t limit, tk::QHead* hq) {
  if (rid_type == TK_RID_U32)
    return sort_t<KT, uint32_t>(keys, rids, n, order, ok, orr, ws, st, rid_type, limit, hq);
  return sort_t<KT, unsigned long long>(keys, rids, n, order, ok, orr, ws, st, rid_type, limit, hq);
}

int sort_any(const void* keys, const void* rowids, uint64_t n, int key_type, int rid_type, int order,
             void* out_keys, void* out_rowids, void* ws, hipStream_t st, uint64_t limit,
             tk::QHead* hq) {
  switch (key_type) {
    case TK_KEY_I32: return sort_rid<tk::KEY_I32>(keys, rowids, n, rid_type, order, out_keys, out_rowids, ws, st, limit, hq);
    case TK_KEY_I64: return sort_rid<tk::KEY_I64>(keys, rowids, n, rid_type, order, out_keys, out_rowids, ws, st, limit, hq);
    case TK_KEY_F32: return sort_rid<tk::KEY_F32>(keys, rowids, n, rid_type, order, out_keys, out_rowids, ws, st, limit, hq);
    default: return sort_rid<tk::KEY_F64>(keys, rowids, n, rid_type, order, out_keys, out_rowids, ws, st, limit, hq);
  }
}

}  // namespace

namespace tk {

// The Top-K of a query by its full sort: the first k_eff pairs of the order
// are written to the outputs (the last pass writes nothing past them).
int topk_by_sort(const void* keys, const void* rowids, uint64_t n, uint64_t k_eff, int key_type,
                 int rid_type, int order, void* out_keys, void* out_rowids, void* scratch,
                 QHead* h, hipStream_t st) {
  return sort_any(keys, rowids, n, key_type, rid_type, order, out_keys, out_rowids, scratch, st,
                  k_eff, h);
}

}  // namespace tk

extern "C" size_t tk_sort_workspace_size(uint64_t n, int key_type, int rid_type) {
  if (key_type < TK_KEY_I32 || key_type > TK_KEY_F64 || (rid_type != TK_RID_U32 && rid_type != TK_RID_U64))
    return 0;
  return (size_t)layout(n, key_type, rid_type).bytes;
}

extern "C" int tk_sort(const void* keys, const void* rowids, uint64_t n, int key_type, int rid_type,
                       int order, void* out_keys, void* out_rowids, void* workspace,
                       size_t workspace_bytes, void* stream) {
  if (key_type < TK_KEY_I32 || key_type > TK_KEY_F64 || (rid_type != TK_RID_U32 && rid_type != TK_RID_U64) ||
      (order != TK_DESC && order != TK_ASC))
    return TK_EINVAL;
  if (n == 0) return TK_OK;
  if (!keys || !out_rowids || !workspace) return TK_EINVAL;
  if (((uintptr_t)workspace & 255) != 0) return TK_EINVAL;
  if (workspace_bytes < layout(n, key_type, rid_type).bytes) return TK_EINVAL;
  if (!rowids && rid_type == TK_RID_U32 && n > (1ull << 32)) return TK_EINVAL;
  if (n >= (1ull << 32)) return TK_EUNSUPPORTED;  // 32-bit digit counts and offsets
  return sort_any(keys, rowids, n, key_type, rid_type, order, out_keys, out_rowids, workspace,
                  (hipStream_t)stream, n, nullptr);
}
