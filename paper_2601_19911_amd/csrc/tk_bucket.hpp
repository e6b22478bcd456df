// Tail of the sampled single query for large K: the exact best K of the
// filter's survivors, over the whole GPU.
//
//   k_bhist     workgroups take slices of the survivors and count them by a
//               logarithmic bucket of their distance D = c - T to the
//               threshold (c the composite read as one wide integer, 2^s
//               buckets per octave: tk_wide.hpp), first in LDS, then added
//               into the query's global histogram (cleared by the sample
//               launch) over the range of buckets the slice reached.  Few
//               workgroups: every bucket counter they share takes one atomic
//               from each.
//   k_bscatter  every workgroup derives from the histogram the boundary
//               bucket b* holding rank K and the exclusive offset of every
//               bucket, reserves room in each hot bucket (b >= b*) for its
//               slice of the survivors with one global atomic per bucket, and
//               scatters its hot survivors there: the hot set grouped by
//               bucket, best bucket first.  Workgroup 0 also cuts the hot set
//               into chunks of whole buckets that fit one LDS tile.
//   k_bsort     each workgroup orders chunks in LDS (a finer bin histogram
//               and counting inside each bin, bin_sort_emit; the bitonic sort
//               when a bin is too full) and writes every member at chunk
//               offset + rank, up to K.
// The bucket is monotone in the composite, so a chunk's members take the
// output positions [offset, offset + size).  A query this path cannot finish
// (survivor count outside [K, capacity], or a hot bucket larger than one LDS
// tile) is finished by workgroup 0 of k_bsort with the one-workgroup select +
// sort.
#pragma once

#include "tk_rank.hpp"

namespace tk {

constexpr int BT_NT = 256;           // k_bhist
constexpr int BSC_NT = 1024;         // k_bscatter
constexpr uint32_t BT_SLICES = 128;  // workgroups of k_bhist
// workgroups of k_bscatter: every one takes a global atomic on each hot
// bucket its slice reaches (64 measured best against 16, 32, 128 and 256)
constexpr uint32_t BT_SCATTER = 64;
constexpr uint32_t BT_GRID = 256;    // workgroups of k_bsort

// Query state of the bucketed tail.
struct BMeta {
  uint32_t bstar;     // boundary bucket
  uint32_t fallback;  // 1: workgroup 0 of k_bsort finishes the query in one workgroup
  uint32_t hot;       // members of the buckets >= bstar
  uint32_t nchunk;    // chunks of the hot set
  uint32_t pad[12];
};

// The bucketed tail's region: gh[NB] (histogram), cur[NB] (scatter cursors),
// chunk[NB] (chunk starts), the state, then the hot set.
struct BTailArgs {
  TailArgs1 t;     // the query (survivors, outputs, fallback workspace)
  uint32_t* gh;
  uint32_t* cur;
  uint32_t* chunk;
  BMeta* meta;
  void* hk;        // hot set, grouped by bucket: key images
  void* hf;        //                             flipped row-ids
};

// A workgroup's slice of the survivors: j = blockIdx.x * NT + threadIdx.x +
// i * stride, stride = gridDim.x * NT (NT threads per workgroup); loads go
// BT_BATCH at a time.
constexpr int BT_BATCH = 8;

// The first BT_BATCH visits of a workgroup's slice, loaded before the
// survivor count is read (every slot below the capacity is in the buffer;
// slots at or past the count are ignored), so that the count and the
// survivors arrive in one round trip.
template <typename U, typename R, int NT>
struct HeldSlice {
  U u[BT_BATCH];
  R f[BT_BATCH];
  uint64_t j0, stride;
  __device__ __forceinline__ void load(const U* sk, const R* sf, uint64_t cap) {
    stride = (uint64_t)gridDim.x * NT;
    j0 = (uint64_t)blockIdx.x * NT + threadIdx.x;
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint64_t j = j0 + (uint64_t)q * stride;
      u[q] = j < cap ? sk[j] : (U)0;
      f[q] = j < cap ? sf[j] : (R)0;
    }
  }
  __device__ __forceinline__ bool valid(int q, uint64_t C) const {
    return j0 + (uint64_t)q * stride < C;
  }
  // whether the held visits cover the whole slice of C survivors
  __device__ __forceinline__ bool covers(uint64_t C) const { return C <= BT_BATCH * stride; }
  // the slice's visits past the held ones
  template <typename Fn>
  __device__ __forceinline__ void rest(const U* sk, const R* sf, uint64_t C, Fn&& fn) const {
    for (uint64_t k0 = j0 + BT_BATCH * stride; k0 < C; k0 += BT_BATCH * stride) {
      U v[BT_BATCH];
      R g[BT_BATCH];
#pragma unroll
      for (int q = 0; q < BT_BATCH; ++q) {
        const uint64_t j = k0 + (uint64_t)q * stride;
        v[q] = j < C ? sk[j] : (U)0;
        g[q] = j < C ? sf[j] : (R)0;
      }
#pragma unroll
      for (int q = 0; q < BT_BATCH; ++q)
        if (k0 + (uint64_t)q * stride < C) fn(v[q], g[q]);
    }
  }
};

template <int KT, int RT>
__device__ __forceinline__ void bhist_body(const BTailArgs& b, uint32_t* lh, uint32_t* red) {
  using B = BT<KT, RT>;
  using U = typename B::U;
  using R = typename B::R;
  constexpr uint32_t NB = B::NB;
  const TailArgs1& a = b.t;
  const U* sk = static_cast<const U*>(a.sk);
  const R* sf = static_cast<const R*>(a.sf);
  HeldSlice<U, R, BT_NT> hs;
  hs.load(sk, sf, a.cap);
  const uint64_t C = a.h->surv_count;
  const typename B::T base = wide((U)a.h->thr_k, (R)a.h->thr_f);
  if (!(C >= a.k_eff && C <= a.cap)) return;  // uniform; k_bscatter flags the fallback
  const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
  // the range of buckets this workgroup touches: only it is cleared and added
  // into the global histogram (all of them when the slice is not all held)
  uint32_t bk[BT_BATCH];
  uint32_t lo = NB, hi = 0;
#pragma unroll
  for (int q = 0; q < BT_BATCH; ++q) {
    bk[q] = B::bucket(hs.u[q], hs.f[q], base);
    if (hs.valid(q, C)) {
      lo = bk[q] < lo ? bk[q] : lo;
      hi = bk[q] > hi ? bk[q] : hi;
    }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if (lane == 0) {
    red[w] = lo;
    red[8 + w] = hi;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < BT_NT / 64; ++i) {
    lo = red[i] < lo ? red[i] : lo;
    hi = red[8 + i] > hi ? red[8 + i] : hi;
  }
  if (!hs.covers(C)) {
    lo = 0;
    hi = NB - 1;
  }
  for (uint32_t i = lo + t; i <= hi; i += BT_NT) lh[i] = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BT_BATCH; ++q)
    if (hs.valid(q, C)) atomicAdd(&lh[bk[q]], 1u);
  hs.rest(sk, sf, C, [&](U u, R f) { atomicAdd(&lh[B::bucket(u, f, base)], 1u); });
  __syncthreads();
  for (uint32_t i = lo + t; i <= hi; i += BT_NT) {
    const uint32_t c = lh[i];
    if (c) atomicAdd(&b.gh[i], c);
  }
}

// k_bscatter's LDS copy of the histogram is read by each thread over BPT
// consecutive buckets; a word of padding after every 32 keeps a wave's lanes
// on distinct banks.
__device__ __forceinline__ uint32_t bs_pad(uint32_t bin) { return bin + (bin >> 5); }
template <uint32_t NB>
constexpr uint32_t bs_padded() { return NB + (NB >> 5) + 1; }

// From the global histogram: the boundary bucket b* (holding rank K), the
// hot set's size and every bucket's exclusive offset (members of better
// buckets, into loff at bs_pad), and the chunks.  Every workgroup of
// k_bscatter derives the same; workgroup 0 also writes the chunk starts and
// the tail's state.  Returns false (workgroup 0 having flagged the fallback)
// when the survivor count or a hot bucket is outside this path's limits.
// Every thread calls it.
template <int KT, int RT>
__device__ __forceinline__ bool bucket_offsets(const BTailArgs& b, uint64_t C, uint32_t* loff,
                                               uint32_t* red, uint32_t& bstar_out) {
  using B = BT<KT, RT>;
  constexpr uint32_t NB = B::NB, BPT = (NB + BSC_NT - 1) / BSC_NT;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const TailArgs1& a = b.t;
  const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
  const bool lead = blockIdx.x == 0;
  const uint64_t K = a.k_eff;
  if (!(C >= K && C <= a.cap)) {
    if (lead && t == 0) b.meta->fallback = 1u;
    return false;
  }
  __syncthreads();  // the histogram is in loff
  // suffix sums: thread t holds buckets [t BPT, t BPT + BPT)
  uint32_t s = 0;
#pragma unroll
  for (uint32_t i = 0; i < BPT; ++i) {
    const uint32_t bin = t * BPT + i;
    s += bin < NB ? loff[bs_pad(bin)] : 0u;
  }
  const uint32_t x = wave_suffix_sum(s);  // sum over lanes >= this one
  if (lane == 0) red[w] = x;
  __syncthreads();
  uint32_t above = x - s;
#pragma unroll
  for (int i = 0; i < BSC_NT / 64; ++i) above += (uint32_t)i > w ? red[i] : 0u;
  // exclusive offsets; a bucket is hot while its offset is below K; the
  // boundary bucket is the one that reaches K
  uint32_t mx = 0;
#pragma unroll
  for (int i = (int)BPT - 1; i >= 0; --i) {
    const uint32_t bin = t * BPT + (uint32_t)i;
    if (bin >= NB) continue;
    const uint32_t c = loff[bs_pad(bin)];
    loff[bs_pad(bin)] = above;
    if (above < K) mx = c > mx ? c : mx;
    if (above < K && K <= (uint64_t)above + c) {
      red[16] = bin;
      red[17] = above + c;
    }
    above += c;
  }
  mx = wave_max(mx);
  if (lane == 0) red[32 + w] = mx;
  __syncthreads();
  const uint32_t bstar = red[16], H = red[17];
#pragma unroll
  for (int i = 0; i < BSC_NT / 64; ++i) mx = red[32 + i] > mx ? red[32 + i] : mx;
  // chunks of whole buckets: chunk c holds the buckets whose offset lies in
  // [c tgt, (c + 1) tgt), at most tgt - 1 + mx <= CAP members
  // tgt = 2^sh: about one chunk per k_bsort workgroup, and tgt - 1 + mx <= CAP
  const uint32_t want = (H + BT_GRID - 1) / BT_GRID;
  const uint32_t lim = mx <= CAP ? CAP - mx + 1 : 1u;
  uint32_t sh = 0;
  while ((2u << sh) <= lim && (1u << sh) < want) ++sh;
  const uint32_t nch = (H + (1u << sh) - 1) >> sh;
  if (mx > CAP || nch + 1 > NB) {
    if (lead && t == 0) b.meta->fallback = 1u;
    return false;
  }
  if (lead) {
    for (uint32_t c = t; c <= nch; c += BSC_NT) b.chunk[c] = H;
    __syncthreads();
    // bucket bin starts the chunks c with off[bin + 1] < c tgt <= off[bin]
#pragma unroll
    for (uint32_t i = 0; i < BPT; ++i) {
      const uint32_t bin = t * BPT + i;
      if (bin >= NB || bin < bstar) continue;
      const uint32_t o = loff[bs_pad(bin)];
      const uint32_t c1 = o >> sh;
      const uint32_t c0 = bin + 1 < NB ? (loff[bs_pad(bin + 1)] >> sh) + 1 : 0u;
      for (uint32_t c = c0; c <= c1; ++c) b.chunk[c] = o;
    }
    if (t == 0) {
      b.meta->bstar = bstar;
      b.meta->hot = H;
      b.meta->nchunk = nch;
      b.meta->fallback = 0u;
    }
  }
  bstar_out = bstar;
  return true;
}

// k_bscatter: each workgroup derives the offsets (bucket_offsets), counts its
// slice's hot survivors per bucket, reserves room in each hot bucket with one
// global atomic on the bucket's cursor (cleared by the sample launch), and
// places them.  Only the hot buckets (>= the boundary) are counted.
template <int KT, int RT>
__device__ __forceinline__ void bscatter_body(const BTailArgs& b, uint32_t* loff, uint32_t* lcnt,
                                              uint32_t* red) {
  using B = BT<KT, RT>;
  using U = typename B::U;
  using R = typename B::R;
  constexpr uint32_t NB = B::NB, BPT = (NB + BSC_NT - 1) / BSC_NT;
  const TailArgs1& a = b.t;
  const U* sk = static_cast<const U*>(a.sk);
  const R* sf = static_cast<const R*>(a.sf);
  const uint32_t t = threadIdx.x;
  // the survivors, the histogram and the query state, read together: every
  // load in flight at once, none waiting for the survivor count
  HeldSlice<U, R, BSC_NT> hs;
  hs.load(sk, sf, a.cap);
  {
    uint32_t c[BPT];
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t i = q * BSC_NT + t;
      c[q] = i < NB ? b.gh[i] : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t i = q * BSC_NT + t;
      if (i < NB) loff[bs_pad(i)] = c[q];
    }
  }
  const uint64_t C = a.h->surv_count;
  const typename B::T base = wide((U)a.h->thr_k, (R)a.h->thr_f);
  uint32_t bstar = 0;
  if (!bucket_offsets<KT, RT>(b, C, loff, red, bstar)) return;  // uniform
  const uint32_t nh = NB - bstar;
  for (uint32_t i = t; i < nh; i += BSC_NT) lcnt[i] = 0;
  uint32_t bk[BT_BATCH];
#pragma unroll
  for (int q = 0; q < BT_BATCH; ++q) bk[q] = B::bucket(hs.u[q], hs.f[q], base);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BT_BATCH; ++q)
    if (hs.valid(q, C) && bk[q] >= bstar) atomicAdd(&lcnt[bk[q] - bstar], 1u);
  hs.rest(sk, sf, C, [&](U u, R f) {
    const uint32_t k = B::bucket(u, f, base);
    if (k >= bstar) atomicAdd(&lcnt[k - bstar], 1u);
  });
  __syncthreads();
  // reserve room in each hot bucket: BT_BATCH atomics in flight per thread
  for (uint32_t i0 = t; i0 < nh; i0 += BT_BATCH * BSC_NT) {
    uint32_t c[BT_BATCH], r[BT_BATCH];
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint32_t i = i0 + (uint32_t)q * BSC_NT;
      c[q] = i < nh ? lcnt[i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint32_t i = i0 + (uint32_t)q * BSC_NT;
      r[q] = c[q] ? atomicAdd(&b.cur[bstar + i], c[q]) : 0u;
    }
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint32_t i = i0 + (uint32_t)q * BSC_NT;
      if (c[q]) lcnt[i] = loff[bs_pad(bstar + i)] + r[q];
    }
  }
  __syncthreads();
  U* hk = static_cast<U*>(b.hk);
  R* hf = static_cast<R*>(b.hf);
#pragma unroll
  for (int q = 0; q < BT_BATCH; ++q) {
    if (hs.valid(q, C) && bk[q] >= bstar) {
      const uint32_t pos = atomicAdd(&lcnt[bk[q] - bstar], 1u);
      hk[pos] = hs.u[q];
      hf[pos] = hs.f[q];
    }
  }
  hs.rest(sk, sf, C, [&](U u, R f) {
    const uint32_t k = B::bucket(u, f, base);
    if (k >= bstar) {
      const uint32_t pos = atomicAdd(&lcnt[k - bstar], 1u);
      hk[pos] = u;
      hf[pos] = f;
    }
  });
}

template <int KT, int RT>
__device__ __noinline__ void bsort_fallback(const TailArgs1 a, unsigned char* smem) {
  LdsTile<KT, RT>& t = *reinterpret_cast<LdsTile<KT, RT>*>(smem);
  SelScratch& sc =
      *reinterpret_cast<SelScratch*>(smem + (sizeof(LdsTile<KT, RT>) + 15) / 16 * 16);
  tail_body<KT, RT>(a, t, sc);
}

// Chunks up to BIN_SORT_MAX members are ordered without a sort network: an
// LDS histogram over (bucket, the BIN_G bits of the distance under the
// bucket's) -- at most BIN_COUNT bins, best first -- gives every bin its
// start, the members are scattered into bin order, and each ranks itself
// within its bin by counting the better members there (bins hold a member or
// two for spread-out keys).  A chunk whose largest bin exceeds BIN_MAX_FILL
// (keys tied on every bit the bins look at) keeps the sort network.
constexpr uint32_t BIN_SORT_MAX = 2048;
constexpr uint32_t BIN_COUNT = 4096;
constexpr int BIN_G = 10;
constexpr uint32_t BIN_MAX_FILL = 32;

// LDS of the bin sort, carved from the second half of the chunk's tile (the
// chunk itself sits in the first half): the histogram, then the scattered
// keys and flips, each region in whichever half has room.
template <typename U, typename R, uint32_t CAP>
struct BinLds {
  static constexpr size_t A = CAP / 2 * sizeof(U), B = CAP / 2 * sizeof(R);
  static constexpr size_t HIST = BIN_COUNT * 4, DK = BIN_SORT_MAX * sizeof(U),
                          DF = BIN_SORT_MAX * sizeof(R);
  static constexpr bool KEYS_IN_A = A >= HIST + DK;
  static_assert(KEYS_IN_A ? B >= DF : (A >= HIST && B >= DK + DF), "the bin sort fits its tile");
  uint32_t* hist;
  U* dk;
  R* df;
  __device__ BinLds(U* k, R* f) {
    unsigned char* a = reinterpret_cast<unsigned char*>(k + CAP / 2);
    unsigned char* bb = reinterpret_cast<unsigned char*>(f + CAP / 2);
    hist = reinterpret_cast<uint32_t*>(a);
    if (KEYS_IN_A) {
      dk = reinterpret_cast<U*>(a + HIST);
      df = reinterpret_cast<R*>(bb);
    } else {
      dk = reinterpret_cast<U*>(bb);
      df = reinterpret_cast<R*>(bb + DK);
    }
  }
};

// The chunk's m members (tile.k/f [0, m), buckets in order, best first) at
// their ranks: emit(rank, u, f).  Returns false, having emitted nothing, when
// a bin is too full (then the caller sorts the chunk).  Every thread calls it.
template <int KT, int RT, int NT, typename Emit>
__device__ __forceinline__ bool bin_sort_emit(uint32_t m, LdsTile<KT, RT>& tile,
                                              typename BT<KT, RT>::T base, uint32_t* red,
                                              Emit&& emit) {
  using B = BT<KT, RT>;
  using U = typename B::U;
  using R = typename B::R;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  constexpr int E = (int)((BIN_SORT_MAX + NT - 1) / NT);
  static_assert(BIN_SORT_MAX <= CAP / 2, "the chunk and the bin sort's regions share the tile");
  const BinLds<U, R, CAP> L(tile.k, tile.f);
  const uint32_t t = threadIdx.x;
  // buckets of the chunk: the first member is in its best, the last in its worst
  const uint32_t bhi = B::bucket(tile.k[0], tile.f[0], base);
  const uint32_t blo = B::bucket(tile.k[m - 1], tile.f[m - 1], base);
  const uint32_t nbk = bhi - blo + 1;
  int G = BIN_G;
  while (G > 0 && (nbk << G) > BIN_COUNT) --G;
  const uint32_t nbin = nbk << G;
  if (nbin > BIN_COUNT) return false;
  for (uint32_t i = t; i < nbin; i += NT) L.hist[i] = 0;
  if (t == 0) red[48] = 0u;
  __syncthreads();
  uint32_t bin[E], slot[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t i = (uint32_t)e * NT + t;
    if (i < m) {
      const U u = tile.k[i];
      const R f = tile.f[i];
      const uint32_t bk = B::bucket(u, f, base);
      const uint32_t sd = B::subdigit(u, f, base, G);
      if (bk < blo || bk > bhi) {  // not in bucket order: leave the chunk to the sort
        red[48] = 1u;
        bin[e] = 0u;
        continue;
      }
      bin[e] = ((bhi - bk) << G) | (((1u << G) - 1u) - sd);  // best bin first
      slot[e] = atomicAdd(&L.hist[bin[e]], 1u);
    }
  }
  __syncthreads();
  if (red[48] != 0u) return false;  // uniform: read after the barrier by every thread
  // exclusive scan of the bins, BPT consecutive bins per thread; the fullest bin
  constexpr uint32_t BPT = BIN_COUNT / NT;
  uint32_t c[BPT], s = 0, mx = 0;
#pragma unroll
  for (uint32_t q = 0; q < BPT; ++q) {
    const uint32_t i = t * BPT + q;
    c[q] = i < nbin ? L.hist[i] : 0u;
    s += c[q];
    mx = c[q] > mx ? c[q] : mx;
  }
  mx = wave_max(mx);
  if (lane_id() == 0) red[32 + (t >> 6)] = mx;
  uint32_t tot = 0;
  uint32_t off = block_excl_scan<NT>(s, red, tot);  // its barriers order the red writes
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) mx = red[32 + i] > mx ? red[32 + i] : mx;
  if (mx > BIN_MAX_FILL) return false;  // uniform: every thread read the same maxima
#pragma unroll
  for (uint32_t q = 0; q < BPT; ++q) {
    const uint32_t i = t * BPT + q;
    if (i < nbin) L.hist[i] = off;
    off += c[q];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t i = (uint32_t)e * NT + t;
    if (i < m) {
      const uint32_t p = L.hist[bin[e]] + slot[e];
      L.dk[p] = tile.k[i];
      L.df[p] = tile.f[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t i = (uint32_t)e * NT + t;
    if (i < m) {
      const uint32_t st = L.hist[bin[e]];
      const uint32_t p = st + slot[e];
      const uint32_t en = bin[e] + 1 < nbin ? L.hist[bin[e] + 1] : m;
      const U u = L.dk[p];
      const R f = L.df[p];
      uint32_t r = st;
      for (uint32_t q = st; q < en; ++q) {
        const U uq = L.dk[q];
        const R fq = L.df[q];
        r += (uq > u || (uq == u && (fq > f || (fq == f && q < p)))) ? 1u : 0u;
      }
      emit(r, u, f);
    }
  }
  __syncthreads();
  return true;
}

template <int KT, int RT>
__device__ __forceinline__ void bsort_body(const BTailArgs& b, unsigned char* smem) {
  using B = BT<KT, RT>;
  using U = typename B::U;
  using R = typename B::R;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const TailArgs1& a = b.t;
  if (b.meta->fallback) {
    if (blockIdx.x == 0) bsort_fallback<KT, RT>(a, smem);
    return;
  }
  LdsTile<KT, RT>& tile = *reinterpret_cast<LdsTile<KT, RT>*>(smem);
  SelScratch& sc =
      *reinterpret_cast<SelScratch*>(smem + (sizeof(LdsTile<KT, RT>) + 15) / 16 * 16);
  const typename B::T base = wide((U)a.h->thr_k, (R)a.h->thr_f);
  const uint32_t nch = b.meta->nchunk;
  const uint64_t K = a.k_eff;
  const U dmask = (U)a.dmask;
  void* const ok = a.out_keys;
  void* const orr = a.out_rids;
  const U* hk = static_cast<const U*>(b.hk);
  const R* hf = static_cast<const R*>(b.hf);
  for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t o = b.chunk[c];
    const uint32_t e = b.chunk[c + 1];
    if (o >= e || o >= K) continue;
    const uint32_t m = e - o;  // <= CAP by construction of the chunks
    for (uint32_t i = threadIdx.x; i < m; i += TAIL_NT) {
      tile.k[i] = hk[o + i];
      tile.f[i] = hf[o + i];
    }
    __syncthreads();
    auto emit = [=](uint64_t j, U u, R f) {
      if (o + j < K) write_out<KT, RT>(o + j, u, f, dmask, ok, orr);
    };
    if (m > BIN_SORT_MAX ||
        !bin_sort_emit<KT, RT, TAIL_NT>(m, tile, base, reinterpret_cast<uint32_t*>(sc.hist), emit))
      block_sort_emit<TAIL_NT, U, R>(m, true, tile.k, tile.f, CAP, nullptr, nullptr, nullptr,
                                     nullptr, emit);
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.h->path = 6u;
}

}  // namespace tk
