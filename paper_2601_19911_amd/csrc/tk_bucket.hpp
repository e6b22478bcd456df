// Tail of the sampled single query for large K: the exact best K of the
// filter's survivors, over the whole GPU.
//
//   k_bhist     workgroups take slices of the survivors and count them by a
//               logarithmic bucket of their distance D = c - T to the
//               threshold (c the composite read as one wide integer, 2^s
//               buckets per octave: tk_wide.hpp), first in LDS, then added
//               into the query's global histogram (cleared by the sample
//               launch).  Few workgroups: every bucket counter they share
//               takes one atomic from each.
//   k_bscatter  every workgroup derives from the histogram the boundary
//               bucket b* holding rank K and the exclusive offset of every
//               bucket, reserves room in each hot bucket (b >= b*) for its
//               slice of the survivors with one global atomic per bucket, and
//               scatters its hot survivors there: the hot set grouped by
//               bucket, best bucket first.  Workgroup 0 also cuts the hot set
//               into chunks of whole buckets that fit one LDS tile.
//   k_bsort     each workgroup sorts chunks in LDS and writes every member at
//               chunk offset + rank, up to K.
// The bucket is monotone in the composite, so a chunk's members take the
// output positions [offset, offset + size).  A query this path cannot finish
// (survivor count outside [K, capacity], or a hot bucket larger than one LDS
// tile) is finished by workgroup 0 of k_bsort with the one-workgroup select +
// sort.
#pragma once

#include "tk_rank.hpp"

namespace tk {

constexpr int BT_NT = 256;           // k_bhist, k_bscatter
constexpr uint32_t BT_SLICES = 128;  // workgroups of k_bhist
constexpr uint32_t BT_SCATTER = 256; // workgroups of k_bscatter
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

// Visits survivors j = blockIdx.x * BT_NT + threadIdx.x + i * stride below C,
// BT_BATCH at a time: the loads of a batch are issued before any is used.
constexpr int BT_BATCH = 8;
template <typename U, typename R, typename Fn>
__device__ __forceinline__ void bt_slice(const U* sk, const R* sf, uint64_t C, Fn&& fn) {
  const uint64_t stride = (uint64_t)gridDim.x * BT_NT;
  for (uint64_t j0 = (uint64_t)blockIdx.x * BT_NT + threadIdx.x; j0 < C; j0 += BT_BATCH * stride) {
    U u[BT_BATCH];
    R f[BT_BATCH];
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint64_t j = j0 + (uint64_t)q * stride;
      u[q] = j < C ? sk[j] : (U)0;
      f[q] = j < C ? sf[j] : (R)0;
    }
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q)
      if (j0 + (uint64_t)q * stride < C) fn(u[q], f[q]);
  }
}

template <int KT, int RT>
__device__ __forceinline__ void bhist_body(const BTailArgs& b, uint32_t* lh) {
  using B = BT<KT, RT>;
  using U = typename B::U;
  using R = typename B::R;
  constexpr uint32_t NB = B::NB;
  const TailArgs1& a = b.t;
  const uint64_t C = a.h->surv_count;
  if (!(C >= a.k_eff && C <= a.cap)) return;  // uniform; k_bscatter flags the fallback
  const uint32_t t = threadIdx.x;
  for (uint32_t i = t; i < NB; i += BT_NT) lh[i] = 0;
  const typename B::T base = wide((U)a.h->thr_k, (R)a.h->thr_f);
  const U* sk = static_cast<const U*>(a.sk);
  const R* sf = static_cast<const R*>(a.sf);
  __syncthreads();
  bt_slice(sk, sf, C, [&](U u, R f) { atomicAdd(&lh[B::bucket(u, f, base)], 1u); });
  __syncthreads();
  for (uint32_t i = t; i < NB; i += BT_NT) {
    const uint32_t c = lh[i];
    if (c) atomicAdd(&b.gh[i], c);
  }
}

template <int KT, int RT>
__device__ __forceinline__ void bscatter_body(const BTailArgs& b, uint32_t* loff, uint32_t* lcnt,
                                              uint32_t* red) {
  using B = BT<KT, RT>;
  using U = typename B::U;
  using R = typename B::R;
  constexpr uint32_t NB = B::NB, BPT = (NB + BT_NT - 1) / BT_NT;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const TailArgs1& a = b.t;
  const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
  const uint64_t C = a.h->surv_count;
  const uint64_t K = a.k_eff;
  if (!(C >= K && C <= a.cap)) {
    if (blockIdx.x == 0 && t == 0) b.meta->fallback = 1u;
    return;
  }
  // the histogram into LDS: every load of the thread in flight at once
  {
    uint32_t c[BPT];
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t i = q * BT_NT + t;
      c[q] = i < NB ? b.gh[i] : 0u;
    }
#pragma unroll
    for (uint32_t q = 0; q < BPT; ++q) {
      const uint32_t i = q * BT_NT + t;
      if (i < NB) {
        loff[i] = c[q];
        lcnt[i] = 0;
      }
    }
  }
  __syncthreads();
  // suffix sums: thread t holds buckets [t BPT, t BPT + BPT)
  uint32_t s = 0;
  for (uint32_t i = 0; i < BPT; ++i) {
    const uint32_t bin = t * BPT + i;
    s += bin < NB ? loff[bin] : 0u;
  }
  uint32_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_down(x, o, 64);
    if (lane + (uint32_t)o < 64) x += y;
  }
  if (lane == 0) red[w] = x;
  __syncthreads();
  uint32_t above = x - s;
#pragma unroll
  for (int i = 0; i < BT_NT / 64; ++i) above += (uint32_t)i > w ? red[i] : 0u;
  // exclusive offsets (members of better buckets); a bucket is hot while its
  // offset is below K; the boundary bucket is the one that reaches K
  uint32_t mx = 0;
  for (int i = (int)BPT - 1; i >= 0; --i) {
    const uint32_t bin = t * BPT + (uint32_t)i;
    if (bin >= NB) continue;
    const uint32_t c = loff[bin];
    loff[bin] = above;
    if (above < K) mx = c > mx ? c : mx;
    if (above < K && K <= (uint64_t)above + c) {
      red[8] = bin;
      red[9] = above + c;
    }
    above += c;
  }
  mx = wave_max(mx);
  if (lane == 0) red[16 + w] = mx;
  __syncthreads();
  const uint32_t bstar = red[8], H = red[9];
#pragma unroll
  for (int i = 0; i < BT_NT / 64; ++i) mx = red[16 + i] > mx ? red[16 + i] : mx;
  // chunks of whole buckets: chunk c holds the buckets whose offset lies in
  // [c tgt, (c + 1) tgt), at most tgt - 1 + mx <= CAP members
  // tgt = 2^sh: about one chunk per k_bsort workgroup, and tgt - 1 + mx <= CAP
  const uint32_t want = (H + BT_GRID - 1) / BT_GRID;
  const uint32_t lim = mx <= CAP ? CAP - mx + 1 : 1u;
  uint32_t sh = 0;
  while ((2u << sh) <= lim && (1u << sh) < want) ++sh;
  const uint32_t nch = (H + (1u << sh) - 1) >> sh;
  if (mx > CAP || nch + 1 > NB) {
    if (blockIdx.x == 0 && t == 0) b.meta->fallback = 1u;
    return;
  }
  if (blockIdx.x == 0) {
    for (uint32_t c = t; c <= nch; c += BT_NT) b.chunk[c] = H;
    __syncthreads();
    // bucket bin starts the chunks c with off[bin + 1] < c tgt <= off[bin]
    for (uint32_t i = 0; i < BPT; ++i) {
      const uint32_t bin = t * BPT + i;
      if (bin >= NB || bin < bstar) continue;
      const uint32_t o = loff[bin];
      const uint32_t c1 = o >> sh;
      const uint32_t c0 = bin + 1 < NB ? (loff[bin + 1] >> sh) + 1 : 0u;
      for (uint32_t c = c0; c <= c1; ++c) b.chunk[c] = o;
    }
    if (t == 0) {
      b.meta->bstar = bstar;
      b.meta->hot = H;
      b.meta->nchunk = nch;
      b.meta->fallback = 0u;
    }
  }
  // this workgroup's slice: count its hot survivors per bucket, reserve room
  // in each bucket, then place them
  const typename B::T base = wide((U)a.h->thr_k, (R)a.h->thr_f);
  const U* sk = static_cast<const U*>(a.sk);
  const R* sf = static_cast<const R*>(a.sf);
  bt_slice(sk, sf, C, [&](U u, R f) {
    const uint32_t bk = B::bucket(u, f, base);
    if (bk >= bstar) atomicAdd(&lcnt[bk], 1u);
  });
  __syncthreads();
  // reserve room in each hot bucket: BT_BATCH atomics in flight per thread
  for (uint32_t i0 = bstar + t; i0 < NB; i0 += BT_BATCH * BT_NT) {
    uint32_t c[BT_BATCH], r[BT_BATCH];
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint32_t i = i0 + (uint32_t)q * BT_NT;
      c[q] = i < NB ? lcnt[i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint32_t i = i0 + (uint32_t)q * BT_NT;
      r[q] = c[q] ? atomicAdd(&b.cur[i], c[q]) : 0u;
    }
#pragma unroll
    for (int q = 0; q < BT_BATCH; ++q) {
      const uint32_t i = i0 + (uint32_t)q * BT_NT;
      if (c[q]) lcnt[i] = loff[i] + r[q];
    }
  }
  __syncthreads();
  U* hk = static_cast<U*>(b.hk);
  R* hf = static_cast<R*>(b.hf);
  bt_slice(sk, sf, C, [&](U u, R f) {
    const uint32_t bk = B::bucket(u, f, base);
    if (bk >= bstar) {
      const uint32_t pos = atomicAdd(&lcnt[bk], 1u);
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
    block_sort_emit<TAIL_NT, U, R>(m, true, tile.k, tile.f, CAP, nullptr, nullptr, nullptr,
                                   nullptr, emit);
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.h->path = 6u;
}

}  // namespace tk
