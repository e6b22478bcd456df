// Tail of the sampled single query over many workgroups: the exact best K
// of the filter's survivors, written in order, without a sort.
//
// Every survivor is at or above the sampled threshold T.  Each workgroup
//   1. loads all C survivors into registers and builds an LDS histogram of
//      a logarithmic bucket of their distance D = c - T (c the composite,
//      key image above flipped row-id, read as one wide integer): 64 exact
//      buckets for D < 64, then 32 per octave.  The bucket is monotone in the
//      composite, so everything better than an element lies in its bucket or
//      above;
//   2. finds the boundary bucket b*, the one holding rank K counted from the
//      top, and collects the hot set H (bucket >= b*, |H| >= K) in LDS;
//   3. counts, for each hot survivor it owns (a range of survivor indices),
//      the members of H better than it: that count is the survivor's rank,
//      and ranks below K are its output position.  Identical composites
//      (possible only with repeated row-ids) are ordered by survivor index.
// All workgroups build the same H, so the ranks agree and each output slot is
// written exactly once.  The histogram keeps H near K + C/64 for spread-out
// keys; ties on the key are split by the row-id bits of D.  A query outside
// this path's limits (survivors beyond the register capacity, or a hot set
// beyond the LDS capacity) is finished by workgroup 0 with the one-workgroup
// select + sort.
#pragma once

#include "tk_sampled.hpp"

namespace tk {

constexpr int RANK_NT = 1024;
constexpr uint32_t RANK_E = 16;                    // survivors per thread
constexpr uint32_t RANK_CMAX = RANK_NT * RANK_E;  // survivors one workgroup holds
constexpr uint32_t RANK_HMAX = 4096;               // hot set capacity
constexpr uint32_t RANK_GMIN = 16, RANK_GMAX = 64;
constexpr uint32_t RANK_MMAX = (RANK_CMAX + RANK_GMIN - 1) / RANK_GMIN;  // owned per workgroup

template <int KT, int RT>
struct RankLds {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  static constexpr uint32_t NB = 32u * Wide<U, R>::W - 128u;
  using T = typename Wide<U, R>::T;
  T hw[RANK_HMAX];             // hot composites, as one wide integer each
  uint32_t hist[NB];
  uint32_t hi[RANK_HMAX];      // survivor index
  uint32_t mine[RANK_MMAX];    // hot-set slots this workgroup ranks
  uint32_t gt[RANK_MMAX];      // members of H better than it
  uint32_t eq[RANK_MMAX];      // members of H equal to it (itself included)
  uint32_t wsum[RANK_NT / 64];
  unsigned long long redk[RANK_NT / 64], redf[RANK_NT / 64];  // minimum of the input
  uint32_t bstar, hcount;
};

// Bytes of LDS for the tail kernel: the rank state, or the one-workgroup
// select + sort state (tile, then scratch at a 16-byte boundary).
template <int KT, int RT>
constexpr size_t rank_smem_bytes() {
  const size_t tile = (sizeof(LdsTile<KT, RT>) + 15) / 16 * 16 + sizeof(SelScratch);
  return sizeof(RankLds<KT, RT>) > tile ? sizeof(RankLds<KT, RT>) : tile;
}

template <int KT, int RT>
__device__ __noinline__ void rank_tail_fallback(const TailArgs1 a, unsigned char* smem) {
  LdsTile<KT, RT>& t = *reinterpret_cast<LdsTile<KT, RT>*>(smem);
  SelScratch& sc =
      *reinterpret_cast<SelScratch*>(smem + (sizeof(LdsTile<KT, RT>) + 15) / 16 * 16);
  tail_body<KT, RT>(a, t, sc);
}

// The tail over G workgroups of RANK_NT threads, this one being workgroup me
// (a single query's launch: RANK_GMIN <= G <= RANK_GMAX; a batched launch: one
// workgroup, G = 1).  INPUT = false: over the filter's survivors
// (TAIL_SURVIVORS), distances taken from the threshold.  INPUT = true: over
// the whole input of a query with n <= RANK_CMAX (TAIL_INPUT), distances taken
// from the input's smallest composite; a.h may be null.  A query outside this
// path's limits is finished by workgroup 0 with the one-workgroup tail.
template <int KT, int RT, bool INPUT = false>
__device__ __forceinline__ void rank_tail_body(const TailArgs1& a, unsigned char* smem,
                                               uint32_t me, uint32_t G) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  using T = typename Wide<U, R>::T;
  using Lds = RankLds<KT, RT>;
  constexpr int NT = RANK_NT, E = (int)RANK_E;
  constexpr uint32_t NB = Lds::NB, BPT = (NB + NT - 1) / NT;
  QHead* h = a.h;
  Lds& L = *reinterpret_cast<Lds*>(smem);
  const uint32_t t = threadIdx.x, lane = lane_id(), w = t >> 6;
  // The survivor loads do not wait for the survivor count: every slot below
  // min(capacity, RANK_CMAX) is in the buffer, and slots past the count are
  // ignored.  The count decides after the histogram (which consumes the
  // loads) whether this path applies.
  const U* sk = static_cast<const U*>(a.sk);
  const R* sf = static_cast<const R*>(a.sf);
  const InputSrc<KT, RT> in{(const typename Key<KT>::Raw*)a.keys, (const R*)a.rids, (U)a.dmask};
  const uint32_t lim = INPUT ? (uint32_t)a.n
                             : (a.cap < (uint64_t)RANK_CMAX ? (uint32_t)a.cap : RANK_CMAX);
  U k[E];
  R f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t j = (uint32_t)e * NT + t;
    if constexpr (INPUT) {
      k[e] = j < lim ? in.key(j) : (U)0;
      f[e] = j < lim ? in.flip(j) : (R)0;
    } else {
      k[e] = j < lim ? sk[j] : (U)0;
      f[e] = j < lim ? sf[j] : (R)0;
    }
  }
  for (uint32_t i = t; i < NB; i += NT) L.hist[i] = 0;
  const uint64_t C64 = INPUT ? a.n : h->surv_count;
  const uint64_t K = a.k_eff;
  const bool ok = INPUT || (C64 >= K && C64 <= a.cap && C64 <= RANK_CMAX);
  const uint32_t C = ok ? (uint32_t)C64 : 0u;
  T base;
  if constexpr (INPUT) {
    // the smallest composite of the input: every distance is >= 0
    U mk = (U)~(U)0;
    R mf = (R)~(R)0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t j = (uint32_t)e * NT + t;
      if (j < C && (k[e] < mk || (k[e] == mk && f[e] < mf))) {
        mk = k[e];
        mf = f[e];
      }
    }
    const U wk = wave_min(mk);
    const R wf = wave_min(mk == wk ? mf : (R)~(R)0);
    if (lane == 0) {
      L.redk[w] = (unsigned long long)wk;
      L.redf[w] = (unsigned long long)wf;
    }
    __syncthreads();  // histogram cleared, wave minima written
    mk = (U)~(U)0;
    mf = (R)~(R)0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
      const U ck = (U)L.redk[i];
      const R cf = (R)L.redf[i];
      if (ck < mk || (ck == mk && cf < mf)) {
        mk = ck;
        mf = cf;
      }
    }
    base = wide(mk, mf);
  } else {
    base = wide((U)h->thr_k, (R)h->thr_f);
    __syncthreads();  // histogram cleared
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t j = (uint32_t)e * NT + t;
    if (j < C) atomicAdd(&L.hist[log_bucket_s<5, T>(wide(k[e], f[e]) - base)], 1u);
  }
  __syncthreads();
  if (!ok) {  // uniform; every thread is past its histogram updates (never with INPUT)
    if (me == 0) rank_tail_fallback<KT, RT>(a, smem);
    return;
  }
  // boundary bucket: thread t holds buckets [t BPT, t BPT + BPT); suffix sums
  // from the top find the one where the count reaches K
  uint32_t s = 0;
#pragma unroll
  for (uint32_t i = 0; i < BPT; ++i) {
    const uint32_t bin = t * BPT + i;
    s += bin < NB ? L.hist[bin] : 0u;
  }
  const uint32_t x = wave_suffix_sum(s);  // sum over lanes >= this one
  if (lane == 0) L.wsum[w] = x;
  __syncthreads();
  uint32_t above = x - s;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) above += (uint32_t)i > w ? L.wsum[i] : 0u;
  if (above < K && K <= (uint64_t)above + s) {
    uint32_t acc = above;
    for (int i = (int)BPT - 1; i >= 0; --i) {
      const uint32_t bin = t * BPT + (uint32_t)i;
      if (bin >= NB) continue;
      acc += L.hist[bin];
      if (acc >= K) {
        L.bstar = bin;
        L.hcount = acc;
        break;
      }
    }
  }
  __syncthreads();
  const uint32_t bstar = L.bstar, H = L.hcount;
  // workgroup me owns survivor indices [me * per, me * per + per); it ranks
  // its hot members among them, at most RANK_MMAX (always so on RANK_GMIN or
  // more workgroups; on one, the whole hot set must fit)
  const uint32_t per = (C + G - 1) / G, jlo = me * per, jhi = jlo + per;
  if (H > RANK_HMAX || (H < per ? H : per) > RANK_MMAX) {
    __syncthreads();  // every thread has read the boundary before the LDS is reused
    if (me == 0) rank_tail_fallback<KT, RT>(a, smem);
    return;
  }
  // the hot set, and the part of it this workgroup ranks: per-thread counts,
  // one block-wide exclusive scan of (hot << 16 | owned), then plain stores
  // hot iff D reaches the lower edge of the boundary bucket (the bucket is
  // monotone in D): D itself below 64, then (32 + sub) << (octave - 6)
  const T dlo = bstar < 64u ? (T)bstar
                            : (T)(32u + (bstar - 64u) % 32u) << ((bstar - 64u) / 32u + 1u);
  uint32_t hot_bits = 0, own_bits = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t j = (uint32_t)e * NT + t;
    const bool hot = j < C && wide(k[e], f[e]) - base >= dlo;
    hot_bits |= hot ? 1u << e : 0u;
    own_bits |= hot && j >= jlo && j < jhi ? 1u << e : 0u;
  }
  const uint32_t packed = ((uint32_t)__popc(hot_bits) << 16) | (uint32_t)__popc(own_bits);
  const uint32_t incl = wave_incl_scan(packed);  // inclusive scan over the lanes
  if (lane == 63) L.wsum[w] = incl;
  __syncthreads();
  uint32_t excl = incl - packed, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    const uint32_t v = L.wsum[i];
    excl += (uint32_t)i < w ? v : 0u;
    tot += v;
  }
  uint32_t pos = excl >> 16, qo = excl & 0xFFFFu;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (hot_bits & (1u << e)) {
      L.hw[pos] = wide(k[e], f[e]);
      L.hi[pos] = (uint32_t)e * NT + t;
      if (own_bits & (1u << e)) {
        L.mine[qo] = pos;
        L.gt[qo] = 0;
        L.eq[qo] = 1;  // itself
        ++qo;
      }
      ++pos;
    }
  }
  __syncthreads();
  // ranks: thread -> (owned element q, slice s of H), every thread busy
  const uint32_t M = tot & 0xFFFFu;
  if (M > 0) {
    const uint32_t Mr = M < (uint32_t)NT ? M : (uint32_t)NT;
    const uint32_t P = (uint32_t)NT / Mr;  // slices of H
    const uint32_t sl = t / Mr;
    const uint32_t hs = (H + P - 1) / P;
    const uint32_t j0 = sl * hs < H ? sl * hs : H;
    const uint32_t j1 = j0 + hs < H ? j0 + hs : H;
    for (uint32_t q0 = 0; q0 < M; q0 += Mr) {
      const uint32_t q = q0 + t % Mr;
      const bool act = sl < P && q < M;
      const uint32_t p = act ? L.mine[q] : 0u;
      const T ci = L.hw[p];
      uint32_t gt = 0, eq = 0;
      if (act) {
        for (uint32_t jj = j0; jj < j1; ++jj) {
          const T cj = L.hw[jj];
          gt += cj > ci ? 1u : 0u;
          eq += (cj == ci && jj != p) ? 1u : 0u;
        }
      }
      if (gt) atomicAdd(&L.gt[q], gt);
      if (eq) atomicAdd(&L.eq[q], eq);
    }
  }
  __syncthreads();
  const U dmask = (U)a.dmask;
  for (uint32_t q = t; q < M; q += NT) {
    const uint32_t p = L.mine[q];
    const T ci = L.hw[p];
    uint64_t rank = L.gt[q];
    if (L.eq[q] > 1) {  // identical composites: the lower survivor index goes first
      const uint32_t ii = L.hi[p];
      for (uint32_t jj = 0; jj < H; ++jj) rank += (L.hw[jj] == ci && L.hi[jj] < ii) ? 1u : 0u;
    }
    if (rank < K)
      write_out<KT, RT>(rank, (U)(ci >> (8 * sizeof(R))), (R)ci, dmask, a.out_keys, a.out_rids);
  }
  if (me == 0 && t == 0 && h) h->path = INPUT ? 7u : 3u;
}

// Workgroups of the tail for k results: enough that each ranks a few dozen
// hot survivors.
inline uint32_t rank_grid(uint64_t k_eff) {
  uint64_t g = (k_eff + 15) / 16;
  if (g < RANK_GMIN) g = RANK_GMIN;
  if (g > RANK_GMAX) g = RANK_GMAX;
  return (uint32_t)g;
}

}  // namespace tk
