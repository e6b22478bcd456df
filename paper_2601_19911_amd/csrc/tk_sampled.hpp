// Device bodies of the sampled Top-K (ordering primitive, paper sec. III-A):
// the stratified sample and its threshold, the streaming filter, and the tail
// (exact select + sort of the survivors).  One query's work is described by
// argument records; the single-query kernels (tk_sampled.hip) and the batched
// kernels (tk_multi.hip) run the same bodies, a batched workgroup first
// looking up which query and which of its workgroups it is.
#pragma once

#include <hip/hip_runtime.h>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_internal.hpp"
#include "tk_plan.hpp"
#include "tk_select.hpp"
#include "tk_src.hpp"
#include "tk_wide.hpp"

namespace tk {

typedef uint32_t u32x4s __attribute__((ext_vector_type(4)));

constexpr int SAMP_NT = 256;
constexpr int FILT_NT = 256;
constexpr int TAIL_NT = 1024;

struct SampArgs {
  const void* keys;
  const void* rids;
  uint64_t n;
  uint64_t dmask;
  uint32_t S, r1;
  QHead* h;
  void* ck;
  void* cf;
  uint32_t nblk;  // sample workgroups of this query
  uint32_t clear_exact;  // 1: also clear the exact select's state in the query header (a
                         // single query whose misjudged sample is taken over by it)
  uint32_t* zero;  // nzero words the sample workgroups clear for later launches, or nullptr
  uint64_t nzero;
};

struct FiltArgs {
  const void* keys;
  const void* rids;
  uint64_t n;
  uint64_t dmask;
  QHead* h;
  void* sk;
  void* sf;
  uint64_t cap;
  uint32_t nblk;   // filter workgroups of this query
  uint32_t r1;     // sample rank of the threshold
  const void* ck;  // the sample's candidates: ncand composites (key images, flipped row-ids)
  const void* cf;
  uint32_t ncand;
  uint32_t pad;
};

struct TailArgs1 {
  const void* keys;
  const void* rids;
  uint64_t n;
  uint64_t dmask;
  QHead* h;
  void* sk;
  void* sf;
  uint64_t cap;
  void* ck;
  void* cf;
  void* tk;
  void* tf;
  uint64_t k_eff;
  void* out_keys;
  void* out_rids;
  uint32_t mode;   // TAIL_SURVIVORS or TAIL_INPUT
  uint32_t defer;  // 1: a misjudged sample is left to the cooperative exact select that
                   // follows (path 4 recorded, nothing written); 0: one workgroup selects
                   // over the input
};

// TAIL_SURVIVORS: select over the survivors of the filter (falling back to
// the input if their count is outside [K, capacity]); TAIL_INPUT: select
// over the whole input (small queries, and those the sample cannot serve).
constexpr uint32_t TAIL_SURVIVORS = 0, TAIL_INPUT = 1;

// ---- k_sample ----------------------------------------------------------------------------------

// 64 uniform bits from a chunk index: the SplitMix64 finalizer (Steele, Lea,
// Flood 2014) of the index times its increment.
__device__ __forceinline__ uint64_t sample_hash(uint64_t c) {
  uint64_t z = (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// ---- small sample ranks: a tournament instead of the radix select ------------------------------
//
// With r1 at most SMALL_R_MAX (and 8-byte composites), the r1 best of a
// workgroup's composites take no radix rounds: each lane sorts its few
// composites in registers, each wave pops its r1 best with r1 wave-wide maxima
// of the lanes' heads, and one wave ranks the waves' lists (at most 64
// entries, one per lane) by counting.  One barrier in all, where the radix
// select takes several per digit.
constexpr uint32_t SMALL_R_MAX = 16;

// The tournament shortens one query's latency for 8-byte composites.  With
// wider ones (two 64-bit words per DPP move and compare) the radix select was
// faster on MI355X by 2-3 us a launch, and in the batched launches, where
// thousands of sample workgroups share the device and throughput counts, it
// was faster for every width (float32: 88 + 13 against 106 + 18 us a batch).
template <typename U, typename R, bool LATENCY>
constexpr bool tournament_shape() {
  return LATENCY && sizeof(U) + sizeof(R) == 8;
}

// Wave-wide maximum through DPP lane moves (a few cycles each, where a
// shuffle goes through the LDS crossbar): xor 1 and xor 2 (quad
// permutations), the half-row and row mirrors (xor 4 and xor 8 once the quads
// and half-rows are uniform), then row 0 into row 1 and row 2 into row 3
// (broadcast of lane 15) and rows 0-1 into rows 2-3 (broadcast of lane 31):
// lane 63 ends up holding the maximum, which is read into every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_max_step(uint64_t v) {
  const uint32_t hi = (uint32_t)(v >> 32), lo = (uint32_t)v;
  const uint64_t w = ((uint64_t)dpp_move<CTRL, ROWS>(hi, hi) << 32) | dpp_move<CTRL, ROWS>(lo, lo);
  return w > v ? w : v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = dpp_max_step<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v = dpp_max_step<0x4E, 0xF>(v);   // quad_perm [2, 3, 0, 1]
  v = dpp_max_step<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_max_step<0x140, 0xF>(v);  // row_mirror
  v = dpp_max_step<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_max_step<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
  return ((uint64_t)hi << 32) | lo;
}

// odd-even transposition sort of a lane's E composites, best (largest) first
template <typename T, int E>
__device__ __forceinline__ void regs_sort_desc(T (&v)[E]) {
#pragma unroll
  for (int i = 0; i < E; ++i) {
#pragma unroll
    for (int j = i & 1; j + 1 < E; j += 2) {
      const T x = v[j], y = v[j + 1];
      v[j] = x < y ? y : x;
      v[j + 1] = x < y ? x : y;
    }
  }
}

// The r best 8-byte composites of a workgroup of NT threads, each holding E of
// them (padding: 0, the smallest composite), as a multiset: out (LDS, 64
// words) ends up holding them in rank order for ranks < r; lst is LDS of 64
// words for the waves' lists.  Every thread must call it (it holds barriers);
// on return the list is visible to all.
template <int NT, int E>
__device__ __forceinline__ void block_top_small(uint64_t (&v)[E], uint32_t r, uint64_t* out,
                                                uint64_t* lst) {
  constexpr uint32_t NW = NT / 64;
  static_assert(NW * SMALL_R_MAX <= 64, "the waves' lists fit one wave");
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  regs_sort_desc(v);
  for (uint32_t i = 0; i < r; ++i) {
    const uint64_t m = wave_max_u64(v[0]);
    const uint64_t hit = ballot(v[0] == m);
    if (lane == (uint32_t)__builtin_ctzll(hit)) {
#pragma unroll
      for (int e = 0; e + 1 < E; ++e) v[e] = v[e + 1];
      v[E - 1] = 0;
    }
    if (lane == 0) lst[w * r + i] = m;
  }
  __syncthreads();
  if (w == 0) {
    const uint32_t tot = NW * r;
    const uint64_t c = lane < tot ? lst[lane] : 0ull;
    uint32_t rank = 0;
#pragma unroll 4
    for (uint32_t j = 0; j < tot; ++j) {
      const uint64_t x = lst[j];
      rank += (x > c || (x == c && j < lane)) ? 1u : 0u;
    }
    if (lane < tot && rank < r) out[rank] = c;
  }
  __syncthreads();
}

// blk: this workgroup's index among the query's a.nblk sample workgroups.
// Each keeps the best r1 composites of its SAMPLE_PER_BLOCK sampled keys
// (the union of these holds the sample's best r1); the next launch selects
// the r1-th best of the union, so no workgroup hands data to another inside
// a kernel.  LATENCY: a single query's launch (the tournament may serve
// small r1), not a batched one.
template <int KT, int RT, bool LATENCY>
__device__ __forceinline__ void sample_body(const SampArgs& a, SelScratch& sc, uint32_t blk) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = SAMP_NT, E = SAMPLE_PER_BLOCK / SAMP_NT;
  QHead* h = a.h;
  if (blk == 0 && threadIdx.x == 0) {
    h->surv_count = 0;
    h->status = 0;
    h->path = 0;
  }
  if (a.zero)
    for (uint64_t i = (uint64_t)blk * NT + threadIdx.x; i < a.nzero; i += (uint64_t)a.nblk * NT)
      a.zero[i] = 0u;
  if (a.clear_exact) {  // the words of the header past the query state
    uint32_t* w = reinterpret_cast<uint32_t*>(reinterpret_cast<Header*>(h)) + sizeof(QHead) / 4;
    constexpr uint32_t NW = (uint32_t)((sizeof(Header) - sizeof(QHead)) / 4);
    for (uint32_t i = blk * NT + threadIdx.x; i < NW; i += a.nblk * NT) w[i] = 0u;
  }
  const InputSrc<KT, RT> src{(const typename Key<KT>::Raw*)a.keys, (const R*)a.rids, (U)a.dmask};
  // Chunk c of 16 keys lies at a pseudo-random offset inside stratum c (of
  // `stride` keys): a column periodic in the stride cannot line its extremes
  // up with every sampled chunk, as it could with one fixed offset.
  const uint64_t nchunks = a.S / SAMPLE_CHUNK;
  const uint64_t stride = a.n / nchunks;  // >= 16: n >= 16 * S
  const uint64_t span = stride - SAMPLE_CHUNK + 1;
  U k[E];
  R f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t j = (uint64_t)blk * SAMPLE_PER_BLOCK + (uint64_t)e * NT + threadIdx.x;
    const uint64_t c = j / SAMPLE_CHUNK;
    const uint64_t pos = c * stride + __umul64hi(sample_hash(c), span) + (j % SAMPLE_CHUNK);
    k[e] = src.key(pos);
    f[e] = src.flip(pos);
  }
  U* ck = static_cast<U*>(a.ck);
  R* cf = static_cast<R*>(a.cf);
  if constexpr (tournament_shape<U, R, LATENCY>()) {
    if (a.r1 <= SMALL_R_MAX) {
      uint64_t v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = wide(k[e], f[e]);
      uint64_t* sh = reinterpret_cast<uint64_t*>(sc.hist);  // 128 words: list, then result
      block_top_small<NT, E>(v, a.r1, sh + 64, sh);
      if (threadIdx.x < a.r1) {
        const uint64_t c = sh[64 + threadIdx.x];
        ck[(uint64_t)blk * a.r1 + threadIdx.x] = (U)(c >> 32);
        cf[(uint64_t)blk * a.r1 + threadIdx.x] = (R)c;
      }
      return;
    }
  }
  U lmin = k[0];
#pragma unroll
  for (int e = 1; e < E; ++e) lmin = k[e] < lmin ? k[e] : lmin;
  const U base = block_min<NT, U>(lmin, sc);
  const RegElems<U, R, E> el{k, f, E};
  const Sel<U, R> s = block_radix_select<NT, U, R>(el, a.r1, base, sc);
  block_compact_regs<NT, U, R, E>(el, s, a.r1, ck + (uint64_t)blk * a.r1,
                                  cf + (uint64_t)blk * a.r1, sc);
}

// ---- k_filter ----------------------------------------------------------------------------------

// Survivors of one filter workgroup are staged in LDS and appended to the
// query's survivor buffer with one global atomic at the end: a global atomic
// per wave that meets a survivor costs far more than the pass itself once the
// survivors number thousands.  A stage that fills up sends the rest straight
// to the buffer (one atomic per wave).
constexpr uint32_t FILT_STAGE = 1024;
static_assert(FILT_STAGE % FILT_NT == 0, "the final append covers the stage in whole rounds");

template <typename U, typename R>
struct SurvStage {
  U k[FILT_STAGE];
  R f[FILT_STAGE];
  uint32_t cnt;
  uint32_t pad;
  unsigned long long base;
};

template <typename U, typename R>
__device__ __forceinline__ void stage_survivor(bool pass, U kk, R ff, SurvStage<U, R>& st, QHead* h,
                                               U* sk, R* sf, uint64_t cap, const R* drids) {
  const uint64_t m = ballot(pass);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  uint32_t b = 0;
  if (lane_id() == leader) b = atomicAdd(&st.cnt, (uint32_t)__popcll(m));
  b = __shfl(b, (int)leader, 64);
  const uint32_t p = b + lanes_below(m);
  const bool spill = pass && p >= FILT_STAGE;
  if (pass && !spill) {
    st.k[p] = kk;
    st.f[p] = ff;
  }
  const uint64_t ms = ballot(spill);
  if (ms == 0) return;
  const uint32_t l2 = (uint32_t)__builtin_ctzll(ms);
  uint64_t g = 0;
  if (lane_id() == l2) g = atomicAdd(&h->surv_count, (unsigned long long)__popcll(ms));
  g = __shfl(g, (int)l2, 64);
  if (spill) {
    const uint64_t pos = g + lanes_below(ms);
    if (pos < cap) {
      sk[pos] = kk;
      sf[pos] = drids ? (R)~drids[ff] : ff;
    }
  }
}

// blk: this workgroup's index among the query's a.nblk filter workgroups,
// which stride over the query's tiles of NT * VEC * UNR keys.  Tiles start at
// the first 16-byte boundary of the key array; the keys before it and the
// ones after the last whole tile are read one per thread.
// The threshold: the r1-th best of the sample workgroups' candidates (at most
// SAMPLE_FINAL_MAX, held in registers), selected by one workgroup of FILT_NT
// threads in a launch of its own and recorded in the query state.
template <int KT, int RT, bool LATENCY>
__device__ __forceinline__ void sample_final_body(const FiltArgs& a, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = FILT_NT, EF = SAMPLE_FINAL_MAX / FILT_NT;
  const U* ck = static_cast<const U*>(a.ck);
  const R* cf = static_cast<const R*>(a.cf);
  U k2[EF];
  R f2[EF];
  int nv = 0;
  U cmin = (U)~(U)0;
#pragma unroll
  for (int e = 0; e < EF; ++e) {
    const uint32_t j = (uint32_t)e * NT + threadIdx.x;
    if (j < a.ncand) {
      k2[e] = ck[j];
      f2[e] = cf[j];
      nv = e + 1;
      cmin = k2[e] < cmin ? k2[e] : cmin;
    } else {
      k2[e] = 0;
      f2[e] = 0;
    }
  }
  U mk = (U)~(U)0;
  R mf = (R)~(R)0;
  bool done = false;
  if constexpr (tournament_shape<U, R, LATENCY>()) {
    if (a.r1 <= SMALL_R_MAX) {
      // the r1-th entry of the tournament's list (padding 0 never ranks above
      // a candidate it is not equal to)
      uint64_t v[EF];
#pragma unroll
      for (int e = 0; e < EF; ++e) v[e] = wide(k2[e], f2[e]);
      uint64_t* sh = reinterpret_cast<uint64_t*>(sc.hist);  // 128 words: list, then result
      block_top_small<NT, EF>(v, a.r1, sh + 64, sh);
      const uint64_t c = sh[64 + a.r1 - 1];
      mk = (U)(c >> 32);
      mf = (R)c;
      done = true;
    }
  }
  if (!done) {
    const U base = block_min<NT, U>(cmin, sc);
    const RegElems<U, R, EF> el{k2, f2, nv};
    const Sel<U, R> s = block_radix_select<NT, U, R>(el, a.r1, base, sc);
    // The threshold is the r1-th best candidate itself, the smallest of the
    // selected ones.  The select may stop with low digits unresolved (its
    // bucket held exactly the count needed); the prefix padded with zeros
    // would also admit every key between it and that candidate, which for
    // clustered keys (a presorted column) is a large share of the input.
    const U lo = s.base + s.P;
    const R lof = s.kind == SEL_KEY ? (R)0 : s.Pf;
#pragma unroll
    for (int e = 0; e < EF; ++e) {
      const bool in = e < nv && (k2[e] > lo || (k2[e] == lo && f2[e] >= lof));
      if (in && (k2[e] < mk || (k2[e] == mk && f2[e] < mf))) {
        mk = k2[e];
        mf = f2[e];
      }
    }
    block_min_comp<NT, U, R>(mk, mf, sc);
  }
  // candidates sharing the threshold's key: when they are most of them, keys
  // tied with the threshold are common and the streaming pass reads row-ids
  // along with the keys
  uint64_t ties = 0;
#pragma unroll
  for (int e = 0; e < EF; ++e) ties += (e < nv && k2[e] == mk) ? 1u : 0u;
  ties = wave_sum64(ties);
  __syncthreads();  // block_min_comp's reads of the scratch are done
  if (lane_id() == 0) sc.red[threadIdx.x >> 6] = ties;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) tot += sc.red[i];
    a.h->thr_k = (unsigned long long)mk;
    a.h->thr_f = (unsigned long long)mf;
    a.h->tie_heavy = 2 * tot >= a.ncand ? 1u : 0u;
  }
}

// Row-ids of VEC consecutive keys: 16-byte loads when the rows allow.
template <typename R, int VEC>
__device__ __forceinline__ void load_rowids(const R* p, bool aligned16, R (&out)[VEC]) {
  if constexpr ((VEC * sizeof(R)) % 16 == 0) {
    if (aligned16) {
      constexpr int NQ = (int)(VEC * sizeof(R) / 16);
#pragma unroll
      for (int c = 0; c < NQ; ++c) {
        const u32x4s q = __builtin_nontemporal_load(reinterpret_cast<const u32x4s*>(p) + c);
        if constexpr (sizeof(R) == 4) {
          out[4 * c] = q.x; out[4 * c + 1] = q.y; out[4 * c + 2] = q.z; out[4 * c + 3] = q.w;
        } else {
          out[2 * c] = (uint64_t)q.x | ((uint64_t)q.y << 32);
          out[2 * c + 1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
        }
      }
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < VEC; ++e) out[e] = p[e];
}

// Stages the survivors among one VEC-key vector of every lane of the wave:
// one LDS reservation for all of them; the ones past the stage go straight to
// the survivor buffer (one global reservation).
template <typename U, typename R, int VEC>
__device__ __forceinline__ void stage_vector(const bool (&pass)[VEC], const U (&kk)[VEC],
                                             const R (&ff)[VEC], SurvStage<U, R>& st, QHead* h,
                                             U* sk, R* sf, uint64_t cap, const R* drids) {
  uint64_t m[VEC];
  uint32_t pre[VEC], tot = 0;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    m[e] = ballot(pass[e]);
    pre[e] = tot;
    tot += (uint32_t)__popcll(m[e]);
  }
  if (tot == 0) return;
  uint32_t b = 0;
  if (lane_id() == 0) b = atomicAdd(&st.cnt, tot);
  b = __shfl(b, 0, 64);
  const uint32_t sb = b > FILT_STAGE ? b : FILT_STAGE;  // first position past the stage
  const uint32_t nspill = b + tot > sb ? b + tot - sb : 0u;
  uint64_t g = 0;
  if (nspill) {
    if (lane_id() == 0) g = atomicAdd(&h->surv_count, (unsigned long long)nspill);
    g = __shfl(g, 0, 64);
  }
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    if (!pass[e]) continue;
    const uint32_t p = b + pre[e] + lanes_below(m[e]);
    if (p < FILT_STAGE) {
      st.k[p] = kk[e];
      st.f[p] = ff[e];
    } else {
      const uint64_t pos = g + (p - sb);
      if (pos < cap) {
        sk[pos] = kk[e];
        sf[pos] = drids ? (R)~drids[ff[e]] : ff[e];
      }
    }
  }
}

// One tile of the streaming pass: UNR 16-byte nontemporal loads per thread
// (or one key per thread for VEC = 1), NT threads apart.
template <typename Raw, int VEC, int UNR, int NT>
__device__ __forceinline__ void load_key_tile(const Raw* keys, uint64_t base, Raw (&v)[UNR][VEC]) {
#pragma unroll
  for (int u = 0; u < UNR; ++u) {
    const uint64_t i0 = base + ((uint64_t)u * NT + threadIdx.x) * VEC;
    if constexpr (VEC * sizeof(Raw) == 16) {
      const u32x4s q = __builtin_nontemporal_load(reinterpret_cast<const u32x4s*>(keys + i0));
      if constexpr (sizeof(Raw) == 4) {
        v[u][0] = q.x; v[u][1] = q.y; v[u][2] = q.z; v[u][3] = q.w;
      } else {
        v[u][0] = (uint64_t)q.x | ((uint64_t)q.y << 32);
        v[u][1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
      }
    } else {
      v[u][0] = keys[i0];
    }
  }
}

template <int KT, int RT, int VEC, int UNR>
__device__ __forceinline__ void filter_body(const FiltArgs& a, uint32_t blk,
                                            SurvStage<typename Key<KT>::U, typename Rid<RT>::R>& st) {
  using Raw = typename Key<KT>::Raw;
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = FILT_NT;
  static_assert(VEC * sizeof(Raw) == 16 || VEC == 1, "vector loads are 16 bytes");
  if (threadIdx.x == 0) st.cnt = 0;
  __syncthreads();
  QHead* h = a.h;
  const U Tk = (U)h->thr_k;
  const R Tf = (R)h->thr_f;
  const R* rids = static_cast<const R*>(a.rids);
  const bool tie_rows = rids != nullptr && h->tie_heavy != 0;
  // Otherwise, explicit row-ids are looked up once per workgroup at the final
  // append: the stage holds the survivor's index, so a wave that reaches the
  // threshold does not wait on a scattered row-id load (needs indices that
  // fit a row-id)
  const R* drids = rids != nullptr && !tie_rows && (sizeof(R) == 8 || a.n <= (1ull << 32))
                       ? rids : nullptr;
  const Raw* keys = static_cast<const Raw*>(a.keys);
  const InputSrc<KT, RT> src{keys, (const R*)a.rids, (U)a.dmask};
  const U dmask = (U)a.dmask;
  U* sk = static_cast<U*>(a.sk);
  R* sf = static_cast<R*>(a.sf);
  constexpr uint64_t TILE = (uint64_t)NT * VEC * UNR;
  uint64_t head = VEC > 1 ? ((16u - ((uintptr_t)keys & 15u)) & 15u) / sizeof(Raw) : 0;
  if (head > a.n) head = a.n;
  // every lane's row-id vector starts head + a multiple of VEC rows in
  const bool ralign = rids != nullptr && (((uintptr_t)(rids + head)) & 15u) == 0;
  const uint64_t ntiles = (a.n - head) / TILE;
  // tile t + nblk is loaded while tile t is checked: twice the bytes in
  // flight per wave at the same occupancy
  // (and, when row-ids go with the keys, its row-ids likewise)
  Raw v[UNR][VEC];
  R rv[UNR][VEC];
  auto load_rows = [=](uint64_t b, R (&r)[UNR][VEC]) {
#pragma unroll
    for (int u = 0; u < UNR; ++u)
      load_rowids<R, VEC>(rids + b + ((uint64_t)u * NT + threadIdx.x) * VEC, ralign, r[u]);
  };
  if (blk < ntiles) {
    load_key_tile<Raw, VEC, UNR, NT>(keys, head + blk * TILE, v);
    if (tie_rows) load_rows(head + blk * TILE, rv);
  }
  for (uint64_t t = blk; t < ntiles; t += a.nblk) {
    const uint64_t base = head + t * TILE;
    Raw nv[UNR][VEC];
    R nrv[UNR][VEC];
    if (t + a.nblk < ntiles) {
      load_key_tile<Raw, VEC, UNR, NT>(keys, base + a.nblk * TILE, nv);
      if (tie_rows) load_rows(base + a.nblk * TILE, nrv);
    }
    bool any = false;
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) any |= (Key<KT>::enc(v[u][e]) ^ dmask) >= Tk;
    if (ballot(any) != 0) {
      // A vector some lane of the wave reaches the threshold with.  When a key
      // of the wave ties with the threshold (common in skewed columns) the
      // row-ids of the whole vector are read at once, coalesced; otherwise only
      // the lanes above the threshold read theirs.  Then survivors are staged.
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        U kk[VEC];
        bool hit = false, tie = false;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          kk[e] = Key<KT>::enc(v[u][e]) ^ dmask;
          hit |= kk[e] >= Tk;
          tie |= kk[e] == Tk;
        }
        if (ballot(hit) == 0) continue;
        const uint64_t i0 = base + ((uint64_t)u * NT + threadIdx.x) * VEC;
        R ff[VEC];
        bool pass[VEC];
        bool pv = false;
        if (tie_rows) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) ff[e] = ~rv[u][e];
        } else if (ballot(tie)) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) ff[e] = src.flip(i0 + e);
        } else if (!drids) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) ff[e] = kk[e] > Tk ? src.flip(i0 + e) : (R)0;
        } else {  // no key of the wave ties: the key alone decides
#pragma unroll
          for (int e = 0; e < VEC; ++e) ff[e] = (R)0;
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          pass[e] = kk[e] > Tk || (kk[e] == Tk && ff[e] >= Tf);
          pv |= pass[e];
        }
        if (ballot(pv) == 0) continue;
        if (drids) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) ff[e] = (R)(i0 + e);
        }
        stage_vector<U, R, VEC>(pass, kk, ff, st, h, sk, sf, a.cap, drids);
      }
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        v[u][e] = nv[u][e];
        if (tie_rows) rv[u][e] = nrv[u][e];
      }
  }
  // the head and the remainder (fewer than VEC + TILE keys), one per thread:
  // position p < head is key p, the others follow the last whole tile
  const uint64_t tail0 = head + ntiles * TILE;
  const uint64_t nrest = head + (a.n - tail0);
  const uint64_t stride = (uint64_t)a.nblk * NT;
  for (uint64_t p0 = (uint64_t)blk * NT; p0 < nrest; p0 += stride) {
    const uint64_t p = p0 + threadIdx.x;
    bool pass = false;
    U kk = 0;
    R ff = 0;
    if (p < nrest) {
      const uint64_t i = p < head ? p : tail0 + (p - head);
      kk = src.key(i);
      pass = kk > Tk;
      if (kk >= Tk) {
        ff = src.flip(i);
        pass = pass || ff >= Tf;
      }
      if (drids) ff = (R)i;
    }
    stage_survivor<U, R>(pass, kk, ff, st, h, sk, sf, a.cap, drids);
  }
  // append the stage to the query's survivor buffer: the whole stage's
  // row-id loads and the reservation in the buffer in flight together
  __syncthreads();
  const uint32_t c = st.cnt < FILT_STAGE ? st.cnt : FILT_STAGE;
  constexpr int FL = FILT_STAGE / NT;
  R fv[FL];
#pragma unroll
  for (int q = 0; q < FL; ++q) {
    const uint32_t j = (uint32_t)q * NT + threadIdx.x;
    if (j < c) fv[q] = drids ? (R)~drids[st.f[j]] : st.f[j];
  }
  if (threadIdx.x == 0) st.base = c ? atomicAdd(&h->surv_count, (unsigned long long)c) : 0ull;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < FL; ++q) {
    const uint32_t j = (uint32_t)q * NT + threadIdx.x;
    const uint64_t pos = st.base + j;
    if (j < c && pos < a.cap) {
      sk[pos] = st.k[j];
      sf[pos] = fv[q];
    }
  }
}

// ---- k_tail ------------------------------------------------------------------------------------

// Where a tail writes its results (scalars, so the kernel arguments stay in
// registers on the fast path).
struct TailOut {
  uint64_t k_eff, dmask;
  void *out_keys, *out_rids, *ck, *cf, *tk, *tf;
};

// Select + sort over an array in global memory (survivors beyond the register
// capacity, or the whole input when the sample misjudged): out of line, so
// its registers do not weigh on the register-resident fast path.
template <int KT, int RT, typename Src>
__device__ __noinline__ void select_sort_write(const Src src, uint64_t n, typename Key<KT>::U base,
                                               const TailOut o, LdsTile<KT, RT>& t, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = TAIL_NT;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const U dmask = (U)o.dmask;
  void* const ok = o.out_keys;
  void* const orr = o.out_rids;
  // captures by value: a reference to the arguments handed to the out-of-line
  // sort would move them to scratch and serialize every load behind them
  auto emit = [=](uint64_t j, U u, R f) { write_out<KT, RT>(j, u, f, dmask, ok, orr); };
  const GlobElems<NT, Src> el{src, n};
  const Sel<U, R> s = block_radix_select<NT, U, R>(el, o.k_eff, base, sc);
  if (o.k_eff <= CAP) {
    block_compact_glob<NT, U, R>(src, n, s, o.k_eff, t.k, t.f, sc);
    block_sort_emit<NT, U, R>(o.k_eff, true, t.k, t.f, CAP, nullptr, nullptr, nullptr, nullptr, emit);
  } else {
    U* ck = static_cast<U*>(o.ck);
    R* cf = static_cast<R*>(o.cf);
    block_compact_glob<NT, U, R>(src, n, s, o.k_eff, ck, cf, sc);
    block_sort_emit<NT, U, R>(o.k_eff, false, t.k, t.f, CAP, ck, cf, static_cast<U*>(o.tk),
                              static_cast<R*>(o.tf), emit);
  }
}

__device__ __forceinline__ TailOut tail_out(const TailArgs1& a) {
  return TailOut{a.k_eff, a.dmask, a.out_keys, a.out_rids, a.ck, a.cf, a.tk, a.tf};
}

// Survivors that fit the registers of the workgroup (16 per thread) are
// loaded once and selected there.
constexpr int TAIL_E = 16;

template <int KT, int RT, typename Src>
__device__ __forceinline__ void select_sort_write_regs(const TailArgs1& a, const Src& src, uint32_t C,
                                                       typename Key<KT>::U base, LdsTile<KT, RT>& t,
                                                       SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = TAIL_NT, E = TAIL_E;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const U dmask = (U)a.dmask;
  U k[E];
  R f[E];
  int nv = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t j = (uint32_t)e * NT + threadIdx.x;
    if (j < C) {
      k[e] = src.key(j);
      f[e] = src.flip(j);
      nv = e + 1;
    } else {
      k[e] = 0;
      f[e] = 0;
    }
  }
  if (base == (U)~(U)0) {  // the caller did not know a lower bound: use the minimum
    U lmin = (U)~(U)0;
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (e < nv) lmin = k[e] < lmin ? k[e] : lmin;
    base = block_min<NT, U>(lmin, sc);
  }
  void* const ok = a.out_keys;
  void* const orr = a.out_rids;
  auto emit = [=](uint64_t j, U u, R f_) { write_out<KT, RT>(j, u, f_, dmask, ok, orr); };
  const RegElems<U, R, E> el{k, f, nv};
  const Sel<U, R> s = block_radix_select<NT, U, R>(el, a.k_eff, base, sc);
  if (a.k_eff <= CAP) {
    block_compact_regs<NT, U, R, E>(el, s, a.k_eff, t.k, t.f, sc);
    block_sort_emit<NT, U, R>(a.k_eff, true, t.k, t.f, CAP, nullptr, nullptr, nullptr, nullptr, emit);
  } else {
    U* ck = static_cast<U*>(a.ck);
    R* cf = static_cast<R*>(a.cf);
    block_compact_regs<NT, U, R, E>(el, s, a.k_eff, ck, cf, sc);
    block_sort_emit<NT, U, R>(a.k_eff, false, t.k, t.f, CAP, ck, cf, static_cast<U*>(a.tk),
                              static_cast<R*>(a.tf), emit);
  }
}

template <int KT, int RT>
__device__ __forceinline__ void tail_body(const TailArgs1& a, LdsTile<KT, RT>& t, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  const InputSrc<KT, RT> in{(const typename Key<KT>::Raw*)a.keys, (const R*)a.rids, (U)a.dmask};
  if (a.mode == TAIL_INPUT) {
    if (a.n <= (uint64_t)TAIL_NT * TAIL_E) select_sort_write_regs<KT, RT>(a, in, (uint32_t)a.n, (U)~(U)0, t, sc);
    else select_sort_write<KT, RT>(in, a.n, (U)0, tail_out(a), t, sc);
    if (a.h && threadIdx.x == 0) {  // a single query's header (the batched form passes none)
      a.h->path = 8u;
      a.h->status = 0u;
    }
    return;
  }
  QHead* h = a.h;
  const uint64_t C = h->surv_count;
  const bool ok = C >= a.k_eff && C <= a.cap;
  if (ok && C <= (uint64_t)TAIL_NT * TAIL_E) {
    const BufSrc<U, R> src{static_cast<const U*>(a.sk), static_cast<const R*>(a.sf)};
    select_sort_write_regs<KT, RT>(a, src, (uint32_t)C, (U)h->thr_k, t, sc);
  } else if (ok) {
    const BufSrc<U, R> src{static_cast<const U*>(a.sk), static_cast<const R*>(a.sf)};
    select_sort_write<KT, RT>(src, C, (U)h->thr_k, tail_out(a), t, sc);
  } else if (!a.defer) {
    select_sort_write<KT, RT>(in, a.n, (U)0, tail_out(a), t, sc);
  }
  // path 4 with defer set hands the query to the cooperative exact select
  if (threadIdx.x == 0) h->path = ok ? 2u : 4u;
}

}  // namespace tk
