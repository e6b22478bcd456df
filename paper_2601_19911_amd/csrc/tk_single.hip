// Single-query entry point of key-only Top-K (ordering primitive, paper
// sec. III-A) and the two paths that do not go through the engine:
//   - queries that fit one LDS tile: for K up to 2048 ranked across
//     workgroups over the whole input (k_rsmall, tk_rank.hpp); for larger K,
//     or as a tuning choice, by one workgroup (k_small): the keys are loaded
//     once, the best K found by radix select and bitonic-sorted in LDS;
//   - queries whose K is a large share of N (or forced, for tests): an exact
//     radix select over the whole input by a cooperative grid (k_tail with
//     exact_only): 8-bit digits of the key image from the top, then of the
//     flipped row-id, each digit found from a global histogram; then the
//     selected composites are sorted (one LDS tile, or tiles plus
//     merge-path merges).
// Every other query takes the sampled path (tk_sampled.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_internal.hpp"
#include "tk_plan.hpp"
#include "tk_rank.hpp"
#include "tk_select.hpp"
#include "tk_src.hpp"

namespace tk {

// ---- kernel 0: header reset (exact-only path) ----------------------------------------------

__global__ void k_init(Header* h) {
  uint32_t* w = reinterpret_cast<uint32_t*>(h);
  for (uint32_t i = threadIdx.x; i < sizeof(Header) / 4; i += blockDim.x) w[i] = 0u;
}

__device__ __forceinline__ void header_reset_block(Header* h) {
  uint32_t* w = reinterpret_cast<uint32_t*>(h);
  for (uint32_t i = threadIdx.x; i < sizeof(Header) / 4; i += blockDim.x) w[i] = 0u;
}

// ---- one-workgroup select + sort in LDS ------------------------------------------------------

// Selects the best k_eff of cnt (<= CAP) composites from `src` and writes them
// sorted to the outputs.  Whole workgroup of NT threads.
template <int KT, int RT, int NT, typename Src>
__device__ void lds_select_sort(const Src& src, uint32_t cnt, uint32_t k_eff,
                                typename Key<KT>::U dmask, void* out_keys, void* out_rids,
                                LdsTile<KT, RT>& t, uint64_t* red, uint32_t* ws) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  constexpr int E = CAP / NT;
  U k[E];
  R f[E];
  int nv = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t j = (uint32_t)e * NT + threadIdx.x;
    if (j < cnt) {
      k[e] = src.key(j);
      f[e] = src.flip(j);
      nv = e + 1;
    } else {
      k[e] = 0;
      f[e] = 0;
    }
  }
  int parity = 0;
  U Tk;
  R Tf;
  block_select<U, R, E, NT>(k, f, nv, k_eff, Tk, Tf, red, parity);
  block_emit_top<U, R, E, NT>(k, f, nv, k_eff, Tk, Tf, t.k, t.f, ws);
  uint32_t P = 1;
  while (P < k_eff) P <<= 1;
  for (uint32_t i = k_eff + threadIdx.x; i < P; i += NT) {
    t.k[i] = 0;
    t.f[i] = 0;
  }
  bitonic_desc<U, R, NT>(t.k, t.f, P);
  for (uint32_t j = threadIdx.x; j < k_eff; j += NT) write_out<KT, RT>(j, t.k[j], t.f[j], dmask, out_keys, out_rids);
}

// ---- kernel: whole query in one workgroup (n <= LDS capacity) -------------------------------

template <int KT, int RT>
__global__ __launch_bounds__(1024) void k_small(const typename Key<KT>::Raw* keys,
                                                const typename Rid<RT>::R* rids, uint32_t n,
                                                uint32_t k_eff, typename Key<KT>::U dmask,
                                                void* out_keys, void* out_rids) {
  constexpr int NT = 1024;
  __shared__ LdsTile<KT, RT> t;
  __shared__ uint64_t red[2 * NT / 64];
  __shared__ uint32_t ws[NT / 64];
  const InputSrc<KT, RT> src{keys, rids, dmask};
  lds_select_sort<KT, RT, NT>(src, n, k_eff, dmask, out_keys, out_rids, t, red, ws);
}

// ---- kernel: whole query ranked across workgroups (n <= LDS capacity) ----------------------

template <int KT, int RT>
__global__ __launch_bounds__(RANK_NT) void k_rsmall(TailArgs1 a) {
  __shared__ __align__(16) unsigned char smem[rank_smem_bytes<KT, RT>()];
  rank_tail_body<KT, RT, true>(a, smem, blockIdx.x, gridDim.x);
}

// ---- kernel 4: tail (cooperative) -----------------------------------------------------------

struct TailArgs {
  const void* keys;
  const void* rids;
  uint64_t n;
  uint64_t dmask;
  Header* h;
  void* ck;
  void* cf;
  void* tk;
  void* tf;
  uint64_t k_eff;
  void* out_keys;
  void* out_rids;
  int exact_only;
};

template <typename U, typename R>
struct SelState {
  U Pk;
  R Pf;
  uint64_t need;  // elements still to take from the boundary bucket
  int dup;        // 1: all bits resolved, `need` copies of (Pk, Pf) are taken
};

// Exact radix select over src[0..n) by all blocks: 8-bit digits of the key
// image from the top, then of the flipped row-id, each digit found from a
// global histogram.  Writes exactly k_eff composites to (ck, cf), unsorted.
// Returns false if a grid barrier failed.
template <int NT, typename U, typename R, typename Src>
__device__ bool exact_select(const Src& src, uint64_t n, uint64_t k_eff, Header* h, U* ck, R* cf,
                             uint32_t* lh, unsigned long long* lh64, uint32_t* sh_u32,
                             int* s_flag) {
  const uint32_t G = gridDim.x;
  const uint64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  constexpr int WU = (int)sizeof(U) * 8, WR = (int)sizeof(R) * 8;
  U Pk = 0, mk = 0;
  R Pf = 0, mf = 0;
  uint64_t need = k_eff;
  bool rid_phase = false;
  int shift = WU - 8;
  int dup = 0;
  for (int pass = 0;; ++pass) {
    for (uint32_t d = threadIdx.x; d < 256; d += NT) lh[d] = 0;
    __syncthreads();
    for (uint64_t i = lo + threadIdx.x; i < hi; i += NT) {
      const U u = src.key(i);
      if (!rid_phase) {
        if ((u & mk) == Pk) atomicAdd(&lh[(uint32_t)(u >> shift) & 0xFFu], 1u);
      } else if (u == Pk) {
        const R f = src.flip(i);
        if ((f & mf) == Pf) atomicAdd(&lh[(uint32_t)(f >> shift) & 0xFFu], 1u);
      }
    }
    __syncthreads();
    unsigned long long* gh = h->hist[pass % 3];
    for (uint32_t d = threadIdx.x; d < 256; d += NT)
      if (lh[d]) atomicAdd(&gh[d], (unsigned long long)lh[d]);
    if (!grid_sync(&h->gs, G, &h->q.status, s_flag)) return false;
    if (blockIdx.x == 0) {
      unsigned long long* old = h->hist[(pass + 2) % 3];
      for (uint32_t d = threadIdx.x; d < 256; d += NT) old[d] = 0;
    }
    for (uint32_t d = threadIdx.x; d < 256; d += NT)
      lh64[d] = __hip_atomic_load(&gh[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t cum = 0;
      int d = 255;
      for (; d > 0; --d) {
        if (cum + lh64[d] >= need) break;
        cum += lh64[d];
      }
      sh_u32[0] = (uint32_t)d;
      sh_u32[1] = (uint32_t)cum;
      sh_u32[2] = (uint32_t)(cum >> 32);
    }
    __syncthreads();
    const uint32_t d = sh_u32[0];
    const uint64_t above = (uint64_t)sh_u32[1] | ((uint64_t)sh_u32[2] << 32);
    const uint64_t bucket = lh64[d];
    __syncthreads();
    need -= above;
    if (!rid_phase) {
      Pk |= (U)d << shift;
      mk |= (U)0xFF << shift;
    } else {
      Pf |= (R)d << shift;
      mf |= (R)0xFF << shift;
    }
    if (bucket == need) break;  // the whole bucket is taken: boundary resolved
    if (shift == 0) {
      if (!rid_phase) {
        rid_phase = true;
        shift = WR - 8;
      } else {
        dup = 1;  // identical composites straddle the boundary
        break;
      }
    } else {
      shift -= 8;
    }
  }
  // compaction: c > B (or >= B when resolved) to the front, copies of B after
  const uint64_t n_gt = k_eff - need;
  const uint64_t gt_end = dup ? n_gt : k_eff;
  for (uint64_t i0 = lo; i0 < hi; i0 += NT) {
    const uint64_t i = i0 + threadIdx.x;
    bool take = false, eq = false;
    U u = 0;
    R f = 0;
    if (i < hi) {
      u = src.key(i);
      if (u >= Pk) {
        f = src.flip(i);
        if (dup) {
          take = cgt(u, f, Pk, Pf);
          eq = (u == Pk && f == Pf);
        } else {
          take = cge(u, f, Pk, Pf);
        }
      }
    }
    const uint64_t mt = ballot(take);
    if (mt) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(mt);
      uint64_t base = 0;
      if (lane_id() == leader) base = atomicAdd(&h->sel_gt, (unsigned long long)__popcll(mt));
      base = __shfl(base, (int)leader, 64);
      if (take) {
        const uint64_t pos = base + lanes_below(mt);
        if (pos < gt_end) {
          ck[pos] = u;
          cf[pos] = f;
        }
      }
    }
    const uint64_t me = ballot(eq);
    if (me) {
      const uint32_t leader = (uint32_t)__builtin_ctzll(me);
      uint64_t base = 0;
      if (lane_id() == leader) base = atomicAdd(&h->sel_eq, (unsigned long long)__popcll(me));
      base = __shfl(base, (int)leader, 64);
      if (eq) {
        const uint64_t pos = n_gt + base + lanes_below(me);
        if (pos < k_eff) {
          ck[pos] = u;
          cf[pos] = f;
        }
      }
    }
  }
  return grid_sync(&h->gs, G, &h->q.status, s_flag);
}

// Sorts ck/cf[0..m) best first with all blocks and writes the outputs.
template <int KT, int RT, int NT>
__device__ bool sort_and_write(uint64_t m, typename Key<KT>::U* ck, typename Rid<RT>::R* cf,
                               typename Key<KT>::U* tk, typename Rid<RT>::R* tf,
                               typename Key<KT>::U dmask, void* out_keys, void* out_rids,
                               Header* h, LdsTile<KT, RT>& t, int* s_flag) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const uint32_t G = gridDim.x;
  if (m <= CAP) {
    if (blockIdx.x != 0) return true;
    uint32_t P = 1;
    while (P < m) P <<= 1;
    for (uint32_t i = threadIdx.x; i < P; i += NT) {
      t.k[i] = i < m ? ck[i] : (U)0;
      t.f[i] = i < m ? cf[i] : (R)0;
    }
    bitonic_desc<U, R, NT>(t.k, t.f, P);
    for (uint32_t j = threadIdx.x; j < m; j += NT) write_out<KT, RT>(j, t.k[j], t.f[j], dmask, out_keys, out_rids);
    return true;
  }
  // 1) sort tiles of CAP in LDS
  const uint64_t ntiles = (m + CAP - 1) / CAP;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += G) {
    const uint64_t base = tile * CAP;
    const uint64_t len = m - base < CAP ? m - base : CAP;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < CAP; i += NT) {
      t.k[i] = i < len ? ck[base + i] : (U)0;
      t.f[i] = i < len ? cf[base + i] : (R)0;
    }
    bitonic_desc<U, R, NT>(t.k, t.f, CAP);
    for (uint32_t i = threadIdx.x; i < len; i += NT) {
      ck[base + i] = t.k[i];
      cf[base + i] = t.f[i];
    }
  }
  if (!grid_sync(&h->gs, G, &h->q.status, s_flag)) return false;
  // 2) merge runs pairwise until one run is left
  U* sk = ck;
  R* sf = cf;
  U* dk = tk;
  R* df = tf;
  constexpr uint64_t ITEMS = 8;
  for (uint64_t run = CAP; run < m; run <<= 1) {
    for (uint64_t o0 = ((uint64_t)blockIdx.x * NT + threadIdx.x) * ITEMS; o0 < m;
         o0 += (uint64_t)G * NT * ITEMS) {
      const uint64_t s = o0 / (2 * run) * (2 * run);
      const uint64_t amid = s + run < m ? s + run : m;
      const uint64_t aend = s + 2 * run < m ? s + 2 * run : m;
      const uint64_t na = amid - s, nb = aend - amid;
      const uint64_t d = o0 - s;
      uint64_t i = merge_split<U, R>(sk + s, sf + s, na, sk + amid, sf + amid, nb, d);
      uint64_t j = d - i;
      const uint64_t cnt = aend - o0 < ITEMS ? aend - o0 : ITEMS;
      for (uint64_t q = 0; q < cnt; ++q) {
        bool from_a;
        if (i >= na) from_a = false;
        else if (j >= nb) from_a = true;
        else from_a = cge(sk[s + i], sf[s + i], sk[amid + j], sf[amid + j]);
        if (from_a) {
          dk[o0 + q] = sk[s + i];
          df[o0 + q] = sf[s + i];
          ++i;
        } else {
          dk[o0 + q] = sk[amid + j];
          df[o0 + q] = sf[amid + j];
          ++j;
        }
      }
    }
    if (!grid_sync(&h->gs, G, &h->q.status, s_flag)) return false;
    U* xk = sk; sk = dk; dk = xk;
    R* xf = sf; sf = df; df = xf;
  }
  for (uint64_t j = (uint64_t)blockIdx.x * NT + threadIdx.x; j < m; j += (uint64_t)G * NT)
    write_out<KT, RT>(j, sk[j], sf[j], dmask, out_keys, out_rids);
  return true;
}

template <int KT, int RT>
__global__ __launch_bounds__(1024) void k_tail(TailArgs a) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = 1024;
  __shared__ LdsTile<KT, RT> t;
  __shared__ uint64_t red[2 * NT / 64];
  __shared__ uint32_t ws[NT / 64];
  __shared__ uint32_t lh[256];
  __shared__ unsigned long long lh64[256];
  __shared__ uint32_t sh_u32[4];
  __shared__ int s_flag;
  Header* h = a.h;
  const U dmask = (U)a.dmask;
  if (a.exact_only == 2) {
    // after a sampled query: only when its tail found the sample misjudged
    // (path 4, left by the previous launch); its sample workgroups cleared the
    // select's counters, histograms and barrier
    if (h->q.path != 4u) return;
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->q.path = 5u;
  }
  const InputSrc<KT, RT> src{(const typename Key<KT>::Raw*)a.keys, (const R*)a.rids, dmask};
  const bool ok =
      exact_select<NT, U, R>(src, a.n, a.k_eff, h, (U*)a.ck, (R*)a.cf, lh, lh64, sh_u32, &s_flag);
  if (!ok) return;
  sort_and_write<KT, RT, NT>(a.k_eff, (U*)a.ck, (R*)a.cf, (U*)a.tk, (R*)a.tf, dmask, a.out_keys,
                             a.out_rids, h, t, &s_flag);
}

// ---- host side -------------------------------------------------------------------------------

namespace {

std::mutex g_mu;
Tuning g_tuning;

// Event pairs around the streaming pass, recorded while profiling is on.
struct Profile {
  std::mutex mu;
  bool on = false;
  uint32_t max = 0;
  std::vector<hipEvent_t> ev;  // 2 per launch
  uint32_t used = 0;
} g_prof;

template <typename T>
T* ws_ptr(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

template <int KT, int RT>
int coop_grid_tail(int dev) {
  static std::mutex mu;
  static std::vector<int> cache;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_tail<KT, RT>, 1024, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    cache[dev] = nb * device_cus(dev);
  }
  return cache[dev];
}

}  // namespace

// Records the start (begin=true) or end of a profiled kernel on `st`.
void profile_mark(hipStream_t st, bool begin) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.on) return;
  if (begin && g_prof.used + 2 > g_prof.ev.size()) return;
  const uint32_t slot = begin ? g_prof.used : g_prof.used + 1;
  if (!begin && slot >= g_prof.ev.size()) return;
  (void)hipEventRecord(g_prof.ev[slot], st);
  if (!begin) g_prof.used += 2;
}

int profile_begin(uint32_t max_launches) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto e : g_prof.ev)
    if (e) (void)hipEventDestroy(e);
  g_prof.ev.assign(2 * (size_t)max_launches, nullptr);
  for (auto& e : g_prof.ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& x : g_prof.ev)
        if (x) (void)hipEventDestroy(x);
      g_prof.ev.clear();
      return TK_EHIP;
    }
  g_prof.used = 0;
  g_prof.max = max_launches;
  g_prof.on = true;
  return TK_OK;
}

// Reads the recorded pairs and releases the events, so that no HIP object of
// the library outlives the measurement (nothing is left for process teardown).
int profile_end(double* total_ms, uint64_t* launches) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = false;
  double tot = 0;
  int rc = TK_OK;
  for (uint32_t i = 0; i + 1 < g_prof.used && rc == TK_OK; i += 2) {
    float ms = 0;
    if (hipEventSynchronize(g_prof.ev[i + 1]) != hipSuccess ||
        hipEventElapsedTime(&ms, g_prof.ev[i], g_prof.ev[i + 1]) != hipSuccess)
      rc = TK_EHIP;
    tot += ms;
  }
  const uint64_t n = g_prof.used / 2;
  for (auto e : g_prof.ev)
    if (e) (void)hipEventDestroy(e);
  g_prof.ev.clear();
  g_prof.used = 0;
  if (rc != TK_OK) return rc;
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  return TK_OK;
}

Tuning current_tuning() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tuning;
}

void set_tuning(const tk_tuning* t) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (t->sample_sigma > 0) g_tuning.sample_sigma = t->sample_sigma;
  if (t->recover_min_log2 > 0) g_tuning.recover_min_log2 = (uint32_t)t->recover_min_log2;
  if (t->recover_min_log2 < 0) g_tuning.recover_min_log2 = 0;
  if (t->cap_sigma > 0) g_tuning.cap_sigma = t->cap_sigma;
  if (t->max_sample_log2 > 0) g_tuning.max_sample_log2 = (uint32_t)t->max_sample_log2;
  if (t->filter_grid > 0) g_tuning.filter_grid = (uint32_t)t->filter_grid;
  if (t->force_cap > 0) g_tuning.force_cap = (uint64_t)t->force_cap;
  if (t->force_cap < 0) g_tuning.force_cap = 0;
  if (t->force_exact == 1) g_tuning.force_exact = 1;
  if (t->force_exact == 2) g_tuning.force_exact = 0;
  if (t->tail_mode == 1) g_tuning.rank_tail = 1;
  if (t->tail_mode == 2) g_tuning.rank_tail = 0;
  if (t->filter_unroll == 4 || t->filter_unroll == 8) g_tuning.filter_unroll = (uint32_t)t->filter_unroll;
  if (t->filter_grid < 0) g_tuning.filter_grid = 0;
  if (t->join_bloom == 1) g_tuning.join_bloom = 1;
  if (t->join_bloom == 2) g_tuning.join_bloom = 0;
}

// with_sort: the bytes tk_workspace_size reports; else the least workspace a
// query runs with (queries without a usable sample then take the grid-wide
// select instead of the sort)
size_t single_ws_bytes(uint64_t n, uint64_t k_eff, uint32_t kb, uint32_t rb, const Tuning& t,
                       bool with_sort = true) {
  const SamplePlan p = plan_sample(n, k_eff, t);
  const WsLayout L = ws_layout(n, k_eff, kb, rb, p);
  return with_sort ? L.total : L.base;
}

template <int KT, int RT>
int run_single(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int order,
               void* out_keys, void* out_rids, void* ws, size_t ws_bytes, hipStream_t st,
               const Tuning& tun) {
  using Raw = typename Key<KT>::Raw;
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  const U dmask = order == TK_ASC ? (U)~(U)0 : (U)0;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  // the header reports the path of the small routes when the caller passed a workspace
  QHead* const hq = ws && ws_bytes >= HEADER_BYTES && !((uintptr_t)ws & 255u)
                        ? &ws_ptr<Header>(ws, 0)->q : nullptr;
  if (!tun.force_exact && tun.rank_tail && n <= RANK_CMAX && !bucket_tail_for(k_eff)) {
    // ranked over the input by several workgroups
    const TailArgs1 ta{keys, rids, n, (uint64_t)dmask, hq, nullptr, nullptr, 0, nullptr, nullptr,
                       nullptr, nullptr, k_eff, out_keys, out_rids, TAIL_INPUT, 0};
    hipLaunchKernelGGL((k_rsmall<KT, RT>), dim3(rank_grid(k_eff)), dim3(RANK_NT), 0, st, ta);
    return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
  }
  if (n <= CAP && !tun.force_exact) {
    hipLaunchKernelGGL((k_small<KT, RT>), dim3(1), dim3(1024), 0, st, (const Raw*)keys,
                       (const R*)rids, (uint32_t)n, (uint32_t)k_eff, dmask, out_keys, out_rids);
    return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
  }
  const SamplePlan p = plan_sample(n, k_eff, tun);
  const WsLayout L = ws_layout(n, k_eff, sizeof(U), sizeof(R), p);
  int exact_mode = 1;
  if (p.fast) {
    const int rc = run_sampled<KT, RT>(keys, rids, n, k_eff, order, out_keys, out_rids, ws, ws_bytes,
                                       st, tun, p);
    if (rc != TK_OK || !recover_on_device(n, tun)) return rc;
    exact_mode = 2;  // returns at once unless the sample misjudged
  }
  if (!ws || ws_bytes < L.base || ((uintptr_t)ws & 255u)) return TK_EINVAL;
  if (exact_mode == 1 && !tun.force_exact && n < ONE_WG_INPUT_MAX) {
    // no usable sample and a small input: one workgroup selects over it (the
    // cooperative launch of the grid-wide select costs more than it saves here)
    return run_input_one_wg<KT, RT>(keys, rids, n, k_eff, order, out_keys, out_rids, ws, st, L);
  }
  if (exact_mode == 1 && !tun.force_exact && L.sort && ws_bytes >= L.total) {
    // no usable sample and K a large share of N: the full radix sort is a few
    // streaming passes, where the grid-wide select takes a round per digit plus
    // merge-path merges of K elements (a workspace without room for the sort's
    // scratch keeps the grid-wide select)
    return topk_by_sort(keys, rids, n, k_eff, KT, RT, order, out_keys, out_rids,
                        ws_ptr<char>(ws, L.sort), &ws_ptr<Header>(ws, 0)->q, st);
  }
  Header* h = ws_ptr<Header>(ws, 0);
  U* cand_k = ws_ptr<U>(ws, L.cand);
  R* cand_f = ws_ptr<R>(ws, L.cand + align_up((size_t)k_eff * sizeof(U), 16));
  U* tmp_k = ws_ptr<U>(ws, L.tmp);
  R* tmp_f = ws_ptr<R>(ws, L.tmp + align_up((size_t)k_eff * sizeof(U), 16));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TK_EHIP;
  if (exact_mode == 1) {
    hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, st, h);
    if (hipGetLastError() != hipSuccess) return TK_EHIP;
  }
  TailArgs a{keys, rids, n, (uint64_t)dmask, h, cand_k, cand_f, tmp_k, tmp_f, k_eff, out_keys,
             out_rids, exact_mode};
  void* args[] = {&a};
  // one workgroup per 16 Ki keys, up to what the device holds at once: every
  // digit round ends in a grid barrier whose cost grows with the grid, so a
  // small input is not spread over the whole device
  const uint64_t want = (n + 16383) / 16384;
  const int full = coop_grid_tail<KT, RT>(dev);
  const int grid = want < (uint64_t)full ? (int)want : full;
  if (hipLaunchCooperativeKernel((const void*)k_tail<KT, RT>, dim3(grid), dim3(1024), args, 0, st) !=
      hipSuccess)
    return TK_EHIP;
  return TK_OK;
}

template int run_single<KEY_I32, RID_U32>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_I32, RID_U64>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_F32, RID_U32>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_F32, RID_U64>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_I64, RID_U32>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_I64, RID_U64>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_F64, RID_U32>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);
template int run_single<KEY_F64, RID_U64>(const void*, const void*, uint64_t, uint64_t, int, void*, void*, void*, size_t, hipStream_t, const Tuning&);

}  // namespace tk

// ---- C ABI -----------------------------------------------------------------------------------

using namespace tk;

extern "C" size_t tk_workspace_size(uint64_t n, uint64_t k, int key_type, int rid_type) {
  const uint64_t k_eff = k < n ? k : n;
  const uint32_t kb = key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  return single_ws_bytes(n, k_eff, kb, rb, current_tuning());
}

extern "C" size_t tk_workspace_min_size(uint64_t n, uint64_t k, int key_type, int rid_type) {
  const uint64_t k_eff = k < n ? k : n;
  const uint32_t kb = key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  return single_ws_bytes(n, k_eff, kb, rb, current_tuning(), false);
}

extern "C" int tk_topk(const void* keys, const void* rowids, uint64_t n, uint64_t k, int key_type,
                       int rid_type, int order, void* out_keys, void* out_rowids,
                       uint64_t* out_count, void* workspace, size_t workspace_bytes, void* stream) {
  if (key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1 || order < 0 || order > 1)
    return TK_EINVAL;
  const uint64_t k_eff = k < n ? k : n;
  if (n > 0 && !keys) return TK_EINVAL;
  if (!rowids && rid_type == TK_RID_U32 && n > (1ull << 32)) return TK_EINVAL;
  if (n >= (1ull << 40)) return TK_EUNSUPPORTED;
  if (out_count) *out_count = k_eff;
  if (k_eff == 0) return TK_OK;
  const Tuning t = current_tuning();
  hipStream_t st = (hipStream_t)stream;
#define TK_RUN(KT, RT) \
  return run_single<KT, RT>(keys, rowids, n, k_eff, order, out_keys, out_rowids, workspace, workspace_bytes, st, t)
  if (key_type == TK_KEY_I32) { if (rid_type == TK_RID_U32) TK_RUN(KEY_I32, RID_U32); TK_RUN(KEY_I32, RID_U64); }
  if (key_type == TK_KEY_F32) { if (rid_type == TK_RID_U32) TK_RUN(KEY_F32, RID_U32); TK_RUN(KEY_F32, RID_U64); }
  if (key_type == TK_KEY_F64) { if (rid_type == TK_RID_U32) TK_RUN(KEY_F64, RID_U32); TK_RUN(KEY_F64, RID_U64); }
  if (rid_type == TK_RID_U32) TK_RUN(KEY_I64, RID_U32);
  TK_RUN(KEY_I64, RID_U64);
#undef TK_RUN
}

// ---- allocation-free variant of tk_topk ------------------------------------------------------
//
// The workspace of tk_topk lives in a file-scope device array instead of a
// caller buffer, for callers that cannot allocate device memory.  Each device
// the library runs on holds its own copy of the array (loaded with the code
// object, kept until the process ends); its device address is looked up once
// per device on the first call there and cached.  Every call on one device
// uses the same array: calls that overlap on one device (different streams,
// different host threads without ordering between their streams) race on it.
// The kernels set up every word of the workspace they read, so nothing has to
// be cleared between calls.

static __device__ __align__(256) unsigned char scratch[TK_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of `scratch`, per device

// Device address of this device's copy of `scratch` (nullptr on failure).
void* scratch_on(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int tk_topk_noalloc(const void* keys, const void* rowids, uint64_t n, uint64_t k,
                               int key_type, int rid_type, int order, void* out_keys,
                               void* out_rowids, uint64_t* out_count, void* stream) {
  if (key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1 || order < 0 || order > 1)
    return TK_EINVAL;
  if (n > 0 && !keys) return TK_EINVAL;
  const uint64_t k_eff = k < n ? k : n;
  if (k_eff == 0) {
    if (out_count) *out_count = 0;
    return TK_OK;
  }
  // the least workspace the query runs with: a query without a usable sample
  // whose sort scratch does not fit takes the grid-wide select
  if (tk_workspace_min_size(n, k, key_type, rid_type) > TK_NOALLOC_SCRATCH_BYTES)
    return TK_EUNSUPPORTED;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TK_EHIP;
  void* ws = scratch_on(dev);
  if (!ws) return TK_EHIP;
  return tk_topk(keys, rowids, n, k, key_type, rid_type, order, out_keys, out_rowids, out_count, ws,
                 TK_NOALLOC_SCRATCH_BYTES, stream);
}

extern "C" int tk_query_info(const void* workspace, tk_info* info) {
  if (!workspace || !info) return TK_EINVAL;
  Header h;
  if (hipMemcpy(&h, workspace, sizeof(Header), hipMemcpyDeviceToHost) != hipSuccess) return TK_EHIP;
  info->path = h.q.path;
  info->status = h.q.status;
  info->survivors = h.q.surv_count;
  info->threshold_key = h.q.thr_k;
  return h.q.status ? TK_EDEVICE : TK_OK;
}

extern "C" int tk_set_tuning(const tk_tuning* t) {
  if (!t) return TK_EINVAL;
  set_tuning(t);
  return TK_OK;
}

extern "C" int tk_profile_begin(uint32_t max_launches) { return profile_begin(max_launches); }

extern "C" int tk_profile_end(double* total_ms, uint64_t* launches) {
  return profile_end(total_ms, launches);
}

extern "C" const char* tk_status_string(int s) {
  switch (s) {
    case TK_OK: return "ok";
    case TK_EINVAL: return "invalid argument";
    case TK_ENOMEM: return "out of host memory";
    case TK_EHIP: return "HIP runtime error";
    case TK_EUNSUPPORTED: return "unsupported device or size";
    case TK_EDEVICE: return "device-side failure";
    case TK_EAGAIN: return "not finished";
    default: return "unknown status";
  }
}
