// The batch engine: many Top-K queries of uneven size (ordering primitive,
// paper sec. III-A, with the key-only contract of sec. II-C) in three
// kernels on the caller's stream.  No workgroup ever waits for another:
// every hand-off between workgroups is either a kernel boundary or an atomic
// ticket whose last taker does the follow-up work itself.
//
//   k_reset   zeroes the per-query state of the launch.
//   k_bprep   the sample workgroups of every sampled query: each reads 1024
//             keys in 16-key chunks spread over its query and keeps its best
//             r1 composites.  The query's last sample workgroup (ticket)
//             selects the r1-th best of them: the query's threshold.
//   k_engine  a persistent grid taking items from one queue, in order:
//               TILE   one streaming pass over a slice of a sampled query:
//                      composites >= threshold go to the query's survivor
//                      buffer.  The workgroup that finishes the query's last
//                      tile (ticket) radix-selects the best K of the survivors
//                      (of the whole query if the sample misjudged), sorts
//                      them in LDS and writes the query's result;
//               EXACT  a small query (or one whose K is a large share of its
//                      keys), radix-selected by one workgroup over its keys.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_engine.hpp"
#include "tk_internal.hpp"
#include "tk_plan.hpp"
#include "tk_select.hpp"
#include "tk_src.hpp"

namespace tk {

typedef uint32_t u32x4e __attribute__((ext_vector_type(4)));

constexpr int PREP_NT = 256;
#ifndef TK_ENG_NT
#define TK_ENG_NT 512
#endif
constexpr int ENG_NT = TK_ENG_NT;
constexpr uint32_t ENG_LDS_BYTES = 49152;

template <int KT, int RT>
struct QSrc {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  const typename Key<KT>::Raw* keys;
  const R* rids;
  uint64_t rid_base;
  U dmask;
  __device__ __forceinline__ U key(uint64_t i) const { return Key<KT>::enc(keys[i]) ^ dmask; }
  __device__ __forceinline__ R flip(uint64_t i) const {
    return ~(rids ? rids[i] : (R)(rid_base + i));
  }
};

template <typename T>
__device__ __forceinline__ T* at(char* scratch, uint64_t off) {
  return reinterpret_cast<T*>(scratch + off);
}

template <int KT, int RT>
__device__ __forceinline__ QSrc<KT, RT> query_src(const EngineArgs& a, const QDesc& d) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  QSrc<KT, RT> s;
  s.keys = reinterpret_cast<const typename Key<KT>::Raw*>(a.keys_base + d.keys);
  s.rids = d.has_rids ? reinterpret_cast<const R*>(a.rids_base + d.rids) : nullptr;
  s.rid_base = d.rid_base;
  s.dmask = d.order ? (U)~(U)0 : (U)0;
  return s;
}

template <typename U, typename R>
struct EngTile {
  static constexpr uint32_t CAP = (sizeof(U) + sizeof(R)) <= 12 ? 4096u : 2048u;
  static_assert(CAP * (sizeof(U) + sizeof(R)) <= ENG_LDS_BYTES, "sort tile must fit the LDS");
};

struct EngShared {
  alignas(16) char buf[ENG_LDS_BYTES];
  SelScratch sc;
  uint32_t idx;
  uint32_t flag;
};

// ---- k_reset -----------------------------------------------------------------------------------

__device__ void reset_body(const EngineArgs& a) {
  uint32_t* qs = reinterpret_cast<uint32_t*>(a.qs);
  const uint64_t words = (uint64_t)a.nq * sizeof(QState) / 4;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (uint64_t)gridDim.x * blockDim.x)
    qs[i] = 0;
  if (blockIdx.x == 0) {
    uint32_t* w = reinterpret_cast<uint32_t*>(a.ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(EngineCtl) / 4; i += blockDim.x) w[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) a.ctl->t_start = wall_clock64();
  }
}

// ---- k_bprep -----------------------------------------------------------------------------------

template <int KT, int RT>
__device__ __forceinline__ void sample_query(const EngineArgs& a, uint32_t q, uint32_t local,
                                             SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = PREP_NT, E = SAMPLE_PER_BLOCK / PREP_NT;
  const QDesc& d = a.qd[q];
  const QSrc<KT, RT> src = query_src<KT, RT>(a, d);
  const uint64_t nchunks = (uint64_t)d.S / SAMPLE_CHUNK;
  const uint64_t stride = d.n / nchunks;  // >= 16: n >= 16 * S
  const uint64_t off0 = (stride - SAMPLE_CHUNK) / 2;
  U k[E];
  R f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t j = (uint64_t)local * SAMPLE_PER_BLOCK + (uint64_t)e * NT + threadIdx.x;
    const uint64_t pos = (j / SAMPLE_CHUNK) * stride + off0 + (j % SAMPLE_CHUNK);
    k[e] = src.key(pos);
    f[e] = src.flip(pos);
  }
  U lmin = k[0];
#pragma unroll
  for (int e = 1; e < E; ++e) lmin = k[e] < lmin ? k[e] : lmin;
  const U base = block_min<NT, U>(lmin, sc);
  const RegElems<U, R, E> el{k, f, E};
  const Sel<U, R> s = block_radix_select<NT, U, R>(el, d.r1, base, sc);
  U* ck = at<U>(a.scratch, d.samp_k);
  R* cf = at<R>(a.scratch, d.samp_f);
  block_compact_regs<NT, U, R, E>(el, s, d.r1, ck + (uint64_t)local * d.r1,
                                  cf + (uint64_t)local * d.r1, sc);
  // the query's last sample workgroup computes its threshold
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = atomicAdd(&a.qs[q].samp_done, 1u);
    sc.cnt[0] = (old == d.samp_blocks - 1) ? 1u : 0u;
  }
  __syncthreads();
  const bool last = sc.cnt[0] != 0;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const uint64_t m = (uint64_t)d.samp_blocks * d.r1;
  const BufSrc<U, R> cs{ck, cf};
  U cmin = (U)~(U)0;
  for (uint64_t i = threadIdx.x; i < m; i += NT) {
    const U u = cs.key(i);
    cmin = u < cmin ? u : cmin;
  }
  const U base2 = block_min<NT, U>(cmin, sc);
  const GlobElems<NT, BufSrc<U, R>> el2{cs, m};
  const Sel<U, R> s2 = block_radix_select<NT, U, R>(el2, d.r1, base2, sc);
  if (threadIdx.x == 0) {
    a.qs[q].thr_k = (unsigned long long)(U)(s2.base + s2.P);
    a.qs[q].thr_f = s2.kind == SEL_KEY ? 0ull : (unsigned long long)s2.Pf;
  }
}

template <int RT>
__device__ void bprep_body(const EngineArgs& a, SelScratch& sc) {
  if (a.nprep == 0) return;
  const uint2 p = a.prep[blockIdx.x];
  switch (a.qd[p.x].key_type) {
    case KEY_I32: sample_query<KEY_I32, RT>(a, p.x, p.y, sc); break;
    case KEY_F32: sample_query<KEY_F32, RT>(a, p.x, p.y, sc); break;
    default: sample_query<KEY_I64, RT>(a, p.x, p.y, sc); break;
  }
}

// ---- k_engine ----------------------------------------------------------------------------------

template <int KT, int RT>
__device__ __forceinline__ void out_write(const EngineArgs& a, const QDesc& d, uint64_t j,
                                          typename Key<KT>::U u, typename Rid<RT>::R f) {
  using U = typename Key<KT>::U;
  const U dmask = d.order ? (U)~(U)0 : (U)0;
  if (d.has_out_keys)
    reinterpret_cast<typename Key<KT>::Raw*>(a.out_keys_base + d.out_keys)[j] = Key<KT>::dec(u ^ dmask);
  if (d.has_out_rids) reinterpret_cast<typename Rid<RT>::R*>(a.out_rids_base + d.out_rids)[j] = ~f;
}

template <int KT, int RT, typename Src>
__device__ __forceinline__ void select_sort_emit(const EngineArgs& a, const QDesc& d, const Src& src,
                                                 uint64_t n, typename Key<KT>::U base,
                                                 EngShared& sm) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr uint32_t CAP = EngTile<U, R>::CAP;
  U* lk = reinterpret_cast<U*>(sm.buf);
  R* lf = reinterpret_cast<R*>(sm.buf + CAP * sizeof(U));
  auto emit = [&](uint64_t j, U u, R f) { out_write<KT, RT>(a, d, j, u, f); };
  const GlobElems<ENG_NT, Src> el{src, n};
  const Sel<U, R> s = block_radix_select<ENG_NT, U, R>(el, d.k_eff, base, sm.sc);
  if (d.k_eff <= CAP) {
    block_compact_glob<ENG_NT, U, R>(src, n, s, d.k_eff, lk, lf, sm.sc);
    block_sort_emit<ENG_NT, U, R>(d.k_eff, true, lk, lf, CAP, nullptr, nullptr, nullptr, nullptr, emit);
  } else {
    U* ck = at<U>(a.scratch, d.cand_k);
    R* cf = at<R>(a.scratch, d.cand_f);
    block_compact_glob<ENG_NT, U, R>(src, n, s, d.k_eff, ck, cf, sm.sc);
    block_sort_emit<ENG_NT, U, R>(d.k_eff, false, lk, lf, CAP, ck, cf, at<U>(a.scratch, d.tmp_k),
                                  at<R>(a.scratch, d.tmp_f), emit);
  }
}

__device__ __forceinline__ void mark_done(const EngineArgs& a, uint32_t q) {
  if (threadIdx.x == 0) {
    a.qs[q].t_done = wall_clock64();
    a.qs[q].done = 1u;
  }
}

template <typename U, typename R>
__device__ __forceinline__ void emit_surv(bool pass, U kk, R ff, unsigned long long* count, U* sk,
                                          R* sf, uint64_t cap) {
  const uint64_t m = ballot(pass);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  uint64_t b = 0;
  if (lane_id() == leader) b = atomicAdd(count, (unsigned long long)__popcll(m));
  b = __shfl(b, (int)leader, 64);
  if (pass) {
    const uint64_t pos = b + lanes_below(m);
    if (pos < cap) {
      sk[pos] = kk;
      sf[pos] = ff;
    }
  }
}

template <int KT, int RT>
__device__ __forceinline__ void do_tail(const EngineArgs& a, uint32_t q, EngShared& sm) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  const QDesc& d = a.qd[q];
  QState& st = a.qs[q];
  const uint64_t C = __hip_atomic_load(&st.surv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (C >= d.k_eff && C <= d.cap) {
    const BufSrc<U, R> src{at<U>(a.scratch, d.surv_k), at<R>(a.scratch, d.surv_f)};
    select_sort_emit<KT, RT>(a, d, src, C, (U)st.thr_k, sm);
  } else {
    if (threadIdx.x == 0) st.status |= 1u;
    const QSrc<KT, RT> src = query_src<KT, RT>(a, d);
    select_sort_emit<KT, RT>(a, d, src, d.n, (U)0, sm);
  }
  mark_done(a, q);
}

// TILE: streams keys [t * tile_len, ...) of a sampled query.
template <int KT, int RT>
__device__ __forceinline__ void do_tile(const EngineArgs& a, uint32_t q, uint32_t t, EngShared& sm) {
  using Raw = typename Key<KT>::Raw;
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = ENG_NT, VEC = 16 / sizeof(Raw), UNR = 4;
  const QDesc& d = a.qd[q];
  QState& st = a.qs[q];
  const U Tk = (U)st.thr_k;
  const R Tf = (R)st.thr_f;
  const QSrc<KT, RT> src = query_src<KT, RT>(a, d);
  U* sk = at<U>(a.scratch, d.surv_k);
  R* sf = at<R>(a.scratch, d.surv_f);
  unsigned long long* cnt = &st.surv;
  const uint64_t lo = (uint64_t)t * d.tile_len;
  const uint64_t hi = lo + d.tile_len < d.n ? lo + d.tile_len : d.n;
  // vector loads from the first 16-byte boundary; scalar head and tail
  const uint64_t mis = ((uintptr_t)(src.keys + lo) & 15u) / sizeof(Raw);
  uint64_t vlo = lo + (mis ? (VEC - mis) : 0);
  if (vlo > hi) vlo = hi;
  constexpr uint64_t STEP = (uint64_t)NT * VEC * UNR;
  const uint64_t nsteps = (hi - vlo) / STEP;
  const uint64_t vhi = vlo + nsteps * STEP;
  auto scalar = [&](uint64_t i, bool valid) {
    bool pass = false;
    U kk = 0;
    R ff = 0;
    if (valid) {
      kk = src.key(i);
      pass = kk > Tk;
      if (kk >= Tk) {
        ff = src.flip(i);
        pass = pass || ff >= Tf;
      }
    }
    emit_surv<U, R>(pass, kk, ff, cnt, sk, sf, d.cap);
  };
  scalar(lo + threadIdx.x, threadIdx.x < vlo - lo);
  for (uint64_t s = 0; s < nsteps; ++s) {
    const uint64_t base = vlo + s * STEP;
    Raw v[UNR][VEC];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const uint64_t i0 = base + ((uint64_t)u * NT + threadIdx.x) * VEC;
      const u32x4e qv = __builtin_nontemporal_load(reinterpret_cast<const u32x4e*>(src.keys + i0));
      if constexpr (sizeof(Raw) == 4) {
        v[u][0] = qv.x; v[u][1] = qv.y; v[u][2] = qv.z; v[u][3] = qv.w;
      } else {
        v[u][0] = (uint64_t)qv.x | ((uint64_t)qv.y << 32);
        v[u][1] = (uint64_t)qv.z | ((uint64_t)qv.w << 32);
      }
    }
    bool any = false;
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) any |= (Key<KT>::enc(v[u][e]) ^ src.dmask) >= Tk;
    if (ballot(any) == 0) continue;
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const uint64_t i = base + ((uint64_t)u * NT + threadIdx.x) * VEC + e;
        const U kk = Key<KT>::enc(v[u][e]) ^ src.dmask;
        bool pass = kk > Tk;
        R ff = 0;
        if (kk >= Tk) {
          ff = src.flip(i);
          pass = pass || ff >= Tf;
        }
        emit_surv<U, R>(pass, kk, ff, cnt, sk, sf, d.cap);
      }
  }
  for (uint64_t i0 = vhi; i0 < hi; i0 += NT) scalar(i0 + threadIdx.x, i0 + threadIdx.x < hi);
  // the query's last tile runs its tail
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = atomicAdd(&st.tiles_done, 1u);
    sm.flag = (old == d.ntiles - 1) ? 1u : 0u;
  }
  __syncthreads();
  const bool last = sm.flag != 0;
  __syncthreads();
  if (!last) return;
  __threadfence();
  do_tail<KT, RT>(a, q, sm);
}

// EXACT: radix passes over all of the query's keys by one workgroup.
template <int KT, int RT>
__device__ __forceinline__ void do_exact(const EngineArgs& a, uint32_t q, EngShared& sm) {
  using U = typename Key<KT>::U;
  const QDesc& d = a.qd[q];
  const QSrc<KT, RT> src = query_src<KT, RT>(a, d);
  select_sort_emit<KT, RT>(a, d, src, d.n, (U)0, sm);
  mark_done(a, q);
}

template <int KT, int RT>
__device__ __forceinline__ void run_item(const EngineArgs& a, const Item& it, EngShared& sm) {
  if (it.type == ITEM_TILE) do_tile<KT, RT>(a, it.q, it.a, sm);
  else do_exact<KT, RT>(a, it.q, sm);
}

// KTF: the key type of every query of the launch, or -1 when the queries mix
// key types (each item then dispatches on its query's type).
template <int RT, int KTF>
__device__ void engine_body(const EngineArgs& a, EngShared& sm) {
  for (;;) {
    if (threadIdx.x == 0) sm.idx = atomicAdd(&a.ctl->head, 1u);
    __syncthreads();
    const uint32_t idx = sm.idx;
    __syncthreads();
    if (idx >= a.nitems) break;
    const Item it = a.items[idx];
    if constexpr (KTF >= 0) {
      run_item<KTF, RT>(a, it, sm);
    } else {
      switch (a.qd[it.q].key_type) {
        case KEY_I32: run_item<KEY_I32, RT>(a, it, sm); break;
        case KEY_F32: run_item<KEY_F32, RT>(a, it, sm); break;
        default: run_item<KEY_I64, RT>(a, it, sm); break;
      }
    }
  }
}

// Layout of one query's scratch regions; returns the bytes used.
uint64_t layout_query(QDesc& d, uint64_t off, uint32_t kb, uint32_t rb, const SamplePlan& p) {
  auto region = [&](uint64_t count, uint64_t& ko, uint64_t& fo) {
    ko = off;
    off = align_up(off + count * kb, 16);
    fo = off;
    off = align_up(off + count * rb, 256);
  };
  const uint64_t before = off;
  if (p.fast) {
    region((uint64_t)p.blocks * p.r1, d.samp_k, d.samp_f);
    region(p.cap, d.surv_k, d.surv_f);
  }
  const uint32_t tile = (kb + rb) <= 12 ? 4096u : 2048u;
  if (d.k_eff > tile) {
    region(d.k_eff, d.cand_k, d.cand_f);
    region(d.k_eff, d.tmp_k, d.tmp_f);
  }
  return off - before;
}

#ifndef TK_EMU
__global__ __launch_bounds__(256) void k_reset(EngineArgs a) { reset_body(a); }

template <int RT>
__global__ __launch_bounds__(PREP_NT) void k_bprep(EngineArgs a) {
  __shared__ SelScratch sc;
  bprep_body<RT>(a, sc);
}

template <int RT, int KTF>
__global__ __launch_bounds__(ENG_NT) void k_engine(EngineArgs a) {
  __shared__ EngShared sm;
  engine_body<RT, KTF>(a, sm);
}

// ---- host ------------------------------------------------------------------------------------

namespace {

template <int RT, int KTF>
int engine_grid(int dev) {
  static std::mutex mu;
  static std::vector<int> cache;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1, 0);
  if (cache[dev] == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_engine<RT, KTF>, ENG_NT,
                                                     0) != hipSuccess || nb < 1)
      nb = 1;
    cache[dev] = nb * device_cus(dev);
  }
  return cache[dev];
}

template <int RT, int KTF>
void launch_engine(const EngineArgs& a, uint32_t grid, hipStream_t st) {
  if (grid > a.nitems) grid = a.nitems;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_engine<RT, KTF>), dim3(grid), dim3(ENG_NT), 0, st, a);
}

template <int RT>
uint32_t grid_for(int key_type, int dev) {
  switch (key_type) {
    case KEY_I32: return (uint32_t)engine_grid<RT, KEY_I32>(dev);
    case KEY_F32: return (uint32_t)engine_grid<RT, KEY_F32>(dev);
    case KEY_I64: return (uint32_t)engine_grid<RT, KEY_I64>(dev);
    default: return (uint32_t)engine_grid<RT, -1>(dev);
  }
}

template <int RT>
void launch_all(const EngineArgs& a, int key_type, uint32_t grid, hipStream_t st) {
  const uint32_t rgrid = std::max<uint32_t>(1, std::min<uint32_t>(1024, (a.nq * 16 + 255) / 256));
  hipLaunchKernelGGL(k_reset, dim3(rgrid), dim3(256), 0, st, a);
  if (a.nprep) hipLaunchKernelGGL(k_bprep<RT>, dim3(a.nprep), dim3(PREP_NT), 0, st, a);
  profile_mark(st, true);
  switch (key_type) {
    case KEY_I32: launch_engine<RT, KEY_I32>(a, grid, st); break;
    case KEY_F32: launch_engine<RT, KEY_F32>(a, grid, st); break;
    case KEY_I64: launch_engine<RT, KEY_I64>(a, grid, st); break;
    default: launch_engine<RT, -1>(a, grid, st); break;
  }
  profile_mark(st, false);
}

}  // namespace

uint32_t engine_grid_size(uint32_t rid_type, int key_type) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  return rid_type == RID_U64 ? grid_for<RID_U64>(key_type, dev) : grid_for<RID_U32>(key_type, dev);
}

void engine_enqueue(const EngineArgs& a, uint32_t rid_type, int key_type, uint32_t grid,
                    hipStream_t st) {
  if (rid_type == RID_U64) launch_all<RID_U64>(a, key_type, grid, st);
  else launch_all<RID_U32>(a, key_type, grid, st);
}

int engine_launch(const EngineArgs& a, uint32_t rid_type, int key_type, uint32_t grid_override,
                  hipStream_t st) {
  const uint32_t grid = grid_override ? grid_override : engine_grid_size(rid_type, key_type);
  if (grid == 0) return TK_EHIP;
  engine_enqueue(a, rid_type, key_type, grid, st);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}
#endif  // TK_EMU

}  // namespace tk
