// Sampled single-query Top-K (ordering primitive, paper sec. III-A): three
// plain kernels on the caller's stream, no workgroup ever waits for another.
//
//   k_sample  S keys in 16-key chunks spread over the query, 1024 per
//             workgroup; each workgroup keeps its best r1 composites.  The
//             workgroup that finishes last (an atomic ticket) selects the
//             r1-th best of all of them: the threshold T.
//   k_filter  the single streaming pass over the keys: composites >= T are
//             appended to the survivor buffer (wave ballot, one atomic per
//             wave that has survivors).
//   k_tail    one workgroup: if K <= survivors <= capacity, radix-selects the
//             best K of the survivors, bitonic-sorts them in LDS and writes
//             the result; otherwise (the sample misjudged) it radix-selects
//             over the whole input instead.
// Any threshold with at least K survivors yields the exact answer, and a
// misjudged one falls back to the exact select, so the result never depends on
// the sample.
#include <hip/hip_runtime.h>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_internal.hpp"
#include "tk_plan.hpp"
#include "tk_select.hpp"
#include "tk_src.hpp"

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
  Header* h;
  void* ck;
  void* cf;
};

struct FiltArgs {
  const void* keys;
  const void* rids;
  uint64_t n;
  uint64_t dmask;
  Header* h;
  void* sk;
  void* sf;
  uint64_t cap;
};

struct TailArgs1 {
  const void* keys;
  const void* rids;
  uint64_t n;
  uint64_t dmask;
  Header* h;
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
};

// ---- k_sample ----------------------------------------------------------------------------------

template <int KT, int RT>
__device__ void sample_body(const SampArgs& a, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = SAMP_NT, E = SAMPLE_PER_BLOCK / SAMP_NT;
  Header* h = a.h;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h->surv_count = 0;
    h->status = 0;
    h->path = 0;
  }
  const InputSrc<KT, RT> src{(const typename Key<KT>::Raw*)a.keys, (const R*)a.rids, (U)a.dmask};
  const uint64_t nchunks = a.S / SAMPLE_CHUNK;
  const uint64_t stride = a.n / nchunks;  // >= 16: n >= 16 * S
  const uint64_t off0 = (stride - SAMPLE_CHUNK) / 2;
  U k[E];
  R f[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint64_t j = (uint64_t)blockIdx.x * SAMPLE_PER_BLOCK + (uint64_t)e * NT + threadIdx.x;
    const uint64_t pos = (j / SAMPLE_CHUNK) * stride + off0 + (j % SAMPLE_CHUNK);
    k[e] = src.key(pos);
    f[e] = src.flip(pos);
  }
  U lmin = k[0];
#pragma unroll
  for (int e = 1; e < E; ++e) lmin = k[e] < lmin ? k[e] : lmin;
  const U base = block_min<NT, U>(lmin, sc);
  const RegElems<U, R, E> el{k, f, E};
  const Sel<U, R> s = block_radix_select<NT, U, R>(el, a.r1, base, sc);
  U* ck = static_cast<U*>(a.ck);
  R* cf = static_cast<R*>(a.cf);
  block_compact_regs<NT, U, R, E>(el, s, a.r1, ck + (uint64_t)blockIdx.x * a.r1,
                                  cf + (uint64_t)blockIdx.x * a.r1, sc);
  // the last workgroup to finish turns the candidates into the threshold
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = atomicAdd(&h->samp_ticket, 1u);
    sc.cnt[0] = (old == gridDim.x - 1) ? 1u : 0u;
  }
  __syncthreads();
  const bool last = sc.cnt[0] != 0;
  __syncthreads();
  if (!last) return;
  __threadfence();
  // at most SAMPLE_FINAL_MAX candidates: 16 per thread, held in registers
  constexpr int EF = SAMPLE_FINAL_MAX / NT;
  const uint32_t m = gridDim.x * a.r1;
  U k2[EF];
  R f2[EF];
  int nv = 0;
  U cmin = (U)~(U)0;
#pragma unroll
  for (int e = 0; e < EF; ++e) {
    const uint32_t j = (uint32_t)e * NT + threadIdx.x;
    if (j < m) {
      k2[e] = ck[j];
      f2[e] = cf[j];
      nv = e + 1;
      cmin = k2[e] < cmin ? k2[e] : cmin;
    } else {
      k2[e] = 0;
      f2[e] = 0;
    }
  }
  const U base2 = block_min<NT, U>(cmin, sc);
  const RegElems<U, R, EF> el2{k2, f2, nv};
  const Sel<U, R> s2 = block_radix_select<NT, U, R>(el2, a.r1, base2, sc);
  if (threadIdx.x == 0) {
    h->thr_k = (unsigned long long)(U)(s2.base + s2.P);
    h->thr_f = s2.kind == SEL_KEY ? 0ull : (unsigned long long)s2.Pf;
    h->samp_ticket = 0;  // ready for the next query on this workspace
  }
}

// ---- k_filter ----------------------------------------------------------------------------------

template <typename U, typename R>
__device__ __forceinline__ void emit_survivor(bool pass, U kk, R ff, Header* h, U* sk, R* sf,
                                              uint64_t cap) {
  const uint64_t m = ballot(pass);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  uint64_t b = 0;
  if (lane_id() == leader) b = atomicAdd(&h->surv_count, (unsigned long long)__popcll(m));
  b = __shfl(b, (int)leader, 64);
  if (pass) {
    const uint64_t pos = b + lanes_below(m);
    if (pos < cap) {
      sk[pos] = kk;
      sf[pos] = ff;
    }
  }
}

template <int KT, int RT, int VEC, int UNR>
__device__ void filter_body(const FiltArgs& a) {
  using Raw = typename Key<KT>::Raw;
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = FILT_NT;
  static_assert(VEC * sizeof(Raw) == 16 || VEC == 1, "vector loads are 16 bytes");
  Header* h = a.h;
  const U Tk = (U)h->thr_k;
  const R Tf = (R)h->thr_f;
  const Raw* keys = static_cast<const Raw*>(a.keys);
  const InputSrc<KT, RT> src{keys, (const R*)a.rids, (U)a.dmask};
  const U dmask = (U)a.dmask;
  U* sk = static_cast<U*>(a.sk);
  R* sf = static_cast<R*>(a.sf);
  constexpr uint64_t TILE = (uint64_t)NT * VEC * UNR;
  const uint64_t ntiles = a.n / TILE;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t base = t * TILE;
    Raw v[UNR][VEC];
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
    bool any = false;
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) any |= (Key<KT>::enc(v[u][e]) ^ dmask) >= Tk;
    if (ballot(any) == 0) continue;
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const uint64_t i = base + ((uint64_t)u * NT + threadIdx.x) * VEC + e;
        const U kk = Key<KT>::enc(v[u][e]) ^ dmask;
        bool pass = kk > Tk;
        R ff = 0;
        if (kk >= Tk) {
          ff = src.flip(i);
          pass = pass || ff >= Tf;
        }
        emit_survivor<U, R>(pass, kk, ff, h, sk, sf, a.cap);
      }
  }
  // remainder (less than one tile)
  const uint64_t stride = (uint64_t)gridDim.x * NT;
  for (uint64_t i0 = ntiles * TILE + (uint64_t)blockIdx.x * NT; i0 < a.n; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    bool pass = false;
    U kk = 0;
    R ff = 0;
    if (i < a.n) {
      kk = src.key(i);
      pass = kk > Tk;
      if (kk >= Tk) {
        ff = src.flip(i);
        pass = pass || ff >= Tf;
      }
    }
    emit_survivor<U, R>(pass, kk, ff, h, sk, sf, a.cap);
  }
}

// ---- k_tail ------------------------------------------------------------------------------------

template <int KT, int RT, typename Src>
__device__ void select_sort_write(const TailArgs1& a, const Src& src, uint64_t n,
                                  typename Key<KT>::U base, LdsTile<KT, RT>& t, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = TAIL_NT;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const U dmask = (U)a.dmask;
  auto emit = [&](uint64_t j, U u, R f) { write_out<KT, RT>(j, u, f, dmask, a.out_keys, a.out_rids); };
  const GlobElems<NT, Src> el{src, n};
  const Sel<U, R> s = block_radix_select<NT, U, R>(el, a.k_eff, base, sc);
  if (a.k_eff <= CAP) {
    block_compact_glob<NT, U, R>(src, n, s, a.k_eff, t.k, t.f, sc);
    block_sort_emit<NT, U, R>(a.k_eff, true, t.k, t.f, CAP, nullptr, nullptr, nullptr, nullptr, emit);
  } else {
    U* ck = static_cast<U*>(a.ck);
    R* cf = static_cast<R*>(a.cf);
    block_compact_glob<NT, U, R>(src, n, s, a.k_eff, ck, cf, sc);
    block_sort_emit<NT, U, R>(a.k_eff, false, t.k, t.f, CAP, ck, cf, static_cast<U*>(a.tk),
                              static_cast<R*>(a.tf), emit);
  }
}

// Survivors that fit the registers of the workgroup (16 per thread) are
// loaded once and selected there.
constexpr int TAIL_E = 16;

template <int KT, int RT>
__device__ __forceinline__ void select_sort_write_regs(const TailArgs1& a, uint32_t C, typename Key<KT>::U base,
                                       LdsTile<KT, RT>& t, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  constexpr int NT = TAIL_NT, E = TAIL_E;
  constexpr uint32_t CAP = LdsTile<KT, RT>::CAP;
  const U dmask = (U)a.dmask;
  const U* sk = static_cast<const U*>(a.sk);
  const R* sf = static_cast<const R*>(a.sf);
  U k[E];
  R f[E];
  int nv = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const uint32_t j = (uint32_t)e * NT + threadIdx.x;
    if (j < C) {
      k[e] = sk[j];
      f[e] = sf[j];
      nv = e + 1;
    } else {
      k[e] = 0;
      f[e] = 0;
    }
  }
  auto emit = [&](uint64_t j, U u, R f_) { write_out<KT, RT>(j, u, f_, dmask, a.out_keys, a.out_rids); };
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
__device__ void tail_body(const TailArgs1& a, LdsTile<KT, RT>& t, SelScratch& sc) {
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  Header* h = a.h;
  const uint64_t C = h->surv_count;
  const bool ok = C >= a.k_eff && C <= a.cap;
  if (ok && C <= (uint64_t)TAIL_NT * TAIL_E) {
    select_sort_write_regs<KT, RT>(a, (uint32_t)C, (U)h->thr_k, t, sc);
  } else if (ok) {
    const BufSrc<U, R> src{static_cast<const U*>(a.sk), static_cast<const R*>(a.sf)};
    select_sort_write<KT, RT>(a, src, C, (U)h->thr_k, t, sc);
  } else {
    const InputSrc<KT, RT> src{(const typename Key<KT>::Raw*)a.keys, (const R*)a.rids, (U)a.dmask};
    select_sort_write<KT, RT>(a, src, a.n, (U)0, t, sc);
  }
  if (threadIdx.x == 0) {
    h->path = ok ? 2u : 4u;
    h->samp_ticket = 0;
  }
}

#ifndef TK_EMU
template <int KT, int RT>
__global__ __launch_bounds__(SAMP_NT) void k_sample(SampArgs a) {
  __shared__ SelScratch sc;
  sample_body<KT, RT>(a, sc);
}

template <int KT, int RT, int VEC, int UNR>
__global__ __launch_bounds__(FILT_NT) void k_filter(FiltArgs a) {
  filter_body<KT, RT, VEC, UNR>(a);
}

template <int KT, int RT>
__global__ __launch_bounds__(TAIL_NT) void k_tail1(TailArgs1 a) {
  __shared__ LdsTile<KT, RT> t;
  __shared__ SelScratch sc;
  tail_body<KT, RT>(a, t, sc);
}

// ---- host ------------------------------------------------------------------------------------

template <typename T>
static T* wsp(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

template <int KT, int RT>
int run_sampled(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int order,
                void* out_keys, void* out_rids, void* ws, size_t ws_bytes, hipStream_t st,
                const Tuning& tun, const SamplePlan& p) {
  using Raw = typename Key<KT>::Raw;
  using U = typename Key<KT>::U;
  using R = typename Rid<RT>::R;
  const WsLayout L = ws_layout(n, k_eff, sizeof(U), sizeof(R), p);
  if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) return TK_EINVAL;
  const uint64_t dmask = order == TK_ASC ? (uint64_t)(U)~(U)0 : 0ull;
  Header* h = wsp<Header>(ws, 0);
  void* samp_k = wsp<char>(ws, L.sample);
  void* samp_f = wsp<char>(ws, L.sample + align_up((size_t)p.blocks * p.r1 * sizeof(U), 16));
  void* surv_k = wsp<char>(ws, L.surv);
  void* surv_f = wsp<char>(ws, L.surv + align_up((size_t)p.cap * sizeof(U), 16));
  void* cand_k = wsp<char>(ws, L.cand);
  void* cand_f = wsp<char>(ws, L.cand + align_up((size_t)k_eff * sizeof(U), 16));
  void* tmp_k = wsp<char>(ws, L.tmp);
  void* tmp_f = wsp<char>(ws, L.tmp + align_up((size_t)k_eff * sizeof(U), 16));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TK_EHIP;
  const SampArgs sa{keys, rids, n, dmask, p.S, p.r1, h, samp_k, samp_f};
  hipLaunchKernelGGL((k_sample<KT, RT>), dim3(p.blocks), dim3(SAMP_NT), 0, st, sa);
  const FiltArgs fa{keys, rids, n, dmask, h, surv_k, surv_f, p.cap};
  const uint32_t grid = tun.filter_grid ? tun.filter_grid : (uint32_t)device_cus(dev) * 8u;
  profile_mark(st, true);
  if (((uintptr_t)keys & 15u) == 0) {
    constexpr int VEC = 16 / sizeof(Raw);
    hipLaunchKernelGGL((k_filter<KT, RT, VEC, 4>), dim3(grid), dim3(FILT_NT), 0, st, fa);
  } else {
    hipLaunchKernelGGL((k_filter<KT, RT, 1, 8>), dim3(grid), dim3(FILT_NT), 0, st, fa);
  }
  profile_mark(st, false);
  const TailArgs1 ta{keys, rids, n, dmask, h, surv_k, surv_f, p.cap, cand_k, cand_f,
                     tmp_k, tmp_f, k_eff, out_keys, out_rids};
  hipLaunchKernelGGL((k_tail1<KT, RT>), dim3(1), dim3(TAIL_NT), 0, st, ta);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}

#define TK_INST(KT, RT)                                                                         \
  template int run_sampled<KT, RT>(const void*, const void*, uint64_t, uint64_t, int, void*,    \
                                   void*, void*, size_t, hipStream_t, const Tuning&,           \
                                   const SamplePlan&);
TK_INST(KEY_I32, RID_U32)
TK_INST(KEY_I32, RID_U64)
TK_INST(KEY_F32, RID_U32)
TK_INST(KEY_F32, RID_U64)
TK_INST(KEY_I64, RID_U32)
TK_INST(KEY_I64, RID_U64)
#undef TK_INST
#endif  // TK_EMU

}  // namespace tk
