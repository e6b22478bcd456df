// Batched Top-K in four plain launches (ordering primitive, paper sec.
// III-A, applied to many queries at once):
//
//   k_msample  every sample workgroup of every sampled query;
//   k_msfinal  one workgroup per sampled query: its threshold;
//   k_mfilter  every filter workgroup of every sampled query (slices of
//              64 Ki keys), appending survivors to the query's buffer;
//   k_mtail    one workgroup per non-empty query: the exact select and sort
//              over the query's survivors, or over its whole input for the
//              queries too small (or with too large a K) for the sample.
//
// A workgroup reads which query (and which of its workgroups) it is from a
// block map, then runs the body the single-query kernels run.  No workgroup
// waits for another or hands it data within a kernel: the hand-offs are the
// launch boundaries, as in the single query.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>

#include "tk_multi.hpp"

namespace tk {

template <int KT, int RT>
__global__ __launch_bounds__(SAMP_NT) void k_msample(const SampArgs* __restrict__ sa,
                                                     const uint2* __restrict__ map) {
  __shared__ SelScratch sc;
  const uint2 m = map[blockIdx.x];
  const SampArgs a = sa[m.x];
  sample_body<KT, RT, false>(a, sc, m.y);
}

template <int KT, int RT>
__global__ __launch_bounds__(FILT_NT) void k_msfinal(const FiltArgs* __restrict__ fa) {
  __shared__ SelScratch sc;
  const FiltArgs a = fa[blockIdx.x];
  sample_final_body<KT, RT, false>(a, sc);
}

// Workgroup w streams the slices w, w + grid, w + 2 grid, ... of the block map;
// the next slice's map entry and record are loaded before the current slice
// is streamed, so that looking them up adds no round trip between slices.
template <int KT, int RT>
__global__ __launch_bounds__(FILT_NT) void k_mfilter(const FiltArgs* __restrict__ fa,
                                                     const uint2* __restrict__ map, uint32_t n) {
  __shared__ SurvStage<typename Key<KT>::U, typename Rid<RT>::R> st;
  uint32_t it = blockIdx.x;
  if (it >= n) return;
  uint2 m = map[it];
  FiltArgs a = fa[m.x];
  while (true) {
    const uint32_t nx = it + gridDim.x;
    uint2 mn = m;
    FiltArgs an = a;
    if (nx < n) {
      mn = map[nx];
      an = fa[mn.x];
    }
    filter_body<KT, RT, 16 / sizeof(typename Key<KT>::Raw), 4>(a, m.y, st);
    if (nx >= n) break;
    __syncthreads();  // the stage is reused by the next slice
    it = nx;
    m = mn;
    a = an;
  }
}

// One tail workgroup per query; with stamps, its end on the device clock
// (the constant-rate real-time counter) is recorded as the query's completion.
template <int KT, int RT>
__global__ __launch_bounds__(TAIL_NT) void k_mtail(const TailArgs1* __restrict__ ta,
                                                   const uint32_t* __restrict__ tq,
                                                   unsigned long long* __restrict__ stamps) {
  __shared__ LdsTile<KT, RT> t;
  __shared__ SelScratch sc;
  const TailArgs1 a = ta[blockIdx.x];
  tail_body<KT, RT>(a, t, sc);
  if (stamps) {
    __syncthreads();
    if (threadIdx.x == 0) stamps[1 + tq[blockIdx.x]] = wall_clock64();
  }
}

// The start of a stamped launch, before any of its other kernels.
__global__ void k_mstamp(unsigned long long* stamps) { stamps[0] = wall_clock64(); }

namespace {

constexpr uint32_t DEFAULT_SLICE = 1u << 15;

struct Regions {
  uint64_t samp, surv, cand, tmp, total;  // offsets within the query's regions
};

Regions regions_of(uint64_t k_eff, uint32_t kb, uint32_t rb, const SamplePlan& p, bool sampled) {
  Regions g{};
  uint64_t off = 0;
  if (sampled) {
    g.samp = off;
    off = align_up(off + (uint64_t)p.blocks * p.r1 * (kb + rb) + 64, 256);
    g.surv = off;
    off = align_up(off + p.cap * (kb + rb) + 64, 256);
  }
  if (k_eff > lds_cap_for(kb + rb)) {
    g.cand = off;
    off = align_up(off + k_eff * (kb + rb) + 64, 256);
    g.tmp = off;
    off = align_up(off + k_eff * (kb + rb) + 64, 256);
  }
  g.total = off;
  return g;
}

}  // namespace

uint64_t multi_layout(const std::vector<uint64_t>& n, const std::vector<uint64_t>& k, int key_type,
                      int rid_type, const Tuning& tun, uint32_t slice_keys, MLayout& L) {
  const uint32_t kb = key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  const size_t q = n.size();
  const uint64_t slice = slice_keys ? slice_keys : DEFAULT_SLICE;
  L = MLayout{};
  L.cls.assign(q, MC_EMPTY);
  L.sp.assign(q, SamplePlan{});
  L.head.assign(q, 0);
  L.reg.assign(q, 0);
  L.fblocks.assign(q, 0);
  for (size_t i = 0; i < q; ++i) {
    const uint64_t ke = std::min(k[i], n[i]);
    if (ke == 0) continue;
    L.sp[i] = plan_sample(n[i], ke, tun);
    if (L.sp[i].fast) {
      L.cls[i] = MC_SAMPLED;
      L.head[i] = L.n_sampled++;
      L.fblocks[i] = (uint32_t)((n[i] + slice - 1) / slice);
      L.n_samp_blocks += L.sp[i].blocks;
      L.n_filt_blocks += L.fblocks[i];
    } else {
      L.cls[i] = MC_INPUT;
      ++L.n_input;
    }
  }
  L.heads_bytes = align_up((uint64_t)L.n_sampled * sizeof(QHead), 256);
  uint64_t off = L.heads_bytes;
  for (size_t i = 0; i < q; ++i) {
    if (L.cls[i] == MC_EMPTY) continue;
    const uint64_t ke = std::min(k[i], n[i]);
    L.reg[i] = off;
    off += regions_of(ke, kb, rb, L.sp[i], L.cls[i] == MC_SAMPLED).total;
  }
  L.total = align_up(off, 256);
  return L.total;
}

void multi_records(const std::vector<MQuery>& q, const MLayout& L, int key_type, int rid_type,
                   char* ws, MRecords& r) {
  const uint32_t kb = key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  r.sa.clear();
  r.smap.clear();
  r.fa.clear();
  r.fmap.clear();
  r.ta.clear();
  r.tq.clear();
  // tails of the largest queries first, so the long ones start early
  std::vector<uint32_t> order(q.size());
  std::iota(order.begin(), order.end(), 0u);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return q[a].n > q[b].n; });
  for (uint32_t i : order) {
    if (L.cls[i] == MC_EMPTY) continue;
    const MQuery& Q = q[i];
    const uint64_t ke = std::min(Q.k, Q.n);
    const uint64_t dmask = Q.order == TK_ASC ? (kb == 8 ? ~0ull : 0xFFFFFFFFull) : 0ull;
    const SamplePlan& p = L.sp[i];
    const bool sampled = L.cls[i] == MC_SAMPLED;
    const Regions g = regions_of(ke, kb, rb, p, sampled);
    char* base = ws + L.reg[i];
    auto split = [&](uint64_t off, uint64_t count, void*& kp, void*& fp) {
      kp = base + off;
      fp = base + off + align_up(count * kb, 16);
    };
    void *ck = nullptr, *cf = nullptr, *tk_ = nullptr, *tf = nullptr;
    if (ke > lds_cap_for(kb + rb)) {
      split(g.cand, ke, ck, cf);
      split(g.tmp, ke, tk_, tf);
    }
    QHead* h = nullptr;
    void *sk = nullptr, *sf = nullptr;
    if (sampled) {
      h = reinterpret_cast<QHead*>(ws) + L.head[i];
      void *pk, *pf;
      split(g.samp, (uint64_t)p.blocks * p.r1, pk, pf);
      split(g.surv, p.cap, sk, sf);
      const uint32_t si = (uint32_t)r.sa.size();
      r.sa.push_back(SampArgs{Q.keys, Q.rids, Q.n, dmask, p.S, p.r1, h, pk, pf, p.blocks, 0});
      for (uint32_t b = 0; b < p.blocks; ++b) r.smap.push_back(uint2{si, b});
      const uint32_t fi = (uint32_t)r.fa.size();
      r.fa.push_back(FiltArgs{Q.keys, Q.rids, Q.n, dmask, h, sk, sf, p.cap, L.fblocks[i], p.r1, pk,
                              pf, p.blocks * p.r1, 0});
      for (uint32_t b = 0; b < L.fblocks[i]; ++b) r.fmap.push_back(uint2{fi, b});
    }
    r.ta.push_back(TailArgs1{Q.keys, Q.rids, Q.n, dmask, h, sk, sf, sampled ? p.cap : 0, ck, cf,
                             tk_, tf, ke, Q.out_keys, Q.out_rids,
                             sampled ? TAIL_SURVIVORS : TAIL_INPUT, 0});
    r.tq.push_back(i);
  }
}

uint64_t multi_pack_bytes(const MRecords& r) {
  return align_up(r.sa.size() * sizeof(SampArgs), 256) + align_up(r.smap.size() * sizeof(uint2), 256) +
         align_up(r.fa.size() * sizeof(FiltArgs), 256) + align_up(r.fmap.size() * sizeof(uint2), 256) +
         align_up(r.ta.size() * sizeof(TailArgs1), 256) + align_up(r.tq.size() * sizeof(uint32_t), 256);
}

MLaunch multi_pack(const MRecords& r, char* dst, char* dev) {
  MLaunch m;
  uint64_t off = 0;
  auto put = [&](const void* src, uint64_t bytes) {
    const uint64_t at = off;
    if (bytes) std::memcpy(dst + at, src, bytes);
    off = align_up(off + bytes, 256);
    return dev + at;
  };
  m.sa = reinterpret_cast<const SampArgs*>(put(r.sa.data(), r.sa.size() * sizeof(SampArgs)));
  m.smap = reinterpret_cast<const uint2*>(put(r.smap.data(), r.smap.size() * sizeof(uint2)));
  m.fa = reinterpret_cast<const FiltArgs*>(put(r.fa.data(), r.fa.size() * sizeof(FiltArgs)));
  m.fmap = reinterpret_cast<const uint2*>(put(r.fmap.data(), r.fmap.size() * sizeof(uint2)));
  m.ta = reinterpret_cast<const TailArgs1*>(put(r.ta.data(), r.ta.size() * sizeof(TailArgs1)));
  m.tq = reinterpret_cast<const uint32_t*>(put(r.tq.data(), r.tq.size() * sizeof(uint32_t)));
  m.n_samp = (uint32_t)r.smap.size();
  m.n_fa = (uint32_t)r.fa.size();
  m.n_filt = (uint32_t)r.fmap.size();
  m.n_tail = (uint32_t)r.ta.size();
  return m;
}

namespace {

template <int KT, int RT>
void enqueue_typed(const MLaunch& m, hipStream_t st) {
  if (m.stamps) hipLaunchKernelGGL(k_mstamp, dim3(1), dim3(1), 0, st, m.stamps);
  if (m.n_samp) hipLaunchKernelGGL((k_msample<KT, RT>), dim3(m.n_samp), dim3(SAMP_NT), 0, st, m.sa, m.smap);
  if (m.n_fa) hipLaunchKernelGGL((k_msfinal<KT, RT>), dim3(m.n_fa), dim3(FILT_NT), 0, st, m.fa);
  profile_mark(st, true);
  // 0: three workgroups per CU (the streaming pass's occupancy), each looping
  // over slices with the next one's record prefetched; measured 5 % faster at
  // C3 than one workgroup per slice, which pays the record lookups of every
  // slice before its first load
  uint32_t fg = m.filt_grid;
  if (fg == 0) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    fg = 3u * (uint32_t)device_cus(dev);
  }
  if (fg > m.n_filt) fg = m.n_filt;
  if (m.n_filt) hipLaunchKernelGGL((k_mfilter<KT, RT>), dim3(fg), dim3(FILT_NT), 0, st, m.fa, m.fmap, m.n_filt);
  profile_mark(st, false);
  if (m.n_tail)
    hipLaunchKernelGGL((k_mtail<KT, RT>), dim3(m.n_tail), dim3(TAIL_NT), 0, st, m.ta, m.tq, m.stamps);
}

template <int KT>
void enqueue_rid(const MLaunch& m, int rid_type, hipStream_t st) {
  if (rid_type == TK_RID_U64) enqueue_typed<KT, RID_U64>(m, st);
  else enqueue_typed<KT, RID_U32>(m, st);
}

}  // namespace

void multi_enqueue(const MLaunch& m, int key_type, int rid_type, hipStream_t st) {
  switch (key_type) {
    case TK_KEY_I32: enqueue_rid<KEY_I32>(m, rid_type, st); break;
    case TK_KEY_F32: enqueue_rid<KEY_F32>(m, rid_type, st); break;
    case TK_KEY_F64: enqueue_rid<KEY_F64>(m, rid_type, st); break;
    default: enqueue_rid<KEY_I64>(m, rid_type, st); break;
  }
}

}  // namespace tk
