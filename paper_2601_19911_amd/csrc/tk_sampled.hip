// Sampled single-query Top-K (ordering primitive, paper sec. III-A): four
// plain kernels on the caller's stream; no workgroup waits for or hands data
// to another within a kernel, so no device-wide fence is needed.
//
//   k_sample  S keys in 16-key chunks spread over the query, 2048 per
//             workgroup; each workgroup keeps its best r1 composites.
//   k_sfinal  one workgroup selects the r1-th best of those candidates: the
//             threshold T.
//   k_filter  the single streaming pass over the keys: composites >= T are
//             staged in LDS (wave ballot + LDS atomic) and appended to the
//             survivor buffer with one global atomic per workgroup.
//   k_rtail   the best K of the survivors over many workgroups: one
//             histogram of the survivors' distance to the threshold bounds a
//             small hot set, whose members are ranked by counting and written
//             at their rank (tk_rank.hpp).
//   k_bhist, k_bscatter, k_bsort   the tail for large K (tk_bucket.hpp):
//             survivors grouped by a logarithmic bucket of their distance to
//             the threshold, runs of whole hot buckets sorted in LDS and
//             written at their offset.
//   k_tail1   the one-workgroup tail (the fallback of both, and a tuning
//             choice): if K <= survivors <= capacity, radix-selects the best
//             K of the survivors, bitonic-sorts them in LDS and writes the
//             result; otherwise (the sample misjudged) it radix-selects over
//             the whole input instead, or, for large inputs, leaves the query
//             to the cooperative exact select over the whole device that the
//             caller enqueues next (it returns at once when the sample held).
// Any threshold with at least K survivors yields the exact answer, and a
// misjudged one falls back to the exact select, so the result never depends on
// the sample.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "tk_bucket.hpp"
#include "tk_rank.hpp"
#include "tk_sampled.hpp"

namespace tk {

template <int KT, int RT>
__global__ __launch_bounds__(SAMP_NT) void k_sample(SampArgs a) {
  __shared__ SelScratch sc;
  sample_body<KT, RT, true>(a, sc, blockIdx.x);
}

template <int KT, int RT>
__global__ __launch_bounds__(FILT_NT) void k_sfinal(FiltArgs a) {
  __shared__ SelScratch sc;
  sample_final_body<KT, RT, true>(a, sc);
}

template <int KT, int RT, int VEC, int UNR>
__global__ __launch_bounds__(FILT_NT) void k_filter(FiltArgs a) {
  __shared__ SurvStage<typename Key<KT>::U, typename Rid<RT>::R> st;
  filter_body<KT, RT, VEC, UNR>(a, blockIdx.x, st);
}

template <int KT, int RT>
__global__ __launch_bounds__(TAIL_NT) void k_tail1(TailArgs1 a) {
  __shared__ LdsTile<KT, RT> t;
  __shared__ SelScratch sc;
  tail_body<KT, RT>(a, t, sc);
}

template <int KT, int RT>
__global__ __launch_bounds__(RANK_NT) void k_rtail(TailArgs1 a) {
  __shared__ __align__(16) unsigned char smem[rank_smem_bytes<KT, RT>()];
  rank_tail_body<KT, RT>(a, smem, blockIdx.x, gridDim.x);
}

template <int KT, int RT>
__global__ __launch_bounds__(BT_NT) void k_bhist(BTailArgs b) {
  __shared__ uint32_t lh[BT<KT, RT>::NB];
  __shared__ uint32_t red[16];
  bhist_body<KT, RT>(b, lh, red);
}

template <int KT, int RT>
__global__ __launch_bounds__(BSC_NT) void k_bscatter(BTailArgs b) {
  __shared__ uint32_t loff[bs_padded<BT<KT, RT>::NB>()];
  __shared__ uint32_t lcnt[BT<KT, RT>::NB];
  __shared__ uint32_t red[48];
  bscatter_body<KT, RT>(b, loff, lcnt, red);
}

template <int KT, int RT>
__global__ __launch_bounds__(TAIL_NT) void k_bsort(BTailArgs b) {
  __shared__ __align__(16) unsigned char smem[(sizeof(LdsTile<KT, RT>) + 15) / 16 * 16 +
                                              sizeof(SelScratch)];
  bsort_body<KT, RT>(b, smem);
}

// ---- host ------------------------------------------------------------------------------------

// Workgroups of the streaming pass: FILT_WG_PER_CU per CU, each striding over
// many tiles.  Fewer, longer-lived workgroups stream faster than a full-
// occupancy grid: at N = 2^28 on MI355X, 2-3 per CU read at 6.9-7.2 TB/s
// against 6.2-6.5 TB/s for 8 per CU (float32 and int64 keys).
constexpr uint32_t FILT_WG_PER_CU = 3;

static uint32_t filter_grid(int dev) { return FILT_WG_PER_CU * (uint32_t)device_cus(dev); }

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
  QHead* h = &wsp<Header>(ws, 0)->q;
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
  const bool bucketed = tun.rank_tail && bucket_tail_for(k_eff);
  const uint32_t nb = bucket_count(8 * (uint32_t)(sizeof(U) + sizeof(R)));
  uint32_t* bt_words = bucketed ? wsp<uint32_t>(ws, L.btail) : nullptr;  // gh, cur, chunk
  const uint32_t defer = recover_on_device(n, tun) ? 1u : 0u;
  const SampArgs sa{keys, rids, n, dmask, p.S, p.r1, h, samp_k, samp_f, p.blocks, defer,
                    bt_words, bucketed ? 2ull * nb : 0ull};
  hipLaunchKernelGGL((k_sample<KT, RT>), dim3(p.blocks), dim3(SAMP_NT), 0, st, sa);
  constexpr int VEC = 16 / sizeof(Raw);
  const bool u8 = tun.filter_unroll == 8;
  const uint32_t grid = tun.filter_grid ? tun.filter_grid : filter_grid(dev);
  const FiltArgs fa{keys, rids, n, dmask, h, surv_k, surv_f, p.cap, grid, p.r1, samp_k, samp_f,
                    p.blocks * p.r1, 0};
  hipLaunchKernelGGL((k_sfinal<KT, RT>), dim3(1), dim3(FILT_NT), 0, st, fa);
  profile_mark(st, true);
  if (u8)
    hipLaunchKernelGGL((k_filter<KT, RT, VEC, 8>), dim3(grid), dim3(FILT_NT), 0, st, fa);
  else
    hipLaunchKernelGGL((k_filter<KT, RT, VEC, 4>), dim3(grid), dim3(FILT_NT), 0, st, fa);
  profile_mark(st, false);
  const TailArgs1 ta{keys, rids, n, dmask, h, surv_k, surv_f, p.cap, cand_k, cand_f,
                     tmp_k, tmp_f, k_eff, out_keys, out_rids, TAIL_SURVIVORS, defer};
  if (bucketed) {
    const size_t hot = align_up((size_t)3 * nb * 4 + 64, 256);
    const BTailArgs bt{ta, bt_words, bt_words + nb, bt_words + 2 * nb,
                       wsp<BMeta>(ws, L.btail + (size_t)3 * nb * 4), wsp<char>(ws, L.btail + hot),
                       wsp<char>(ws, L.btail + hot + align_up((size_t)p.cap * sizeof(U), 256))};
    hipLaunchKernelGGL((k_bhist<KT, RT>), dim3(BT_SLICES), dim3(BT_NT), 0, st, bt);
    hipLaunchKernelGGL((k_bscatter<KT, RT>), dim3(BT_SCATTER), dim3(BSC_NT), 0, st, bt);
    hipLaunchKernelGGL((k_bsort<KT, RT>), dim3(BT_GRID), dim3(TAIL_NT), 0, st, bt);
  } else if (tun.rank_tail)
    hipLaunchKernelGGL((k_rtail<KT, RT>), dim3(rank_grid(k_eff)), dim3(RANK_NT), 0, st, ta);
  else
    hipLaunchKernelGGL((k_tail1<KT, RT>), dim3(1), dim3(TAIL_NT), 0, st, ta);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}

template <int KT, int RT>
int run_input_one_wg(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int order,
                     void* out_keys, void* out_rids, void* ws, hipStream_t st, const WsLayout& L) {
  using U = typename Key<KT>::U;
  const uint64_t dmask = order == TK_ASC ? (uint64_t)(U)~(U)0 : 0ull;
  QHead* h = &wsp<Header>(ws, 0)->q;
  void* cand_k = wsp<char>(ws, L.cand);
  void* cand_f = wsp<char>(ws, L.cand + align_up((size_t)k_eff * sizeof(U), 16));
  void* tmp_k = wsp<char>(ws, L.tmp);
  void* tmp_f = wsp<char>(ws, L.tmp + align_up((size_t)k_eff * sizeof(U), 16));
  const TailArgs1 ta{keys, rids, n, dmask, h, nullptr, nullptr, 0, cand_k, cand_f,
                     tmp_k, tmp_f, k_eff, out_keys, out_rids, TAIL_INPUT, 0};
  hipLaunchKernelGGL((k_tail1<KT, RT>), dim3(1), dim3(TAIL_NT), 0, st, ta);
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}

#define TK_INST(KT, RT)                                                                         \
  template int run_sampled<KT, RT>(const void*, const void*, uint64_t, uint64_t, int, void*,    \
                                   void*, void*, size_t, hipStream_t, const Tuning&,           \
                                   const SamplePlan&);                                          \
  template int run_input_one_wg<KT, RT>(const void*, const void*, uint64_t, uint64_t, int,      \
                                        void*, void*, void*, hipStream_t, const WsLayout&);
TK_INST(KEY_I32, RID_U32)
TK_INST(KEY_I32, RID_U64)
TK_INST(KEY_F32, RID_U32)
TK_INST(KEY_F32, RID_U64)
TK_INST(KEY_I64, RID_U32)
TK_INST(KEY_I64, RID_U64)
TK_INST(KEY_F64, RID_U32)
TK_INST(KEY_F64, RID_U64)
#undef TK_INST

}  // namespace tk
