// Batched Top-K plans: thousands of independent queries of uneven N and K
// over one packed key buffer, run as one multi-query launch (tk_multi.hip):
// sample, threshold, filter and tail workgroups of every query in four
// kernels, replayed from a hipGraph once the pointer set is known.  Host code
// only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "mitopk.h"
#include "tk_internal.hpp"
#include "tk_multi.hpp"
#include "tk_plan.hpp"

using namespace tk;

struct tk_plan {
  int key_type = 0, rid_type = 0;
  uint32_t q = 0;
  tk_plan_params params{};
  Tuning tun;
  std::vector<uint64_t> n, k, off;
  std::vector<int> order;
  std::vector<uint64_t> out_off;  // q + 1 entries
  MLayout L;
  uint64_t rec_bytes = 0;         // argument records, after the layout
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // records on the device match this pointer set
  bool uploaded = false;
  uint64_t u_keys = 0, u_rids = 0, u_ok = 0, u_or = 0;
  MLaunch launch;
  // graph of the launch for one (pointers, stream) combination
  bool have_graph = false;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t g_stream = nullptr;
  bool warm = false;              // this pointer set has run once on g_stream
  // pinned staging of the records: the upload is an asynchronous copy on the
  // launch stream; the event marks when the copy has read the staging
  char* h_stage = nullptr;
  hipEvent_t staged = nullptr;
  bool stage_pending = false;
  std::mutex mu;
};

namespace {

constexpr uint32_t PLAN_MAX_SAMPLE_LOG2 = 14;

Tuning plan_tuning(const tk_plan_params* p) {
  Tuning t = current_tuning();
  t.force_exact = 0;
  t.force_cap = 0;
  t.min_sample_log2 = 12;
  // a batch's samples are read by one launch before any filter: at most 2^14
  // keys per query keeps that launch short (2^20 cost 7 % of the C3 batch)
  t.max_sample_log2 = PLAN_MAX_SAMPLE_LOG2;
  if (p) {
    if (p->min_sample_log2) t.min_sample_log2 = p->min_sample_log2;
    if (p->max_sample_log2) t.max_sample_log2 = p->max_sample_log2;
    if (p->sample_sigma > 0) t.sample_sigma = p->sample_sigma;
    if (p->cap_sigma > 0) t.cap_sigma = p->cap_sigma;
  }
  return t;
}

bool valid_inputs(const uint64_t* offsets, const uint32_t* ks, const uint8_t* orders, uint32_t q,
                  int key_type, int rid_type, const tk_plan_params* params) {
  if (!offsets || !ks || !orders || q == 0) return false;
  if (key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1) return false;
  if (params && ((params->tile_keys && params->tile_keys < 4096) ||
                 params->min_sample_log2 > 24 || params->max_sample_log2 > 24))
    return false;
  for (uint32_t i = 0; i < q; ++i) {
    if (offsets[i + 1] < offsets[i]) return false;
    if (orders[i] > 1) return false;
    if (rid_type == TK_RID_U32 && offsets[i + 1] - offsets[i] > (1ull << 32)) return false;
  }
  return true;
}

// Layout of the plan; returns the workspace bytes.
size_t build(tk_plan& P, const uint64_t* offsets, const uint32_t* ks, const uint8_t* orders) {
  const uint32_t q = P.q;
  P.n.resize(q);
  P.k.resize(q);
  P.off.assign(offsets, offsets + q + 1);
  P.order.resize(q);
  P.out_off.assign(q + 1, 0);
  for (uint32_t i = 0; i < q; ++i) {
    P.n[i] = offsets[i + 1] - offsets[i];
    P.k[i] = ks[i];
    P.order[i] = orders[i];
    P.out_off[i + 1] = P.out_off[i] + std::min<uint64_t>(ks[i], P.n[i]);
  }
  const uint64_t lay = multi_layout(P.n, P.k, P.key_type, P.rid_type, P.tun, P.params.tile_keys, P.L);
  MRecords sizes;
  sizes.sa.resize(P.L.n_sampled);
  sizes.smap.resize(P.L.n_samp_blocks);
  sizes.fa.resize(P.L.n_sampled);
  sizes.fmap.resize(P.L.n_filt_blocks);
  sizes.ta.resize(P.L.n_sampled + P.L.n_input);
  sizes.tq.resize(P.L.n_sampled + P.L.n_input);
  P.rec_bytes = multi_pack_bytes(sizes);
  return lay + P.rec_bytes + align_up((uint64_t)(q + 1) * sizeof(unsigned long long), 256);
}

// Device address of the plan's completion stamps: after the layout and the records.
unsigned long long* stamps_of(tk_plan& P) {
  return reinterpret_cast<unsigned long long*>(P.ws + P.L.total + P.rec_bytes);
}

int upload(tk_plan& P, const void* keys, const void* rowids, void* out_keys, void* out_rowids,
           hipStream_t st) {
  const uint32_t kb = key_bytes(P.key_type), rb = P.rid_type == TK_RID_U64 ? 8 : 4;
  std::vector<MQuery> qs(P.q);
  for (uint32_t i = 0; i < P.q; ++i) {
    MQuery& m = qs[i];
    m.keys = static_cast<const char*>(keys) + P.off[i] * kb;
    m.rids = rowids ? static_cast<const char*>(rowids) + P.off[i] * rb : nullptr;
    m.n = P.n[i];
    m.k = P.k[i];
    m.order = P.order[i];
    m.out_keys = out_keys ? static_cast<char*>(out_keys) + P.out_off[i] * kb : nullptr;
    m.out_rids = static_cast<char*>(out_rowids) + P.out_off[i] * rb;
  }
  MRecords r;
  multi_records(qs, P.L, P.key_type, P.rid_type, P.ws, r);
  const uint64_t bytes = multi_pack_bytes(r);
  if (bytes != P.rec_bytes) return TK_EINVAL;
  // the staging is rewritten only once the previous upload's copy has read it
  // (in practice long done: uploads happen when the pointer set changes)
  if (P.stage_pending && hipEventSynchronize(P.staged) != hipSuccess) return TK_EHIP;
  P.stage_pending = false;
  char* dev = P.ws + P.L.total;
  P.launch = multi_pack(r, P.h_stage, dev);
  P.launch.filt_grid = P.params.filter_grid;
  P.launch.stamps = stamps_of(P);
  if (hipMemcpyAsync(dev, P.h_stage, bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(P.staged, st) != hipSuccess)
    return TK_EHIP;
  P.stage_pending = true;
  return TK_OK;
}

void release(tk_plan* P) {
  if (P->stage_pending) (void)hipEventSynchronize(P->staged);
  if (P->staged) (void)hipEventDestroy(P->staged);
  if (P->h_stage) (void)hipHostFree(P->h_stage);
  delete P;
}

void drop_graph(tk_plan& P) {
  if (P.have_graph) {
    (void)hipGraphExecDestroy(P.gexec);
    (void)hipGraphDestroy(P.graph);
    P.have_graph = false;
  }
}

}  // namespace

extern "C" size_t tk_plan_workspace_size(const uint64_t* offsets, const uint32_t* ks,
                                         const uint8_t* orders, uint32_t q, int key_type,
                                         int rid_type, const tk_plan_params* params) {
  if (!valid_inputs(offsets, ks, orders, q, key_type, rid_type, params)) return 0;
  tk_plan P;
  P.key_type = key_type;
  P.rid_type = rid_type;
  P.q = q;
  if (params) P.params = *params;
  P.tun = plan_tuning(params);
  return build(P, offsets, ks, orders);
}

extern "C" int tk_plan_create(const uint64_t* offsets, const uint32_t* ks, const uint8_t* orders,
                              uint32_t q, int key_type, int rid_type,
                              const tk_plan_params* params, void* workspace,
                              size_t workspace_bytes, tk_plan** out) {
  if (!out || !valid_inputs(offsets, ks, orders, q, key_type, rid_type, params)) return TK_EINVAL;
  if (!workspace || ((uintptr_t)workspace & 255u)) return TK_EINVAL;
  tk_plan* P = new (std::nothrow) tk_plan;
  if (!P) return TK_ENOMEM;
  P->key_type = key_type;
  P->rid_type = rid_type;
  P->q = q;
  if (params) P->params = *params;
  P->tun = plan_tuning(params);
  const size_t need = build(*P, offsets, ks, orders);
  if (workspace_bytes < need) {
    delete P;
    return TK_EINVAL;
  }
  if (hipHostMalloc((void**)&P->h_stage, P->rec_bytes ? P->rec_bytes : 256, hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&P->staged, hipEventDisableTiming) != hipSuccess) {
    release(P);
    return TK_EHIP;
  }
  P->ws = static_cast<char*>(workspace);
  P->ws_bytes = workspace_bytes;
  *out = P;
  return TK_OK;
}

extern "C" int tk_plan_output_offsets(const tk_plan* P, uint64_t* out_offsets) {
  if (!P || !out_offsets) return TK_EINVAL;
  std::memcpy(out_offsets, P->out_off.data(), P->out_off.size() * sizeof(uint64_t));
  return TK_OK;
}

extern "C" int tk_plan_info(const tk_plan* P, uint32_t* n_sampled, uint32_t* n_exact,
                            uint32_t* n_items) {
  if (!P) return TK_EINVAL;
  if (n_sampled) *n_sampled = P->L.n_sampled;
  if (n_exact) *n_exact = P->L.n_input;
  if (n_items)
    *n_items = (uint32_t)(P->L.n_samp_blocks + P->L.n_sampled + P->L.n_filt_blocks +
                          P->L.n_sampled + P->L.n_input);
  return TK_OK;
}

extern "C" int tk_plan_launch(tk_plan* P, const void* keys, const void* rowids, void* out_keys,
                              void* out_rowids, void* stream) {
  if (!P || !keys || !out_rowids) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(P->mu);
  hipStream_t st = (hipStream_t)stream;
  const uint64_t gk = (uint64_t)(uintptr_t)keys, gr = (uint64_t)(uintptr_t)rowids,
                 go = (uint64_t)(uintptr_t)out_keys, gq = (uint64_t)(uintptr_t)out_rowids;
  if (!P->uploaded || P->u_keys != gk || P->u_rids != gr || P->u_ok != go || P->u_or != gq) {
    drop_graph(*P);
    P->warm = false;
    const int rc = upload(*P, keys, rowids, out_keys, out_rowids, st);
    if (rc != TK_OK) return rc;
    P->uploaded = true;
    P->u_keys = gk;
    P->u_rids = gr;
    P->u_ok = go;
    P->u_or = gq;
  }
  // graphs need a created stream; the first launch of a pointer set on a
  // stream runs eagerly (it also loads the kernels' code object)
  const bool graph = P->params.use_graph >= 0 && st != nullptr;
  if (!graph || !P->warm || P->g_stream != st) {
    if (P->g_stream != st) drop_graph(*P);
    P->g_stream = st;
    P->warm = true;
    multi_enqueue(P->launch, P->key_type, P->rid_type, st);
    return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
  }
  if (!P->have_graph) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return TK_EHIP;
    multi_enqueue(P->launch, P->key_type, P->rid_type, st);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || !g || hipGetLastError() != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return TK_EHIP;
    }
    if (hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return TK_EHIP;
    }
    P->graph = g;
    P->have_graph = true;
  }
  return hipGraphLaunch(P->gexec, st) == hipSuccess ? TK_OK : TK_EHIP;
}

extern "C" int tk_plan_query_times(const tk_plan* P, double* seconds) {
  if (!P || !seconds) return TK_EINVAL;
  if (!P->uploaded) return TK_EINVAL;  // no launch yet
  std::vector<unsigned long long> st(P->q + 1);
  if (hipMemcpy(st.data(), const_cast<tk_plan*>(P)->ws + P->L.total + P->rec_bytes,
                st.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
    return TK_EHIP;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return TK_EHIP;
  const double hz = (double)khz * 1e3;
  for (uint32_t i = 0; i < P->q; ++i)
    seconds[i] = P->L.cls[i] == MC_EMPTY ? 0.0 : (double)(int64_t)(st[1 + i] - st[0]) / hz;
  return TK_OK;
}

extern "C" int tk_plan_stats(const tk_plan* P, uint32_t* fallbacks, uint32_t* unfinished) {
  if (!P) return TK_EINVAL;
  std::vector<QHead> hs(P->L.n_sampled);
  if (!hs.empty() &&
      hipMemcpy(hs.data(), P->ws, hs.size() * sizeof(QHead), hipMemcpyDeviceToHost) != hipSuccess)
    return TK_EHIP;
  uint32_t fb = 0, un = 0;
  for (const QHead& h : hs) {
    if (h.path == 4u) ++fb;
    if (h.path != 2u && h.path != 4u) ++un;
  }
  if (fallbacks) *fallbacks = fb;
  if (unfinished) *unfinished = un;
  return TK_OK;
}

extern "C" void tk_plan_destroy(tk_plan* P) {
  if (!P) return;
  drop_graph(*P);
  release(P);
}

// ---- per-query launches from C: the baseline of the batched form ---------------------------

extern "C" size_t tk_topk_each_workspace_size(const uint64_t* offsets, const uint32_t* ks,
                                              uint32_t q, int key_type, int rid_type) {
  if (!offsets || !ks || key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1) return 0;
  size_t m = 256;
  for (uint32_t i = 0; i < q; ++i) {
    if (offsets[i + 1] < offsets[i]) return 0;
    const size_t w = tk_workspace_size(offsets[i + 1] - offsets[i], ks[i], key_type, rid_type);
    m = w > m ? w : m;
  }
  return align_up(m, 256);
}

extern "C" int tk_topk_each(const void* keys, const void* rowids, const uint64_t* offsets,
                            const uint32_t* ks, const uint8_t* orders, uint32_t q, int key_type,
                            int rid_type, void* out_keys, void* out_rowids, void* workspace,
                            size_t workspace_bytes, void* const* streams, uint32_t nstreams,
                            double* seconds) {
  if (!keys || !out_rowids || !offsets || !ks || !orders || !workspace || !streams || nstreams == 0)
    return TK_EINVAL;
  if (key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1) return TK_EINVAL;
  const size_t per = tk_topk_each_workspace_size(offsets, ks, q, key_type, rid_type);
  if (per == 0 || workspace_bytes < per * nstreams || ((uintptr_t)workspace & 255u)) return TK_EINVAL;
  const uint32_t kb = key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  // events: one start on stream 0 that every stream waits for, one per query
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  };
  if (seconds) {
    ev.assign((size_t)q + 1, nullptr);
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        cleanup();
        return TK_EHIP;
      }
    if (hipEventRecord(ev[0], (hipStream_t)streams[0]) != hipSuccess) {
      cleanup();
      return TK_EHIP;
    }
    for (uint32_t s = 1; s < nstreams; ++s)
      if (hipStreamWaitEvent((hipStream_t)streams[s], ev[0], 0) != hipSuccess) {
        cleanup();
        return TK_EHIP;
      }
  }
  uint64_t out = 0;
  int rc = TK_OK;
  for (uint32_t i = 0; i < q && rc == TK_OK; ++i) {
    const uint32_t s = i % nstreams;
    const uint64_t n = offsets[i + 1] - offsets[i];
    rc = tk_topk(static_cast<const char*>(keys) + offsets[i] * kb,
                 rowids ? static_cast<const char*>(rowids) + offsets[i] * rb : nullptr, n, ks[i],
                 key_type, rid_type, orders[i],
                 out_keys ? static_cast<char*>(out_keys) + out * kb : nullptr,
                 static_cast<char*>(out_rowids) + out * rb, nullptr,
                 static_cast<char*>(workspace) + (size_t)s * per, per, streams[s]);
    if (rc == TK_OK && seconds && hipEventRecord(ev[1 + i], (hipStream_t)streams[s]) != hipSuccess)
      rc = TK_EHIP;
    out += ks[i] < n ? ks[i] : n;
  }
  if (rc == TK_OK && seconds) {
    for (uint32_t i = 0; i < q && rc == TK_OK; ++i) {
      float ms = 0;
      if (hipEventSynchronize(ev[1 + i]) != hipSuccess ||
          hipEventElapsedTime(&ms, ev[0], ev[1 + i]) != hipSuccess)
        rc = TK_EHIP;
      seconds[i] = ms * 1e-3;
    }
  }
  cleanup();
  return rc;
}
