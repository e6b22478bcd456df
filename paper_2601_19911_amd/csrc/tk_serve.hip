// Served form: continuous batching of Top-K requests over key columns, with
// the cost-accounted gate of the paper (sec. II-B, the "Risky Gate"): a
// request goes to the GPU only when the estimated CPU cost exceeds the
// estimated offload cost (host-link transfer of a host-resident column's rows,
// kernels, result return) by more than a margin; otherwise it runs on the
// host with the multithreaded CPU path.  Host code only.
//
// Threads: the caller submits; a batcher thread forms micro-batches of one key
// type whenever a slot (stream + device arena + pinned staging) is free,
// admitting requests while the slot's arena has room, and enqueues the
// batch's multi-query launch (tk_multi.hip) on that slot's stream followed by
// an asynchronous copy of the results to pinned host memory and an event; a
// completion thread waits on
// the slots' events in launch order and publishes the results; CPU workers run
// the gated-off requests.  With two or more slots, micro-batches overlap on
// the device, and requests that arrive while others run join the next batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mitopk.h"
#include "tk_internal.hpp"
#include "tk_multi.hpp"
#include "tk_plan.hpp"

using namespace tk;

namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Column {
  const void* d_keys;  // nullptr: host-resident, the GPU route copies the rows it needs
  const void* h_keys;  // nullptr: no host copy, GPU route only
  uint64_t n;
  int key_type;
};

struct Req {
  uint64_t id;
  uint32_t col;
  uint64_t offset, n;
  uint32_t k;
  int order;
  int route;  // 0 GPU, 1 CPU
  std::atomic<int> state{0};  // 0 queued, 1 running, 2 done (released when taken)
  int status = 0;
  uint64_t t_submit = 0, t_start = 0, t_done = 0;
  std::vector<uint8_t> out_keys;
  std::vector<uint64_t> out_rids;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* arena = nullptr;      // device
  size_t arena_bytes = 0;
  char* h_stage = nullptr;    // pinned: descriptors, queue, sample map
  char* h_out = nullptr;      // pinned: results
  size_t stage_bytes = 0, out_bytes = 0;
  std::vector<uint64_t> reqs;
  std::vector<uint64_t> out_off;
  uint64_t out_rid_base = 0;   // where row-ids start in h_out
  int key_type = 0;
  bool busy = false;
};

}  // namespace

struct tk_server {
  tk_server_cfg cfg{};
  std::vector<Column> cols;
  // live requests by id (stable addresses); a request is released once its
  // result is taken, so the server holds only queued, running and untaken ones
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  uint64_t next_id = 0;
  std::mutex mu;
  std::condition_variable cv_batch, cv_cpu, cv_done, cv_slot;
  std::deque<uint64_t> gpu_q[4];  // per key type
  std::deque<uint64_t> cpu_q;
  std::vector<Slot> slots;
  std::deque<int> inflight;  // slot indices in launch order
  std::vector<std::thread> workers;
  std::thread batcher, completer;
  bool stop = false;
  uint64_t submitted = 0, completed = 0, n_gpu = 0, n_cpu = 0, n_batches = 0, n_batched = 0;
  uint64_t n_failed = 0;
  int dev = 0;
  Req& req(uint64_t id) { return *reqs.at(id); }
};

namespace {

double cpu_cost(const tk_cost_model& c, uint64_t n, uint32_t k) {
  return c.cpu_a * (double)n + c.cpu_b * (double)k * std::log2((double)k + 1.0) + c.cpu_c;
}
// offload cost: kernels and result return, plus the host-link transfer of the
// request's key bytes when the column has no device copy (the gate's B)
double gpu_cost(const tk_cost_model& c, uint64_t n, uint32_t k, double bytes, double h2d) {
  return c.gpu_a * (double)n + c.gpu_b * (double)k + c.gpu_c + bytes / h2d;
}

bool all_zero(const tk_cost_model& c) {
  return c.cpu_a == 0 && c.cpu_b == 0 && c.cpu_c == 0 && c.gpu_a == 0 && c.gpu_b == 0 && c.gpu_c == 0;
}

// Default cost models per key type (tk_key_t order): fits on relative
// residuals of measured request times over N = 2^10 .. 2^20 and K in {10,
// 100, 1000, 10000} on an MI355X (device-resident keys, launch to results on
// the host) and of the CPU route on 16 host threads.
constexpr tk_cost_model DEFAULT_COST[4] = {
    {5.09e-10, 2.36e-9, 2.56e-5, 1.49e-11, 6.62e-9, 3.40e-5},  // int32
    {4.88e-10, 2.67e-9, 2.14e-5, 1.54e-11, 6.96e-9, 3.71e-5},  // int64
    {5.01e-10, 2.45e-9, 2.31e-5, 1.39e-11, 6.54e-9, 3.53e-5},  // float32
    {4.88e-10, 2.41e-9, 2.58e-5, 1.39e-11, 6.89e-9, 3.88e-5},  // float64
};
constexpr double DEFAULT_H2D = 5.0e10;

void finish(tk_server* s, uint64_t id) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    Req& r = s->req(id);
    r.t_done = now_ns();
    r.state.store(2);
    if (r.status != TK_OK) ++s->n_failed;
    ++s->completed;
  }
  s->cv_done.notify_all();
}

void cpu_worker(tk_server* s) {
  for (;;) {
    uint64_t id;
    Req* rp;
    Column c;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_cpu.wait(lk, [&] { return s->stop || !s->cpu_q.empty(); });
      if (s->stop && s->cpu_q.empty()) return;
      id = s->cpu_q.front();
      s->cpu_q.pop_front();
      rp = &s->req(id);
      c = s->cols[rp->col];
    }
    Req& r = *rp;
    r.t_start = now_ns();
    const uint32_t kb = key_bytes(c.key_type);
    const uint64_t ke = std::min<uint64_t>(r.k, r.n);
    r.out_keys.resize(ke * kb);
    r.out_rids.resize(ke);
    uint64_t cnt = 0;
    r.status = tk_cpu_topk(static_cast<const char*>(c.h_keys) + r.offset * kb, nullptr, r.n, r.k,
                           c.key_type, TK_RID_U64, r.order, r.out_keys.data(), r.out_rids.data(),
                           &cnt, 1);
    for (auto& x : r.out_rids) x += r.offset;
    finish(s, id);
  }
}

struct Taken {
  Req* r;
  const void* d_keys;  // column's device keys, or nullptr (host-resident: staged in the arena)
  const void* h_keys;  // column's host keys
  uint64_t offset, n;
  uint32_t k;
  int order;
};

// A micro-batch laid out in a slot's arena:
//   [batch workspace: query states, then each query's regions][argument
//   records][result keys][result row-ids][rows of host-resident requests]
struct BatchBuild {
  MLayout L;
  MRecords rec;
  std::vector<uint64_t> out_off;
  std::vector<uint64_t> stage_off;  // arena offset of each host-resident request's rows
  uint64_t off_rec = 0, rec_bytes = 0, off_out_k = 0, off_out_r = 0, off_rows = 0, end = 0;
  size_t stage_need = 0, out_need = 0;  // pinned staging and result bytes the batch needs
};

// Lays out a micro-batch for a slot; returns false if it does not fit the
// slot's arena, its pinned staging or its pinned result buffer.
bool build_batch(const std::vector<Taken>& ids, int key_type, const Slot& sl, BatchBuild& b) {
  const uint32_t kb = key_bytes(key_type), rb = 8;
  const size_t q = ids.size();
  Tuning t = current_tuning();
  t.force_exact = 0;
  t.force_cap = 0;
  t.min_sample_log2 = 12;
  t.max_sample_log2 = 14;  // as for plans: the batch's samples precede every filter
  std::vector<uint64_t> n(q), k(q);
  b.out_off.assign(q + 1, 0);
  for (size_t i = 0; i < q; ++i) {
    n[i] = ids[i].n;
    k[i] = ids[i].k;
    b.out_off[i + 1] = b.out_off[i] + std::min<uint64_t>(ids[i].k, ids[i].n);
  }
  uint64_t off = multi_layout(n, k, key_type, TK_RID_U64, t, 0, b.L);
  // records need the output addresses, which follow the records: size them first
  MRecords sizes;
  sizes.sa.resize(b.L.n_sampled);
  sizes.smap.resize(b.L.n_samp_blocks);
  sizes.fa.resize(b.L.n_sampled);
  sizes.fmap.resize(b.L.n_filt_blocks);
  sizes.ta.resize(b.L.n_sampled + b.L.n_input);
  sizes.tq.resize(b.L.n_sampled + b.L.n_input);
  b.off_rec = off;
  b.rec_bytes = multi_pack_bytes(sizes);
  off = align_up(off + b.rec_bytes, 256);
  b.off_out_k = off;
  off = align_up(off + b.out_off[q] * kb, 256);
  b.off_out_r = off;
  off = align_up(off + b.out_off[q] * rb, 256);
  b.off_rows = off;
  b.stage_off.assign(q, 0);
  for (size_t i = 0; i < q; ++i)
    if (!ids[i].d_keys) {
      b.stage_off[i] = off;
      off = align_up(off + ids[i].n * kb, 256);
    }
  b.end = off;
  b.stage_need = b.L.heads_bytes + b.rec_bytes;
  b.out_need = b.off_rows - b.off_out_k;
  if (off > sl.arena_bytes || b.stage_need > sl.stage_bytes || b.out_need > sl.out_bytes) return false;
  std::vector<MQuery> qs(q);
  for (size_t i = 0; i < q; ++i) {
    MQuery& m = qs[i];
    m.keys = ids[i].d_keys ? static_cast<const char*>(ids[i].d_keys) + ids[i].offset * kb
                           : static_cast<const char*>(sl.arena + b.stage_off[i]);
    m.rids = nullptr;  // local index; the column offset is added on the host
    m.n = ids[i].n;
    m.k = ids[i].k;
    m.order = ids[i].order;
    m.out_keys = sl.arena + b.off_out_k + b.out_off[i] * kb;
    m.out_rids = sl.arena + b.off_out_r + b.out_off[i] * rb;
  }
  multi_records(qs, b.L, key_type, TK_RID_U64, sl.arena, b.rec);
  return true;
}

void batcher_loop(tk_server* s) {
  hipSetDevice(s->dev);
  const double window_ns = s->cfg.window_us * 1e3;
  for (;;) {
    int slot = -1;
    std::vector<Taken> take;
    int kt = 0;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_batch.wait(lk, [&] {
        if (s->stop) return true;
        bool any = false;
        for (const auto& q : s->gpu_q) any = any || !q.empty();
        if (!any) return false;
        for (auto& sl : s->slots)
          if (!sl.busy) return true;
        return false;
      });
      if (s->stop) return;
      // the key type whose oldest request waited longest
      uint64_t best = UINT64_MAX;
      for (int t = 0; t < 4; ++t)
        if (!s->gpu_q[t].empty() && s->req(s->gpu_q[t].front()).t_submit < best) {
          best = s->req(s->gpu_q[t].front()).t_submit;
          kt = t;
        }
      // a short window lets a batch fill when it would otherwise be tiny
      if (window_ns > 0 && s->gpu_q[kt].size() < s->cfg.max_batch) {
        const uint64_t deadline = best + (uint64_t)window_ns;
        const uint64_t tn = now_ns();
        if (tn < deadline) {
          lk.unlock();
          std::this_thread::sleep_for(std::chrono::nanoseconds(std::min<uint64_t>(deadline - tn, 200000)));
          lk.lock();
          if (s->stop) return;
        }
      }
      for (size_t i = 0; i < s->slots.size(); ++i)
        if (!s->slots[i].busy) {
          slot = (int)i;
          break;
        }
      if (slot < 0) continue;
      auto& q = s->gpu_q[kt];
      while (!q.empty() && take.size() < s->cfg.max_batch) {
        Req& r = s->req(q.front());
        const Column& c = s->cols[r.col];
        take.push_back(Taken{&r, c.d_keys, c.h_keys, r.offset, r.n, r.k, r.order});
        q.pop_front();
      }
      s->slots[slot].busy = true;
    }
    Slot& sl = s->slots[slot];
    // admission by memory: shrink the batch until it fits the slot's arena,
    // staging and result buffers
    BatchBuild b;
    bool fits = false;
    while (!take.empty() && !(fits = build_batch(take, kt, sl, b))) {
      if (take.size() == 1) break;
      std::lock_guard<std::mutex> lk(s->mu);
      s->gpu_q[kt].push_front(take.back().r->id);
      take.pop_back();
    }
    if (!fits) {
      // a single request larger than a slot: the CPU route takes it when its
      // column has a host copy; otherwise it fails (no valid host address)
      bool any_cpu = false;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        for (const Taken& t : take) {
          if (t.h_keys) {
            t.r->route = 1;
            ++s->n_cpu;
            --s->n_gpu;
            s->cpu_q.push_back(t.r->id);
            any_cpu = true;
          } else {
            t.r->status = TK_ENOMEM;
            t.r->t_start = t.r->t_done = now_ns();
            t.r->state.store(2);
            ++s->n_failed;
            ++s->completed;
          }
        }
        sl.busy = false;
      }
      if (any_cpu) s->cv_cpu.notify_all();
      s->cv_done.notify_all();
      s->cv_batch.notify_all();
      continue;
    }
    const uint64_t t0 = now_ns();
    const uint32_t kb = key_bytes(kt);
    // staging: zeroed query states, then the argument records
    std::memset(sl.h_stage, 0, b.L.heads_bytes);
    const MLaunch m = multi_pack(b.rec, sl.h_stage + b.L.heads_bytes, sl.arena + b.off_rec);
    int rc = TK_OK;
    for (size_t i = 0; rc == TK_OK && i < take.size(); ++i)
      if (!take[i].d_keys &&
          hipMemcpyAsync(sl.arena + b.stage_off[i], static_cast<const char*>(take[i].h_keys) + take[i].offset * kb,
                         take[i].n * kb, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
        rc = TK_EHIP;
    if (rc == TK_OK && b.L.heads_bytes &&
        hipMemcpyAsync(sl.arena, sl.h_stage, b.L.heads_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
      rc = TK_EHIP;
    if (rc == TK_OK && b.rec_bytes &&
        hipMemcpyAsync(sl.arena + b.off_rec, sl.h_stage + b.L.heads_bytes, b.rec_bytes,
                       hipMemcpyHostToDevice, sl.stream) != hipSuccess)
      rc = TK_EHIP;
    if (rc == TK_OK) {
      multi_enqueue(m, kt, TK_RID_U64, sl.stream);
      if (hipGetLastError() != hipSuccess) rc = TK_EHIP;
    }
    if (rc == TK_OK)
      rc = hipMemcpyAsync(sl.h_out, sl.arena + b.off_out_k, b.out_need, hipMemcpyDeviceToHost,
                          sl.stream) == hipSuccess ? TK_OK : TK_EHIP;
    if (rc == TK_OK) rc = hipEventRecord(sl.done, sl.stream) == hipSuccess ? TK_OK : TK_EHIP;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      sl.reqs.clear();
      for (const Taken& t : take) sl.reqs.push_back(t.r->id);
      sl.out_off = b.out_off;
      sl.out_rid_base = b.off_out_r - b.off_out_k;
      sl.key_type = kt;
      for (const Taken& t : take) {
        t.r->t_start = t0;
        t.r->status = rc;
        t.r->state.store(1);
      }
      s->inflight.push_back(slot);
      ++s->n_batches;
      s->n_batched += take.size();
    }
    s->cv_slot.notify_all();
  }
}

void completer_loop(tk_server* s) {
  hipSetDevice(s->dev);
  for (;;) {
    int slot;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_slot.wait(lk, [&] { return s->stop || !s->inflight.empty(); });
      if (s->inflight.empty()) return;
      slot = s->inflight.front();
      s->inflight.pop_front();
    }
    Slot& sl = s->slots[slot];
    const hipError_t e = hipEventSynchronize(sl.done);
    const uint32_t kb = key_bytes(sl.key_type);
    const uint64_t tdone = now_ns();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (size_t i = 0; i < sl.reqs.size(); ++i) {
        Req& r = s->req(sl.reqs[i]);
        const uint64_t a = sl.out_off[i], c = sl.out_off[i + 1] - a;
        r.out_keys.assign(sl.h_out + a * kb, sl.h_out + (a + c) * kb);
        r.out_rids.resize(c);
        std::memcpy(r.out_rids.data(), sl.h_out + sl.out_rid_base + a * 8, c * 8);
        for (auto& x : r.out_rids) x += r.offset;  // local index -> column row
        if (e != hipSuccess) r.status = TK_EHIP;
        if (r.status != TK_OK) ++s->n_failed;
        r.t_done = tdone;
        r.state.store(2);
        ++s->completed;
      }
      sl.reqs.clear();
      sl.busy = false;
    }
    s->cv_done.notify_all();
    s->cv_batch.notify_all();
  }
}

}  // namespace

extern "C" int tk_server_create(const tk_server_cfg* cfg, void* arena, size_t arena_bytes,
                                tk_server** out) {
  if (!cfg || !out || !arena || ((uintptr_t)arena & 255u)) return TK_EINVAL;
  tk_server* s = new (std::nothrow) tk_server;
  if (!s) return TK_ENOMEM;
  s->cfg = *cfg;
  for (int t = 0; t < 4; ++t)
    if (all_zero(s->cfg.cost[t])) s->cfg.cost[t] = DEFAULT_COST[t];
  if (!(s->cfg.h2d_bytes_per_s > 0)) s->cfg.h2d_bytes_per_s = DEFAULT_H2D;
  if (s->cfg.max_batch == 0) s->cfg.max_batch = 256;
  if (s->cfg.slots == 0) s->cfg.slots = 2;
  if (s->cfg.cpu_threads <= 0) s->cfg.cpu_threads = 4;
  if (hipGetDevice(&s->dev) != hipSuccess) {
    delete s;
    return TK_EHIP;
  }
  const size_t per = (arena_bytes / s->cfg.slots) & ~(size_t)255;
  s->slots.resize(s->cfg.slots);
  for (uint32_t i = 0; i < s->cfg.slots; ++i) {
    Slot& sl = s->slots[i];
    sl.arena = static_cast<char*>(arena) + i * per;
    sl.arena_bytes = per;
    sl.stage_bytes = std::min<size_t>(per, (size_t)64 << 20);
    sl.out_bytes = std::min<size_t>(per, (size_t)64 << 20);
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.h_stage, sl.stage_bytes, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.h_out, sl.out_bytes, hipHostMallocDefault) != hipSuccess) {
      tk_server_destroy(s);
      return TK_EHIP;
    }
  }
  s->batcher = std::thread(batcher_loop, s);
  s->completer = std::thread(completer_loop, s);
  for (int i = 0; i < s->cfg.cpu_threads; ++i) s->workers.emplace_back(cpu_worker, s);
  *out = s;
  return TK_OK;
}

extern "C" int tk_server_add_column(tk_server* s, const void* d_keys, const void* h_keys,
                                    uint64_t n, int key_type, uint32_t* col) {
  if (!s || !col || key_type < 0 || key_type > 3 || (n && !d_keys && !h_keys)) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  s->cols.push_back(Column{d_keys, h_keys, n, key_type});
  *col = (uint32_t)(s->cols.size() - 1);
  return TK_OK;
}

extern "C" int tk_server_submit(tk_server* s, uint32_t col, uint64_t offset, uint64_t n,
                                uint32_t k, int order, uint64_t* req_id) {
  if (!s || !req_id || order < 0 || order > 1) return TK_EINVAL;
  const uint64_t t = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (col >= s->cols.size() || offset > s->cols[col].n || n > s->cols[col].n - offset) return TK_EINVAL;
  const Column& c = s->cols[col];
  std::unique_ptr<Req> rp(new (std::nothrow) Req);
  if (!rp) return TK_ENOMEM;
  const uint64_t id = s->next_id++;
  Req& r = *rp;
  r.id = id;
  r.col = col;
  r.offset = offset;
  r.n = n;
  r.k = k;
  r.order = order;
  r.t_submit = t;
  // the gate: CPU unless offloading saves more than the margin; a column with
  // no device copy pays the transfer of the request's rows on the GPU route
  int route = 0;
  if (s->cfg.gate == 2) route = 1;
  else if (s->cfg.gate == 1 && c.h_keys) {
    const uint32_t ke = (uint64_t)k < n ? k : (uint32_t)n;  // the work is min(k, n) results
    const tk_cost_model& m = s->cfg.cost[c.key_type];
    const double bytes = c.d_keys ? 0.0 : (double)n * key_bytes(c.key_type);
    const double saving = cpu_cost(m, n, ke) - gpu_cost(m, n, ke, bytes, s->cfg.h2d_bytes_per_s);
    route = saving > s->cfg.margin_ms * 1e-3 ? 0 : 1;
  }
  if (route == 1 && !c.h_keys) route = 0;
  r.route = route;
  s->reqs.emplace(id, std::move(rp));
  ++s->submitted;
  if (route == 1) {
    ++s->n_cpu;
    s->cpu_q.push_back(id);
    s->cv_cpu.notify_one();
  } else {
    ++s->n_gpu;
    s->gpu_q[c.key_type].push_back(id);
    s->cv_batch.notify_one();
  }
  *req_id = id;
  return TK_OK;
}

extern "C" int tk_server_result(tk_server* s, uint64_t id, void* h_keys, uint64_t* h_rowids,
                                tk_req_info* info) {
  if (!s) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return TK_EINVAL;
  Req& r = *it->second;
  if (r.state.load() < 2) return TK_EAGAIN;
  if (h_keys && !r.out_keys.empty()) std::memcpy(h_keys, r.out_keys.data(), r.out_keys.size());
  if (h_rowids && !r.out_rids.empty()) std::memcpy(h_rowids, r.out_rids.data(), r.out_rids.size() * 8);
  if (info) {
    info->t_submit_ns = r.t_submit;
    info->t_start_ns = r.t_start;
    info->t_done_ns = r.t_done;
    info->route = r.route;
    info->status = r.status;
    info->count = r.out_rids.size();
  }
  const int st = r.status;
  s->reqs.erase(it);  // taken: the request and its results are released
  return st;
}

extern "C" int tk_server_drain(tk_server* s) {
  if (!s) return TK_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->completed >= s->submitted; });
  return TK_OK;
}

extern "C" int tk_server_stats(tk_server* s, tk_server_counters* st) {
  if (!s || !st) return TK_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->completed = s->completed;
  st->routed_gpu = s->n_gpu;
  st->routed_cpu = s->n_cpu;
  st->batches = s->n_batches;
  st->batched_requests = s->n_batched;
  st->live = s->reqs.size();
  st->failed = s->n_failed;
  return TK_OK;
}

extern "C" int tk_server_replay(tk_server* s, uint64_t count, const double* t_arrival_s,
                                const uint32_t* cols, const uint64_t* offsets, const uint64_t* ns,
                                const uint32_t* ks, const uint8_t* orders, uint64_t* req_ids) {
  if (!s || !t_arrival_s || !cols || !offsets || !ns || !ks || !orders || !req_ids) return TK_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint64_t i = 0; i < count; ++i) {
    const auto due = t0 + std::chrono::nanoseconds((int64_t)(t_arrival_s[i] * 1e9));
    while (std::chrono::steady_clock::now() < due) {
      const auto left = due - std::chrono::steady_clock::now();
      if (left > std::chrono::microseconds(200)) std::this_thread::sleep_for(left - std::chrono::microseconds(100));
    }
    const int rc = tk_server_submit(s, cols[i], offsets[i], ns[i], ks[i], orders[i], &req_ids[i]);
    if (rc != TK_OK) return rc;
  }
  return TK_OK;
}

extern "C" void tk_server_destroy(tk_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_batch.notify_all();
  s->cv_cpu.notify_all();
  s->cv_slot.notify_all();
  if (s->batcher.joinable()) s->batcher.join();
  if (s->completer.joinable()) s->completer.join();
  for (auto& w : s->workers)
    if (w.joinable()) w.join();
  for (auto& sl : s->slots) {
    if (sl.stream) {
      hipStreamSynchronize(sl.stream);
      hipStreamDestroy(sl.stream);
    }
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.h_stage) hipHostFree(sl.h_stage);
    if (sl.h_out) hipHostFree(sl.h_out);
  }
  delete s;
}
