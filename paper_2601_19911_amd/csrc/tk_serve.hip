// Served form: continuous batching of Top-K requests over device-resident key
// columns, with the cost-accounted gate of the paper (sec. II-B, the "Risky
// Gate"): a request goes to the GPU only when the estimated CPU cost exceeds
// the estimated offload cost by more than a margin; otherwise it runs on the
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
#include <thread>
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
  const void* d_keys;
  const void* h_keys;
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
  std::atomic<int> state{0};  // 0 queued, 1 running, 2 done, 3 taken
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
  std::deque<Req> reqs;  // stable addresses; index = request id
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
  int dev = 0;
};

namespace {

double cpu_cost(const tk_server_cfg& c, uint64_t n, uint32_t k) {
  return c.cpu_a * (double)n + c.cpu_b * (double)k * std::log2((double)k + 1.0) + c.cpu_c;
}
double gpu_cost(const tk_server_cfg& c, uint64_t n, uint32_t k) {
  return c.gpu_a * (double)n + c.gpu_b * (double)k + c.gpu_c;
}

void finish(tk_server* s, uint64_t id) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->reqs[id].t_done = now_ns();
    s->reqs[id].state.store(2);
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
      rp = &s->reqs[id];
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
  const void* d_keys;
  uint64_t offset, n;
  uint32_t k;
  int order;
};

// A micro-batch laid out in a slot's arena:
//   [batch workspace: query states, then each query's regions][argument
//   records][result keys][result row-ids]
struct BatchBuild {
  MLayout L;
  MRecords rec;
  std::vector<uint64_t> out_off;
  uint64_t off_rec = 0, rec_bytes = 0, off_out_k = 0, off_out_r = 0, end = 0;
};

// Lays out a micro-batch for `arena`; returns false if it does not fit.
bool build_batch(const std::vector<Taken>& ids, int key_type, char* arena, size_t arena_bytes,
                 BatchBuild& b, size_t* needed) {
  const uint32_t kb = key_bytes(key_type), rb = 8;
  const size_t q = ids.size();
  Tuning t = current_tuning();
  t.force_exact = 0;
  t.force_cap = 0;
  t.min_sample_log2 = 12;
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
  b.off_rec = off;
  b.rec_bytes = multi_pack_bytes(sizes);
  off = align_up(off + b.rec_bytes, 256);
  b.off_out_k = off;
  off = align_up(off + b.out_off[q] * kb, 256);
  b.off_out_r = off;
  off = align_up(off + b.out_off[q] * rb, 256);
  b.end = off;
  if (needed) *needed = off;
  if (off > arena_bytes) return false;
  std::vector<MQuery> qs(q);
  for (size_t i = 0; i < q; ++i) {
    MQuery& m = qs[i];
    m.keys = static_cast<const char*>(ids[i].d_keys) + ids[i].offset * kb;
    m.rids = nullptr;  // local index; the column offset is added on the host
    m.n = ids[i].n;
    m.k = ids[i].k;
    m.order = ids[i].order;
    m.out_keys = arena + b.off_out_k + b.out_off[i] * kb;
    m.out_rids = arena + b.off_out_r + b.out_off[i] * rb;
  }
  multi_records(qs, b.L, key_type, TK_RID_U64, arena, b.rec);
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
        if (!s->gpu_q[t].empty() && s->reqs[s->gpu_q[t].front()].t_submit < best) {
          best = s->reqs[s->gpu_q[t].front()].t_submit;
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
        Req& r = s->reqs[q.front()];
        take.push_back(Taken{&r, s->cols[r.col].d_keys, r.offset, r.n, r.k, r.order});
        q.pop_front();
      }
      s->slots[slot].busy = true;
    }
    Slot& sl = s->slots[slot];
    // admission by memory: shrink the batch until it fits the slot's arena
    BatchBuild b;
    size_t need = 0;
    while (!take.empty() && !build_batch(take, kt, sl.arena, sl.arena_bytes, b, &need)) {
      if (take.size() == 1) break;
      std::lock_guard<std::mutex> lk(s->mu);
      s->gpu_q[kt].push_front(take.back().r->id);
      take.pop_back();
    }
    const size_t stage = b.L.heads_bytes + b.rec_bytes;
    const size_t outb = b.end - b.off_out_k;
    if (take.empty() || need > sl.arena_bytes || stage > sl.stage_bytes || outb > sl.out_bytes) {
      // a single request larger than a slot: it goes to the CPU path instead
      std::lock_guard<std::mutex> lk(s->mu);
      for (const Taken& t : take) {
        t.r->route = 1;
        s->cpu_q.push_back(t.r->id);
      }
      sl.busy = false;
      s->cv_cpu.notify_all();
      continue;
    }
    const uint64_t t0 = now_ns();
    // staging: zeroed query states, then the argument records
    std::memset(sl.h_stage, 0, b.L.heads_bytes);
    const MLaunch m = multi_pack(b.rec, sl.h_stage + b.L.heads_bytes, sl.arena + b.off_rec);
    int rc = TK_OK;
    if (b.L.heads_bytes &&
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
      rc = hipMemcpyAsync(sl.h_out, sl.arena + b.off_out_k, outb, hipMemcpyDeviceToHost, sl.stream) ==
                   hipSuccess ? TK_OK : TK_EHIP;
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
        Req& r = s->reqs[sl.reqs[i]];
        const uint64_t a = sl.out_off[i], c = sl.out_off[i + 1] - a;
        r.out_keys.assign(sl.h_out + a * kb, sl.h_out + (a + c) * kb);
        r.out_rids.resize(c);
        std::memcpy(r.out_rids.data(), sl.h_out + sl.out_rid_base + a * 8, c * 8);
        for (auto& x : r.out_rids) x += r.offset;  // local index -> column row
        if (e != hipSuccess) r.status = TK_EHIP;
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
  const tk_server_cfg& c = s->cfg;
  if (c.cpu_a == 0 && c.cpu_b == 0 && c.cpu_c == 0 && c.gpu_a == 0 && c.gpu_b == 0 && c.gpu_c == 0) {
    // no cost model given: least-squares fit of measured request times for
    // N = 2^8 .. 2^22, K in {10, 100, 1000}, int32/int64/float32 keys, on an
    // MI355X (device-resident keys, launch to results on the host) against the
    // CPU route on 16 host threads
    s->cfg.cpu_a = 1.79e-10;
    s->cfg.cpu_b = 1.26e-8;
    s->cfg.cpu_c = 4.36e-5;
    s->cfg.gpu_a = 0.0;
    s->cfg.gpu_b = 1.48e-8;
    s->cfg.gpu_c = 5.30e-5;
  }
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
  if (!s || !col || key_type < 0 || key_type > 3 || (n && !d_keys)) return TK_EINVAL;
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
  if (col >= s->cols.size() || offset + n > s->cols[col].n) return TK_EINVAL;
  const Column& c = s->cols[col];
  s->reqs.emplace_back();
  const uint64_t id = s->reqs.size() - 1;
  Req& r = s->reqs.back();
  r.id = id;
  r.col = col;
  r.offset = offset;
  r.n = n;
  r.k = k;
  r.order = order;
  r.t_submit = t;
  // the gate: CPU unless offloading saves more than the margin
  int route = 0;
  if (s->cfg.gate == 2) route = 1;
  else if (s->cfg.gate == 1 && c.h_keys) {
    const uint32_t ke = (uint64_t)k < n ? k : (uint32_t)n;  // the work is min(k, n) results
    const double saving = cpu_cost(s->cfg, n, ke) - gpu_cost(s->cfg, n, ke);
    route = saving > s->cfg.margin_ms * 1e-3 ? 0 : 1;
  }
  if (route == 1 && !c.h_keys) route = 0;
  r.route = route;
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
  if (id >= s->reqs.size()) return TK_EINVAL;
  Req& r = s->reqs[id];
  if (r.state.load() < 2) return TK_EAGAIN;
  if (h_keys) std::memcpy(h_keys, r.out_keys.data(), r.out_keys.size());
  if (h_rowids) std::memcpy(h_rowids, r.out_rids.data(), r.out_rids.size() * 8);
  if (info) {
    info->t_submit_ns = r.t_submit;
    info->t_start_ns = r.t_start;
    info->t_done_ns = r.t_done;
    info->route = r.route;
    info->status = r.status;
    info->count = r.out_rids.size();
  }
  return r.status;
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
