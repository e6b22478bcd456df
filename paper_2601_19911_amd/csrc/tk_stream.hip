// Chunk-pipelined key-only streaming (paper sec. II-C, transmission: only
// keys and row-ids cross the host link; sec. IV-A: that link, not the device,
// bounds the end-to-end time): Top-K over a key column that stays in host
// memory, however large, through two device staging buffers.
//
//   copy stream    chunk i+1's keys (and row-ids) host -> staging buffer
//                  (i+1) mod 2, after the query that last read that buffer;
//   compute stream chunk i's Top-K (tk_topk on the staging buffer), its
//                  row-ids moved from chunk-local to column positions, then
//                  merged with the running Top-K of chunks 0..i-1: one more
//                  tk_topk over the two lists, with their row-ids.
// The merge keeps the exact result: the best K of the column are among the
// union of the chunks' best K, and ties resolve by row-id in every step.  The
// device holds two chunks and a few K-sized lists, so a column larger than
// HBM streams like any other; with pinned host memory the copies of one
// chunk overlap the query of the previous one, and the end-to-end time
// approaches the copy time of the key bytes.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_plan.hpp"

namespace {

constexpr uint64_t STREAM_DEFAULT_CHUNK = 1ull << 24;

template <typename R>
__global__ __launch_bounds__(256) void k_add_base(R* __restrict__ r, uint64_t cnt, uint64_t base) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * 256)
    r[i] = (R)((uint64_t)r[i] + base);
}

struct StreamLayout {
  uint64_t chunk, kk;           // keys per chunk, min(k, n)
  uint64_t stage_k[2], stage_r[2], list_k[2], list_r[2], ws, ws_bytes, total;
};

uint64_t a256(uint64_t b) { return (b + 255) & ~255ull; }

StreamLayout stream_layout(uint64_t n, uint64_t k, uint64_t chunk, int kt, int rt, bool rids) {
  StreamLayout L{};
  L.chunk = chunk ? chunk : STREAM_DEFAULT_CHUNK;
  if (L.chunk > n) L.chunk = n ? n : 1;
  L.kk = k < n ? k : n;
  const uint64_t kb = tk::key_bytes(kt), rb = rt == TK_RID_U64 ? 8 : 4;
  // the largest workspace of the call's tk_topk queries: every chunk (all of
  // `chunk` keys but the last) and every merge of the running list with a
  // chunk's best (its length settles after two chunks)
  uint64_t wmax = 0, prev_q = ~0ull, prev_m = ~0ull, run = 0;
  const uint64_t nch = n ? (n + L.chunk - 1) / L.chunk : 0;
  for (uint64_t c = 0; c < nch; ++c) {
    const uint64_t len = n - c * L.chunk < L.chunk ? n - c * L.chunk : L.chunk;
    const uint64_t kc = L.kk < len ? L.kk : len;
    if (len != prev_q) {
      const uint64_t w = tk_workspace_size(len, k, kt, rt);
      wmax = w > wmax ? w : wmax;
      prev_q = len;
    }
    if (c == 0) {
      run = kc;
      continue;
    }
    const uint64_t m = run + kc;
    if (m != prev_m) {
      const uint64_t w = tk_workspace_size(m, k, kt, rt);
      wmax = w > wmax ? w : wmax;
      prev_m = m;
    }
    run = m < L.kk ? m : L.kk;
  }
  L.ws_bytes = a256(wmax ? wmax : 256);
  uint64_t o = 0;
  for (int b = 0; b < 2; ++b) {
    L.stage_k[b] = o;
    o += a256(L.chunk * kb);
    L.stage_r[b] = o;
    o += rids ? a256(L.chunk * rb) : 0;
  }
  for (int b = 0; b < 2; ++b) {
    L.list_k[b] = o;
    o += a256(2 * L.kk * kb);
    L.list_r[b] = o;
    o += a256(2 * L.kk * rb);
  }
  L.ws = o;
  o += L.ws_bytes;
  L.total = o;
  return L;
}

// ready[b]: staging buffer b holds its chunk; freed[b]: its query has read
// it; entry: the compute stream's work before the call (the copies must not
// overwrite a workspace that earlier work on the compute stream still reads).
struct Events {
  hipEvent_t ready[2] = {nullptr, nullptr}, freed[2] = {nullptr, nullptr}, entry = nullptr;
  bool ok = true;
  Events() {
    ok = hipEventCreateWithFlags(&entry, hipEventDisableTiming) == hipSuccess;
    for (int b = 0; b < 2; ++b)
      ok = ok && hipEventCreateWithFlags(&ready[b], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&freed[b], hipEventDisableTiming) == hipSuccess;
  }
  // waits already enqueued on these events stay valid after the destroy
  ~Events() {
    if (entry) (void)hipEventDestroy(entry);
    for (int b = 0; b < 2; ++b) {
      if (ready[b]) (void)hipEventDestroy(ready[b]);
      if (freed[b]) (void)hipEventDestroy(freed[b]);
    }
  }
};

}  // namespace

extern "C" size_t tk_stream_workspace_size(uint64_t n, uint64_t k, uint64_t chunk, int key_type,
                                           int rid_type, int with_rowids) {
  if (key_type < TK_KEY_I32 || key_type > TK_KEY_F64 || (rid_type != TK_RID_U32 && rid_type != TK_RID_U64))
    return 0;
  return (size_t)stream_layout(n, k, chunk, key_type, rid_type, with_rowids != 0).total;
}

extern "C" int tk_topk_stream(const void* h_keys, const void* h_rowids, uint64_t n, uint64_t k,
                              int key_type, int rid_type, int order, uint64_t chunk, void* out_keys,
                              void* out_rowids, uint64_t* out_count, void* workspace,
                              size_t workspace_bytes, void* stream, void* copy_stream) {
  if (key_type < TK_KEY_I32 || key_type > TK_KEY_F64 || (rid_type != TK_RID_U32 && rid_type != TK_RID_U64) ||
      (order != TK_DESC && order != TK_ASC))
    return TK_EINVAL;
  const uint64_t kk = k < n ? k : n;
  if (n > 0 && !h_keys) return TK_EINVAL;
  if (!h_rowids && rid_type == TK_RID_U32 && n > (1ull << 32)) return TK_EINVAL;
  if (out_count) *out_count = kk;
  if (kk == 0) return TK_OK;
  if (!out_rowids && !out_keys) return TK_EINVAL;
  const StreamLayout L = stream_layout(n, k, chunk, key_type, rid_type, h_rowids != nullptr);
  if (!workspace || workspace_bytes < L.total || ((uintptr_t)workspace & 255u)) return TK_EINVAL;
  char* w = static_cast<char*>(workspace);
  const uint64_t kb = tk::key_bytes(key_type), rb = rid_type == TK_RID_U64 ? 8 : 4;
  hipStream_t st = (hipStream_t)stream;
  hipStream_t cs = copy_stream ? (hipStream_t)copy_stream : st;
  Events ev;
  if (!ev.ok) return TK_EHIP;
  const uint64_t nch = (n + L.chunk - 1) / L.chunk;
  auto copy_in = [&](uint64_t c) -> bool {
    const int b = (int)(c & 1);
    const uint64_t off = c * L.chunk, len = n - off < L.chunk ? n - off : L.chunk;
    // the buffer's previous chunk (c - 2) has been queried
    if (c >= 2 && hipStreamWaitEvent(cs, ev.freed[b], 0) != hipSuccess) return false;
    if (hipMemcpyAsync(w + L.stage_k[b], static_cast<const char*>(h_keys) + off * kb, len * kb,
                       hipMemcpyHostToDevice, cs) != hipSuccess)
      return false;
    if (h_rowids && hipMemcpyAsync(w + L.stage_r[b], static_cast<const char*>(h_rowids) + off * rb,
                                   len * rb, hipMemcpyHostToDevice, cs) != hipSuccess)
      return false;
    return hipEventRecord(ev.ready[b], cs) == hipSuccess;
  };
  if (cs != st && (hipEventRecord(ev.entry, st) != hipSuccess ||
                   hipStreamWaitEvent(cs, ev.entry, 0) != hipSuccess))
    return TK_EHIP;
  if (!copy_in(0)) return TK_EHIP;
  int cur = 0;       // the list holding the running result
  uint64_t run = 0;  // its length
  for (uint64_t c = 0; c < nch; ++c) {
    const int b = (int)(c & 1);
    const uint64_t off = c * L.chunk, len = n - off < L.chunk ? n - off : L.chunk;
    // the next chunk's copy goes out before this chunk's query is enqueued
    if (c + 1 < nch && !copy_in(c + 1)) return TK_EHIP;
    if (hipStreamWaitEvent(st, ev.ready[b], 0) != hipSuccess) return TK_EHIP;
    const uint64_t kc = kk < len ? kk : len;
    const bool only = nch == 1;
    char* qk = only ? static_cast<char*>(out_keys) : w + L.list_k[cur] + run * kb;
    char* qr = only ? static_cast<char*>(out_rowids) : w + L.list_r[cur] + run * rb;
    int rc = tk_topk(w + L.stage_k[b], h_rowids ? w + L.stage_r[b] : nullptr, len, k, key_type,
                     rid_type, order, qk, qr, nullptr, w + L.ws, L.ws_bytes, st);
    if (rc != TK_OK) return rc;
    if (hipEventRecord(ev.freed[b], st) != hipSuccess) return TK_EHIP;
    if (!h_rowids && off > 0 && qr) {
      const unsigned g = (unsigned)((kc + 255) / 256 < 1024 ? (kc + 255) / 256 : 1024);
      if (rid_type == TK_RID_U32)
        hipLaunchKernelGGL(k_add_base<uint32_t>, dim3(g), dim3(256), 0, st, reinterpret_cast<uint32_t*>(qr), kc, off);
      else
        hipLaunchKernelGGL(k_add_base<unsigned long long>, dim3(g), dim3(256), 0, st,
                           reinterpret_cast<unsigned long long*>(qr), kc, off);
      if (hipGetLastError() != hipSuccess) return TK_EHIP;
    }
    if (only) break;
    if (c == 0) {
      run = kc;
      continue;
    }
    // merge the running list with this chunk's best, both with column row-ids
    const uint64_t m = run + kc;
    const bool last = c + 1 == nch;
    char* dk = last ? static_cast<char*>(out_keys) : w + L.list_k[cur ^ 1];
    char* dr = last ? static_cast<char*>(out_rowids) : w + L.list_r[cur ^ 1];
    rc = tk_topk(w + L.list_k[cur], w + L.list_r[cur], m, k, key_type, rid_type, order, dk, dr,
                 nullptr, w + L.ws, L.ws_bytes, st);
    if (rc != TK_OK) return rc;
    run = m < kk ? m : kk;
    cur ^= 1;
  }
  return TK_OK;
}
