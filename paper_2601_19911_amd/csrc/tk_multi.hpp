// Batched Top-K: many queries of uneven N and K in four launches (sample,
// threshold, filter, tail), each workgroup running the same body as in the
// single-query kernels for the query and slice its block map names.  Shared
// by the plan
// API (tk_batched.hip) and the served form (tk_serve.hip).  Host code.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "tk_sampled.hpp"

namespace tk {

// One query of a batch, as device addresses.
struct MQuery {
  const void* keys;  // its first key
  const void* rids;  // its row-ids, or nullptr: row-id = index within the query
  uint64_t n, k;
  int order;
  void* out_keys;  // min(k, n) entries, or nullptr
  void* out_rids;  // min(k, n) entries
};

enum MClass : uint8_t { MC_EMPTY = 0, MC_SAMPLED = 1, MC_INPUT = 2 };

// Where each query's scratch lives, relative to the batch workspace:
//   [QHead of every sampled query][each query's regions]
struct MLayout {
  std::vector<uint8_t> cls;
  std::vector<SamplePlan> sp;
  std::vector<uint32_t> head;     // index of the query's QHead (sampled queries)
  std::vector<uint64_t> reg;      // offset of the query's scratch regions
  std::vector<uint32_t> fblocks;  // filter workgroups of each sampled query
  uint64_t heads_bytes = 0;       // the QHead array at offset 0
  uint64_t total = 0;
  uint32_t n_sampled = 0, n_input = 0;
  uint64_t n_samp_blocks = 0, n_filt_blocks = 0;
};

// Classifies and lays out a batch.  slice_keys: keys per filter workgroup
// (0: 64 Ki).  Returns the workspace bytes (multiple of 256).
uint64_t multi_layout(const std::vector<uint64_t>& n, const std::vector<uint64_t>& k, int key_type,
                      int rid_type, const Tuning& tun, uint32_t slice_keys, MLayout& L);

// Argument records and block maps of one launch.
struct MRecords {
  std::vector<SampArgs> sa;
  std::vector<uint2> smap;  // (sa index, workgroup within the query)
  std::vector<FiltArgs> fa;
  std::vector<uint2> fmap;  // (fa index, workgroup within the query)
  std::vector<TailArgs1> ta;
  std::vector<uint32_t> tq;  // query index of each tail record
};

// Fills the records for queries q (absolute device addresses; ws is the
// batch workspace on the device).
void multi_records(const std::vector<MQuery>& q, const MLayout& L, int key_type, int rid_type,
                   char* ws, MRecords& r);

// Device copies of the records.
struct MLaunch {
  const SampArgs* sa = nullptr;
  const uint2* smap = nullptr;
  uint32_t n_samp = 0;
  const FiltArgs* fa = nullptr;
  uint32_t n_fa = 0;  // sampled queries (one threshold workgroup each)
  const uint2* fmap = nullptr;
  uint32_t n_filt = 0;
  const TailArgs1* ta = nullptr;
  const uint32_t* tq = nullptr;  // query index of each tail record
  uint32_t n_tail = 0;
  uint32_t filt_grid = 0;  // filter workgroups looping over the slices; 0: three per CU
                           // (at least the slice count: one per slice)
  // per-query completion stamps (device clock), or nullptr: stamps[0] is the
  // launch's start, stamps[1 + i] the end of query i's tail
  unsigned long long* stamps = nullptr;
};

// Byte sizes of the records as laid out by multi_pack (each part 256-aligned).
uint64_t multi_pack_bytes(const MRecords& r);
// Packs the records into host memory `dst` (multi_pack_bytes(r) bytes) and
// returns the launch description for the same layout at device address dev.
MLaunch multi_pack(const MRecords& r, char* dst, char* dev);

// Enqueues the four launches on st.  Makes no runtime query, so it may run
// inside a stream capture; launch errors surface through hipGetLastError.
void multi_enqueue(const MLaunch& m, int key_type, int rid_type, hipStream_t st);

}  // namespace tk
