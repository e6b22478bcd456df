// Data structures shared by the batch engine kernels and their host drivers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tk_plan.hpp"

namespace tk {

enum ItemType : uint32_t { ITEM_TILE = 1, ITEM_EXACT = 3 };
enum QueryClass : uint8_t { CLS_SAMPLED = 0, CLS_EXACT = 1, CLS_EMPTY = 2 };

// One query, as the engine sees it.  Key, row-id and output locations are
// byte offsets added to the launch's base addresses (bases of 0 make them
// absolute addresses).  Scratch offsets are relative to the launch's scratch.
struct QDesc {
  uint64_t keys, rids, out_keys, out_rids;
  uint64_t n;
  uint64_t rid_base;   // implicit row-id = rid_base + local index
  uint64_t cap;        // survivor capacity
  uint64_t samp_k, samp_f, surv_k, surv_f, cand_k, cand_f, tmp_k, tmp_f;
  uint32_t k_eff;
  uint32_t r1;         // sample rank (1-based) of the threshold
  uint32_t S;          // sample size
  uint32_t samp_blocks;
  uint32_t ntiles;
  uint32_t tile_len;
  uint8_t key_type, order, has_rids, has_out_keys;
  uint8_t has_out_rids, cls, pad0, pad1;
};

// Per-query state of one launch; zeroed by k_reset.
struct QState {
  unsigned long long surv;   // survivors appended so far
  unsigned long long thr_k;  // threshold: key image
  unsigned long long thr_f;  //            flipped row-id
  unsigned long long t_done; // wall clock (100 MHz) when the result was written
  uint32_t samp_done;        // sample workgroups finished
  uint32_t tiles_done;       // streaming tiles finished
  uint32_t status;           // 1: the sample misjudged, the exact select over the input ran
  uint32_t done;             // 1: results written
  uint32_t pad[4];
};
static_assert(sizeof(QState) == 64, "QState is 64 bytes");

struct Item {
  uint32_t type, q, a, pad;
};

struct EngineCtl {
  uint32_t head;               // next queue item
  uint32_t pad[31];
  unsigned long long t_start;  // wall clock when k_reset ran
  unsigned long long pad2[15];
};
static_assert(sizeof(EngineCtl) == 256, "EngineCtl is 256 bytes");

struct EngineArgs {
  const QDesc* qd;      // per-query descriptors (device memory)
  QState* qs;           // per-query state (device memory)
  EngineCtl* ctl;
  const Item* items;    // the queue, in order
  const uint2* prep;    // (query, sample workgroup) of every k_bprep workgroup
  char* scratch;
  uint32_t nitems;
  uint32_t nq;
  uint32_t nprep;
  uint32_t pad;
  uint64_t keys_base, rids_base, out_keys_base, out_rids_base;
};

// scratch bytes of one query's regions, placed at `off`
uint64_t layout_query(QDesc& d, uint64_t off, uint32_t kb, uint32_t rb, const SamplePlan& p);
// Enqueues k_reset, k_bprep and k_engine.  key_type: the type of every query,
// or -1 for a launch that mixes key types.  grid_override 0: the occupancy grid.
int engine_launch(const EngineArgs& a, uint32_t rid_type, int key_type, uint32_t grid_override,
                  hipStream_t st);
// The occupancy grid of k_engine on the current device (0 on a HIP error).
// Queries the runtime, so it is called before a stream capture begins.
uint32_t engine_grid_size(uint32_t rid_type, int key_type);
// engine_launch with a given grid and no runtime queries: safe inside a stream
// capture (launch errors surface when the capture ends).
void engine_enqueue(const EngineArgs& a, uint32_t rid_type, int key_type, uint32_t grid,
                    hipStream_t st);

// keys per streaming tile (256 KiB of keys)
inline uint32_t tile_len_for(uint32_t kb) { return kb == 8 ? (1u << 15) : (1u << 16); }

}  // namespace tk
