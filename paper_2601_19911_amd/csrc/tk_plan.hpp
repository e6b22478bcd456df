// Host-side planning shared by the single-query and batched paths: sample
// size, sample rank, survivor capacity and workspace layout.  Pure arithmetic,
// no HIP calls, so it also builds into the host unit tests.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

namespace tk {

// LDS capacity (elements) of the one-workgroup select/sort stage for a
// composite of `cb` bytes (key image + row-id): 128 KiB of LDS.
inline uint32_t lds_cap_for(uint32_t cb) { return cb <= 8 ? 16384u : 8192u; }

constexpr uint32_t SAMPLE_CHUNK = 16;        // contiguous keys per sample chunk
constexpr uint32_t SAMPLE_PER_BLOCK = 2048;  // sample keys per local-select block
constexpr uint32_t SAMPLE_FINAL_MAX = 2048;  // candidates of the final select (registers of a
                                             // filter workgroup)
// Largest N sampled with K > N / 16: the survivors (up to ~N / 2) then stay
// below 2^20, so that no bucket of the large-K tail (128 or 256 per octave)
// outgrows one LDS tile
constexpr uint64_t SAMPLE_WIDE_K_MAX_N = 1ull << 20;

struct SamplePlan {
  bool fast = false;     // sample -> filter -> tail; else exact radix select
  uint32_t S = 0;        // sample size (multiple of SAMPLE_PER_BLOCK)
  uint32_t blocks = 0;   // S / SAMPLE_PER_BLOCK
  uint32_t r1 = 0;       // sample rank (1-based) used as the threshold
  uint64_t cap = 0;      // survivor capacity
};

struct Tuning {
  double sample_sigma = 4.0;   // safety margin on the sample rank, in std devs
  double cap_sigma = 6.0;      // survivor capacity margin, in std devs
  uint32_t max_sample_log2 = 20;
  uint32_t min_sample_log2 = 11;
  uint32_t filter_grid = 0;    // 0: automatic
  uint32_t filter_unroll = 4;  // 16-byte loads in flight per thread and tile: 4 or 8
  uint64_t force_cap = 0;      // >0: override the survivor capacity (tests)
  int force_exact = 0;         // 1: always take the exact radix path (tests)
  uint32_t tile_len = 0;       // keys per streaming tile of the engine (0: 256 KiB of keys)
  int rank_tail = 1;           // 1: survivors ranked across workgroups when they fit; 0: one
                               // workgroup selects and sorts them
  uint32_t recover_min_log2 = 29;  // sampled queries of at least 2^this keys hand a misjudged
                                   // sample to a cooperative exact select over the device (0:
                                   // never; one workgroup selects over the input instead).
                                   // The conditional cooperative launch costs about 21 us on
                                   // every query (MI355X), 11 % at N = 2^28 float32
  int join_bloom = 1;              // 1: join tables carry the bloom prefilter
};

// Whether a sampled query of n keys enqueues the cooperative exact select that
// takes over when its sample misjudged.
inline bool recover_on_device(uint64_t n, const Tuning& t) {
  return t.recover_min_log2 > 0 && t.recover_min_log2 < 63 && n >= (1ull << t.recover_min_log2);
}

// Chooses the sample for a query of n keys and k_eff results.  The threshold
// is the r1-th best of S sampled keys; survivors ~ r1 * n / S.  The sample is
// as large as allowed while the final select still fits one workgroup.
inline SamplePlan plan_sample(uint64_t n, uint64_t k_eff, const Tuning& t) {
  SamplePlan p;
  if (t.force_exact || k_eff == 0 || n < (1ull << t.min_sample_log2) * 16) return p;
  // K beyond N / 16: a sample still bounds the survivors to ~K when N is
  // moderate; past SAMPLE_WIDE_K_MAX_N (or K beyond N / 2) the exact select
  // over the input is used instead
  if (k_eff * 16 > n && (n > SAMPLE_WIDE_K_MAX_N || k_eff * 2 > n)) return p;
  for (int lg = (int)t.max_sample_log2; lg >= (int)t.min_sample_log2; --lg) {
    const uint64_t S = 1ull << lg;
    if (S * 16 > n) continue;
    const double m = (double)k_eff * (double)S / (double)n;
    const uint64_t r1 = (uint64_t)ceil(m + t.sample_sigma * sqrt(m) + 3.0);
    const uint64_t blocks = S / SAMPLE_PER_BLOCK;
    if (r1 > SAMPLE_PER_BLOCK || r1 * blocks > SAMPLE_FINAL_MAX) continue;
    p.fast = true;
    p.S = (uint32_t)S;
    p.blocks = (uint32_t)blocks;
    p.r1 = (uint32_t)r1;
    const double unit = (double)n / (double)S;
    double cap = ((double)r1 + t.cap_sigma * sqrt((double)r1) + 12.0) * unit + 4096.0;
    if ((double)k_eff * 2.0 + 4096.0 > cap) cap = (double)k_eff * 2.0 + 4096.0;
    if (cap > (double)n) cap = (double)n;
    p.cap = t.force_cap ? t.force_cap : (uint64_t)cap;
    return p;
  }
  return p;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bytes of the full sort's scratch for n pairs (tk_sort's layout): two
// ping-pong copies of the keys and row-ids, a 4-byte count per digit and tile
// of 4096 pairs, and the digit totals.
inline size_t sort_scratch_bytes(uint64_t n, uint32_t kb, uint32_t rb) {
  const uint64_t ntiles = n ? (n + 4095) / 4096 : 1;
  return 2 * (align_up((size_t)n * kb, 256) + align_up((size_t)n * rb, 256)) +
         align_up((size_t)ntiles * 256 * 4, 256) + align_up(256 * 4, 256);
}

// Queries without a usable sample from this size on are answered by the full
// sort, keeping the first K (path 9); below it by one workgroup (path 8).
constexpr uint64_t SORT_ROUTE_MIN_N = 1ull << 16;

// The bucketed tail (large K): logarithmic buckets of a W-bit composite
// distance with 2^sub buckets per octave.
constexpr uint64_t BUCKET_TAIL_MIN_K = 2049;  // smaller K: the survivors are ranked directly
inline uint32_t bucket_sub(uint32_t w) { return w == 64 ? 8u : 7u; }
inline uint32_t bucket_count(uint32_t w) { return (1u << bucket_sub(w)) * (w - bucket_sub(w) + 1); }
inline bool bucket_tail_for(uint64_t k_eff) { return k_eff >= BUCKET_TAIL_MIN_K; }

constexpr size_t HEADER_BYTES = 8192;

// Byte offsets inside the caller's workspace for one query.
struct WsLayout {
  size_t sample = 0;   // sample candidates: blocks * r1 composites
  size_t surv = 0;     // survivors: cap composites (key image, flipped row-id), SoA
  size_t cand = 0;     // exact selection: k_eff composites, SoA
  size_t tmp = 0;      // merge ping-pong: k_eff composites, SoA
  size_t btail = 0;    // bucketed tail (large K): histogram, cursors, offsets, state, and
                       // cap composites grouped by bucket (0 when not used)
  size_t sort = 0;     // full sort's scratch (queries the sort answers; 0 when not used)
  size_t base = 0;     // bytes without the sort's scratch (the exact select's minimum)
  size_t total = 0;
};

// Bytes of the bucketed tail's region for a query with survivor capacity cap.
inline size_t btail_bytes(uint64_t cap, uint32_t kb, uint32_t rb) {
  const size_t nb = bucket_count(8 * (kb + rb));
  return align_up(3 * nb * 4 + 64, 256) + align_up(cap * kb, 256) + align_up(cap * rb, 256);
}

inline WsLayout ws_layout(uint64_t n, uint64_t k_eff, uint32_t kb, uint32_t rb, const SamplePlan& p) {
  WsLayout L;
  size_t off = HEADER_BYTES;
  L.sample = off;
  off = align_up(off + (size_t)p.blocks * p.r1 * (kb + rb) + 64, 256);
  L.surv = off;
  off = align_up(off + (size_t)p.cap * (kb + rb) + 64, 256);
  L.cand = off;
  off = align_up(off + (size_t)k_eff * (kb + rb) + 64, 256);
  L.tmp = off;
  const uint32_t cap = lds_cap_for(kb + rb);
  if (k_eff > cap) off = align_up(off + (size_t)k_eff * (kb + rb) + 64, 256);
  if (p.fast && bucket_tail_for(k_eff)) {
    L.btail = off;
    off += btail_bytes(p.cap, kb, rb);
  }
  L.base = off;
  if (!p.fast && n >= SORT_ROUTE_MIN_N && n < (1ull << 32)) {  // the sort route's scratch
    L.sort = align_up(off, 256);
    off = L.sort + sort_scratch_bytes(n, kb, rb);
  }
  L.total = off;
  return L;
}

}  // namespace tk
