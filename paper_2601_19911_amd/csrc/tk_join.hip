// Matching primitive (paper sec. III-B): the probe phase of an inner equi-join,
// key-only.  The build side's (key, row-id) pairs go into a device hash table;
// every probe key is looked up in parallel and each match returns the pair
// (probe row-id, build row-id): the "set of matched pointers" of sec. II-C,
// which the host late-materializes.
//
// Table (caller-owned device buffer, see tk_join_table_size):
//   [header, 256 B][slots: S slots of (key word, row-id word)][side list][bloom words]
//   [repeat filter words]
// S is a power of two >= 2 * n_build, so the load factor is at most 1/2.  Open
// addressing with linear probing; duplicate build keys take one slot each, so
// a probe walks its run until an empty slot and returns every equal key.  The
// empty marker is the key whose bits are 1 << (width - 1) (INT_MIN); build keys
// equal to it are not hashed but appended to the side list, which a probe of
// that key reads in full.  The header counts the side list and records whether
// any build key occurs twice; without duplicates a probe stops at its first
// hit.  With some, a small filter of the repeated keys (REPEAT_WORDS words, 3
// bits per key, set by the insert that meets an equal key) lets a probe stop
// at its first hit whenever its key is not among them.
//
// The bloom prefilter (sec. III-B names a bloom filter as another form of the
// matching primitive; here it sits in front of the table): S / 16 words of 64 bits (8-16 bits per build key), each hashed
// key setting 3 bits of one word.  A probe key reads its word first and walks
// the slots only when all 3 bits are set, so most probes of absent keys touch
// one word of a small array (L2- or last-level-cache resident) instead of
// the slot lines in HBM.
//
// Memory behaviour on MI355X: the probe is bound by random reads of slots
// (one slot usually, in one 128-byte line; adjacent slots of a run share it).
// Probe keys stream in coalesced; matches are staged per workgroup in LDS and
// written out contiguously behind one global atomic per stage flush.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mitopk.h"
#include "tk_device.hpp"
#include "tk_internal.hpp"

namespace {

constexpr uint64_t JOIN_HEADER_BYTES = 256;
constexpr uint64_t JOIN_MAX_BUILD = 1ull << 31;
constexpr int PROBE_NT = 256;   // threads per probe workgroup
constexpr int PROBE_PER = 4;    // probe keys per thread per tile
constexpr int PROBE_WG_PER_CU = 6;  // 16 KiB stages: 6 fit the LDS of a CU
constexpr uint64_t REPEAT_WORDS = 1024;  // 8 KiB: cache-resident for every probe

struct JoinHeader {
  unsigned long long side_count;  // build keys equal to the empty marker
  uint32_t dup;                   // 1: some build key occurs more than once
  uint32_t pad[61];
};
static_assert(sizeof(JoinHeader) == JOIN_HEADER_BYTES, "join header is 256 bytes");

// A slot: key bits and row-id in words of one width (4 bytes when both are
// 4-byte types, else 8), so one aligned 8- or 16-byte load reads a slot.
template <typename W>
struct alignas(2 * sizeof(W)) Slot {
  W key;
  W rid;
};

template <int KT> struct JKey;
template <> struct JKey<TK_KEY_I32> {
  using Raw = uint32_t;
  static constexpr Raw EMPTY = 0x80000000u;
};
template <> struct JKey<TK_KEY_I64> {
  using Raw = unsigned long long;
  static constexpr Raw EMPTY = 0x8000000000000000ull;
};

// Slot index: the key's bits folded and multiplied by 2^64 / golden ratio
// (Knuth's multiplicative hashing); the top log2(S) bits of the product.
__device__ __forceinline__ uint64_t slot_of(uint64_t x, uint32_t shift) {
  x ^= x >> 31;
  x *= 0x9E3779B97F4A7C15ull;
  return x >> shift;
}

// Bloom word and bits of a key: the 64-bit finalizer of MurmurHash3 (Appleby),
// a hash independent of the slot's; the top bits pick the word, three 6-bit
// fields of the low bits the bits inside it.
__device__ __forceinline__ uint64_t bloom_hash(uint64_t x) {
  x ^= x >> 33;
  x *= 0xFF51AFD7ED558CCDull;
  x ^= x >> 33;
  x *= 0xC4CEB9FE1A85EC53ull;
  x ^= x >> 33;
  return x;
}
__device__ __forceinline__ unsigned long long bloom_bits(uint64_t z) {
  return (1ull << (z & 63)) | (1ull << ((z >> 6) & 63)) | (1ull << ((z >> 12) & 63));
}
// The repeat filter's hash: the same finalizer over the key xor a constant,
// so that its words and bits are not those of the bloom prefilter.
__device__ __forceinline__ uint64_t repeat_hash(uint64_t x) {
  return bloom_hash(x ^ 0x5851F42D4C957F2Dull);
}
__device__ __forceinline__ uint64_t repeat_word(uint64_t z) { return z >> 54; }  // < 1024

uint64_t slots_for(uint64_t n_build) {
  uint64_t s = 64;
  while (s < 2 * n_build) s <<= 1;
  return s;
}

bool wide_slot(int key_type, int rid_type) {
  return key_type == TK_KEY_I64 || rid_type == TK_RID_U64;
}

uint64_t round256(uint64_t b) { return (b + 255) & ~255ull; }

uint64_t bloom_words_for(uint64_t nslots) { return nslots / 16; }

// Byte offsets of the side list and the bloom words inside the table.
uint64_t side_offset(uint64_t nslots, uint64_t slot_b) {
  return JOIN_HEADER_BYTES + round256(nslots * slot_b);
}
uint64_t bloom_offset(uint64_t n_build, uint64_t nslots, uint64_t slot_b, uint64_t rid_b) {
  return side_offset(nslots, slot_b) + round256((n_build ? n_build : 1) * rid_b);
}

uint64_t repeat_offset(uint64_t n_build, uint64_t nslots, uint64_t slot_b, uint64_t rid_b) {
  return bloom_offset(n_build, nslots, slot_b, rid_b) + round256(bloom_words_for(nslots) * 8);
}

size_t table_bytes_for(uint64_t n_build, int key_type, int rid_type) {
  const uint64_t slot_b = wide_slot(key_type, rid_type) ? 16 : 8;
  const uint64_t rid_b = rid_type == TK_RID_U64 ? 8 : 4;
  const uint64_t nslots = slots_for(n_build);
  return (size_t)(repeat_offset(n_build, nslots, slot_b, rid_b) + REPEAT_WORDS * 8);
}

// ---- build ------------------------------------------------------------------------------

template <typename W>
__global__ __launch_bounds__(256) void k_jfill(Slot<W>* __restrict__ slots, uint64_t nslots,
                                               W empty, JoinHeader* __restrict__ hdr,
                                               unsigned long long* __restrict__ bloom,
                                               uint64_t nwords,
                                               unsigned long long* __restrict__ rep) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hdr->side_count = 0;
    hdr->dup = 0;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += stride) {
    Slot<W> s;
    s.key = empty;
    s.rid = 0;
    slots[i] = s;
  }
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride)
    bloom[i] = 0ull;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < REPEAT_WORDS; i += stride)
    rep[i] = 0ull;
}

template <int KT, typename W, typename BR>
__global__ __launch_bounds__(256) void k_jbuild(const typename JKey<KT>::Raw* __restrict__ keys,
                                                const BR* __restrict__ rids, uint64_t n,
                                                Slot<W>* __restrict__ slots, uint64_t mask,
                                                uint32_t shift, BR* __restrict__ side,
                                                JoinHeader* __restrict__ hdr,
                                                unsigned long long* __restrict__ bloom,
                                                uint32_t bshift,
                                                unsigned long long* __restrict__ rep) {
  using Raw = typename JKey<KT>::Raw;
  constexpr Raw EMPTY = JKey<KT>::EMPTY;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const Raw key = keys[i];
    const BR r = rids ? rids[i] : (BR)i;
    if (key == EMPTY) {
      const unsigned long long at = atomicAdd(&hdr->side_count, 1ull);
      side[at] = r;
      continue;
    }
    if (bloom) {
      const uint64_t z = bloom_hash((uint64_t)key);
      atomicOr(&bloom[z >> bshift], bloom_bits(z));
    }
    const W w = (W)key;
    uint64_t p = slot_of((uint64_t)key, shift);
    // at most n < S keys are hashed, so an empty slot is always ahead
    bool met = false;
    for (uint64_t step = 0; step <= mask; ++step) {
      const W prev = atomicCAS(&slots[p].key, (W)EMPTY, w);
      if (prev == (W)EMPTY) {
        slots[p].rid = (W)r;
        break;
      }
      if (prev == w && !met) {  // of two equal keys the later insert always meets the earlier
        met = true;
        if (hdr->dup == 0) hdr->dup = 1;
        const uint64_t z = repeat_hash((uint64_t)key);
        atomicOr(&rep[repeat_word(z)], bloom_bits(z));
      }
      p = (p + 1) & mask;
    }
  }
}

// ---- probe ------------------------------------------------------------------------------

template <typename W, typename BR, typename PR>
struct ProbeArgs {
  const void* keys;
  const PR* rids;         // null: probe row-id = position
  uint64_t n;
  const Slot<W>* slots;
  uint64_t mask;
  uint32_t shift;
  const BR* side;
  const JoinHeader* hdr;
  const unsigned long long* bloom;  // null: no prefilter
  uint32_t bshift;                  // 64 - log2(bloom words)
  const unsigned long long* rep;    // repeat filter
  PR* out_p;
  BR* out_b;
  uint64_t cap;
  unsigned long long* count;
};

// Matches are staged per workgroup in LDS and written out behind one global
// atomic per flush: the output counter is a single address that every
// workgroup of the device updates, so the number of updates, not the bytes,
// bounds the probe when they are frequent (a flush per wave and 256 matches
// took 2.4 ms for 2^26 probes at a hit rate of 1/2, whatever the table size).
// A stage of 16 KiB is flushed once it holds 3/4 of its capacity; matches
// that find it full go straight to the output behind one atomic per wave.
// (16 KiB lets 6 workgroups share a CU: at 2^26 probes 2-19 % faster than 4
// workgroups with 32 KiB stages.)
template <typename BR, typename PR>
struct ProbeStage {
  static constexpr uint32_t CAP = 16384u / (uint32_t)(sizeof(PR) + sizeof(BR));
  PR p[CAP];
  BR b[CAP];
  unsigned long long fill;  // reservations made (may pass CAP; those past it were spilled)
  unsigned long long base;
};

template <typename BR, typename PR>
__device__ __forceinline__ void stage_match(bool emit, PR pr, BR br, ProbeStage<BR, PR>& st,
                                            PR* __restrict__ out_p, BR* __restrict__ out_b,
                                            uint64_t cap, unsigned long long* count) {
  constexpr uint32_t CAP = ProbeStage<BR, PR>::CAP;
  const uint64_t m = tk::ballot(emit);
  if (m == 0) return;
  const uint32_t leader = (uint32_t)__builtin_ctzll(m);
  unsigned long long b = 0;
  if (tk::lane_id() == leader) b = atomicAdd(&st.fill, (unsigned long long)__popcll(m));
  b = __shfl(b, (int)leader, 64);
  const uint64_t pos = b + tk::lanes_below(m);
  if (emit && pos < CAP) {
    st.p[pos] = pr;
    st.b[pos] = br;
  }
  const bool spill = emit && pos >= CAP;
  const uint64_t ms = tk::ballot(spill);
  if (ms == 0) return;
  const uint32_t l2 = (uint32_t)__builtin_ctzll(ms);
  unsigned long long g = 0;
  if (tk::lane_id() == l2) g = atomicAdd(count, (unsigned long long)__popcll(ms));
  g = __shfl(g, (int)l2, 64);
  if (spill) {
    const uint64_t o = g + tk::lanes_below(ms);
    if (o < cap) {
      out_p[o] = pr;
      out_b[o] = br;
    }
  }
}

// Whole workgroup: writes the staged matches behind one global atomic and
// empties the stage.  Pairs past the output capacity are counted, not written.
template <typename BR, typename PR>
__device__ __forceinline__ void flush_stage(ProbeStage<BR, PR>& st, PR* __restrict__ out_p,
                                            BR* __restrict__ out_b, uint64_t cap,
                                            unsigned long long* count) {
  constexpr uint32_t CAP = ProbeStage<BR, PR>::CAP;
  __syncthreads();  // every stage write is done
  const uint32_t c = st.fill < CAP ? (uint32_t)st.fill : CAP;
  if (threadIdx.x == 0) st.base = c ? atomicAdd(count, (unsigned long long)c) : 0ull;
  __syncthreads();
  const uint64_t base = st.base;
  for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
    const uint64_t o = base + i;
    if (o < cap) {
      out_p[o] = st.p[i];
      out_b[o] = st.b[i];
    }
  }
  __syncthreads();  // the stage has been read
  if (threadIdx.x == 0) st.fill = 0;
  __syncthreads();
}

// Every tile: each thread's PROBE_PER keys are loaded, then (in one round)
// their repeat-filter words when the table has repeated keys and their bloom
// words when it has the prefilter, then the first slots of the keys still in
// play; the linear-probing walks of all of them advance together, one slot
// each per round, so a thread has up to PROBE_PER dependent slot loads in
// flight.  Keys equal to the empty marker are served from the side list
// afterwards.
template <int KT, typename W, typename BR, typename PR>
__global__ __launch_bounds__(PROBE_NT) void k_jprobe(ProbeArgs<W, BR, PR> a) {
  using Raw = typename JKey<KT>::Raw;
  constexpr Raw EMPTY = JKey<KT>::EMPTY;
  constexpr uint64_t TILE = (uint64_t)PROBE_NT * PROBE_PER;
  constexpr uint32_t FLUSH_AT = ProbeStage<BR, PR>::CAP / 4 * 3;
  __shared__ ProbeStage<BR, PR> st;
  if (threadIdx.x == 0) st.fill = 0;
  __syncthreads();
  const Raw* __restrict__ keys = static_cast<const Raw*>(a.keys);
  const bool dup = a.hdr->dup != 0;
  const uint64_t side_n = a.hdr->side_count;

  for (uint64_t base = (uint64_t)blockIdx.x * TILE; base < a.n; base += (uint64_t)gridDim.x * TILE) {
    Raw key[PROBE_PER];
    uint64_t pos[PROBE_PER];
    Slot<W> cur[PROBE_PER];
    bool act[PROBE_PER], side[PROBE_PER];
#pragma unroll
    for (int q = 0; q < PROBE_PER; ++q) {
      const uint64_t j = base + (uint64_t)q * PROBE_NT + threadIdx.x;
      key[q] = j < a.n ? keys[j] : EMPTY;
      side[q] = j < a.n && key[q] == EMPTY;
      act[q] = j < a.n && key[q] != EMPTY;
    }
    // with repeated build keys: whether each key may be one of them (its walk
    // then goes on past a hit), read beside the bloom words
    unsigned long long rw[PROBE_PER], rneed[PROBE_PER];
#pragma unroll
    for (int q = 0; q < PROBE_PER; ++q) {
      rw[q] = rneed[q] = 0;
      if (dup) {
        const uint64_t z = repeat_hash((uint64_t)key[q]);
        rneed[q] = bloom_bits(z);
        if (act[q]) rw[q] = a.rep[repeat_word(z)];
      }
    }
    if (a.bloom) {  // keys whose 3 bits are not all set are absent from the build side
      unsigned long long word[PROBE_PER], need[PROBE_PER];
#pragma unroll
      for (int q = 0; q < PROBE_PER; ++q) {
        const uint64_t z = bloom_hash((uint64_t)key[q]);
        need[q] = bloom_bits(z);
        word[q] = act[q] ? a.bloom[z >> a.bshift] : 0ull;
      }
#pragma unroll
      for (int q = 0; q < PROBE_PER; ++q) act[q] = act[q] && (word[q] & need[q]) == need[q];
    }
#pragma unroll
    for (int q = 0; q < PROBE_PER; ++q) {
      pos[q] = slot_of((uint64_t)key[q], a.shift);
      cur[q].key = (W)EMPTY;
      cur[q].rid = 0;
      if (act[q]) cur[q] = a.slots[pos[q]];
    }
    while (true) {
      bool any = false;
#pragma unroll
      for (int q = 0; q < PROBE_PER; ++q) {
        bool emit = false;
        BR brid = 0;
        if (act[q]) {
          if (cur[q].key == (W)EMPTY) {
            act[q] = false;
          } else {
            if (cur[q].key == (W)key[q]) {
              emit = true;
              brid = (BR)cur[q].rid;
              if (!dup || (rw[q] & rneed[q]) != rneed[q]) act[q] = false;  // no other equal key
            }
            if (act[q]) pos[q] = (pos[q] + 1) & a.mask;
          }
        }
        const uint64_t j = base + (uint64_t)q * PROBE_NT + threadIdx.x;
        stage_match<BR, PR>(emit, emit ? (a.rids ? a.rids[j] : (PR)j) : (PR)0, brid, st, a.out_p,
                            a.out_b, a.cap, a.count);
        any |= act[q];
      }
      if (tk::ballot(any) == 0) break;
#pragma unroll
      for (int q = 0; q < PROBE_PER; ++q)
        if (act[q]) cur[q] = a.slots[pos[q]];
    }
#pragma unroll
    for (int q = 0; q < PROBE_PER; ++q) {
      if (tk::ballot(side[q]) == 0 || side_n == 0) continue;
      const uint64_t j = base + (uint64_t)q * PROBE_NT + threadIdx.x;
      const PR pr = side[q] ? (a.rids ? a.rids[j] : (PR)j) : (PR)0;
      for (uint64_t t = 0; t < side_n; ++t)
        stage_match<BR, PR>(side[q], pr, side[q] ? a.side[t] : (BR)0, st, a.out_p, a.out_b, a.cap,
                            a.count);
    }
    __syncthreads();
    if (st.fill >= FLUSH_AT) flush_stage<BR, PR>(st, a.out_p, a.out_b, a.cap, a.count);
  }
  flush_stage<BR, PR>(st, a.out_p, a.out_b, a.cap, a.count);
}

__global__ void k_jclear(unsigned long long* count) { *count = 0; }

int launch_grid(int dev_cus, uint64_t work, uint64_t per_wg, int wg_per_cu) {
  uint64_t g = (work + per_wg - 1) / per_wg;
  const uint64_t lim = (uint64_t)dev_cus * wg_per_cu;
  if (g > lim) g = lim;
  return (int)(g ? g : 1);
}

int cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
    return 256;
  return v;
}

uint32_t log2_of(uint64_t pow2) {
  uint32_t lg = 0;
  while ((1ull << lg) < pow2) ++lg;
  return lg;
}

unsigned long long* words_at(void* table, uint64_t off) {
  return reinterpret_cast<unsigned long long*>(static_cast<char*>(table) + off);
}

// nwords: bloom words to fill (0: the table is built without the prefilter)
template <int KT, typename W, typename BR>
int build_t(const void* keys, const void* rids, uint64_t n, void* table, uint64_t nslots,
            uint64_t nwords, hipStream_t st) {
  auto* hdr = static_cast<JoinHeader*>(table);
  auto* slots = reinterpret_cast<Slot<W>*>(static_cast<char*>(table) + JOIN_HEADER_BYTES);
  auto* side = reinterpret_cast<BR*>(static_cast<char*>(table) + side_offset(nslots, sizeof(Slot<W>)));
  auto* bloom = nwords ? words_at(table, bloom_offset(n, nslots, sizeof(Slot<W>), sizeof(BR)))
                       : nullptr;
  auto* rep = words_at(table, repeat_offset(n, nslots, sizeof(Slot<W>), sizeof(BR)));
  const int c = cus();
  hipLaunchKernelGGL(k_jfill<W>, dim3(launch_grid(c, nslots, 256 * 8, 8)), dim3(256), 0, st, slots,
                     nslots, (W)JKey<KT>::EMPTY, hdr, bloom, nwords, rep);
  if (n) {
    hipLaunchKernelGGL((k_jbuild<KT, W, BR>), dim3(launch_grid(c, n, 256 * 4, 16)), dim3(256), 0, st,
                       static_cast<const typename JKey<KT>::Raw*>(keys), static_cast<const BR*>(rids),
                       n, slots, nslots - 1, 64u - log2_of(nslots), side, hdr, bloom,
                       nwords ? 64u - log2_of(nwords) : 0u, rep);
  }
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}

template <int KT, typename W, typename BR, typename PR>
int probe_t(const tk_join_table* t, const void* keys, const void* rids, uint64_t n, void* out_p,
            void* out_b, uint64_t cap, uint64_t* d_count, hipStream_t st) {
  auto* hdr = static_cast<const JoinHeader*>(t->table);
  auto* slots = reinterpret_cast<const Slot<W>*>(static_cast<const char*>(t->table) + JOIN_HEADER_BYTES);
  auto* side = reinterpret_cast<const BR*>(static_cast<const char*>(t->table) +
                                           side_offset(t->slots, sizeof(Slot<W>)));
  auto* cnt = reinterpret_cast<unsigned long long*>(d_count);
  hipLaunchKernelGGL(k_jclear, dim3(1), dim3(1), 0, st, cnt);
  if (n) {
    ProbeArgs<W, BR, PR> a;
    a.keys = keys;
    a.rids = static_cast<const PR*>(rids);
    a.n = n;
    a.slots = slots;
    a.mask = t->slots - 1;
    a.shift = 64u - log2_of(t->slots);
    a.side = side;
    a.hdr = hdr;
    a.bloom = t->bloom_words ? words_at(t->table, bloom_offset(t->n_build, t->slots, sizeof(Slot<W>),
                                                               sizeof(BR)))
                             : nullptr;
    a.bshift = t->bloom_words ? 64u - log2_of(t->bloom_words) : 0u;
    a.rep = words_at(t->table, repeat_offset(t->n_build, t->slots, sizeof(Slot<W>), sizeof(BR)));
    a.out_p = static_cast<PR*>(out_p);
    a.out_b = static_cast<BR*>(out_b);
    a.cap = (out_p && out_b) ? cap : 0;
    a.count = cnt;
    hipLaunchKernelGGL((k_jprobe<KT, W, BR, PR>),
                       dim3(launch_grid(cus(), n, (uint64_t)PROBE_NT * PROBE_PER, PROBE_WG_PER_CU)),
                       dim3(PROBE_NT), 0, st, a);
  }
  return hipGetLastError() == hipSuccess ? TK_OK : TK_EHIP;
}

template <int KT, typename W, typename BR>
int probe_rid(const tk_join_table* t, const void* keys, const void* rids, uint64_t n, int prt,
              void* out_p, void* out_b, uint64_t cap, uint64_t* d_count, hipStream_t st) {
  if (prt == TK_RID_U32)
    return probe_t<KT, W, BR, uint32_t>(t, keys, rids, n, out_p, out_b, cap, d_count, st);
  return probe_t<KT, W, BR, unsigned long long>(t, keys, rids, n, out_p, out_b, cap, d_count, st);
}

}  // namespace

extern "C" size_t tk_join_table_size(uint64_t n_build, int key_type, int rid_type) {
  if ((key_type != TK_KEY_I32 && key_type != TK_KEY_I64) ||
      (rid_type != TK_RID_U32 && rid_type != TK_RID_U64) || n_build > JOIN_MAX_BUILD)
    return 0;
  return table_bytes_for(n_build, key_type, rid_type);
}

extern "C" int tk_join_build(const void* keys, const void* rowids, uint64_t n_build, int key_type,
                             int rid_type, void* table, size_t table_bytes, tk_join_table* out,
                             void* stream) {
  if (key_type == TK_KEY_F32 || key_type == TK_KEY_F64) return TK_EUNSUPPORTED;
  if ((key_type != TK_KEY_I32 && key_type != TK_KEY_I64) ||
      (rid_type != TK_RID_U32 && rid_type != TK_RID_U64) || !out || !table)
    return TK_EINVAL;
  if (n_build > JOIN_MAX_BUILD) return TK_EUNSUPPORTED;
  if (n_build && !keys) return TK_EINVAL;
  if (rid_type == TK_RID_U32 && !rowids && n_build > (1ull << 32)) return TK_EINVAL;
  if (((uintptr_t)table & 255) != 0) return TK_EINVAL;
  if (table_bytes < table_bytes_for(n_build, key_type, rid_type)) return TK_EINVAL;
  const uint64_t nslots = slots_for(n_build);
  const uint64_t nwords = tk::current_tuning().join_bloom ? bloom_words_for(nslots) : 0;
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (key_type == TK_KEY_I32 && rid_type == TK_RID_U32)
    rc = build_t<TK_KEY_I32, uint32_t, uint32_t>(keys, rowids, n_build, table, nslots, nwords, st);
  else if (key_type == TK_KEY_I32)
    rc = build_t<TK_KEY_I32, unsigned long long, unsigned long long>(keys, rowids, n_build, table,
                                                                     nslots, nwords, st);
  else if (rid_type == TK_RID_U32)
    rc = build_t<TK_KEY_I64, unsigned long long, uint32_t>(keys, rowids, n_build, table, nslots,
                                                           nwords, st);
  else
    rc = build_t<TK_KEY_I64, unsigned long long, unsigned long long>(keys, rowids, n_build, table,
                                                                     nslots, nwords, st);
  if (rc != TK_OK) return rc;
  out->table = table;
  out->table_bytes = table_bytes;
  out->n_build = n_build;
  out->slots = nslots;
  out->key_type = key_type;
  out->rid_type = rid_type;
  out->bloom_words = nwords;
  return TK_OK;
}

extern "C" int tk_join_probe(const tk_join_table* t, const void* keys, const void* rowids,
                             uint64_t n_probe, int rid_type, void* out_probe_rowids,
                             void* out_build_rowids, uint64_t capacity, uint64_t* d_count,
                             void* stream) {
  if (!t || !t->table || !d_count) return TK_EINVAL;
  if ((t->key_type != TK_KEY_I32 && t->key_type != TK_KEY_I64) ||
      (t->rid_type != TK_RID_U32 && t->rid_type != TK_RID_U64) ||
      (rid_type != TK_RID_U32 && rid_type != TK_RID_U64))
    return TK_EINVAL;
  if (t->slots != slots_for(t->n_build) ||
      t->table_bytes < table_bytes_for(t->n_build, t->key_type, t->rid_type) ||
      (t->bloom_words != 0 && t->bloom_words != bloom_words_for(t->slots)))
    return TK_EINVAL;
  if (n_probe && !keys) return TK_EINVAL;
  if (capacity && (!out_probe_rowids || !out_build_rowids)) return TK_EINVAL;
  if (rid_type == TK_RID_U32 && !rowids && n_probe > (1ull << 32)) return TK_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (t->key_type == TK_KEY_I32 && t->rid_type == TK_RID_U32)
    return probe_rid<TK_KEY_I32, uint32_t, uint32_t>(t, keys, rowids, n_probe, rid_type,
                                                     out_probe_rowids, out_build_rowids, capacity,
                                                     d_count, st);
  if (t->key_type == TK_KEY_I32)
    return probe_rid<TK_KEY_I32, unsigned long long, unsigned long long>(
        t, keys, rowids, n_probe, rid_type, out_probe_rowids, out_build_rowids, capacity, d_count, st);
  if (t->rid_type == TK_RID_U32)
    return probe_rid<TK_KEY_I64, unsigned long long, uint32_t>(
        t, keys, rowids, n_probe, rid_type, out_probe_rowids, out_build_rowids, capacity, d_count, st);
  return probe_rid<TK_KEY_I64, unsigned long long, unsigned long long>(
      t, keys, rowids, n_probe, rid_type, out_probe_rowids, out_build_rowids, capacity, d_count, st);
}
