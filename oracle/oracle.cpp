// ORACLE — test infrastructure only.  Only the tests, __graft_entry__.smoke()
// and the bench's cpu_baseline leg may load this library.  The product (the HIP
// library and its binding) never calls it.
//
// What it computes: the ordering primitive of the paper (sec. III-A): the
// ORDER BY key LIMIT K result over (key, row-id) pairs, key-only, returning
// the row-ids in sorted order (sec. II-C, "Processing"), with the query
// template of sec. V-B (ORDER BY value DESC LIMIT 100).
//
// Definition written out (readings where the paper is silent are listed in the
// design notes):
//   pair a comes before pair b
//     descending: key_a > key_b, or key_a = key_b and rowid_a < rowid_b
//     ascending:  key_a < key_b, or key_a = key_b and rowid_a < rowid_b
//   where < is numeric order for int32/int64 and the IEEE 754-2019 totalOrder
//   predicate (clause 5.10) for float32 and float64.  The result is the first
//   K_eff = min(K, N) pairs of the input sorted by that relation, best first:
//   the original key bits and the paired row-id.
//
// Steps: an index array 0..N-1; std::nth_element with the comparator puts the
// K_eff best first; std::sort orders those.  Both are library primitives; there
// is no other selection logic.  Single-threaded, slow, obviously correct.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

enum { KEY_I32 = 0, KEY_I64 = 1, KEY_F32 = 2, KEY_F64 = 3 };
enum { RID_U32 = 0, RID_U64 = 1 };
enum { ORDER_DESC = 0, ORDER_ASC = 1 };

// Three-way comparison of two float32 keys under IEEE 754-2019 totalOrder,
// written from the clauses of 5.10 (not from any bit trick):
//  - two numbers that compare unequal keep their numeric order;
//  - numerically equal values differ only as -0 < +0;
//  - a NaN with the sign bit set is below every other datum, one without it
//    above every other datum;
//  - two NaNs of the same sign: for positive sign the smaller significand
//    field (quiet bit included) comes first, for negative sign the larger.
int cmp_f32(float a, float b) {
  const bool an = std::isnan(a), bn = std::isnan(b);
  const bool sa = std::signbit(a), sb = std::signbit(b);
  if (!an && !bn) {
    if (a < b) return -1;
    if (a > b) return 1;
    if (sa == sb) return 0;
    return sa ? -1 : 1;
  }
  if (an && bn) {
    if (sa != sb) return sa ? -1 : 1;
    uint32_t ba, bb;
    std::memcpy(&ba, &a, 4);
    std::memcpy(&bb, &b, 4);
    const uint32_t fa = ba & 0x7FFFFFu, fb = bb & 0x7FFFFFu;
    if (fa == fb) return 0;
    const int c = fa < fb ? -1 : 1;
    return sa ? -c : c;
  }
  if (an) return sa ? -1 : 1;
  return sb ? 1 : -1;
}

// The same clauses for float64 (binary64 significand field: 52 bits).
int cmp_f64(double a, double b) {
  const bool an = std::isnan(a), bn = std::isnan(b);
  const bool sa = std::signbit(a), sb = std::signbit(b);
  if (!an && !bn) {
    if (a < b) return -1;
    if (a > b) return 1;
    if (sa == sb) return 0;
    return sa ? -1 : 1;
  }
  if (an && bn) {
    if (sa != sb) return sa ? -1 : 1;
    uint64_t ba, bb;
    std::memcpy(&ba, &a, 8);
    std::memcpy(&bb, &b, 8);
    const uint64_t fa = ba & 0xFFFFFFFFFFFFFull, fb = bb & 0xFFFFFFFFFFFFFull;
    if (fa == fb) return 0;
    const int c = fa < fb ? -1 : 1;
    return sa ? -c : c;
  }
  if (an) return sa ? -1 : 1;
  return sb ? 1 : -1;
}

template <typename K>
int cmp_int(K a, K b) { return a < b ? -1 : (a > b ? 1 : 0); }

template <typename K, typename R>
struct Before {
  const K* keys;
  const R* rids;  // null: row-id = index
  int key_type;
  int order;
  int key_cmp(uint64_t i, uint64_t j) const {
    if (key_type == KEY_F32) {
      float a, b;
      std::memcpy(&a, &keys[i], 4);
      std::memcpy(&b, &keys[j], 4);
      return cmp_f32(a, b);
    }
    if (key_type == KEY_F64) {
      double a, b;
      std::memcpy(&a, &keys[i], 8);
      std::memcpy(&b, &keys[j], 8);
      return cmp_f64(a, b);
    }
    return cmp_int(keys[i], keys[j]);
  }
  uint64_t rid(uint64_t i) const { return rids ? (uint64_t)rids[i] : i; }
  bool operator()(uint64_t i, uint64_t j) const {
    const int c = key_cmp(i, j);
    if (c != 0) return order == ORDER_DESC ? c > 0 : c < 0;
    return rid(i) < rid(j);
  }
};

template <typename K, typename R>
void run(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int key_type, int order,
         void* out_keys, void* out_rids) {
  std::vector<uint64_t> idx(n);
  for (uint64_t i = 0; i < n; ++i) idx[i] = i;
  Before<K, R> before{(const K*)keys, (const R*)rids, key_type, order};
  std::nth_element(idx.begin(), idx.begin() + (k_eff - 1), idx.end(), before);
  std::sort(idx.begin(), idx.begin() + k_eff, before);
  for (uint64_t j = 0; j < k_eff; ++j) {
    if (out_keys) ((K*)out_keys)[j] = ((const K*)keys)[idx[j]];
    if (out_rids) ((R*)out_rids)[j] = (R)before.rid(idx[j]);
  }
}

template <typename K>
void dispatch_rid(int rid_type, const void* keys, const void* rids, uint64_t n, uint64_t k_eff,
                  int key_type, int order, void* ok, void* orid) {
  if (rid_type == RID_U32) run<K, uint32_t>(keys, rids, n, k_eff, key_type, order, ok, orid);
  else run<K, uint64_t>(keys, rids, n, k_eff, key_type, order, ok, orid);
}

}  // namespace

extern "C" {

// One query.  keys: n keys of key_type (0 int32, 1 int64, 2 float32, 3 float64).  rowids:
// n row-ids of rid_type (0 uint32, 1 uint64), or null for row-id = index.
// order: 0 descending, 1 ascending.  Writes K_eff = min(k, n) results to
// out_keys (key bits, may be null) and out_rowids (rid_type, may be null) and
// K_eff to *out_count.  Returns 0, or -1 on a bad argument.
int oracle_topk(const void* keys, const void* rowids, uint64_t n, uint64_t k, int key_type,
                int rid_type, int order, void* out_keys, void* out_rowids, uint64_t* out_count) {
  if (key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1 || order < 0 || order > 1)
    return -1;
  if (n > 0 && !keys) return -1;
  const uint64_t k_eff = k < n ? k : n;
  if (out_count) *out_count = k_eff;
  if (k_eff == 0) return 0;
  if (key_type == KEY_I32 || key_type == KEY_F32)
    dispatch_rid<int32_t>(rid_type, keys, rowids, n, k_eff, key_type, order, out_keys, out_rowids);
  else
    dispatch_rid<int64_t>(rid_type, keys, rowids, n, k_eff, key_type, order, out_keys, out_rowids);
  return 0;
}

// Batched form: query q covers keys[offsets[q] .. offsets[q+1]) with its own
// k[q] and order[q]; row-ids are the local index inside the query when rowids
// is null, else rowids[offsets[q] + i].  Query q's results go to position
// out_offsets[q] of out_keys/out_rowids, where out_offsets is the exclusive
// prefix sum of min(k[q], n_q) (computed here).  Returns 0 or -1.
int oracle_topk_batched(const void* keys, const void* rowids, const uint64_t* offsets,
                        const uint32_t* ks, const uint8_t* orders, uint32_t q, int key_type,
                        int rid_type, void* out_keys, void* out_rowids) {
  if (!offsets || !ks || !orders) return -1;
  const size_t kb = key_type == KEY_I64 || key_type == KEY_F64 ? 8 : 4, rb = rid_type == RID_U64 ? 8 : 4;
  uint64_t out_pos = 0;
  for (uint32_t i = 0; i < q; ++i) {
    const uint64_t lo = offsets[i], n = offsets[i + 1] - offsets[i];
    uint64_t cnt = 0;
    const void* kq = (const char*)keys + lo * kb;
    const void* rq = rowids ? (const void*)((const char*)rowids + lo * rb) : nullptr;
    void* ok = out_keys ? (void*)((char*)out_keys + out_pos * kb) : nullptr;
    void* orr = out_rowids ? (void*)((char*)out_rowids + out_pos * rb) : nullptr;
    int rc = oracle_topk(kq, rq, n, ks[i], key_type, rid_type, orders[i], ok, orr, &cnt);
    if (rc) return rc;
    out_pos += cnt;
  }
  return 0;
}

}  // extern "C"
