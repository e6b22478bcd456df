// ORACLE — test infrastructure only.  Only the tests, __graft_entry__.smoke()
// and the bench's cpu_baseline leg may load this library.  The product (the HIP
// library and its binding) never calls it.
//
// What it computes: the matching primitive of the paper (sec. III-B), the probe
// phase of a key-based equi-join done key-only.  The build side is a list of
// (key, row-id) pairs, the probe side another; the result is the set of matched
// pointers (sec. II-C, "Processing"), i.e. every pair
//     (probe row-id p_j, build row-id b_i)   with   probe_key_j == build_key_i,
// once per (j, i), for an inner equi-join.  Keys are integers (int32 or int64)
// and compare by numeric equality.  The result is a multiset; it is returned in
// one canonical order, ascending by (probe row-id, build row-id), so that two
// correct results compare equal element by element.
//
// Steps, each a library primitive:
//   1. sort the build positions by (key, row-id)            (std::sort)
//   2. for every probe key, the run of equal build keys      (std::equal_range)
//      contributes one pair per member
//   3. sort the pairs by (probe row-id, build row-id)       (std::sort)
// Single-threaded, slow, obviously correct.  The nested loop over all (j, i)
// is the pure-Python brute force this is pinned against on tiny inputs.
#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace {

enum { KEY_I32 = 0, KEY_I64 = 1 };
enum { RID_U32 = 0, RID_U64 = 1 };

uint64_t rid_at(const void* rids, int rid_type, uint64_t i) {
  if (!rids) return i;
  return rid_type == RID_U32 ? (uint64_t)((const uint32_t*)rids)[i] : ((const uint64_t*)rids)[i];
}

template <typename K>
std::vector<std::pair<uint64_t, uint64_t>> join(const K* bk, const void* br, int br_type,
                                                uint64_t nb, const K* pk, const void* pr,
                                                int pr_type, uint64_t np) {
  // step 1: build side sorted by key, equal keys by row-id
  std::vector<std::pair<K, uint64_t>> build(nb);
  for (uint64_t i = 0; i < nb; ++i) build[i] = {bk[i], rid_at(br, br_type, i)};
  std::sort(build.begin(), build.end());
  // step 2: one pair per equal build key
  std::vector<std::pair<uint64_t, uint64_t>> out;
  for (uint64_t j = 0; j < np; ++j) {
    const K key = pk[j];
    auto lo = std::lower_bound(build.begin(), build.end(), key,
                               [](const std::pair<K, uint64_t>& e, K v) { return e.first < v; });
    auto hi = std::upper_bound(build.begin(), build.end(), key,
                               [](K v, const std::pair<K, uint64_t>& e) { return v < e.first; });
    const uint64_t p = rid_at(pr, pr_type, j);
    for (auto it = lo; it != hi; ++it) out.push_back({p, it->second});
  }
  // step 3: canonical order
  std::sort(out.begin(), out.end());
  return out;
}

std::vector<std::pair<uint64_t, uint64_t>> g_last;

}  // namespace

extern "C" {

// Runs the join and keeps its result; returns the number of matched pairs, or
// -1 on a bad argument.  build_rowids / probe_rowids may be null (row-id =
// position).  key_type: 0 int32, 1 int64.  *_rid_type: 0 uint32, 1 uint64 (the
// type of the given row-id array; ignored when it is null).
int64_t oracle_join(const void* build_keys, const void* build_rowids, uint64_t n_build,
                    int build_rid_type, const void* probe_keys, const void* probe_rowids,
                    uint64_t n_probe, int probe_rid_type, int key_type) {
  if (key_type < 0 || key_type > 1 || build_rid_type < 0 || build_rid_type > 1 ||
      probe_rid_type < 0 || probe_rid_type > 1)
    return -1;
  if ((n_build > 0 && !build_keys) || (n_probe > 0 && !probe_keys)) return -1;
  if (key_type == KEY_I32)
    g_last = join<int32_t>((const int32_t*)build_keys, build_rowids, build_rid_type, n_build,
                           (const int32_t*)probe_keys, probe_rowids, probe_rid_type, n_probe);
  else
    g_last = join<int64_t>((const int64_t*)build_keys, build_rowids, build_rid_type, n_build,
                           (const int64_t*)probe_keys, probe_rowids, probe_rid_type, n_probe);
  return (int64_t)g_last.size();
}

// Copies the pairs of the last oracle_join into two uint64 arrays of its size.
void oracle_join_fetch(uint64_t* out_probe_rowids, uint64_t* out_build_rowids) {
  for (size_t i = 0; i < g_last.size(); ++i) {
    out_probe_rowids[i] = g_last[i].first;
    out_build_rowids[i] = g_last[i].second;
  }
  g_last.clear();
  g_last.shrink_to_fit();
}

}  // extern "C"
