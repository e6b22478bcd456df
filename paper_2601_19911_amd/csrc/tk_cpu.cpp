// Multithreaded CPU Top-K: the CPU route of the cost gate (paper sec. II-B,
// "Risky Gate": small inputs stay on the host).  Same result definition as
// the device path; independent code.
//
// Each thread streams its slice and keeps candidates at or above a running
// threshold in a buffer; when the buffer fills, a partial selection keeps the
// best K and raises the threshold.  The per-thread results are then merged
// with one more selection and a sort.
#include <sched.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <thread>
#include <vector>

#include "mitopk.h"

namespace {

template <typename U, typename R>
struct Comp {
  U u;  // order-preserving key image (ascending queries use its complement)
  R f;  // complemented row-id, so larger is better
  bool operator>(const Comp& o) const { return u > o.u || (u == o.u && f > o.f); }
  bool operator>=(const Comp& o) const { return u > o.u || (u == o.u && f >= o.f); }
};

inline uint32_t img(uint32_t bits, int kt) {
  if (kt == TK_KEY_F32) return bits ^ ((uint32_t)((int32_t)bits >> 31) | 0x80000000u);
  return bits ^ 0x80000000u;
}
inline uint64_t img(uint64_t bits, int kt) {
  if (kt == TK_KEY_F64) return bits ^ ((uint64_t)((int64_t)bits >> 63) | 0x8000000000000000ull);
  return bits ^ 0x8000000000000000ull;
}
inline uint32_t unimg(uint32_t u, int kt) {
  if (kt == TK_KEY_F32) return u ^ (((u >> 31) - 1u) | 0x80000000u);
  return u ^ 0x80000000u;
}
inline uint64_t unimg(uint64_t u, int kt) {
  if (kt == TK_KEY_F64) return u ^ (((u >> 63) - 1ull) | 0x8000000000000000ull);
  return u ^ 0x8000000000000000ull;
}

template <typename U, typename R>
void keep_best(std::vector<Comp<U, R>>& v, size_t k) {
  if (v.size() <= k) return;
  std::nth_element(v.begin(), v.begin() + (k - 1), v.end(),
                   [](const Comp<U, R>& a, const Comp<U, R>& b) { return a > b; });
  v.resize(k);
}

template <typename U, typename R>
void slice_topk(const U* keys, const R* rids, uint64_t lo, uint64_t hi, size_t k, int kt, U dmask,
                std::vector<Comp<U, R>>& out) {
  const size_t cap = std::max<size_t>(4 * k, 4096);
  out.clear();
  out.reserve(cap + 1);
  bool have_thr = false;
  Comp<U, R> thr{0, 0};
  for (uint64_t i = lo; i < hi; ++i) {
    const U u = img(keys[i], kt) ^ dmask;
    if (have_thr && u < thr.u) continue;
    const Comp<U, R> c{u, (R) ~(rids ? rids[i] : (R)i)};
    if (have_thr && !(c >= thr)) continue;
    out.push_back(c);
    if (out.size() >= cap) {
      keep_best(out, k);
      thr = *std::min_element(out.begin(), out.end(),
                              [](const Comp<U, R>& a, const Comp<U, R>& b) { return b > a; });
      have_thr = true;
    }
  }
  keep_best(out, k);
}

template <typename U, typename R>
int run(const void* keys, const void* rids, uint64_t n, uint64_t k_eff, int kt, int order,
        void* out_keys, void* out_rids, int nthreads) {
  const U dmask = order == TK_ASC ? (U) ~(U)0 : (U)0;
  uint64_t per = (n + nthreads - 1) / nthreads;
  if (per < (1u << 15)) {
    nthreads = (int)std::max<uint64_t>(1, n >> 15);
    per = (n + nthreads - 1) / nthreads;
  }
  std::vector<std::vector<Comp<U, R>>> parts(nthreads);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) {
    const uint64_t lo = std::min(n, per * t), hi = std::min(n, per * (t + 1));
    th.emplace_back([=, &parts] {
      slice_topk<U, R>((const U*)keys, (const R*)rids, lo, hi, k_eff, kt, dmask, parts[t]);
    });
  }
  for (auto& x : th) x.join();
  std::vector<Comp<U, R>> all;
  for (auto& p : parts) all.insert(all.end(), p.begin(), p.end());
  keep_best(all, k_eff);
  std::sort(all.begin(), all.end(), [](const Comp<U, R>& a, const Comp<U, R>& b) { return a > b; });
  for (uint64_t j = 0; j < k_eff; ++j) {
    if (out_keys) ((U*)out_keys)[j] = unimg((U)(all[j].u ^ dmask), kt);
    if (out_rids) ((R*)out_rids)[j] = (R)~all[j].f;
  }
  return TK_OK;
}

}  // namespace

extern "C" int tk_cpu_topk(const void* keys, const void* rowids, uint64_t n, uint64_t k,
                           int key_type, int rid_type, int order, void* out_keys,
                           void* out_rowids, uint64_t* out_count, int nthreads) {
  if (key_type < 0 || key_type > 3 || rid_type < 0 || rid_type > 1 || order < 0 || order > 1)
    return TK_EINVAL;
  if (n > 0 && !keys) return TK_EINVAL;
  const uint64_t k_eff = k < n ? k : n;
  if (out_count) *out_count = k_eff;
  if (k_eff == 0) return TK_OK;
  if (nthreads <= 0) {
    cpu_set_t set;
    nthreads = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set) : 1;
    if (nthreads < 1) nthreads = 1;
  }
  try {
    if (key_type == TK_KEY_I64 || key_type == TK_KEY_F64) {
      if (rid_type == TK_RID_U32)
        return run<uint64_t, uint32_t>(keys, rowids, n, k_eff, key_type, order, out_keys, out_rowids, nthreads);
      return run<uint64_t, uint64_t>(keys, rowids, n, k_eff, key_type, order, out_keys, out_rowids, nthreads);
    }
    if (rid_type == TK_RID_U32)
      return run<uint32_t, uint32_t>(keys, rowids, n, k_eff, key_type, order, out_keys, out_rowids, nthreads);
    return run<uint32_t, uint64_t>(keys, rowids, n, k_eff, key_type, order, out_keys, out_rowids, nthreads);
  } catch (...) {
    return TK_ENOMEM;
  }
}

namespace {

template <typename R>
int gather_host(const double* cols, uint32_t ncols, uint64_t n, const R* rids, uint64_t k,
                double* out, int nthreads) {
  for (uint64_t j = 0; j < k; ++j)
    if ((uint64_t)rids[j] >= n) return TK_EINVAL;
  auto work = [&](uint32_t c0, uint32_t c1) {
    for (uint32_t c = c0; c < c1; ++c) {
      const double* col = cols + (uint64_t)c * n;
      double* o = out + (uint64_t)c * k;
      for (uint64_t j = 0; j < k; ++j) o[j] = col[rids[j]];
    }
  };
  const uint32_t t = (uint32_t)std::max(1, std::min<int>(nthreads, (int)ncols));
  if (t == 1 || (uint64_t)ncols * k < 65536) {
    work(0, ncols);
    return TK_OK;
  }
  std::vector<std::thread> th;
  for (uint32_t i = 0; i < t; ++i)
    th.emplace_back(work, (uint32_t)((uint64_t)ncols * i / t), (uint32_t)((uint64_t)ncols * (i + 1) / t));
  for (auto& x : th) x.join();
  return TK_OK;
}

}  // namespace

extern "C" int tk_gather_f64_host(const double* cols, uint32_t ncols, uint64_t n,
                                  const void* rowids, int rid_type, uint64_t k, double* out,
                                  int nthreads) {
  if (rid_type != TK_RID_U32 && rid_type != TK_RID_U64) return TK_EINVAL;
  if (k == 0 || ncols == 0) return TK_OK;
  if (!cols || !rowids || !out) return TK_EINVAL;
  if (nthreads <= 0) nthreads = 1;
  try {
    if (rid_type == TK_RID_U32)
      return gather_host(cols, ncols, n, static_cast<const uint32_t*>(rowids), k, out, nthreads);
    return gather_host(cols, ncols, n, static_cast<const uint64_t*>(rowids), k, out, nthreads);
  } catch (...) {
    return TK_ENOMEM;
  }
}
