// Serving policy: admission of queued requests to executor slots under an
// HBM budget, packet-count buckets and p-cell box alignment (the last two
// make request shapes repeat, so that captured graphs are replayed).
// Header-only and free of HIP so that the host tests compile it with g++.
#ifndef FGGC_ADMISSION_H
#define FGGC_ADMISSION_H

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <vector>

namespace fggc {

struct SlotState {
  size_t cap;  // device bytes the slot holds now
  bool busy;   // running a request
};

struct Admission {
  int slot = -1;             // slot that takes the request; -1: wait
  std::vector<int> release;  // idle slots whose memory is freed first
  size_t limit = 0;          // the most memory the chosen slot may then hold
};

// Decide where the head-of-queue request (needing `need` bytes) runs.
// An idle slot that already holds enough memory is preferred (the smallest
// such); otherwise the idle slot holding the most grows, if the total stays
// within the budget, after freeing other idle slots (largest first) when
// that is what makes it fit.  Otherwise the request waits for a running one
// to finish.  A request with need > budget must be rejected before this.
inline Admission plan_admission(const std::vector<SlotState> &s, size_t need, size_t budget) {
  Admission r;
  size_t total = 0;
  for (const auto &x : s) total += x.cap;
  int best = -1;
  for (int i = 0; i < (int)s.size(); ++i)
    if (!s[i].busy && s[i].cap >= need && (best < 0 || s[i].cap < s[best].cap)) best = i;
  if (best >= 0) {
    if (total <= budget) {
      r.slot = best;
      r.limit = s[best].cap;
      return r;
    }
  }
  best = -1;
  for (int i = 0; i < (int)s.size(); ++i)
    if (!s[i].busy && (best < 0 || s[i].cap > s[best].cap)) best = i;
  if (best < 0) return r;
  size_t others = total - s[best].cap;
  std::vector<int> idle;
  for (int i = 0; i < (int)s.size(); ++i)
    if (i != best && !s[i].busy && s[i].cap > 0) idle.push_back(i);
  std::sort(idle.begin(), idle.end(), [&](int a, int b) { return s[a].cap > s[b].cap; });
  for (int j : idle) {
    if (others + need <= budget) break;
    others -= s[j].cap;
    r.release.push_back(j);
  }
  if (others + need <= budget) {
    r.slot = best;
    r.limit = budget - others;
    return r;
  }
  r.release.clear();
  return r;
}

// Smallest m * 2^e >= N with m in {4, 5, 6, 7, 8} (quarter-octave steps, so
// at most 25% padding); at least 64.
inline int64_t padded_count(int64_t N) {
  if (N <= 64) return 64;
  int e = 0;
  while ((N >> e) >= 8) ++e;
  // now 4 <= N / 2^e < 8 up to the truncated bits
  e = e >= 1 ? e - 1 : 0;
  while ((int64_t(8) << e) < N) ++e;
  const int64_t u = int64_t(1) << e;
  const int64_t m = (N + u - 1) / u;
  return m * u;
}

inline int64_t floor_div(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// Widen the p-cell box [lo, lo + n) to multiples of `a` at both ends.
inline void align_box(int64_t &lo, int64_t &n, int64_t a) {
  const int64_t hi = lo + n;
  lo = floor_div(lo, a) * a;
  n = -floor_div(-hi, a) * a - lo;
}

}  // namespace fggc
#endif
