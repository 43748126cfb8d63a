// HBM accounting of the request server (plain C++, no device code): bytes
// held in plans, workspaces and staging buffers against a budget.
#pragma once

#include <stddef.h>

#include <algorithm>

namespace kp {

struct Budget {
  size_t used = 0;    // bytes accounted now
  size_t high = 0;    // high-water mark
  size_t limit = 0;   // 0: no limit

  void add(long long delta) {
    used = (size_t)((long long)used + delta);
    high = std::max(high, used);
  }
  bool fits(size_t more) const { return limit == 0 || used + more <= limit; }
};

// A buffer of `have` bytes is regrown to `need` > have bytes: the old buffer
// is freed and a new one allocated (`ok`: the allocation succeeded).  The
// growth need - have was accounted before the allocation.  Returns the
// buffer's size afterwards (need, or 0 when the allocation failed, in which
// case the old size and the growth are both released).
inline size_t regrow(Budget& b, size_t have, size_t need, bool ok) {
  if (ok) return need;
  b.add(-(long long)need);   // have + (need - have): nothing is held any more
  return 0;
}

}  // namespace kp
