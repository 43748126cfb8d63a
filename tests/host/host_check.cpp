// Host-side checks of the library's plain C++ parts (closed-form bases, the
// low-rank factor, the request server's HBM accounting), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by test_host_sanitizers.py.
// Prints "host checks ok" and returns 0, or reports the first failure.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_2501_03377_amd/csrc/kp_budget.h"

namespace kp {
int basis_1d(int n, int bc, double* Q, double* lam);
int lowrank_table(const double* ln, int n, const double* lq, int q, int r, double* tab);
}  // namespace kp

static int fail(const char* what, int a, int b) {
  std::printf("FAILED: %s (%d, %d)\n", what, a, b);
  return 1;
}

int main() {
  // every boundary condition of eq. (3.1) at many sizes: the bases are
  // orthonormal and the eigenvalues ascending
  const int sizes[] = {3, 4, 5, 6, 7, 8, 9, 16, 17, 31, 64, 65, 100, 128, 257, 512};
  for (int n : sizes)
    for (int bc = 0; bc < 5; ++bc) {
      std::vector<double> Q((size_t)n * n), lam(n);
      if (kp::basis_1d(n, bc, Q.data(), lam.data()) != 0) return fail("basis_1d", n, bc);
      for (int i = 1; i < n; ++i)
        if (lam[i] < lam[i - 1] - 1e-15) return fail("ascending", n, bc);
      double worst = 0.0;
      for (int a = 0; a < n; ++a)
        for (int b = a; b < n; b += (n > 64 ? 7 : 1)) {
          double d = 0.0;
          for (int j = 0; j < n; ++j) d += Q[(size_t)j * n + a] * Q[(size_t)j * n + b];
          worst = std::fmax(worst, std::fabs(d - (a == b ? 1.0 : 0.0)));
        }
      if (worst > 1e-12) return fail("orthonormal", n, bc);
    }
  // invalid sizes and boundary codes are refused
  {
    std::vector<double> Q(16), lam(4);
    if (kp::basis_1d(2, 0, Q.data(), lam.data()) == 0) return fail("n < 3 accepted", 2, 0);
    if (kp::basis_1d(4, 7, Q.data(), lam.data()) == 0) return fail("bad bc accepted", 4, 7);
  }
  // the low-rank factor on several shapes and ranks
  const int shapes[][3] = {{8, 12, 1}, {20, 30, 2}, {64, 48, 5}, {100, 100, 3}, {33, 17, 16}};
  for (const auto& s : shapes) {
    const int n = s[0], q = s[1], r = s[2];
    std::vector<double> Qn((size_t)n * n), ln(n), Qq((size_t)q * q), lq(q), tab((size_t)n * q);
    kp::basis_1d(n, 1, Qn.data(), ln.data());
    kp::basis_1d(q, 3, Qq.data(), lq.data());
    if (kp::lowrank_table(ln.data(), n, lq.data(), q, r, tab.data()) != 0)
      return fail("lowrank_table", n, r);
    for (double v : tab)
      if (!std::isfinite(v)) return fail("lowrank finite", n, r);
  }
  // HBM accounting with an injected allocation failure: a 300-byte buffer is
  // regrown to 500 bytes (growth reserved first); the allocation fails, so
  // neither the old buffer nor the growth is held any more
  {
    kp::Budget b;
    b.limit = 1000;
    b.add(300);
    if (!b.fits(200)) return fail("fits", (int)b.used, 200);
    b.add(200);
    size_t size = kp::regrow(b, 300, 500, false);
    if (size != 0 || b.used != 0 || b.high != 500) return fail("regrow failure", (int)b.used, (int)size);
    // a later regrowth from nothing succeeds and accounts exactly its size
    b.add(500);
    size = kp::regrow(b, 0, 500, true);
    if (size != 500 || b.used != 500) return fail("regrow success", (int)b.used, (int)size);
    if (b.fits(501) || !b.fits(500)) return fail("budget edge", (int)b.used, 0);
  }
  std::printf("host checks ok\n");
  return 0;
}
