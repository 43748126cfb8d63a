// Closed-form orthonormal eigenbases of the 1D operators L_n(alpha,beta,gamma)
// of eq. (3.1), from the spectral lemmas of Sec. 3.2 (Lemmas 3.1-3.4),
// normalised as eq. (4.5) requires (L = V Lambda V^T with V^T V = I).
//
// Host code only.  Accuracy measures (not in the paper, whose footnote to
// eq. (4.5) reports that entrywise assembly was less accurate than `eig`):
//  * every angle is k*pi*a/b with integers a, b; the numerator is reduced
//    exactly in integer arithmetic to the first octant before one
//    floating-point multiply, so no angle carries a large-argument error;
//  * eigenvalues are evaluated as 4 sin^2(theta/2), which equals the lemmas'
//    2 - 2 cos(theta) but keeps full relative accuracy for small theta.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace kp {

// sin(pi * m / d) for integers m and d > 0, with exact argument reduction.
static double sinpi_frac(int64_t m, int64_t d) {
  int64_t a = m % (2 * d);
  if (a < 0) a += 2 * d;                 // a in [0, 2d)
  double sign = 1.0;
  if (a >= d) { a -= d; sign = -1.0; }   // sin(x + pi) = -sin(x)
  if (2 * a > d) a = d - a;              // sin(pi - x) = sin(x); a/d in [0, 1/2]
  if (4 * a > d) {                       // sin(x) = cos(pi/2 - x), argument <= pi/4
    return sign * std::cos((M_PI * (double)(d - 2 * a)) / (double)(2 * d));
  }
  return sign * std::sin((M_PI * (double)a) / (double)d);
}

// cos(pi * m / d) = sin(pi * (d - 2m) / (2d)).
static double cospi_frac(int64_t m, int64_t d) { return sinpi_frac(d - 2 * m, 2 * d); }

// Fills Q (n x n, row-major, Q[j*n + c] = entry j of eigenvector c) and the
// eigenvalues lam[c] in ascending order.  Returns 0, or -1 for bad input.
int basis_1d(int n, int bc, double* Q, double* lam) {
  if (n < 3 || !Q || !lam) return -1;
  const int64_t N = n;
  switch (bc) {
    case 0: {  // periodic, Lemma 3.1: constant, cos/sin pairs, alternating (n even)
      const double c0 = 1.0 / std::sqrt((double)n), c1 = std::sqrt(2.0 / (double)n);
      int col = 0;
      for (int j = 0; j < n; ++j) Q[j * n + col] = c0;
      lam[col++] = 0.0;
      for (int64_t k = 1; 2 * k < N; ++k) {
        const double s = sinpi_frac(k, N);     // theta_k / 2 = pi k / n
        for (int64_t j = 1; j <= N; ++j) {
          // angle 2 pi j k / n, numerator reduced modulo the period n
          const int64_t m = (j * k) % N;
          Q[(j - 1) * n + col] = c1 * cospi_frac(2 * m, N);
          Q[(j - 1) * n + col + 1] = c1 * sinpi_frac(2 * m, N);
        }
        lam[col] = lam[col + 1] = 4.0 * s * s;
        col += 2;
      }
      if (N % 2 == 0) {
        for (int64_t j = 1; j <= N; ++j) Q[(j - 1) * n + col] = (j % 2 ? -c0 : c0);
        lam[col++] = 4.0;
      }
      return col == n ? 0 : -1;
    }
    case 1: {  // Dirichlet, Lemma 3.2: sin(j k pi / (n+1)), norm^2 = (n+1)/2
      const double c = std::sqrt(2.0 / (double)(N + 1));
      for (int64_t k = 1; k <= N; ++k) {
        const double s = sinpi_frac(k, 2 * (N + 1));
        lam[k - 1] = 4.0 * s * s;
        for (int64_t j = 1; j <= N; ++j)
          Q[(j - 1) * n + (k - 1)] = c * sinpi_frac((j * k) % (2 * (N + 1)), N + 1);
      }
      return 0;
    }
    case 2: {  // Neumann, Lemma 3.3: cos((j - 1/2)(k - 1) pi / n)
      for (int64_t k = 1; k <= N; ++k) {
        const double c = (k == 1) ? 1.0 / std::sqrt((double)N) : std::sqrt(2.0 / (double)N);
        const double s = sinpi_frac(k - 1, 2 * N);
        lam[k - 1] = 4.0 * s * s;
        for (int64_t j = 1; j <= N; ++j)
          Q[(j - 1) * n + (k - 1)] = c * cospi_frac(((2 * j - 1) * (k - 1)) % (4 * N), 2 * N);
      }
      return 0;
    }
    case 3:    // Dirichlet-Neumann, Lemma 3.4: sin(j (2k-1) pi / (2n+1))
    case 4: {  // Neumann-Dirichlet: cos((j - 1/2)(2k-1) pi / (2n+1))
      const int64_t D = 2 * N + 1;
      const double c = 2.0 / std::sqrt((double)D);   // norm^2 = (2n+1)/4
      for (int64_t k = 1; k <= N; ++k) {
        const double s = sinpi_frac(2 * k - 1, 2 * D);
        lam[k - 1] = 4.0 * s * s;
        for (int64_t j = 1; j <= N; ++j) {
          double v;
          if (bc == 3) v = sinpi_frac((j * (2 * k - 1)) % (2 * D), D);
          else v = cospi_frac(((2 * j - 1) * (2 * k - 1)) % (4 * D), 2 * D);
          Q[(j - 1) * n + (k - 1)] = c * v;
        }
      }
      return 0;
    }
    default:
      return -1;
  }
}

}  // namespace kp
