// Low-Kronecker-rank approximation of the 2D pseudoinverse (Sec. 4.3.2),
// host side.  The pseudoinverse is (V_q (x) V_n) diag(g_ij) (V_q (x) V_n)^T
// with the Hadamard pseudoinverse Ghat of the eigenvalue sums (eq. 4.7).
// The low-rank preconditioner keeps the best rank-r approximation G_r of
// Ghat (Eckart-Young-Mirsky); its Kronecker pairs M_{q,rho} (x) M_{n,rho}
// share the eigenbases, so the operator equals
//   (V_q (x) V_n) diag(vec G_r) (V_q (x) V_n)^T,
// which the device applies as the pseudoinverse's mode products with G_r in
// place of Ghat.  This file computes G_r.
//
// Ghat is entrywise 1/(a_i + b_j), a Cauchy-like matrix whose singular values
// fall off quickly, so the leading r singular triplets come from a block
// subspace iteration on Ghat^T Ghat with a few extra columns, followed by a
// Rayleigh-Ritz step; the small symmetric eigenproblems are solved by the
// cyclic Jacobi method (Golub and Van Loan, Sec. 8.5).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace kp {
namespace {

// Eigen-decomposition of a symmetric k x k matrix A (row-major, destroyed):
// eigenvalues in w (descending), eigenvectors in the columns of V.
void jacobi_eigen(std::vector<double>& A, int k, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * k + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        // rotation that zeroes a(p, q): t = tan(theta), the smaller root
        const double tau = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < k; ++r) {   // A <- A J
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = c * arp - s * arq;
          a(r, q) = s * arp + c * arq;
        }
        for (int r = 0; r < k; ++r) {   // A <- J^T A
          const double apr = a(p, r), aqr = a(q, r);
          a(p, r) = c * apr - s * aqr;
          a(q, r) = s * apr + c * aqr;
        }
        for (int r = 0; r < k; ++r) {   // V <- V J
          double& vp = V[(size_t)r * k + p];
          double& vq = V[(size_t)r * k + q];
          const double x = vp, y = vq;
          vp = c * x - s * y;
          vq = s * x + c * y;
        }
      }
  }
  std::vector<int> idx(k);
  for (int i = 0; i < k; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x) > a(y, y); });
  std::vector<double> Vs((size_t)k * k);
  w.resize(k);
  for (int c = 0; c < k; ++c) {
    w[c] = a(idx[c], idx[c]);
    for (int r = 0; r < k; ++r) Vs[(size_t)r * k + c] = V[(size_t)r * k + idx[c]];
  }
  V.swap(Vs);
}

// splitmix64 (Steele, Lea, Flood 2014) as a fixed pseudo-random source.
double mix(uint64_t i) {
  uint64_t z = i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

// Orthonormalises the k columns of Y (q x k, column c at Y[c*q ..]) by
// modified Gram-Schmidt, twice; a column that vanishes (Ghat of lower rank)
// is replaced by a fresh pseudo-random one.
void orthonormalise(std::vector<double>& Y, int q, int k, uint64_t& seed) {
  for (int c = 0; c < k; ++c) {
    double* y = &Y[(size_t)c * q];
    for (int attempt = 0; attempt < 8; ++attempt) {
      double before = 0.0;
      for (int j = 0; j < q; ++j) before += y[j] * y[j];
      for (int pass = 0; pass < 2; ++pass)
        for (int d = 0; d < c; ++d) {
          const double* x = &Y[(size_t)d * q];
          double dot = 0.0;
          for (int j = 0; j < q; ++j) dot += x[j] * y[j];
          for (int j = 0; j < q; ++j) y[j] -= dot * x[j];
        }
      double nrm = 0.0;
      for (int j = 0; j < q; ++j) nrm += y[j] * y[j];
      if (nrm > 1e-24 * before && nrm > 0.0) {
        const double inv = 1.0 / std::sqrt(nrm);
        for (int j = 0; j < q; ++j) y[j] *= inv;
        break;
      }
      for (int j = 0; j < q; ++j) y[j] = mix(seed++);
    }
  }
}

}  // namespace

// G_r, the best rank-r approximation of Ghat with g_ij = 1/(ln_i + lq_j) (0
// where |ln_i + lq_j| < 1e-13), written to tab[j*n + i].  Returns 0, or -1
// for r outside 1..min(n, q).
int lowrank_table(const double* ln, int n, const double* lq, int q, int r, double* tab) {
  const int m = std::min(n, q);
  if (r < 1 || r > m) return -1;
  std::vector<double> G((size_t)n * q);   // row-major [i][j]
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < q; ++j) {
      const double s = ln[i] + lq[j];
      G[(size_t)i * q + j] = std::fabs(s) < 1e-13 ? 0.0 : 1.0 / s;
    }
  const int k = std::min(m, r + 6);
  std::vector<double> Y((size_t)q * k), B((size_t)n * k), C, w, W, prev;
  uint64_t seed = 1;
  for (auto& v : Y) v = mix(seed++);
  orthonormalise(Y, q, k, seed);
  // B = Ghat Y (column c of B at B[c*n ..])
  auto times_g = [&]() {
    std::fill(B.begin(), B.end(), 0.0);
    for (int i = 0; i < n; ++i) {
      const double* g = &G[(size_t)i * q];
      for (int c = 0; c < k; ++c) {
        const double* y = &Y[(size_t)c * q];
        double t = 0.0;
        for (int j = 0; j < q; ++j) t += g[j] * y[j];
        B[(size_t)c * n + i] = t;
      }
    }
  };
  // Ritz values of Ghat^T Ghat on span(Y): eigenvalues of B^T B
  auto ritz = [&]() {
    C.assign((size_t)k * k, 0.0);
    for (int a = 0; a < k; ++a)
      for (int b = a; b < k; ++b) {
        double t = 0.0;
        for (int i = 0; i < n; ++i) t += B[(size_t)a * n + i] * B[(size_t)b * n + i];
        C[(size_t)a * k + b] = C[(size_t)b * k + a] = t;
      }
    jacobi_eigen(C, k, w, W);
  };
  int settled = 0;
  for (int it = 0; it < 500 && settled < 2; ++it) {
    times_g();
    ritz();
    if (!prev.empty()) {
      bool same = true;
      for (int c = 0; c < r; ++c) same = same && std::fabs(w[c] - prev[c]) <= 1e-15 * w[0];
      settled = same ? settled + 1 : 0;
    }
    prev = w;
    // Y <- orth(Ghat^T B)
    for (int c = 0; c < k; ++c) {
      double* y = &Y[(size_t)c * q];
      std::fill(y, y + q, 0.0);
      const double* b = &B[(size_t)c * n];
      for (int i = 0; i < n; ++i) {
        const double bi = b[i];
        const double* g = &G[(size_t)i * q];
        for (int j = 0; j < q; ++j) y[j] += g[j] * bi;
      }
    }
    orthonormalise(Y, q, k, seed);
  }
  // Rayleigh-Ritz on the final basis: G_r = B W_r W_r^T Y^T
  times_g();
  ritz();
  std::vector<double> T((size_t)q * k, 0.0);   // T = Y W_r W_r^T, column c at T[c*q ..]
  for (int c = 0; c < k; ++c)
    for (int d = 0; d < k; ++d) {
      double pcd = 0.0;
      for (int rho = 0; rho < r; ++rho) pcd += W[(size_t)c * k + rho] * W[(size_t)d * k + rho];
      if (pcd == 0.0) continue;
      const double* y = &Y[(size_t)c * q];
      double* t = &T[(size_t)d * q];
      for (int j = 0; j < q; ++j) t[j] += y[j] * pcd;
    }
  for (int j = 0; j < q; ++j)
    for (int i = 0; i < n; ++i) {
      double v = 0.0;
      for (int c = 0; c < k; ++c) v += B[(size_t)c * n + i] * T[(size_t)c * q + j];
      tab[(size_t)j * n + i] = v;
    }
  return 0;
}

}  // namespace kp
