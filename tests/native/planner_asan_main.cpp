// Host-only driver of the planner under AddressSanitizer/UBSan (and ThreadSanitizer):
// the host pool, every table size at the edges (K = 0, single-entry rows, d = 3..8), the
// core quadrature, the Jacobi eigen/SVD routines and both compression routes.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "planner.hpp"

int main() {
  std::mt19937_64 rng(7);
  std::normal_distribution<double> nd;
  for (int d = 3; d <= 8; ++d)
    for (int K = 0; K <= 12; ++K) {
      hdf::ChainCoeffs cc;
      hdf::chain_coeffs(d, K, cc);
    }
  // the host pool: every index runs once, calls back to back, sizes around the worker count
  for (int rep = 0; rep < 300; ++rep) {
    const int n = rep % 41;
    std::vector<int> hit(n, 0);
    hdf::parallel_for(n, [&](int i) { hit[i] += 1; });
    for (int i = 0; i < n; ++i)
      if (hit[i] != 1) {
        std::printf("pool: index %d of %d ran %d times\n", i, n, hit[i]);
        return 1;
      }
  }
  std::vector<double> a(8192);
  hdf::chebyshev_coeffs(1, 2.0, 1.0, 8192, false, a.data());
  {
    // the cores of the degrees run on the pool: the same values on every call
    std::vector<std::vector<double>> c1, c2;
    hdf::radial_cores(a.data(), 20, 5, 0.1, 0.9, c1);
    hdf::radial_cores(a.data(), 20, 5, 0.1, 0.9, c2);
    if (c1 != c2) {
      std::printf("radial cores differ between calls\n");
      return 1;
    }
  }
  for (int d = 3; d <= 8; ++d)
    for (int p = 0; p <= 24; p += 2) {
      std::vector<std::vector<double>> cores;
      hdf::radial_cores(a.data(), p, d, 0.1, 0.9, cores);
      std::vector<int32_t> t;
      hdf::index_set(d, p / 2, t);
    }
  for (int L = 1; L <= 12; ++L) {
    std::vector<double> Yx(40 * L), Yy(30 * L), Gx(L * L, 0.0), Gy(L * L, 0.0), M(L * L);
    for (auto& v : Yx) v = nd(rng);
    for (auto& v : Yy) v = nd(rng);
    for (int i = 0; i < L; ++i)
      for (int j = 0; j < L; ++j) {
        for (int r = 0; r < 40; ++r) Gx[i * L + j] += Yx[r * L + i] * Yx[r * L + j];
        for (int r = 0; r < 30; ++r) Gy[i * L + j] += Yy[r * L + i] * Yy[r * L + j];
        M[i * L + j] = 1.0 / (1.0 + i + j);
      }
    hdf::DegreeFactor df;
    hdf::compress_degree(0, L, Gx.data(), M.data(), 1e-6, 1e-15, df);
    hdf::Precond pc;
    hdf::gram_precondition(L, Gx.data(), 1e-15, pc);
    hdf::compress_degree_refined(0, L, Gx.data(), pc, M.data(), 1e-6, 1e-14, df);
    hdf::SqrtFactor fx, fy;
    hdf::sqrt_factor_single(L, Gx.data(), 1e-15, fx);
    hdf::sqrt_factor_refined(L, Gy.data(), pc, 1e-14, fy);
    hdf::DegreeFactorCross dc;
    hdf::compress_degree_cross(0, L, fx, fy, M.data(), 1e-6, dc);
    // rectangular SVD: A = U S V^T reproduces A
    const int m = L, n = L + 2;
    std::vector<double> A(m * n), U(m * n), S(n), V(n * n);
    for (auto& v : A) v = nd(rng);
    hdf::jacobi_svd(m, n, A.data(), U.data(), S.data(), V.data());
    double err = 0.0, nrm = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += U[i * n + c] * S[c] * V[j * n + c];
        err = std::fmax(err, std::fabs(s - A[i * n + j]));
        nrm = std::fmax(nrm, std::fabs(A[i * n + j]));
      }
    if (err > 1e-12 * nrm) {
      std::printf("svd residual %g at L=%d\n", err, L);
      return 1;
    }
  }
  std::printf("ok\n");
  return 0;
}
