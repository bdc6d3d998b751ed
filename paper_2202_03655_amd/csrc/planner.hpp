// Host planner of the HDF build: the data-free expansion of the kernel and
// the small dense linear algebra of the compression step.
#pragma once
#include <cstddef>
#include <cstdint>
#include <functional>
#include <vector>

namespace hdf {

constexpr int kChebNodes = 8192;     // first-kind nodes of the Chebyshev transform
constexpr int kMaxDim = 8;

// k(r; l) and dk/dl for the four kernels (kind = hdf_kernel value).
double kernel_value(int kind, double r, double l);
double kernel_dl(int kind, double r, double l);

// Chebyshev coefficients of f(s) = k(D|s|; l) from the DCT-II at n first-kind
// nodes (n a power of two); odd coefficients set to zero.
void chebyshev_coeffs(int kind, double D, double l, int n, bool derivative, double* a);

// Smallest even p <= p_max with sum_{i>p}|a_i| <= thr; -1 if none.
int choose_degree(const double* a, int n, double thr, int p_max, double* tail_at_p);

// Radial cores M_k (k = 0..p/2), row-major, L_k = p/2 - k + 1, basis
// T_a(t), t = (2 rho^2 - u0 - u1)/(u1 - u0); Z_k folded in.
void radial_cores(const double* a, int p, int d, double u0, double u1,
                  std::vector<std::vector<double>>& cores);

// Index set H_k (flat, d-2 ints per harmonic) in the enumeration order.
void index_set(int d, int k, std::vector<int32_t>& out);
int64_t index_count(int d, int k);
double sphere_area(int d);

// Symmetric eigendecomposition (cyclic Jacobi): A (n x n row-major, destroyed)
// -> eigenvalues w (unsorted) and eigenvectors as columns of V (row-major).
void jacobi_eigh(int n, double* A, double* w, double* V);

// Interval of rho^2 carrying the radial basis (widened when degenerate).
void radial_interval(double rmin2, double rmax2, double* u0, double* u1);

// Per-degree compression from the radial Gram G (L x L) and core M (L x L).
struct DegreeFactor {
  int k = 0, L = 0, s = 0;
  std::vector<double> lam;   // s kept eigenvalues, ordered
  std::vector<double> E;     // L x s, column-major by l: E[l*L + a]
  std::vector<double> Ep;    // L x s, column-major by l
};
void compress_degree(int k, int L, const double* G, const double* M, double tau,
                     double null_rel, DegreeFactor& out);
// The same from an eigendecomposition G = Vg diag(wg) Vg^T already at hand (Vg row-major L x L).
void compress_degree_eig(int k, int L, const double* wg, const double* Vg, const double* M, double tau,
                         double null_rel, DegreeFactor& out);

// Two-pass (CholeskyQR2-style) compression.  Pass 1: from the radial Gram G1
// (L x L) build the preconditioner T1 = V1 diag(lam1c)^{-1/2} (L x L,
// row-major), eigenvalues clamped from below at floor_rel * max.  Pass 2:
// G2 = (Y T1)^T (Y T1) is recomputed from the data; with G2 = V2 L2 V2^T,
// R = diag(sqrt(L2)) V2^T diag(sqrt(lam1c)) V1^T satisfies Y = Q R with Q
// orthonormal to working accuracy, and the degree is compressed from
// eig(R M R^T) as in the single-pass routine.
struct Precond {
  int L = 0;
  std::vector<double> V1, lam1c, T1;   // L x L row-major; T1 = V1 diag(lam1c^-1/2)
  std::vector<double> w1;              // eigenvalues of G1 before the clamp (G1 = V1 diag(w1) V1^T)
};
void gram_precondition(int L, const double* G1, double floor_rel, Precond& pc);
void compress_degree_refined(int k, int L, const double* G2, const Precond& pc, const double* M,
                             double tau, double null_rel, DegreeFactor& out);

// General case X != Y (Algorithm 1): square-root factors of the two radial
// Grams, Y = Q R with Q orthonormal, R (r x L) and T (L x r) with R T = I
// (row-major); from the single-pass Gram or the refined pair (G2, pc).
struct SqrtFactor {
  int L = 0, r = 0;
  std::vector<double> R, T;
};
void sqrt_factor_single(int L, const double* G, double null_rel, SqrtFactor& f);
void sqrt_factor_refined(int L, const double* G2, const Precond& pc, double null_rel, SqrtFactor& f);
// One-sided Jacobi SVD of A (m x n, row-major): A = U diag(S) V^T, U m x n,
// V n x n (row-major), S unsorted.
void jacobi_svd(int m, int n, const double* A, double* U, double* S, double* V);
// Per-degree compression of the cross radial core: SVD of R_x M R_y^T, the
// singular values above tau kept in descending order; radial coefficients
// Ex = T_x U sqrt(S), Ey = T_y V sqrt(S) (L x s, column-major by l), signed so
// that the largest-magnitude entry of each Ex column is positive.
struct DegreeFactorCross {
  int k = 0, L = 0, s = 0;
  std::vector<double> sig, Ex, Ey;
};
void compress_degree_cross(int k, int L, const SqrtFactor& fx, const SqrtFactor& fy, const double* M,
                           double tau, DegreeFactorCross& out);

// The kernel-matrix threshold tau of the Frobenius-form error budget; N is
// the side of the kernel matrix (sqrt(N_x N_y) for a rectangular one).
// Placement of work items of unequal weight (loads[i] > 0) into workgroups of at most wg
// waves, wave w of a workgroup running on SIMD w % ns: ceil(n / wg) groups, the wg G - n missing
// waves taken one per group from the last groups first, and the items, heaviest first, each given
// to the SIMD of a group with a free wave and the smallest load so far (then the group with the
// smallest load).  order receives the items wave by wave, groups after one another; nw the waves
// of each group.  Returns false (outputs unspecified) if the inputs admit no placement.
bool place_wave_items(const std::vector<int>& loads, int wg, int ns, std::vector<int>& order,
                      std::vector<int>& nw);
// Runs fn(i) for every i in [0, n) on the calling thread and the workers of a process-wide
// pool (at most 8, created on first use), each taking the next index from a shared counter;
// returns when every call has returned.  The calls must be independent of each other and must
// not call parallel_for.  Concurrent callers are served one after the other; in a process forked
// after the pool started, everything runs on the calling thread.
void parallel_for(int n, const std::function<void(int)>& fn);
double tau_threshold(double tol, double nu, double N, int d, int p);

// Tighter degree and rank selection (remark after Eq. bound).  The relative
// Frobenius error is estimated from M sampled pairs, stratified into the
// off-diagonal pairs (a != b) and the diagonal at the pairs' first points:
//   ||E||^2 ~ N (N-1) mean_off e^2 + N mean_diag e^2, the same for ||K||^2.
// Per pair (device, launch_pairs): r = ||x_a - x_b||, rho^2 of both
// normalised points, their dot product, and the indices a, b.
struct PairSample {
  std::vector<double> r, ra2, rb2, dot;
  std::vector<int32_t> a, b;
};
// Smallest even p <= p_max whose sampled truncation error (kernel vs its
// degree-p Chebyshev expansion on [0, D]) is <= eps / 2; -1 if none.  p_hint
// (the budget rule's degree, or -1) only shortens the scan.
int choose_degree_sampled(int kind, double l, const double* a, int n_coef, double D, double N,
                          const PairSample& ps, double eps, int p_max, int p_hint);
// From the factor kept at tau0 (deg[k].lam ordered by |lambda| descending),
// drop eigenpairs in increasing |lambda| (equal |lambda| together) while the
// sampled error of U D U^T stays <= margin * eps.  Returns tau >= tau0 (kept:
// |lambda| > tau) and the final estimate in *err.
double tune_threshold(int kind, double l, int d, double N, double u0, double u1,
                      const std::vector<DegreeFactor>& deg, const PairSample& ps, double eps,
                      double margin, double tau0, double* err);

// Normalised Gegenbauer chain recurrences of the solid harmonics.
//   level j = 1..d-2 (coordinate x_j, partial radius r_j^2), lower index b:
//   P_0 = c0, P_1 = c1 * x, P_{n+1} = A_n x P_n - B_n r^2 P_{n-1}.
// Values are r^n C_n^lam(x/r) / sqrt(h_n^lam), lam = b + (d-j-1)/2.
struct ChainCoeffs {
  int d = 0, K = 0;
  // layout [level-1][b][n] with n = 0..K (entries for n < 2 hold c0, c1)
  std::vector<double> A, B;        // size (d-2)*(K+1)*(K+1)
  double c0(int level, int b) const { return A[idx(level, b, 0)]; }
  double c1(int level, int b) const { return A[idx(level, b, 1)]; }
  std::size_t idx(int level, int b, int n) const {
    return ((std::size_t)(level - 1) * (K + 1) + b) * (K + 1) + n;
  }
};
void chain_coeffs(int d, int K, ChainCoeffs& out);

// Solid harmonics S_h(x) of every degree <= K and their gradients at one point x
// (d coordinates), by the same nested chain recurrences as the device factor
// kernel, in its loop order, forward mode (each level carries P, dP/dx and
// dP/d(r^2)).  Harmonic t of the loop order goes to row col_of[t] (skipped when
// negative): val[row], grad[row * d + j] = dS/dx_j.
void harmonics_and_gradients(int d, int K, const ChainCoeffs& cc, const int32_t* col_of, const double* x,
                             double* val, double* grad);

// Derivative maps of the solid harmonics: the derivative of a harmonic of
// degree k is a harmonic polynomial of degree k - 1, so
//   dS_{k,h}/dx_j = sum_h' G_k^(j)[h][h'] S_{k-1,h'}
// for the orthonormal bases of degrees k and k - 1.  rows_k[k] is the first
// row of degree k among the H rows of `col_of` (-1 if the degree is absent).
// For every k >= 1 with both degrees present, G[k] holds d blocks of
// |H_k| x |H_{k-1}| (j-major), fitted by least squares on points of the unit
// sphere drawn with SplitMix64 (twice as many points as the largest |H_k|, plus
// 32; normal equations in binary64, solved in extended precision); the fit is
// exact up to rounding because the identity holds at every x.  The maps depend
// on d and the degrees only, not on the data.
void harmonic_derivative_maps(int d, int K, const ChainCoeffs& cc, const int32_t* col_of, int H,
                              const std::vector<int>& rows_k, std::vector<std::vector<double>>& G);

}  // namespace hdf
