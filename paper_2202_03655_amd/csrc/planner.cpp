// Host planner: kernel expansion (data-free) and the small compression step.
//
// Radial cores.  The paper (Sec. 3.3 and App. A) expands the degree-p
// Chebyshev series of the kernel through powers of ||x||, ||y|| and cos(g)
// and re-expands the powers of cos(g) in Gegenbauer polynomials.  That route
// needs exact arithmetic (the power coefficients cancel catastrophically,
// Sec. 3.7).  The same degree-k coefficient function is obtained here
// directly, in extended precision, from the Rodrigues form of the Gegenbauer
// projection: with F(S) = f(sqrt(S)) (a Chebyshev series in S = s^2 since f
// is even), U = |z_x|^2, V = |z_y|^2 and w = sqrt(UV),
//
//   coeff of C_k^alpha(t) in F(U + V - 2 w t)
//     = w^k (-1)^k (k+alpha) Gamma(alpha) / (sqrt(pi) Gamma(alpha+k+1/2))
//       * int_{-1}^{1} F^{(k)}(U + V - 2 w t) (1 - t^2)^{k+alpha-1/2} dt,
//
// (k integrations by parts of the projection against Rodrigues' formula),
// so no division by w^k is ever performed.  Multiplying by Z_k (addition
// theorem) and 4^-k (|z| = rho/2) gives the core as a polynomial in
// (rho_x^2, rho_y^2), which is sampled on a tensor Chebyshev grid and turned
// into Chebyshev coefficients by a 2-D DCT (exact for its degree).  The
// integral is exact by Gauss-Legendre (d odd: the weight is a polynomial) or
// Gauss-Chebyshev of the second kind (d even: weight sqrt(1-t^2) times a
// polynomial).
#include "planner.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <limits>
#include <complex>
#include <map>
#include <memory>
#include <mutex>
#include <cstring>
#include <stdexcept>
#include <thread>
#include <atomic>
#include <condition_variable>
#include <unistd.h>

namespace hdf {

typedef long double ld;
static const ld kPiL = 3.141592653589793238462643383279502884L;

double kernel_value(int kind, double r, double l) {
  switch (kind) {
    case 0: return std::exp(-(r * r) / (2.0 * l * l));
    case 1: return 1.0 / (1.0 + (r * r) / (l * l));
    case 2: { double z = std::sqrt(3.0) * r / l; return (1.0 + z) * std::exp(-z); }
    case 3: { double z = std::sqrt(5.0) * r / l; return (1.0 + z + z * z / 3.0) * std::exp(-z); }
  }
  return NAN;
}

double kernel_dl(int kind, double r, double l) {
  switch (kind) {
    case 0: return kernel_value(0, r, l) * r * r / (l * l * l);
    case 1: { double k = kernel_value(1, r, l); return 2.0 * r * r * k * k / (l * l * l); }
    case 2: { double z = std::sqrt(3.0) * r / l; return z * z * std::exp(-z) / l; }
    case 3: { double z = std::sqrt(5.0) * r / l; return (z / 3.0) * (1.0 + z) * z * std::exp(-z) / l; }
  }
  return NAN;
}

// ---------------------------------------------------------------- host pool
namespace {
class Pool {
 public:
  explicit Pool(int n_workers) : pid_(getpid()) {
    for (int i = 0; i < n_workers; ++i) workers_.emplace_back([this] { loop(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : workers_) t.join();
  }
  void run(int n, const std::function<void(int)>& fn) {
    if (workers_.empty() || getpid() != pid_) {
      for (int i = 0; i < n; ++i) fn(i);
      return;
    }
    std::lock_guard<std::mutex> serial(call_mu_);
    {
      std::lock_guard<std::mutex> lk(mu_);
      fn_ = &fn;
      n_ = n;
      next_.store(0);
      finished_ = 0;
      ++gen_;
    }
    cv_.notify_all();
    work(fn, n);
    // every worker takes part in every generation, so none can be left behind on this one
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return finished_ == (int)workers_.size(); });
    fn_ = nullptr;
  }

 private:
  void work(const std::function<void(int)>& fn, int n) {
    for (int i = next_.fetch_add(1); i < n; i = next_.fetch_add(1)) fn(i);
  }
  void loop() {
    uint64_t seen = 0;
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
      if (stop_) return;
      seen = gen_;
      const std::function<void(int)>* fn = fn_;
      const int n = n_;
      lk.unlock();
      work(*fn, n);
      lk.lock();
      if (++finished_ == (int)workers_.size()) done_.notify_all();
    }
  }
  const pid_t pid_;
  std::vector<std::thread> workers_;
  std::mutex mu_, call_mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)>* fn_ = nullptr;
  std::atomic<int> next_{0};
  int n_ = 0, finished_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};
}  // namespace

void parallel_for(int n, const std::function<void(int)>& fn) {
  if (n <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  static Pool pool((int)std::min(8u, std::max(1u, std::thread::hardware_concurrency()) - 1));
  pool.run(n, fn);
}

// ---------------------------------------------------------------- DCT-II
// Tables of a length-n DCT-II (FFT twiddles, post-twiddles, Chebyshev
// nodes), evaluated once per length and kept for the process.
namespace {
struct DctTables {
  std::vector<std::complex<double>> w;    // exp(-2 pi i j / n), j <= n/2
  std::vector<double> pc, ps;             // cos, sin of -pi i / (2n)
  std::vector<double> node;               // cos(pi (j + 1/2) / n)
};
const DctTables& dct_tables(size_t n) {
  static std::mutex mu;
  static std::map<size_t, std::unique_ptr<DctTables>> cache;
  std::lock_guard<std::mutex> lock(mu);
  std::unique_ptr<DctTables>& t = cache[n];
  if (!t) {
    t.reset(new DctTables());
    t->w.resize(n / 2 + 1);
    for (size_t j = 0; j < t->w.size(); ++j) {
      const double ang = -2.0 * M_PI * (double)j / (double)n;
      t->w[j] = std::complex<double>(std::cos(ang), std::sin(ang));
    }
    t->pc.resize(n);
    t->ps.resize(n);
    t->node.resize(n);
    for (size_t i = 0; i < n; ++i) {
      const double ang = -M_PI * (double)i / (2.0 * (double)n);
      t->pc[i] = std::cos(ang);
      t->ps[i] = std::sin(ang);
      t->node[i] = std::cos(M_PI * ((double)i + 0.5) / (double)n);
    }
  }
  return *t;
}
}  // namespace

// Radix-2 iterative complex FFT (in place, forward sign -1), n a power of 2.
static void fft(std::vector<std::complex<double>>& x, const DctTables& tb) {
  const size_t n = x.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t stride = n / len;
    for (size_t i = 0; i < n; i += len) {
      for (size_t k = 0; k < len / 2; ++k) {
        const std::complex<double> u = x[i + k], b = x[i + k + len / 2], t = tb.w[k * stride];
        // plain product (std::complex's operator* takes a slow inf/nan path)
        const std::complex<double> v(b.real() * t.real() - b.imag() * t.imag(),
                                     b.real() * t.imag() + b.imag() * t.real());
        x[i + k] = u + v;
        x[i + k + len / 2] = u - v;
      }
    }
  }
}

// y_i = sum_j f_j cos(pi i (2j+1) / (2n)) via one length-n FFT (Makhoul).
static void dct2(const std::vector<double>& f, std::vector<double>& y, const DctTables& tb) {
  const size_t n = f.size();
  std::vector<std::complex<double>> v(n);
  for (size_t j = 0; j < n / 2; ++j) {
    v[j] = f[2 * j];
    v[n - 1 - j] = f[2 * j + 1];
  }
  fft(v, tb);
  y.resize(n);
  for (size_t i = 0; i < n; ++i) y[i] = v[i].real() * tb.pc[i] - v[i].imag() * tb.ps[i];
}

// The sampled function f(D |x|) is even, so node j and node n - 1 - j carry the
// same value: the odd coefficients vanish and the even ones are a length-n/2
// DCT-II of the first half, sum_j f_j cos(pi (2i) (2j+1) / (2n)) =
// 2 sum_{j < n/2} f_j cos(pi i (2j+1) / n).
void chebyshev_coeffs(int kind, double D, double l, int n, bool derivative, double* a) {
  const DctTables& tn = dct_tables((size_t)n);
  const int h = n / 2;
  std::vector<double> f(h), y;
  for (int j = 0; j < h; ++j) {
    const double r = D * std::fabs(tn.node[j]);
    f[j] = derivative ? kernel_dl(kind, r, l) : kernel_value(kind, r, l);
  }
  dct2(f, y, dct_tables((size_t)h));
  for (int i = 0; i < n; ++i) a[i] = (i % 2) ? 0.0 : y[i / 2] * 4.0 / n;
  a[0] *= 0.5;
}

int choose_degree(const double* a, int n, double thr, int p_max, double* tail_at_p) {
  std::vector<double> tail(n, 0.0);
  double acc = 0.0;
  for (int i = n - 1; i >= 1; --i) {
    acc += std::fabs(a[i]);
    tail[i - 1] = acc;
  }
  for (int p = 0; p <= std::min(p_max, n - 1); p += 2) {
    if (tail[p] <= thr) {
      if (tail_at_p) *tail_at_p = tail[p];
      return p;
    }
  }
  return -1;
}

// ------------------------------------------------------------ quadrature
static void gauss_legendre(int n, std::vector<ld>& x, std::vector<ld>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    ld z = cosl(kPiL * (i + 0.75L) / (n + 0.5L));
    ld dp = 0;
    for (int it = 0; it < 100; ++it) {
      ld p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      ld dz = p1 / dp;
      z -= dz;
      // quadratic convergence: a step within a few ulps means the node is
      // exact to the working precision (a bound below the type's epsilon
      // would never be met and run every iteration)
      if (fabsl(dz) <= 4 * LDBL_EPSILON * (1 + fabsl(z))) {
        // refresh the derivative at the converged node
        p0 = 1; p1 = z;
        for (int k = 2; k <= n; ++k) {
          ld p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1);
        break;
      }
    }
    x[i] = z;
    w[i] = 2 / ((1 - z * z) * dp * dp);
  }
}

// Clenshaw evaluation of sum_n c_n T_n(x).
static ld clenshaw(const std::vector<ld>& c, ld x) {
  ld b1 = 0, b2 = 0;
  for (int n = (int)c.size() - 1; n >= 1; --n) {
    ld b0 = 2 * x * b1 - b2 + c[n];
    b2 = b1;
    b1 = b0;
  }
  return x * b1 - b2 + (c.empty() ? 0 : c[0]);
}

// d/dx of a Chebyshev series (coefficients), length shrinks by one.
static std::vector<ld> cheb_derivative(const std::vector<ld>& c) {
  const int N = (int)c.size() - 1;
  if (N <= 0) return std::vector<ld>(1, 0);
  std::vector<ld> d(N + 2, 0);
  for (int n = N; n >= 1; --n) d[n - 1] = d[n + 1] + 2 * n * c[n];
  d[0] *= 0.5L;
  d.resize(N);
  return d;
}

void radial_interval(double rmin2, double rmax2, double* u0, double* u1) {
  double a = rmin2, b = rmax2;
  if (!(b > a)) {
    a = 0.0;
    if (!(b > 0.0)) b = 1.0;
  }
  *u0 = a;
  *u1 = b;
}

void radial_cores(const double* a, int p, int d, double u0, double u1,
                  std::vector<std::vector<double>>& cores) {
  const int K = p / 2;
  const ld alpha = (ld)(d - 2) / 2;
  // F(S) = sum_n c_n T_n(2S - 1), c_n = a_{2n}; derivatives in S carry 2^k.
  std::vector<std::vector<ld>> der(K + 1);
  std::vector<ld> cur(K + 1);
  for (int n = 0; n <= K; ++n) cur[n] = a[2 * n];
  for (int k = 0; k <= K; ++k) {
    der[k] = cur;
    std::vector<ld> nx = cheb_derivative(cur);
    for (auto& v : nx) v *= 2;
    cur = nx;
  }
  const ld a0 = ((ld)u0 + (ld)u1) / 2, a1 = ((ld)u1 - (ld)u0) / 2;
  cores.assign(K + 1, std::vector<double>());
  // the degrees are independent: largest (k = 0) first
  parallel_for(K + 1, [&](int k) {
    const int L = K - k + 1;
    // quadrature for int F^(k)(A - B t) (1 - t^2)^{k + alpha - 1/2} dt
    std::vector<ld> tq, wq;
    if (d % 2) {
      const int beta = k + (d - 3) / 2;
      const int deg = (K - k) + 2 * beta;
      gauss_legendre(deg / 2 + 1, tq, wq);
      for (size_t q = 0; q < tq.size(); ++q) wq[q] *= powl(1 - tq[q] * tq[q], beta);
    } else {
      const int m = k + (d - 4) / 2;            // (1-t^2)^{m} sqrt(1-t^2)
      const int deg = (K - k) + 2 * m;
      const int nq = deg / 2 + 1;
      tq.resize(nq);
      wq.resize(nq);
      for (int q = 0; q < nq; ++q) {
        const ld th = kPiL * (q + 1) / (nq + 1);
        tq[q] = cosl(th);
        wq[q] = kPiL / (nq + 1) * sinl(th) * sinl(th) * powl(1 - tq[q] * tq[q], m);
      }
    }
    const ld pref = ((k % 2) ? -1 : 1) * 2 * powl(kPiL, alpha + 0.5L) * powl(0.25L, k) /
                    tgammal(alpha + k + 0.5L);
    std::vector<ld> th(L), r2(L);
    for (int i = 0; i < L; ++i) {
      th[i] = kPiL * (i + 0.5L) / L;
      r2[i] = a0 + a1 * cosl(th[i]);
    }
    std::vector<ld> G((size_t)L * L);
    for (int i = 0; i < L; ++i)
      for (int j = i; j < L; ++j) {
        const ld A = (r2[i] + r2[j]) / 4, B = sqrtl(r2[i] * r2[j]) / 2;
        ld acc = 0;
        for (size_t q = 0; q < tq.size(); ++q) acc += wq[q] * clenshaw(der[k], 2 * (A - B * tq[q]) - 1);
        G[(size_t)i * L + j] = G[(size_t)j * L + i] = pref * acc;
      }
    // 2-D DCT: M[a][b] = (2/L)^2 sum_ij G_ij cos(a th_i) cos(b th_j), halved at 0
    std::vector<ld> C((size_t)L * L);
    for (int aa = 0; aa < L; ++aa)
      for (int i = 0; i < L; ++i) C[(size_t)aa * L + i] = cosl(aa * th[i]);
    std::vector<ld> T1((size_t)L * L, 0);
    for (int aa = 0; aa < L; ++aa)
      for (int j = 0; j < L; ++j) {
        ld s = 0;
        for (int i = 0; i < L; ++i) s += C[(size_t)aa * L + i] * G[(size_t)i * L + j];
        T1[(size_t)aa * L + j] = s;
      }
    std::vector<double>& M = cores[k];
    M.assign((size_t)L * L, 0.0);
    for (int aa = 0; aa < L; ++aa)
      for (int bb = 0; bb < L; ++bb) {
        ld s = 0;
        for (int j = 0; j < L; ++j) s += T1[(size_t)aa * L + j] * C[(size_t)bb * L + j];
        s *= (ld)4 / ((ld)L * L);
        if (aa == 0) s *= 0.5L;
        if (bb == 0) s *= 0.5L;
        M[(size_t)aa * L + bb] = (double)s;
      }
    // exact symmetry (the grid values are symmetric; rounding may differ)
    for (int aa = 0; aa < L; ++aa)
      for (int bb = aa + 1; bb < L; ++bb) {
        double v = 0.5 * (M[(size_t)aa * L + bb] + M[(size_t)bb * L + aa]);
        M[(size_t)aa * L + bb] = M[(size_t)bb * L + aa] = v;
      }
  });
}

// ------------------------------------------------------------ harmonics
static void index_rec(int d, int depth, int upper, std::vector<int32_t>& prefix,
                      std::vector<int32_t>& out) {
  if (depth == d - 2) {
    for (int m = -upper; m <= upper; ++m) {
      out.insert(out.end(), prefix.begin(), prefix.end());
      out.push_back(m);
    }
    return;
  }
  for (int mu = 0; mu <= upper; ++mu) {
    prefix.push_back(mu);
    index_rec(d, depth + 1, mu, prefix, out);
    prefix.pop_back();
  }
}

void index_set(int d, int k, std::vector<int32_t>& out) {
  out.clear();
  std::vector<int32_t> prefix;
  index_rec(d, 1, k, prefix, out);
}

static int64_t binom(int64_t n, int64_t k) {
  if (k < 0 || n < 0 || k > n) return 0;
  int64_t r = 1;
  for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

int64_t index_count(int d, int k) {
  if (k < 0) return 0;
  return binom(k + d - 1, k) - (k >= 2 ? binom(k + d - 3, k - 2) : 0);
}

double sphere_area(int d) {
  return (double)(2 * powl(kPiL, (ld)d / 2) / tgammal((ld)d / 2));
}

double tau_threshold(double tol, double nu, double N, int d, int p) {
  const int K = p / 2;
  const double area = sphere_area(d);
  double denom = 0.0;
  for (int k = 0; k <= K; ++k) denom += (double)index_count(d, k) / area * std::sqrt((double)(K - k + 1));
  return (tol * nu * N / 2.0) / denom;
}

void chain_coeffs(int d, int K, ChainCoeffs& out) {
  out.d = d;
  out.K = K;
  const size_t sz = (size_t)(d - 2) * (K + 1) * (K + 1);
  out.A.assign(sz, 0.0);
  out.B.assign(sz, 0.0);
  std::vector<ld> logh((size_t)std::max(2, K + 1));
  // lgamma at the integers the terms below take (n + 2 lam and n + 1 are whole numbers)
  std::vector<ld> lg_int((size_t)(3 * K + d + 4));
  for (size_t m = 1; m < lg_int.size(); ++m) lg_int[m] = lgammal((ld)m);
  for (int level = 1; level <= d - 2; ++level) {
    for (int b = 0; b <= K; ++b) {
      const int two_lam = 2 * b + d - level - 1;
      const ld lam = b + (ld)(d - level - 1) / 2;
      // log h_n^lam = log(pi) + (1 - 2 lam) log 2 + lgamma(n + 2 lam) - lgamma(n + 1)
      //               - log(n + lam) - 2 lgamma(lam), summed in this order; each log h_n once
      // (the steps below read three consecutive ones)
      const ld head = logl(kPiL) + (1 - 2 * lam) * logl(2.0L), tail = 2 * lgammal(lam);
      const int nh = std::max(2, K - b + 1);
      for (int n = 0; n < nh; ++n) logh[n] = head + lg_int[n + two_lam] - lg_int[n + 1] - logl(n + lam) - tail;
      const size_t base = out.idx(level, b, 0);
      out.A[base + 0] = (double)expl(-0.5L * logh[0]);                 // c0
      if (b < K) out.A[base + 1] = (double)(2 * lam * expl(-0.5L * logh[1]));   // c1 (rows of length >= 2)
      for (int n = 1; n + 1 <= K - b; ++n) {
        const ld an = 2 * (n + lam) / (n + 1) * expl(0.5L * (logh[n] - logh[n + 1]));
        const ld bn = (n + 2 * lam - 1) / (n + 1) * expl(0.5L * (logh[n - 1] - logh[n + 1]));
        out.A[base + n + 1] = (double)an;   // step producing P_{n+1}
        out.B[base + n + 1] = (double)bn;
      }
    }
  }
}

// ------------------------------------------------------------ harmonic gradients
namespace {
struct HGState {
  int d, K;
  const ChainCoeffs* cc;
  const int32_t* col_of;
  const double* xt;
  double r2[8];
  int t;
  double* val;
  double* grad;
};

// Chain level `level` (coordinate level - 1) from index b, prefix pre with gradient gpre.
void hg_chain(HGState& st, int level, int b, double pre, const double* gpre) {
  const int d = st.d, cj = level - 1;
  const double x = st.xt[cj], rr = st.r2[cj];
  double pm1 = 0, pxm1 = 0, prm1 = 0;
  double p = st.cc->A[st.cc->idx(level, b, 0)], px = 0, pr = 0;
  for (int nn = 0; nn <= st.K - b; ++nn) {
    if (nn == 1) {
      pm1 = p; pxm1 = px; prm1 = pr;
      const double c1 = st.cc->A[st.cc->idx(level, b, 1)];
      p = c1 * x; px = c1; pr = 0;
    } else if (nn >= 2) {
      const double A = st.cc->A[st.cc->idx(level, b, nn)], B = st.cc->B[st.cc->idx(level, b, nn)];
      const double pn = A * x * p - B * rr * pm1;
      const double pxn = A * (p + x * px) - B * rr * pxm1;
      const double prn = A * x * pr - B * (pm1 + rr * prm1);
      pm1 = p; pxm1 = px; prm1 = pr;
      p = pn; px = pxn; pr = prn;
    }
    // d/dx_q of P(x_cj, r_cj^2): dP/dx on its own coordinate, 2 x_q dP/dr^2 on every q >= cj
    double g[8];
    for (int q = 0; q < d; ++q) {
      double dp = 0;
      if (q == cj) dp += px;
      if (q >= cj) dp += 2 * st.xt[q] * pr;
      g[q] = gpre[q] * p + pre * dp;
    }
    if (level == 1) {
      const int col = st.col_of[st.t++];
      if (col >= 0) {
        st.val[col] = pre * p;
        for (int q = 0; q < d; ++q) st.grad[(size_t)col * d + q] = g[q];
      }
    } else {
      hg_chain(st, level - 1, b + nn, pre * p, g);
    }
  }
}
}  // namespace

void harmonics_and_gradients(int d, int K, const ChainCoeffs& cc, const int32_t* col_of, const double* x,
                             double* val, double* grad) {
  HGState st{};
  st.d = d; st.K = K; st.cc = &cc; st.col_of = col_of; st.xt = x; st.t = 0; st.val = val; st.grad = grad;
  double acc = 0;
  for (int j = d - 1; j >= 0; --j) {
    acc += x[j] * x[j];
    st.r2[j] = acc;
  }
  // azimuthal part (x_{d-2} + i x_{d-1})^m outermost, cosine branch first
  const double ax = x[d - 2], ay = x[d - 1];
  double cr = 1, ci = 0, pcr = 0, pci = 0;
  const double inv_sqrt_2pi = 0.39894228040143267794, inv_sqrt_pi = 0.56418958354775628695;
  for (int mm = 0; mm <= K; ++mm) {
    if (mm > 0) {
      pcr = cr; pci = ci;
      const double ncr = ax * cr - ay * ci;
      ci = ay * cr + ax * ci;
      cr = ncr;
    }
    const double cm = mm == 0 ? inv_sqrt_2pi : inv_sqrt_pi;
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    g[d - 2] = cm * mm * pcr;                  // d Re z^m / dx = m Re z^(m-1), d / dy = -m Im z^(m-1)
    g[d - 1] = -cm * mm * pci;
    hg_chain(st, d - 2, mm, cm * cr, g);
    if (mm > 0) {
      g[d - 2] = cm * mm * pci;                // d Im z^m / dx = m Im z^(m-1), d / dy = m Re z^(m-1)
      g[d - 1] = cm * mm * pcr;
      hg_chain(st, d - 2, mm, cm * ci, g);
    }
  }
}

namespace {
uint64_t splitmix_next(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// Cholesky factor and solve of a symmetric positive definite n x n system with nrhs columns (long double)
void spd_solve(int n, std::vector<long double>& A, int nrhs, std::vector<long double>& B) {
  for (int j = 0; j < n; ++j) {
    long double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    const long double djj = sqrtl(s);
    A[(size_t)j * n + j] = djj;
    for (int i = j + 1; i < n; ++i) {
      long double t = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = t / djj;
    }
  }
  for (int c = 0; c < nrhs; ++c) {
    for (int i = 0; i < n; ++i) {             // L y = b
      long double t = B[(size_t)i * nrhs + c];
      for (int k = 0; k < i; ++k) t -= A[(size_t)i * n + k] * B[(size_t)k * nrhs + c];
      B[(size_t)i * nrhs + c] = t / A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {        // L^T x = y
      long double t = B[(size_t)i * nrhs + c];
      for (int k = i + 1; k < n; ++k) t -= A[(size_t)k * n + i] * B[(size_t)k * nrhs + c];
      B[(size_t)i * nrhs + c] = t / A[(size_t)i * n + i];
    }
  }
}
}  // namespace

void harmonic_derivative_maps(int d, int K, const ChainCoeffs& cc, const int32_t* col_of, int H,
                              const std::vector<int>& rows_k, std::vector<std::vector<double>>& G) {
  G.assign(K + 1, std::vector<double>());
  int nmax = 1;
  for (int k = 0; k <= K; ++k)
    if (rows_k[k] >= 0) nmax = std::max(nmax, (int)index_count(d, k));
  const int M = 2 * nmax + 32;
  // the harmonics and gradients of every row at M points of the unit sphere
  std::vector<double> val((size_t)M * H), grad((size_t)M * H * d);
  uint64_t seed = 0x48444603ull;
  const double two_pi = 6.283185307179586476925;
  for (int p = 0; p < M; ++p) {
    double x[8], nrm = 0;
    for (int j = 0; j < d; ++j) {            // Box-Muller normals from 53-bit uniforms in (0, 1)
      const double u1 = ((splitmix_next(seed) >> 11) + 0.5) * 0x1.0p-53;
      const double u2 = ((splitmix_next(seed) >> 11) + 0.5) * 0x1.0p-53;
      x[j] = std::sqrt(-2.0 * std::log(u1)) * std::cos(two_pi * u2);
      nrm += x[j] * x[j];
    }
    nrm = std::sqrt(nrm);
    for (int j = 0; j < d; ++j) x[j] /= nrm;
    harmonics_and_gradients(d, K, cc, col_of, x, &val[(size_t)p * H], &grad[(size_t)p * H * d]);
  }
  for (int k = 1; k <= K; ++k) {
    if (rows_k[k] < 0 || rows_k[k - 1] < 0) continue;
    const int n0 = (int)index_count(d, k), n1 = (int)index_count(d, k - 1);
    const int r0 = rows_k[k], r1 = rows_k[k - 1];
    // normal equations (A^T A) X = A^T B_j with A = S_{k-1} (M x n1), B_j = dS_k/dx_j (M x n0)
    std::vector<double> Nd((size_t)n1 * n1, 0.0), Rd((size_t)n1 * n0 * d, 0.0), gj((size_t)n0 * d);
    for (int p = 0; p < M; ++p) {
      const double* v = &val[(size_t)p * H];
      const double* gr = &grad[(size_t)p * H * d];
      for (int j = 0; j < d; ++j)
        for (int h = 0; h < n0; ++h) gj[(size_t)j * n0 + h] = gr[(size_t)(r0 + h) * d + j];
      for (int a = 0; a < n1; ++a) {
        const double va = v[r1 + a];
        double* nrow = &Nd[(size_t)a * n1];
        for (int b = 0; b < n1; ++b) nrow[b] += va * v[r1 + b];
        double* rrow = &Rd[(size_t)a * n0 * d];
        for (size_t c = 0; c < gj.size(); ++c) rrow[c] += va * gj[c];
      }
    }
    std::vector<long double> N(Nd.begin(), Nd.end()), R(Rd.begin(), Rd.end());
    spd_solve(n1, N, n0 * d, R);
    std::vector<double>& g = G[k];
    g.assign((size_t)d * n0 * n1, 0.0);
    for (int j = 0; j < d; ++j)
      for (int h = 0; h < n0; ++h)
        for (int a = 0; a < n1; ++a) g[((size_t)j * n0 + h) * n1 + a] = (double)R[(size_t)a * n0 * d + (size_t)j * n0 + h];
  }
}

// ------------------------------------------------------------ eigen
void jacobi_eigh(int n, double* A, double* w, double* V) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  // Cyclic sweeps with the threshold rule: a rotation is skipped when |a_pq| is below half a unit roundoff
  // of sqrt(|a_pp a_qq|) (it would move no diagonal entry), and the iteration ends after a sweep without a
  // rotation.  (An off-diagonal mass test at the unit-roundoff level is never met once rounding noise of
  // order n eps |A| fills the off-diagonal entries.)
  const double eps = std::numeric_limits<double>::epsilon();
  for (int sweep = 0; sweep < 100; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        if (std::fabs(apq) <= 0.5 * eps * std::sqrt(std::fabs(app * aqq))) continue;
        ++rotated;
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {           // A <- A J (columns p, q)
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {           // A <- J^T A (rows p, q)
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        A[p * n + q] = A[q * n + p] = 0.0;
        for (int k = 0; k < n; ++k) {           // V <- V J
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
    if (rotated == 0) break;
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

void compress_degree(int k, int L, const double* G, const double* M, double tau,
                     double null_rel, DegreeFactor& out) {
  out.k = k;
  out.L = L;
  out.s = 0;
  out.lam.clear();
  out.E.clear();
  out.Ep.clear();
  std::vector<double> Gc(G, G + (size_t)L * L), wg(L), Vg((size_t)L * L);
  jacobi_eigh(L, Gc.data(), wg.data(), Vg.data());
  compress_degree_eig(k, L, wg.data(), Vg.data(), M, tau, null_rel, out);
}

void compress_degree_eig(int k, int L, const double* wg, const double* Vg, const double* M, double tau,
                         double null_rel, DegreeFactor& out) {
  out.k = k;
  out.L = L;
  out.s = 0;
  out.lam.clear();
  out.E.clear();
  out.Ep.clear();
  double gmax = 0.0;
  for (int i = 0; i < L; ++i) gmax = std::max(gmax, wg[i]);
  if (!(gmax > 0.0)) return;
  std::vector<int> kept;
  for (int i = 0; i < L; ++i)
    if (wg[i] > null_rel * gmax) kept.push_back(i);
  const int r = (int)kept.size();
  // B = diag(sqrt(w)) V_kept^T  (r x L);  A = B M B^T
  std::vector<double> B((size_t)r * L);
  for (int i = 0; i < r; ++i)
    for (int a = 0; a < L; ++a) B[(size_t)i * L + a] = std::sqrt(wg[kept[i]]) * Vg[(size_t)a * L + kept[i]];
  std::vector<double> BM((size_t)r * L, 0.0), A((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i)
    for (int b = 0; b < L; ++b) {
      double s = 0.0;
      for (int a = 0; a < L; ++a) s += B[(size_t)i * L + a] * M[(size_t)a * L + b];
      BM[(size_t)i * L + b] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int b = 0; b < L; ++b) s += BM[(size_t)i * L + b] * B[(size_t)j * L + b];
      A[(size_t)i * r + j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j) {
      const double v = 0.5 * (A[(size_t)i * r + j] + A[(size_t)j * r + i]);
      A[(size_t)i * r + j] = A[(size_t)j * r + i] = v;
    }
  std::vector<double> mu(r), W((size_t)r * r);
  jacobi_eigh(r, A.data(), mu.data(), W.data());
  std::vector<int> ord(r);
  for (int i = 0; i < r; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    const double ax = std::fabs(mu[x]), ay = std::fabs(mu[y]);
    if (ax != ay) return ax > ay;
    const int nx = mu[x] < 0, ny = mu[y] < 0;
    if (nx != ny) return nx < ny;
    return x < y;
  });
  for (int c = 0; c < r; ++c) {
    const int i = ord[c];
    if (!(std::fabs(mu[i]) > tau)) break;
    std::vector<double> e(L, 0.0), ep(L, 0.0);
    for (int a = 0; a < L; ++a) {
      double s1 = 0.0, s2 = 0.0;
      for (int j = 0; j < r; ++j) {
        const double v = Vg[(size_t)a * L + kept[j]] * W[(size_t)j * r + i];
        s1 += v / std::sqrt(wg[kept[j]]);
        s2 += v * std::sqrt(wg[kept[j]]);
      }
      e[a] = s1;
      ep[a] = s2;
    }
    int piv = 0;
    for (int a = 1; a < L; ++a)
      if (std::fabs(e[a]) > std::fabs(e[piv])) piv = a;
    if (e[piv] < 0)
      for (int a = 0; a < L; ++a) { e[a] = -e[a]; ep[a] = -ep[a]; }
    out.lam.push_back(mu[i]);
    out.E.insert(out.E.end(), e.begin(), e.end());
    out.Ep.insert(out.Ep.end(), ep.begin(), ep.end());
    out.s++;
  }
}

// ------------------------------------------------------------ SVD
// One-sided Jacobi (Hestenes): plane rotations orthogonalise the columns of
// A (m x n, row-major), accumulated in V (n x n); the singular values are the
// final column norms and U holds the normalised columns (zero where the norm
// is zero).  Works on the matrix itself, not on A^T A, so small singular
// values keep their relative accuracy.
void jacobi_svd(int m, int n, const double* A, double* U, double* S, double* V) {
  std::vector<double> W(A, A + (size_t)m * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double worst = 0.0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int i = 0; i < m; ++i) {
          const double wp = W[(size_t)i * n + p], wq = W[(size_t)i * n + q];
          alpha += wp * wp;
          beta += wq * wq;
          gamma += wp * wq;
        }
        if (gamma == 0.0) continue;
        const double rel = std::fabs(gamma) / std::sqrt(alpha * beta);
        worst = std::max(worst, rel);
        if (rel <= 1e-15) continue;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < m; ++i) {
          const double wp = W[(size_t)i * n + p], wq = W[(size_t)i * n + q];
          W[(size_t)i * n + p] = c * wp - sn * wq;
          W[(size_t)i * n + q] = sn * wp + c * wq;
        }
        for (int i = 0; i < n; ++i) {
          const double vp = V[(size_t)i * n + p], vq = V[(size_t)i * n + q];
          V[(size_t)i * n + p] = c * vp - sn * vq;
          V[(size_t)i * n + q] = sn * vp + c * vq;
        }
      }
    if (worst <= 1e-15) break;
  }
  for (int j = 0; j < n; ++j) {
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += W[(size_t)i * n + j] * W[(size_t)i * n + j];
    nrm = std::sqrt(nrm);
    S[j] = nrm;
    for (int i = 0; i < m; ++i) U[(size_t)i * n + j] = nrm > 0.0 ? W[(size_t)i * n + j] / nrm : 0.0;
  }
}

void sqrt_factor_single(int L, const double* G, double null_rel, SqrtFactor& f) {
  f.L = L;
  f.r = 0;
  f.R.clear();
  f.T.clear();
  std::vector<double> Gc(G, G + (size_t)L * L), w(L), Vg((size_t)L * L);
  jacobi_eigh(L, Gc.data(), w.data(), Vg.data());
  double gmax = 0.0;
  for (int i = 0; i < L; ++i) gmax = std::max(gmax, w[i]);
  if (!(gmax > 0.0)) return;
  std::vector<int> kept;
  for (int i = 0; i < L; ++i)
    if (w[i] > null_rel * gmax) kept.push_back(i);
  f.r = (int)kept.size();
  f.R.assign((size_t)f.r * L, 0.0);
  f.T.assign((size_t)L * f.r, 0.0);
  for (int i = 0; i < f.r; ++i) {
    const double sw = std::sqrt(w[kept[i]]);
    for (int a = 0; a < L; ++a) {
      f.R[(size_t)i * L + a] = sw * Vg[(size_t)a * L + kept[i]];
      f.T[(size_t)a * f.r + i] = Vg[(size_t)a * L + kept[i]] / sw;
    }
  }
}

void sqrt_factor_refined(int L, const double* G2, const Precond& pc, double null_rel, SqrtFactor& f) {
  f.L = L;
  f.r = 0;
  f.R.clear();
  f.T.clear();
  std::vector<double> Gc(G2, G2 + (size_t)L * L), w2(L), V2((size_t)L * L);
  jacobi_eigh(L, Gc.data(), w2.data(), V2.data());
  double gmax = 0.0;
  for (int i = 0; i < L; ++i) gmax = std::max(gmax, w2[i]);
  if (!(gmax > 0.0)) return;
  std::vector<int> kept;
  for (int i = 0; i < L; ++i)
    if (w2[i] > null_rel * gmax) kept.push_back(i);
  f.r = (int)kept.size();
  f.R.assign((size_t)f.r * L, 0.0);
  f.T.assign((size_t)L * f.r, 0.0);
  for (int i = 0; i < f.r; ++i) {
    const int ki = kept[i];
    const double s2 = std::sqrt(w2[ki]);
    for (int a = 0; a < L; ++a) {
      double acc = 0.0, acc2 = 0.0;
      for (int j = 0; j < L; ++j) {
        acc += V2[(size_t)j * L + ki] * std::sqrt(pc.lam1c[j]) * pc.V1[(size_t)a * L + j];
        acc2 += pc.V1[(size_t)a * L + j] / std::sqrt(pc.lam1c[j]) * V2[(size_t)j * L + ki];
      }
      f.R[(size_t)i * L + a] = s2 * acc;
      f.T[(size_t)a * f.r + i] = acc2 / s2;
    }
  }
}

void compress_degree_cross(int k, int L, const SqrtFactor& fx, const SqrtFactor& fy, const double* M,
                           double tau, DegreeFactorCross& out) {
  out.k = k;
  out.L = L;
  out.s = 0;
  out.sig.clear();
  out.Ex.clear();
  out.Ey.clear();
  const int rx = fx.r, ry = fy.r;
  if (rx == 0 || ry == 0) return;
  // A = R_x M R_y^T (rx x ry)
  std::vector<double> RM((size_t)rx * L, 0.0), A((size_t)rx * ry, 0.0);
  for (int i = 0; i < rx; ++i)
    for (int b = 0; b < L; ++b) {
      double acc = 0.0;
      for (int a = 0; a < L; ++a) acc += fx.R[(size_t)i * L + a] * M[(size_t)a * L + b];
      RM[(size_t)i * L + b] = acc;
    }
  for (int i = 0; i < rx; ++i)
    for (int j = 0; j < ry; ++j) {
      double acc = 0.0;
      for (int b = 0; b < L; ++b) acc += RM[(size_t)i * L + b] * fy.R[(size_t)j * L + b];
      A[(size_t)i * ry + j] = acc;
    }
  std::vector<double> U((size_t)rx * ry), S(ry), V((size_t)ry * ry);
  jacobi_svd(rx, ry, A.data(), U.data(), S.data(), V.data());
  std::vector<int> ord(ry);
  for (int i = 0; i < ry; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return S[x] > S[y]; });
  for (int c = 0; c < ry; ++c) {
    const int j = ord[c];
    if (!(S[j] > tau)) break;
    const double rs = std::sqrt(S[j]);
    std::vector<double> ex(L, 0.0), ey(L, 0.0);
    for (int a = 0; a < L; ++a) {
      double s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < rx; ++i) s1 += fx.T[(size_t)a * rx + i] * U[(size_t)i * ry + j];
      for (int i = 0; i < ry; ++i) s2 += fy.T[(size_t)a * ry + i] * V[(size_t)i * ry + j];
      ex[a] = s1 * rs;
      ey[a] = s2 * rs;
    }
    int piv = 0;
    for (int a = 1; a < L; ++a)
      if (std::fabs(ex[a]) > std::fabs(ex[piv])) piv = a;
    if (ex[piv] < 0)
      for (int a = 0; a < L; ++a) { ex[a] = -ex[a]; ey[a] = -ey[a]; }
    out.sig.push_back(S[j]);
    out.Ex.insert(out.Ex.end(), ex.begin(), ex.end());
    out.Ey.insert(out.Ey.end(), ey.begin(), ey.end());
    out.s++;
  }
}

void gram_precondition(int L, const double* G1, double floor_rel, Precond& pc) {
  pc.L = L;
  std::vector<double> Gc(G1, G1 + (size_t)L * L), w(L);
  pc.V1.assign((size_t)L * L, 0.0);
  jacobi_eigh(L, Gc.data(), w.data(), pc.V1.data());
  pc.w1 = w;
  double gmax = 0.0;
  for (int i = 0; i < L; ++i) gmax = std::max(gmax, w[i]);
  if (!(gmax > 0.0)) gmax = 1.0;
  const double floor_v = floor_rel * gmax;
  pc.lam1c.resize(L);
  for (int i = 0; i < L; ++i) pc.lam1c[i] = std::max(w[i], floor_v);
  pc.T1.assign((size_t)L * L, 0.0);
  for (int a = 0; a < L; ++a)
    for (int j = 0; j < L; ++j) pc.T1[(size_t)a * L + j] = pc.V1[(size_t)a * L + j] / std::sqrt(pc.lam1c[j]);
}

void compress_degree_refined(int k, int L, const double* G2, const Precond& pc, const double* M,
                             double tau, double null_rel, DegreeFactor& out) {
  out.k = k;
  out.L = L;
  out.s = 0;
  out.lam.clear();
  out.E.clear();
  out.Ep.clear();
  std::vector<double> Gc(G2, G2 + (size_t)L * L), w2(L), V2((size_t)L * L);
  jacobi_eigh(L, Gc.data(), w2.data(), V2.data());
  double gmax = 0.0;
  for (int i = 0; i < L; ++i) gmax = std::max(gmax, w2[i]);
  if (!(gmax > 0.0)) return;
  std::vector<int> kept;
  for (int i = 0; i < L; ++i)
    if (w2[i] > null_rel * gmax) kept.push_back(i);
  const int r = (int)kept.size();
  // R (r x L) = diag(sqrt(w2)) V2_kept^T diag(sqrt(lam1c)) V1^T
  // T (L x r) = V1 diag(lam1c^-1/2) V2_kept diag(w2^-1/2)  (R T = I)
  std::vector<double> R((size_t)r * L, 0.0), T((size_t)L * r, 0.0);
  for (int i = 0; i < r; ++i) {
    const int ki = kept[i];
    const double s2 = std::sqrt(w2[ki]);
    for (int a = 0; a < L; ++a) {
      double acc = 0.0, acc2 = 0.0;
      for (int j = 0; j < L; ++j) {
        acc += V2[(size_t)j * L + ki] * std::sqrt(pc.lam1c[j]) * pc.V1[(size_t)a * L + j];
        acc2 += pc.V1[(size_t)a * L + j] / std::sqrt(pc.lam1c[j]) * V2[(size_t)j * L + ki];
      }
      R[(size_t)i * L + a] = s2 * acc;
      T[(size_t)a * r + i] = acc2 / s2;
    }
  }
  std::vector<double> RM((size_t)r * L, 0.0), A((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i)
    for (int b = 0; b < L; ++b) {
      double s = 0.0;
      for (int a = 0; a < L; ++a) s += R[(size_t)i * L + a] * M[(size_t)a * L + b];
      RM[(size_t)i * L + b] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < r; ++j) {
      double s = 0.0;
      for (int b = 0; b < L; ++b) s += RM[(size_t)i * L + b] * R[(size_t)j * L + b];
      A[(size_t)i * r + j] = s;
    }
  for (int i = 0; i < r; ++i)
    for (int j = i + 1; j < r; ++j) {
      const double v = 0.5 * (A[(size_t)i * r + j] + A[(size_t)j * r + i]);
      A[(size_t)i * r + j] = A[(size_t)j * r + i] = v;
    }
  std::vector<double> mu(r), W((size_t)r * r);
  jacobi_eigh(r, A.data(), mu.data(), W.data());
  std::vector<int> ord(r);
  for (int i = 0; i < r; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    const double ax = std::fabs(mu[x]), ay = std::fabs(mu[y]);
    if (ax != ay) return ax > ay;
    const int nx = mu[x] < 0, ny = mu[y] < 0;
    if (nx != ny) return nx < ny;
    return x < y;
  });
  for (int c = 0; c < r; ++c) {
    const int i = ord[c];
    if (!(std::fabs(mu[i]) > tau)) break;
    std::vector<double> e(L, 0.0), ep(L, 0.0);
    for (int a = 0; a < L; ++a) {
      double s1 = 0.0, s2 = 0.0;
      for (int j = 0; j < r; ++j) {
        s1 += T[(size_t)a * r + j] * W[(size_t)j * r + i];
        s2 += R[(size_t)j * L + a] * W[(size_t)j * r + i];
      }
      e[a] = s1;
      ep[a] = s2;
    }
    int piv = 0;
    for (int a = 1; a < L; ++a)
      if (std::fabs(e[a]) > std::fabs(e[piv])) piv = a;
    if (e[piv] < 0)
      for (int a = 0; a < L; ++a) { e[a] = -e[a]; ep[a] = -ep[a]; }
    out.lam.push_back(mu[i]);
    out.E.insert(out.E.end(), e.begin(), e.end());
    out.Ep.insert(out.Ep.end(), ep.begin(), ep.end());
    out.s++;
  }
}

}  // namespace hdf

namespace hdf {

// ------------------------------------------------------------------ sampled rules
namespace {

// Stratified relative Frobenius error from the off-diagonal sums of squares
// (errors and values over n_off pairs) and the diagonal ones (over n_d points).
double stratified(double N, double e_off, double k_off, int n_off, double e_d, double k_d, int n_d) {
  const double w_off = N * (N - 1.0), w_d = N;
  double num = w_d * e_d / n_d, den = w_d * k_d / n_d;
  if (n_off > 0) {
    num += w_off * e_off / n_off;
    den += w_off * k_off / n_off;
  }
  return std::sqrt(num / den);
}

}  // namespace

int choose_degree_sampled(int kind, double l, const double* a, int n_coef, double D, double N,
                          const PairSample& ps, double eps, int p_max, int p_hint) {
  // the budget rule's degree bounds the answer in exact arithmetic (a max-norm
  // tail <= eps nu / 2 gives a Frobenius truncation error <= eps / 2): scan up
  // to it first, and on to p_max only if no degree qualifies there
  if (p_hint >= 0 && p_hint < p_max) {
    const int p = choose_degree_sampled(kind, l, a, n_coef, D, N, ps, eps, p_hint, -1);
    if (p >= 0) return p;
  }
  const int M = (int)ps.r.size();
  const int top = std::min(p_max, n_coef - 1);
  // e_off[p] = sum over off-diagonal pairs of (k - S_p)^2 for every p <= top
  std::vector<double> e_off(top + 1, 0.0);
  double k_off = 0.0;
  int n_off = 0;
  for (int t = 0; t < M; ++t) {
    if (ps.a[t] == ps.b[t]) continue;
    ++n_off;
    const double kv = kernel_value(kind, ps.r[t], l), s = ps.r[t] / D;
    k_off += kv * kv;
    double Tm = 1.0, T = s, S = a[0];
    e_off[0] += (kv - S) * (kv - S);
    for (int p = 1; p <= top; ++p) {
      if (p >= 2) {
        const double Tn = 2.0 * s * T - Tm;
        Tm = T;
        T = Tn;
      }
      S += a[p] * T;
      e_off[p] += (kv - S) * (kv - S);
    }
  }
  // diagonal: s = 0, T_i(0) = 1, 0, -1, 0, 1, ...
  const double k0 = kernel_value(kind, 0.0, l);
  double S0 = 0.0;
  for (int p = 0; p <= top; ++p) {
    S0 += a[p] * ((p % 2) ? 0.0 : ((p / 2) % 2 ? -1.0 : 1.0));
    if (p % 2) continue;
    const double e_d = (k0 - S0) * (k0 - S0) * M, k_d = k0 * k0 * M;
    if (stratified(N, e_off[p], k_off, n_off, e_d, k_d, M) <= eps / 2.0) return p;
  }
  return -1;
}

double tune_threshold(int kind, double l, int d, double N, double u0, double u1,
                      const std::vector<DegreeFactor>& deg, const PairSample& ps, double eps,
                      double margin, double tau0, double* err) {
  const int M = (int)ps.r.size();
  const int K = (int)deg.size() - 1;
  const double alpha = 0.5 * d - 1.0;
  const double area = sphere_area(d);
  // eigenpairs kept at tau0, in (k, l) order
  std::vector<int> pk, pl;
  std::vector<double> plam;
  for (int k = 0; k <= K; ++k)
    for (int li = 0; li < deg[k].s; ++li) { pk.push_back(k); pl.push_back(li); plam.push_back(deg[k].lam[li]); }
  const int J = (int)pk.size();
  std::vector<double> c1(K + 1, 1.0), hk(K + 1);      // C_k^alpha(1), |H_k| / |S^{d-1}|
  for (int k = 1; k <= K; ++k) c1[k] = c1[k - 1] * (k + 2.0 * alpha - 1.0) / k;
  for (int k = 0; k <= K; ++k) hk[k] = (double)index_count(d, k) / area;
  std::vector<int> off;
  for (int t = 0; t < M; ++t)
    if (ps.a[t] != ps.b[t]) off.push_back(t);
  const int n_off = (int)off.size();
  const int rows = n_off + M;                          // off-diagonal pairs, then diagonal points
  const double k0 = kernel_value(kind, 0.0, l);
  // Dropping a set S of eigenpairs turns the residual r0 = k - K~ of a row
  // into r0 + sum_{j in S} c_j, so per stratum the squared error is
  //   sum r0^2 + 2 sum_{j in S} b_j + sum_{j, j' in S} G_jj',
  // b_j = sum r0 c_j, G = C^T C: one pass over the rows accumulates them.
  struct Acc {
    std::vector<double> G[2], b[2];
    double r2[2] = {0, 0}, k2[2] = {0, 0};
  };
  auto accumulate = [&](int r0, int r1, Acc& A) {
    for (int st = 0; st < 2; ++st) { A.G[st].assign((size_t)J * J, 0.0); A.b[st].assign(J, 0.0); }
    const int Lmax = K + 1;
    std::vector<double> Ta(Lmax), Tb(Lmax), G(K + 1), cj(J);
    for (int row = r0; row < r1; ++row) {
      double ra2, rb2, dot, kv;
      int st;
      if (row < n_off) {
        const int t = off[row];
        ra2 = ps.ra2[t]; rb2 = ps.rb2[t]; dot = ps.dot[t];
        kv = kernel_value(kind, ps.r[t], l);
        st = 0;
      } else {
        ra2 = rb2 = dot = ps.ra2[row - n_off];
        kv = k0;
        st = 1;
      }
      const double ta = (2.0 * ra2 - u0 - u1) / (u1 - u0), tb = (2.0 * rb2 - u0 - u1) / (u1 - u0);
      Ta[0] = Tb[0] = 1.0;
      if (Lmax > 1) { Ta[1] = ta; Tb[1] = tb; }
      for (int q = 2; q < Lmax; ++q) { Ta[q] = 2.0 * ta * Ta[q - 1] - Ta[q - 2]; Tb[q] = 2.0 * tb * Tb[q - 1] - Tb[q - 2]; }
      // (rho_a rho_b)^k C_k^alpha(cos): solid Gegenbauer recurrence in dot and rho_a^2 rho_b^2
      const double rr = ra2 * rb2;
      G[0] = 1.0;
      if (K >= 1) G[1] = 2.0 * alpha * dot;
      for (int k = 2; k <= K; ++k)
        G[k] = (2.0 * (k + alpha - 1.0) * dot * G[k - 1] - (k + 2.0 * alpha - 2.0) * rr * G[k - 2]) / k;
      double kt = 0.0;
      for (int j = 0; j < J; ++j) {
        const DegreeFactor& df = deg[pk[j]];
        const double* e = df.E.data() + (size_t)pl[j] * df.L;
        double qa = 0.0, qb = 0.0;
        for (int q = 0; q < df.L; ++q) { qa += Ta[q] * e[q]; qb += Tb[q] * e[q]; }
        cj[j] = plam[j] * hk[pk[j]] * G[pk[j]] / c1[pk[j]] * qa * qb;
        kt += cj[j];
      }
      const double r = kv - kt;
      A.r2[st] += r * r;
      A.k2[st] += kv * kv;
      double* Gs = A.G[st].data();
      double* bs = A.b[st].data();
      for (int j = 0; j < J; ++j) {
        bs[j] += r * cj[j];
        const double v = cj[j];
        for (int jj = 0; jj <= j; ++jj) Gs[(size_t)j * J + jj] += v * cj[jj];
      }
    }
  };
  const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<Acc> acc(nth);
  {
    const int per = (rows + nth - 1) / nth;
    std::vector<std::thread> th;
    for (int i = 0; i < nth; ++i) {
      const int r0 = std::min(rows, i * per), r1 = std::min(rows, r0 + per);
      th.emplace_back(accumulate, r0, r1, std::ref(acc[i]));
    }
    for (auto& x : th) x.join();
  }
  // fixed-order combination of the thread partials; G symmetric from its lower triangle
  Acc tot;
  for (int st = 0; st < 2; ++st) { tot.G[st].assign((size_t)J * J, 0.0); tot.b[st].assign(J, 0.0); }
  for (const Acc& A : acc)
    for (int st = 0; st < 2; ++st) {
      tot.r2[st] += A.r2[st];
      tot.k2[st] += A.k2[st];
      for (size_t i = 0; i < tot.G[st].size(); ++i) tot.G[st][i] += A.G[st][i];
      for (int j = 0; j < J; ++j) tot.b[st][j] += A.b[st][j];
    }
  for (int st = 0; st < 2; ++st)
    for (int j = 0; j < J; ++j)
      for (int jj = 0; jj < j; ++jj) tot.G[st][(size_t)jj * J + j] = tot.G[st][(size_t)j * J + jj];
  std::vector<char> dropped(J, 0);
  auto error_with = [&](const std::vector<int>& extra) {
    double e2[2];
    for (int st = 0; st < 2; ++st) {
      const std::vector<double>& Gs = tot.G[st];
      double v = tot.r2[st];
      std::vector<int> S;
      for (int j = 0; j < J; ++j)
        if (dropped[j]) S.push_back(j);
      S.insert(S.end(), extra.begin(), extra.end());
      for (int j : S) v += 2.0 * tot.b[st][j];
      for (int j : S)
        for (int jj : S) v += Gs[(size_t)j * J + jj];
      e2[st] = std::max(v, 0.0);
    }
    return stratified(N, e2[0], tot.k2[0], n_off, e2[1], tot.k2[1], M);
  };
  double e = error_with({}), tau = tau0;
  if (e <= margin * eps && J > 0) {
    std::vector<double> mags(J);
    for (int j = 0; j < J; ++j) mags[j] = std::fabs(plam[j]);
    std::vector<double> levels(mags);
    std::sort(levels.begin(), levels.end());
    levels.erase(std::unique(levels.begin(), levels.end()), levels.end());
    std::vector<int> cols;
    for (double m : levels) {                    // ascending |lambda|, equal |lambda| together
      cols.clear();
      for (int j = 0; j < J; ++j)
        if (mags[j] == m) cols.push_back(j);
      const double e2 = error_with(cols);
      if (e2 > margin * eps) break;
      for (int j : cols) dropped[j] = 1;
      e = e2;
      tau = std::max(tau, m);
    }
  }
  if (err) *err = e;
  return tau;
}

bool place_wave_items(const std::vector<int>& loads, int wg, int ns, std::vector<int>& order,
                      std::vector<int>& nw) {
  const int n = (int)loads.size();
  if (n < 1 || wg < 1 || ns < 1 || wg % ns) return false;
  for (int v : loads)
    if (v < 1) return false;
  const int G = (n + wg - 1) / wg;
  nw.assign(G, wg);
  for (int miss = wg * G - n, g = G - 1; miss > 0; --miss) {
    --nw[g];
    g = g == 0 ? G - 1 : g - 1;
  }
  // bin (g, sm): the waves sm, sm + ns, ... < nw[g] of group g
  std::vector<int> cap(G * ns), bin_load(G * ns, 0), grp_load(G, 0);
  for (int g = 0; g < G; ++g)
    for (int sm = 0; sm < ns; ++sm) cap[g * ns + sm] = sm < nw[g] ? (nw[g] - sm + ns - 1) / ns : 0;
  std::vector<int> by_load(n);
  for (int i = 0; i < n; ++i) by_load[i] = i;
  std::stable_sort(by_load.begin(), by_load.end(), [&](int a, int b) { return loads[a] > loads[b]; });
  std::vector<std::vector<int>> bin(G * ns);
  for (int i : by_load) {
    int best = -1;
    for (int bi = 0; bi < G * ns; ++bi) {
      if ((int)bin[bi].size() >= cap[bi]) continue;
      if (best < 0 || bin_load[bi] < bin_load[best] ||
          (bin_load[bi] == bin_load[best] && grp_load[bi / ns] < grp_load[best / ns]))
        best = bi;
    }
    if (best < 0) return false;
    bin[best].push_back(i);
    bin_load[best] += loads[i];
    grp_load[best / ns] += loads[i];
  }
  order.clear();
  std::vector<char> seen(n, 0);
  for (int g = 0; g < G; ++g)
    for (int w = 0; w < nw[g]; ++w) {
      const std::vector<int>& b = bin[g * ns + w % ns];
      const size_t j = (size_t)(w / ns);
      if (j >= b.size() || seen[b[j]]) return false;
      seen[b[j]] = 1;
      order.push_back(b[j]);
    }
  return (int)order.size() == n;
}

}  // namespace hdf
