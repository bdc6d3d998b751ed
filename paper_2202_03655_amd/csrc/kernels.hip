// gfx950 kernels of the HDF hot path: geometry, radial Gram moments, factor
// evaluation and the two contraction passes of the matvec.
//
// Layout in HBM (N points, leading dimension ldN >= roundup(N, 64) + 64, so
// that vector loads of a row may run up to 63 points past N without leaving
// the row):
//   x_soa : d rows of ldN coordinates (input type), one row per coordinate;
//   phi   : H rows of ldN values, row h = solid harmonic h at every point;
//   q     : S rows of ldN values, row (k,l) = radial function l of degree k.
// Every per-point kernel maps consecutive lanes to consecutive points, so a
// wavefront reads/writes one contiguous 256 B (fp32) or 512 B (fp64) segment
// per row.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace hdf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// 16x16x4 MFMA.  Operands: lane r + 16 q supplies A[r][q] and B[q][r].
// Accumulator element e of lane j + 16 g holds D[row(g, e)][j]; the row map
// differs between the two instructions (measured on gfx950):
//   f32: row = 4 g + e        f64: row = g + 4 e
template <> struct Mfma<float> {
  typedef floatx4 V;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
};
template <> struct Mfma<double> {
  typedef doublex4 V;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return g + 4 * e; }
};

template <typename T> struct Vec2;
template <> struct Vec2<float> { typedef float2 type; };
template <> struct Vec2<double> { typedef double2 type; };

__device__ __forceinline__ double kernel_value_dev(int kind, double r, double l) {
  switch (kind) {
    case 0: return exp(-(r * r) / (2.0 * l * l));
    case 1: return 1.0 / (1.0 + (r * r) / (l * l));
    case 2: { double z = 1.7320508075688772 * r / l; return (1.0 + z) * exp(-z); }
    default: { double z = 2.23606797749979 * r / l; return (1.0 + z + z * z / 3.0) * exp(-z); }
  }
}

// SplitMix64 output number q (1-based) of the stream started at `seed`:
// the generator is counter based, state_q = seed + q * gamma.
__device__ __forceinline__ uint64_t splitmix_at(uint64_t seed, uint64_t q) {
  uint64_t z = seed + q * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Fixed-order tree reduction over a 256-thread block (deterministic).
template <typename Op>
__device__ __forceinline__ double block_reduce(double v, double* sh, Op op) {
  const int t = threadIdx.x;
  __syncthreads();
  sh[t] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] = op(sh[t], sh[t + w]);
    __syncthreads();
  }
  return sh[0];
}

struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpAdd { __device__ double operator()(double a, double b) const { return a + b; } };

// ------------------------------------------------------------------ prep
// Partial record per block: [0..7] min, [8..15] max, [16] nu2, [17] nonfinite.
constexpr int kPrepRec = 18;

// block_reduce of the 18 entries of a prep record at once (entries 0..7 min, 8..15 max, 16..17
// sum): the same fixed tree per entry, with one barrier per level for all of them.
__device__ __forceinline__ void block_reduce_rec(double (&v)[kPrepRec], double (*sh)[256]) {
  const int t = threadIdx.x;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPrepRec; ++q) sh[q][t] = v[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int q = 0; q < kPrepRec; ++q) {
        const double a = sh[q][t], b = sh[q][t + w];
        sh[q][t] = q < 8 ? fmin(a, b) : (q < 16 ? fmax(a, b) : a + b);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPrepRec; ++q) v[q] = sh[q][0];
}

template <typename Tin>
__global__ void __launch_bounds__(256) k_prep_minmax(const Tin* __restrict__ pts, int64_t n, int d,
                                                      int64_t ld, Tin* __restrict__ x_soa,
                                                      int64_t ldx, int kind, double l,
                                                      double* __restrict__ part) {
  __shared__ double shr[kPrepRec][256];
  double mn[8], mx[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) { mn[j] = INFINITY; mx[j] = -INFINITY; }
  double nf = 0.0;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gsz) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j < d) {
        const Tin raw = pts[i * ld + j];
        x_soa[(int64_t)j * ldx + i] = raw;
        const double v = (double)raw;
        if (!isfinite(v)) nf += 1.0;
        mn[j] = fmin(mn[j], v);
        mx[j] = fmax(mx[j], v);
      }
    }
  }
  // ||K||_F sample: pair t uses generator outputs 2t+1 and 2t+2
  double nu = 0.0;
  {
#pragma clang fp contract(off)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < kNuPairs; t += gsz) {
      const uint64_t ia = (splitmix_at(kNuSeed, 2 * (uint64_t)t + 1) >> 11) % (uint64_t)n;
      const uint64_t ib = (splitmix_at(kNuSeed, 2 * (uint64_t)t + 2) >> 11) % (uint64_t)n;
      double s = 0.0;
      for (int j = 0; j < d; ++j) {
        const double df = (double)pts[(int64_t)ia * ld + j] - (double)pts[(int64_t)ib * ld + j];
        s = s + df * df;
      }
      const double kv = kernel_value_dev(kind, sqrt(s), l);
      nu = nu + kv * kv;
    }
  }
  double* rec = part + (int64_t)blockIdx.x * kPrepRec;
  double v[kPrepRec];
#pragma unroll
  for (int j = 0; j < 8; ++j) { v[j] = mn[j]; v[8 + j] = mx[j]; }
  v[16] = nu;
  v[17] = nf;
  block_reduce_rec(v, shr);
  if (threadIdx.x < kPrepRec) {
    double r = v[0];
#pragma unroll
    for (int q = 1; q < kPrepRec; ++q) r = threadIdx.x == q ? v[q] : r;
    rec[threadIdx.x] = r;
  }
}

__global__ void __launch_bounds__(256) k_prep_fin1(const double* __restrict__ part, int nblk,
                                                    GeoDev* geo) {
  __shared__ double shr[kPrepRec][256];
  double v[kPrepRec];
#pragma unroll
  for (int q = 0; q < kPrepRec; ++q) v[q] = (q < 8) ? INFINITY : (q < 16 ? -INFINITY : 0.0);
  for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
    for (int q = 0; q < kPrepRec; ++q) {
      const double x = part[(int64_t)b * kPrepRec + q];
      v[q] = (q < 8) ? fmin(v[q], x) : (q < 16 ? fmax(v[q], x) : v[q] + x);
    }
  }
  block_reduce_rec(v, shr);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) geo->c[q] = (v[q] + v[8 + q]) * 0.5;   // centre of the bounding box
    geo->nu2_sum = v[16];
    geo->nonfinite = v[17];
  }
}

template <typename Tin>
__global__ void __launch_bounds__(256) k_prep_radius(const Tin* __restrict__ x_soa, int64_t ldx,
                                                      int64_t n, int d, const GeoDev* geo,
                                                      double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sh[256];
  double mx = 0.0;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gsz) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
      const double t = (double)x_soa[(int64_t)j * ldx + i] - geo->c[j];
      s = s + t * t;
    }
    mx = fmax(mx, s);
  }
  const double r = block_reduce(mx, sh, OpMax());
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_prep_fin2(const double* __restrict__ part, int nblk,
                                                    GeoDev* geo) {
  __shared__ double sh[256];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) v = fmax(v, part[b]);
  const double r = block_reduce(v, sh, OpMax());
  if (threadIdx.x == 0) {
    geo->R2 = r;
    geo->R = sqrt(r);
    geo->Reff = geo->R > 0.0 ? geo->R : 1.0;
  }
}

template <typename Tin>
__global__ void __launch_bounds__(256) k_prep_rho(const Tin* __restrict__ x_soa, int64_t ldx,
                                                   int64_t n, int d, const GeoDev* geo,
                                                   double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sh[256];
  double mn = INFINITY, mx = -INFINITY;
  const double Reff = geo->Reff;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gsz) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) {
      const double t = ((double)x_soa[(int64_t)j * ldx + i] - geo->c[j]) / Reff;
      s = s + t * t;
    }
    mn = fmin(mn, s);
    mx = fmax(mx, s);
  }
  const double a = block_reduce(mn, sh, OpMin());
  const double b = block_reduce(mx, sh, OpMax());
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = b; }
}

__global__ void __launch_bounds__(256) k_prep_fin3(const double* __restrict__ part, int nblk,
                                                    GeoDev* geo) {
  __shared__ double sh[256];
  double mn = INFINITY, mx = -INFINITY;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    mn = fmin(mn, part[2 * b]);
    mx = fmax(mx, part[2 * b + 1]);
  }
  const double a = block_reduce(mn, sh, OpMin());
  const double c = block_reduce(mx, sh, OpMax());
  if (threadIdx.x == 0) { geo->rho2_min = a; geo->rho2_max = c; }
}

hipError_t launch_prep(const void* pts, int dtype, int64_t n, int d, int64_t ld, void* x_soa,
                       int64_t ldx, int kernel, double l, double* partials, GeoDev* geo,
                       hipStream_t s) {
  const int nb = kPrepBlocks;
  if (dtype == 0) {
    k_prep_minmax<float><<<nb, 256, 0, s>>>((const float*)pts, n, d, ld, (float*)x_soa, ldx, kernel, l, partials);
  } else {
    k_prep_minmax<double><<<nb, 256, 0, s>>>((const double*)pts, n, d, ld, (double*)x_soa, ldx, kernel, l, partials);
  }
  k_prep_fin1<<<1, 256, 0, s>>>(partials, nb, geo);
  if (dtype == 0) k_prep_radius<float><<<nb, 256, 0, s>>>((const float*)x_soa, ldx, n, d, geo, partials);
  else k_prep_radius<double><<<nb, 256, 0, s>>>((const double*)x_soa, ldx, n, d, geo, partials);
  k_prep_fin2<<<1, 256, 0, s>>>(partials, nb, geo);
  if (dtype == 0) k_prep_rho<float><<<nb, 256, 0, s>>>((const float*)x_soa, ldx, n, d, geo, partials);
  else k_prep_rho<double><<<nb, 256, 0, s>>>((const double*)x_soa, ldx, n, d, geo, partials);
  k_prep_fin3<<<1, 256, 0, s>>>(partials, nb, geo);
  return hipGetLastError();
}

// Geometry of two point sets (general case X != Y): the existing passes run
// over both sets into adjacent halves of the partial records, so the centre,
// radius and rho^2 interval are those of X u Y.  nu is then replaced by the
// cross-pair estimate: pair t draws generator outputs 2t+1 and 2t+2, a < nx,
// b < ny (the per-set estimates of the min/max pass are discarded).
template <typename Tin>
__global__ void __launch_bounds__(256) k_nu_cross(const Tin* __restrict__ px, int64_t nx, int64_t ldx,
                                                   const Tin* __restrict__ py, int64_t ny, int64_t ldy,
                                                   int d, int kind, double l, double* __restrict__ part) {
  __shared__ double sh[256];
  double nu = 0.0;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  {
#pragma clang fp contract(off)
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < kNuPairs; t += gsz) {
      const uint64_t ia = (splitmix_at(kNuSeed, 2 * (uint64_t)t + 1) >> 11) % (uint64_t)nx;
      const uint64_t ib = (splitmix_at(kNuSeed, 2 * (uint64_t)t + 2) >> 11) % (uint64_t)ny;
      double s = 0.0;
      for (int j = 0; j < d; ++j) {
        const double df = (double)px[(int64_t)ia * ldx + j] - (double)py[(int64_t)ib * ldy + j];
        s = s + df * df;
      }
      const double kv = kernel_value_dev(kind, sqrt(s), l);
      nu = nu + kv * kv;
    }
  }
  const double r = block_reduce(nu, sh, OpAdd());
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_nu_fin(const double* __restrict__ part, int nblk, GeoDev* geo) {
  __shared__ double sh[256];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) v += part[b];
  const double r = block_reduce(v, sh, OpAdd());
  if (threadIdx.x == 0) geo->nu2_sum = r;
}

hipError_t launch_prep_cross(const void* ptsx, int64_t nx, int64_t ldx, const void* ptsy, int64_t ny,
                             int64_t ldy, int dtype, int d, void* soax, int64_t ldsx, void* soay,
                             int64_t ldsy, int kernel, double l, double* partials, GeoDev* geo,
                             hipStream_t s) {
  const int nb = kPrepBlocks;
  double* p1 = partials + (int64_t)nb * kPrepRec;
#define PREP_CROSS(T)                                                                                   \
  k_prep_minmax<T><<<nb, 256, 0, s>>>((const T*)ptsx, nx, d, ldx, (T*)soax, ldsx, kernel, l, partials); \
  k_prep_minmax<T><<<nb, 256, 0, s>>>((const T*)ptsy, ny, d, ldy, (T*)soay, ldsy, kernel, l, p1);       \
  k_prep_fin1<<<1, 256, 0, s>>>(partials, 2 * nb, geo);                                                 \
  k_prep_radius<T><<<nb, 256, 0, s>>>((const T*)soax, ldsx, nx, d, geo, partials);                      \
  k_prep_radius<T><<<nb, 256, 0, s>>>((const T*)soay, ldsy, ny, d, geo, partials + nb);                 \
  k_prep_fin2<<<1, 256, 0, s>>>(partials, 2 * nb, geo);                                                 \
  k_prep_rho<T><<<nb, 256, 0, s>>>((const T*)soax, ldsx, nx, d, geo, partials);                         \
  k_prep_rho<T><<<nb, 256, 0, s>>>((const T*)soay, ldsy, ny, d, geo, partials + 2 * nb);                \
  k_prep_fin3<<<1, 256, 0, s>>>(partials, 2 * nb, geo);                                                 \
  k_nu_cross<T><<<nb, 256, 0, s>>>((const T*)ptsx, nx, ldx, (const T*)ptsy, ny, ldy, d, kernel, l, partials); \
  k_nu_fin<<<1, 256, 0, s>>>(partials, nb, geo);
  if (dtype == 0) {
    PREP_CROSS(float)
  } else {
    PREP_CROSS(double)
  }
#undef PREP_CROSS
  return hipGetLastError();
}

// ------------------------------------------------------------------ sampled pairs
template <typename Tin>
__global__ void __launch_bounds__(256) k_pairs(const Tin* __restrict__ x_soa, int64_t ldx, int64_t n, int d,
                                                const GeoDev* __restrict__ geo, uint64_t seed, int M,
                                                double* __restrict__ out, int32_t* __restrict__ idx) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= M) return;
  const int64_t a = (int64_t)((splitmix_at(seed, 2 * (uint64_t)t + 1) >> 11) % (uint64_t)n);
  const int64_t b = (int64_t)((splitmix_at(seed, 2 * (uint64_t)t + 2) >> 11) % (uint64_t)n);
  const double Reff = geo->Reff;
  double r2 = 0.0, ra2 = 0.0, rb2 = 0.0, dot = 0.0;
  for (int j = 0; j < d; ++j) {
    const double xa = (double)x_soa[(int64_t)j * ldx + a], xb = (double)x_soa[(int64_t)j * ldx + b];
    const double df = xa - xb;
    const double ua = (xa - geo->c[j]) / Reff, ub = (xb - geo->c[j]) / Reff;
    r2 += df * df;
    ra2 += ua * ua;
    rb2 += ub * ub;
    dot += ua * ub;
  }
  out[t] = sqrt(r2);
  out[M + t] = ra2;
  out[2 * M + t] = rb2;
  out[3 * M + t] = dot;
  idx[t] = (int32_t)a;
  idx[M + t] = (int32_t)b;
}

hipError_t launch_pairs(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                        uint64_t seed, int M, double* out, int32_t* idx, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((M + 255) / 256);
  if (dtype == 0) k_pairs<float><<<nb, 256, 0, s>>>((const float*)x_soa, ldx, n, d, geo, seed, M, out, idx);
  else k_pairs<double><<<nb, 256, 0, s>>>((const double*)x_soa, ldx, n, d, geo, seed, M, out, idx);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Gram
// Moments mu[k][c] = sum_i rho_i^{2k} T_c(t_i) as a tall-skinny product
// A^T B on MFMA (A[i][k] = rho_i^{2k}, B[i][c] = T_c(t_i)).  The per-degree
// Gram blocks follow on the host from T_a T_b = (T_{a+b} + T_{|a-b|}) / 2.
constexpr int kGramRowTiles = 2;   // k <= 31
constexpr int kGramColTiles = 4;   // c <= 63
constexpr int kGramWaves = 4096;   // target wavefronts per Gram launch

// Per-point radial variables: rho^2 = ||(x - c)/R||^2 and the Chebyshev
// argument t of the radial basis.
template <typename Tin>
__device__ __forceinline__ void radial_point(const Tin* __restrict__ x_soa, int64_t ldx, int64_t i,
                                             int d, const GeoDev* __restrict__ geo, double Reff,
                                             double u0, double u1, double& rho2, double& t) {
  double s = 0.0;
  for (int j = 0; j < d; ++j) {
    const double v = ((double)x_soa[(int64_t)j * ldx + i] - geo->c[j]) / Reff;
    s += v * v;
  }
  rho2 = s;
  t = (2.0 * s - u0 - u1) / (u1 - u0);
}

// A 16-point tile feeds four MFMA K-steps: in step e, lane group g (lanes
// 16g..16g+15) supplies point tile*16 + g + 4e, lane r of the group supplies
// row / column index r of the two operands.  Any bijection between (g, e)
// and the 16 points is valid because the points are summed over.
// NRT x NCT moment tiles (rows k < 16 NRT, columns c < 16 NCT) are compile-time
// sizes, so the accumulators of unused tiles take no registers.
template <typename Tin, int MODE, int NRT, int NCT>
__global__ void __launch_bounds__(256) k_gram(const Tin* __restrict__ x_soa, int64_t ldx, int64_t n,
                                               int d, const GeoDev* __restrict__ geo, double u0,
                                               double u1, int K, double* __restrict__ part) {
  constexpr int nrt = NRT, nct = NCT;
  typedef typename std::conditional<MODE == 0, double, float>::type T;
  typedef typename Mfma<T>::V V;
  __shared__ double sh[4][4 * 64];
  // T_c(t) (c < 16 NCT) and rho^2 of a tile's 16 points, one row per point, per wavefront
  constexpr int TCS = 16 * NCT + 1;
  __shared__ double tcs[4][16 * TCS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const double Reff = geo->Reff;
  double dacc[NRT][NCT][4];
#pragma unroll
  for (int a = 0; a < NRT; ++a)
#pragma unroll
    for (int b = 0; b < NCT; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) dacc[a][b][e] = 0.0;
  const int64_t ntile = (n + 15) / 16;
  int since_flush = 0;
  V acc[NRT][NCT];
#pragma unroll
  for (int a = 0; a < NRT; ++a)
#pragma unroll
    for (int b = 0; b < NCT; ++b) acc[a][b] = V{0, 0, 0, 0};
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    double w[NRT][4], tc[NCT][4];
    // the radial point and the T_c(t) recurrence of point g + 4 e run once, in lane e of group g,
    // and go through LDS to the sixteen lanes that use them (T_c for c = b*16 + li, rho^2 for
    // the powers rho^(2k), k = a*16 + li)
    double* trow = &tcs[wave][0];
    if (li < 4) {
      const int64_t i = tile * 16 + g + 4 * li;
      double rho2 = 0.0, tp = 0.0;
      if (i < n) radial_point(x_soa, ldx, i, d, geo, Reff, u0, u1, rho2, tp);
      double* dst = trow + (g + 4 * li) * TCS;
      dst[16 * NCT] = rho2;
      double tm1 = 1.0, t0 = tp;
#pragma unroll
      for (int c = 0; c < 16 * NCT; ++c) {
        double cur;
        if (c == 0) cur = 1.0;
        else if (c == 1) cur = tp;
        else { cur = 2.0 * tp * t0 - tm1; tm1 = t0; t0 = cur; }
        dst[c] = cur;
      }
    }
    // the rows are read by the other lanes of the wavefront (wavefront-synchronous exchange; the
    // next tile's rows are written after this tile's MFMAs, which every lane reaches first)
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = tile * 16 + g + 4 * e;
      const double rho2 = trow[(g + 4 * e) * TCS + 16 * NCT];
#pragma unroll
      for (int a = 0; a < NRT; ++a) {
        const int k = a * 16 + li;
        double pw = 0.0;
        if (i < n && a < nrt && k <= K) {
          pw = 1.0;
          double base = rho2;
          for (int q = k; q > 0; q >>= 1) {
            if (q & 1) pw *= base;
            base *= base;
          }
        }
        w[a][e] = pw;
      }
    }
#pragma unroll
    for (int b = 0; b < NCT; ++b) {
      const int c = b * 16 + li;
#pragma unroll
      for (int e = 0; e < 4; ++e) tc[b][e] = (b < nct && c <= 2 * K) ? trow[(g + 4 * e) * TCS + c] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = tile * 16 + g + 4 * e;
#pragma unroll
      for (int a = 0; a < NRT; ++a) {
        if (a >= nrt) continue;
#pragma unroll
        for (int b = 0; b < NCT; ++b) {
          if (b >= nct) continue;
          const double wv = (i < n) ? w[a][e] : 0.0;
          if constexpr (MODE == 2) {
            const float ah = (float)wv, al = (float)(wv - (double)ah);
            const float bh = (float)tc[b][e], bl = (float)(tc[b][e] - (double)bh);
            acc[a][b] = Mfma<float>::run(ah, bh, acc[a][b]);
            acc[a][b] = Mfma<float>::run(ah, bl, acc[a][b]);
            acc[a][b] = Mfma<float>::run(al, bh, acc[a][b]);
          } else {
            acc[a][b] = Mfma<T>::run((T)wv, (T)tc[b][e], acc[a][b]);
          }
        }
      }
    }
    // binary32 accumulators are flushed to binary64 every 4 tiles (64 points)
    if (MODE != 0 && ++since_flush == 4) {
      since_flush = 0;
#pragma unroll
      for (int a = 0; a < NRT; ++a)
#pragma unroll
        for (int b = 0; b < NCT; ++b) {
#pragma unroll
          for (int e = 0; e < 4; ++e) dacc[a][b][e] += (double)acc[a][b][e];
          acc[a][b] = V{0, 0, 0, 0};
        }
    }
  }
#pragma unroll
  for (int a = 0; a < NRT; ++a)
#pragma unroll
    for (int b = 0; b < NCT; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) dacc[a][b][e] += (double)acc[a][b][e];
  // combine the four waves in a fixed order, one 16x16 tile at a time
  const int rows = nrt * 16, cols = nct * 16;
  double* out = part + (int64_t)blockIdx.x * rows * cols;
#pragma unroll
  for (int a = 0; a < NRT; ++a)
#pragma unroll
    for (int b = 0; b < NCT; ++b) {
      if (a >= nrt || b >= nct) continue;
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 4; ++e) sh[wave][e * 64 + lane] = dacc[a][b][e];
      __syncthreads();
      const int idx = threadIdx.x;             // 256 = 4 elements x 64 lanes
      const int ln = idx & 63, e = idx >> 6;
      const double v = sh[0][idx] + sh[1][idx] + sh[2][idx] + sh[3][idx];
      const int row = a * 16 + Mfma<T>::row(ln >> 4, e), col = b * 16 + (ln & 15);
      out[row * cols + col] = v;
    }
}

// Fixed-order sum over block partial records: out[e] = sum_b part[b][e].
// Fixed-order sum of the per-block partial records, out[e] = sum_b part[b][e].
// A block owns 64 consecutive entries; wavefront w takes the records
// b = w, w + 4, ... with eight independent running sums (loads in flight),
// and the four wavefront sums are combined in a fixed order through LDS.
__global__ void __launch_bounds__(256) k_gram_fin(const double* __restrict__ part, int nblk, int total,
                                                   double* __restrict__ out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane;
  const int ee = e < total ? e : 0;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int b = w;
  for (; b + 28 < nblk; b += 32)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += part[(int64_t)(b + 4 * u) * total + ee];
  for (; b < nblk; b += 4) acc[0] += part[(int64_t)b * total + ee];
  red[w][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  __syncthreads();
  if (w == 0 && e < total) out[e] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

int gram_blocks(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  int64_t b = (tiles + 3) / 4;
  if (b > kGramWaves / 4) b = kGramWaves / 4;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_gram(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d,
                       const GeoDev* geo, double u0, double u1, int K, int mode,
                       double* partials, double* moments, hipStream_t s) {
  const int nrt = (K + 1 + 15) / 16, nct = (2 * K + 1 + 15) / 16;
  if (nrt > kGramRowTiles || nct > kGramColTiles) return hipErrorInvalidValue;
  const int nb = gram_blocks(n);
#define GRAM_TILES(TIN, MODE, R, C)                                                               \
  k_gram<TIN, MODE, R, C><<<nb, 256, 0, s>>>((const TIN*)x_soa, ldx, n, d, geo, u0, u1, K, partials)
#define GRAM_LAUNCH(TIN, MODE)                                                                    \
  do {                                                                                            \
    if (nrt == 1 && nct == 1) GRAM_TILES(TIN, MODE, 1, 1);                                         \
    else if (nrt == 1 && nct == 2) GRAM_TILES(TIN, MODE, 1, 2);                                    \
    else if (nrt == 2 && nct == 3) GRAM_TILES(TIN, MODE, 2, 3);                                    \
    else if (nrt == 2 && nct == 4) GRAM_TILES(TIN, MODE, 2, 4);                                    \
    else return hipErrorInvalidValue;                                                             \
  } while (0)
  if (dtype == 0) {
    if (mode == 0) GRAM_LAUNCH(float, 0);
    else if (mode == 1) GRAM_LAUNCH(float, 1);
    else GRAM_LAUNCH(float, 2);
  } else {
    if (mode == 0) GRAM_LAUNCH(double, 0);
    else if (mode == 1) GRAM_LAUNCH(double, 1);
    else GRAM_LAUNCH(double, 2);
  }
#undef GRAM_LAUNCH
#undef GRAM_TILES
  const int total = nrt * 16 * nct * 16;
  k_gram_fin<<<(total + 63) / 64, 256, 0, s>>>(partials, nb, total, moments);
  return hipGetLastError();
}

// Second Gram pass (refinement of the compression, binary64 MFMA): for degree
// k = blockIdx.y, G2_k = sum_i z_i z_i^T with z_i = T1_k^T y_i and
// y_i[a] = rho_i^k T_a(t_i), a < L_k = K - k + 1.  T1_k (L_k x L_k, row-major)
// is the preconditioner from the first pass, so the columns Y_k T1_k are
// nearly orthonormal and their Gram is accurate in binary64 even when Y_k is
// badly conditioned.  z is formed on the VALU (lane r of group g holds z_r
// and z_{16+r} of four points), then accumulated as z z^T on MFMA with the
// same (g, e) -> point bijection as the first pass.  Partial record per
// block and degree: [32][32].
template <typename Tin>
__global__ void __launch_bounds__(256) k_gram2(const Tin* __restrict__ x_soa, int64_t ldx, int64_t n,
                                                int d, const GeoDev* __restrict__ geo, double u0,
                                                double u1, int K, const double* __restrict__ T1,
                                                const int32_t* __restrict__ t1_off,
                                                const int32_t* __restrict__ sel, int n_sel,
                                                double* __restrict__ part) {
  typedef Mfma<double>::V V;
  __shared__ double t1s[32 * 32];
  __shared__ double sh[4][4 * 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int k = sel[blockIdx.y];
  const int L = K - k + 1;
  const int nt = (L + 15) / 16;
  const double Reff = geo->Reff;
  for (int e = threadIdx.x; e < L * L; e += 256) t1s[e] = T1[t1_off[k] + e];
  __syncthreads();
  V acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V{0, 0, 0, 0};
  const bool j0 = li < L, j1 = 16 + li < L;
  const int64_t ntile = (n + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntile; tile += (int64_t)gridDim.x * 4) {
    double t[4], rk[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = tile * 16 + g + 4 * e;
      double rho2 = 0.0, tt = 0.0, pw = 0.0;
      if (i < n) {
        radial_point(x_soa, ldx, i, d, geo, Reff, u0, u1, rho2, tt);
        pw = 1.0;
        double base = sqrt(rho2);
        for (int q = k; q > 0; q >>= 1) {
          if (q & 1) pw *= base;
          base *= base;
        }
      }
      t[e] = tt;
      rk[e] = pw;
    }
    double z0[4] = {0, 0, 0, 0}, z1[4] = {0, 0, 0, 0};
    double tm1[4], tc[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) { tm1[e] = 0.0; tc[e] = 1.0; }
    for (int a = 0; a < L; ++a) {
      const double c0 = j0 ? t1s[a * L + li] : 0.0;
      const double c1 = j1 ? t1s[a * L + 16 + li] : 0.0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (a == 1) { tm1[e] = 1.0; tc[e] = t[e]; }
        else if (a >= 2) { const double tn = 2.0 * t[e] * tc[e] - tm1[e]; tm1[e] = tc[e]; tc[e] = tn; }
        const double ya = rk[e] * tc[e];
        z0[e] += c0 * ya;
        z1[e] += c1 * ya;
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[0][0] = Mfma<double>::run(z0[e], z0[e], acc[0][0]);
      if (nt > 1) {
        acc[0][1] = Mfma<double>::run(z0[e], z1[e], acc[0][1]);
        acc[1][0] = Mfma<double>::run(z1[e], z0[e], acc[1][0]);
        acc[1][1] = Mfma<double>::run(z1[e], z1[e], acc[1][1]);
      }
    }
  }
  double* out = part + ((int64_t)blockIdx.x * n_sel + blockIdx.y) * 1024;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if (a >= nt || b >= nt) continue;
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 4; ++e) sh[wave][e * 64 + lane] = acc[a][b][e];
      __syncthreads();
      const int idx = threadIdx.x, ln = idx & 63, e = idx >> 6;
      const double v = sh[0][idx] + sh[1][idx] + sh[2][idx] + sh[3][idx];
      const int row = a * 16 + Mfma<double>::row(ln >> 4, e), col = b * 16 + (ln & 15);
      out[row * 32 + col] = v;
    }
}

int gram2_blocks(int64_t n, int n_sel) {
  const int64_t tiles = (n + 15) / 16;
  int64_t b = (tiles + 3) / 4;
  const int64_t cap = std::max<int64_t>(1, kGramWaves / (4 * n_sel));
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_gram2(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d,
                        const GeoDev* geo, double u0, double u1, int K, const double* T1,
                        const int32_t* t1_off, const int32_t* sel, int n_sel, double* partials,
                        double* out, hipStream_t s) {
  if (K + 1 > 32 || n_sel < 1) return hipErrorInvalidValue;
  const int nb = gram2_blocks(n, n_sel);
  const dim3 grid(nb, n_sel);
  if (dtype == 0)
    k_gram2<float><<<grid, 256, 0, s>>>((const float*)x_soa, ldx, n, d, geo, u0, u1, K, T1, t1_off, sel,
                                        n_sel, partials);
  else
    k_gram2<double><<<grid, 256, 0, s>>>((const double*)x_soa, ldx, n, d, geo, u0, u1, K, T1, t1_off, sel,
                                         n_sel, partials);
  const int total = n_sel * 1024;
  k_gram_fin<<<(total + 63) / 64, 256, 0, s>>>(partials, nb, total, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ build
// Solid harmonics by nested normalised Gegenbauer chain recurrences.  The
// loops run from the innermost chain level outwards (azimuthal index first,
// degree k last), so each level keeps only its two-term recurrence state in
// registers; every iteration of the innermost loop yields one harmonic,
// stored to its canonical row col_of[t] (the table follows this loop order).
// Each thread evaluates PPT consecutive points (independent recurrence chains
// in flight) and writes them with one 16-byte nontemporal store per row.
typedef double doublex2 __attribute__((ext_vector_type(2)));
template <typename T, int PPT> struct PVec;
template <> struct PVec<float, 4> { typedef floatx4 type; };
template <> struct PVec<double, 2> { typedef doublex2 type; };

template <typename T, int PPT>
__device__ __forceinline__ void store_row(T* __restrict__ dst, const T (&v)[PPT]) {
  typedef typename PVec<T, PPT>::type V;
  V w;
#pragma unroll
  for (int e = 0; e < PPT; ++e) w[e] = v[e];
  __builtin_nontemporal_store(w, reinterpret_cast<V*>(dst));
}

template <typename T, int D, int PPT, int LEVEL>
struct Chain {
  typedef typename Vec2<T>::type T2;
  static __device__ __forceinline__ void run(const T (&xt)[PPT][D], const T (&r2)[PPT][D], int b,
                                             const T (&prefix)[PPT], int K,
                                             const T2* __restrict__ chain,
                                             const int32_t* __restrict__ col_of, int& t,
                                             T* __restrict__ phi_base, int64_t ld) {
    const T2* cf = chain + ((int64_t)(LEVEL - 1) * (K + 1) + b) * (K + 1);
    T pm1[PPT], p[PPT], pre[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) { pm1[e] = 0; p[e] = cf[0].x; }
    for (int nn = 0; nn <= K - b; ++nn) {
      if (nn == 1) {
#pragma unroll
        for (int e = 0; e < PPT; ++e) { pm1[e] = p[e]; p[e] = cf[1].x * xt[e][LEVEL - 1]; }
      } else if (nn >= 2) {
        const T A = cf[nn].x, B = cf[nn].y;
#pragma unroll
        for (int e = 0; e < PPT; ++e) {
          const T pn = A * xt[e][LEVEL - 1] * p[e] - B * r2[e][LEVEL - 1] * pm1[e];
          pm1[e] = p[e];
          p[e] = pn;
        }
      }
#pragma unroll
      for (int e = 0; e < PPT; ++e) pre[e] = prefix[e] * p[e];
      Chain<T, D, PPT, LEVEL - 1>::run(xt, r2, b + nn, pre, K, chain, col_of, t, phi_base, ld);
    }
  }
};
template <typename T, int D, int PPT>
struct Chain<T, D, PPT, 0> {
  typedef typename Vec2<T>::type T2;
  static __device__ __forceinline__ void run(const T (&)[PPT][D], const T (&)[PPT][D], int,
                                             const T (&prefix)[PPT], int, const T2* __restrict__,
                                             const int32_t* __restrict__ col_of, int& t,
                                             T* __restrict__ phi_base, int64_t ld) {
    const int col = col_of[t++];
    if (col >= 0) store_row<T, PPT>(phi_base + (int64_t)col * ld, prefix);
  }
};

template <typename Tin, typename T, int D, int PPT>
__global__ void __launch_bounds__(256) k_build(const Tin* __restrict__ x_soa, int64_t ldx, int64_t n,
                                                const GeoDev* __restrict__ geo, double u0, double u1,
                                                const int32_t* __restrict__ col_of,
                                                const typename Vec2<T>::type* __restrict__ chain,
                                                const int32_t* __restrict__ q_len,
                                                const int32_t* __restrict__ q_off,
                                                const T* __restrict__ q_coef, int K, int S,
                                                T* __restrict__ phi, int64_t ld_phi,
                                                T* __restrict__ q, int64_t ld_q) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * PPT;
  if (i0 >= n) return;      // whole thread past the end (ld is padded to 64)
  T xt[PPT][D], r2[PPT][D], tt[PPT];
  {
#pragma clang fp contract(off)
    const double Reff = geo->Reff;
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int64_t i = (i0 + e < n) ? i0 + e : n - 1;
      double rho2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double v = ((double)x_soa[(int64_t)j * ldx + i] - geo->c[j]) / Reff;
        xt[e][j] = (T)v;
        rho2 = rho2 + v * v;
      }
      tt[e] = (T)((2.0 * rho2 - u0 - u1) / (u1 - u0));
    }
  }
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    T acc = 0;
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
      acc += xt[e][j] * xt[e][j];
      r2[e][j] = acc;
    }
  }
  // harmonics: azimuthal part (x_{D-1} + i x_D)^m outermost
  int t = 0;
  T cr[PPT], ci[PPT], pre[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) { cr[e] = 1; ci[e] = 0; }
  const T inv_sqrt_2pi = (T)0.39894228040143267794, inv_sqrt_pi = (T)0.56418958354775628695;
  T* phi_base = phi + i0;
  for (int mm = 0; mm <= K; ++mm) {
    if (mm > 0) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const T ax = xt[e][D - 2], ay = xt[e][D - 1];
        const T ncr = ax * cr[e] - ay * ci[e];
        ci[e] = ay * cr[e] + ax * ci[e];
        cr[e] = ncr;
      }
    }
    const T cm = (mm == 0) ? inv_sqrt_2pi : inv_sqrt_pi;
#pragma unroll
    for (int e = 0; e < PPT; ++e) pre[e] = cm * cr[e];
    Chain<T, D, PPT, D - 2>::run(xt, r2, mm, pre, K, chain, col_of, t, phi_base, ld_phi);
    if (mm > 0) {
#pragma unroll
      for (int e = 0; e < PPT; ++e) pre[e] = cm * ci[e];
      Chain<T, D, PPT, D - 2>::run(xt, r2, mm, pre, K, chain, col_of, t, phi_base, ld_phi);
    }
  }
  // radial functions: Clenshaw in the basis T_a(t)
  for (int row = 0; row < S; ++row) {
    const int L = q_len[row];
    const T* cf = q_coef + q_off[row];
    T b1[PPT], b2[PPT], val[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) { b1[e] = 0; b2[e] = 0; }
    for (int a = L - 1; a >= 1; --a) {
      const T c = cf[a];
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const T b0 = 2 * tt[e] * b1[e] - b2[e] + c;
        b2[e] = b1[e];
        b1[e] = b0;
      }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) val[e] = tt[e] * b1[e] - b2[e] + cf[0];
    store_row<T, PPT>(q + (int64_t)row * ld_q + i0, val);
  }
}

template <typename Tin, typename T>
static hipError_t launch_build_t(const void* x_soa, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                                 double u0, double u1, const BuildTables& tb, void* phi,
                                 int64_t ld_phi, void* q, int64_t ld_q, hipStream_t s) {
  constexpr int PPT = 16 / sizeof(T);
  const dim3 grid((unsigned)((n + 256 * PPT - 1) / (256 * PPT)));
  typedef typename Vec2<T>::type T2;
#define BUILD_CASE(DD)                                                                        \
  case DD:                                                                                    \
    k_build<Tin, T, DD, PPT><<<grid, 256, 0, s>>>((const Tin*)x_soa, ldx, n, geo, u0, u1,    \
                                                  tb.col_of, (const T2*)tb.chain, tb.q_len,   \
                                                  tb.q_off, (const T*)tb.q_coef, tb.K, tb.S,  \
                                                  (T*)phi, ld_phi, (T*)q, ld_q);              \
    break;
  switch (d) {
    BUILD_CASE(3)
    BUILD_CASE(4)
    BUILD_CASE(5)
    BUILD_CASE(6)
    BUILD_CASE(7)
    BUILD_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef BUILD_CASE
  return hipGetLastError();
}

hipError_t launch_build(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d,
                        const GeoDev* geo, double u0, double u1, const BuildTables& tb,
                        int prec, void* phi, int64_t ld_phi, void* q, int64_t ld_q,
                        hipStream_t s) {
  if (prec == 1 && dtype == 0)
    return launch_build_t<float, float>(x_soa, ldx, n, d, geo, u0, u1, tb, phi, ld_phi, q, ld_q, s);
  if (prec == 0 && dtype == 1)
    return launch_build_t<double, double>(x_soa, ldx, n, d, geo, u0, u1, tb, phi, ld_phi, q, ld_q, s);
  if (prec == 0 && dtype == 0)        // binary64 factor of binary32 points (tolerances below binary32)
    return launch_build_t<float, double>(x_soa, ldx, n, d, geo, u0, u1, tb, phi, ld_phi, q, ld_q, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ adjoint
// dF/dx_i for F = sum_c w_c^T U C U^T v_c, C = diag(lambda) (structure frozen), with
// U[i,(k,h,l)] = S_h(xt_i) q_{k,l}(rho_i^2), xt = (x - c)/R:
//   dF/dx_i = (1/R) sum_{k,h} [ a_h(i) grad S_h(xt_i) + 2 xt_i b_h(i) S_h(xt_i) ],
//   a_h = sum_l q_{k,l} alpha_{h,l},  b_h = sum_l q'_{k,l} alpha_{h,l},
//   alpha_{h,l}(i) = sum_c w_ic Gv[(k,h,l)][c] + v_ic Gw[(k,h,l)][c],  Gv = C U^T V, Gw = C U^T W.
// Both terms are factor contractions: the second is the product of U' (q replaced by q' =
// dq/d(rho^2)) with [Gv | Gw]; the first, since every partial derivative of a degree-k solid
// harmonic is a combination of the degree k-1 ones (dS_{k,h}/dx_j = sum_h' G_k^(j)[h][h'] S_{k-1,h'}),
// is the product of the shifted factor S_{k-1,h'} q_{k,l} with [G^(j)T Gv | G^(j)T Gw] for every j.
// The contractions run through the pass-2 kernel; k_radial evaluates q', k_adj_combine adds up.

// out[row][i] = scale * sum_{a < len} coef[a] T_a(t_i) for the S rows of a coefficient table (the
// radial-function tables with derivative coefficients give q' = dq/d(rho^2)); PPT points per thread.
template <typename Tin, typename T, int PPT>
__global__ void __launch_bounds__(256) k_radial(const Tin* __restrict__ x_soa, int64_t ldx, int64_t n, int d,
                                                 const GeoDev* __restrict__ geo, double u0, double u1,
                                                 const int32_t* __restrict__ q_len, const int32_t* __restrict__ q_off,
                                                 const T* __restrict__ coef, int S, T scale, T* __restrict__ out,
                                                 int64_t ld_out) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * PPT;
  if (i0 >= n) return;      // whole thread past the end (rows are padded past n)
  T tt[PPT];
  {
#pragma clang fp contract(off)
    const double Reff = geo->Reff;
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int64_t i = (i0 + e < n) ? i0 + e : n - 1;
      double rho2 = 0.0;
      for (int j = 0; j < d; ++j) {
        const double v = ((double)x_soa[(int64_t)j * ldx + i] - geo->c[j]) / Reff;
        rho2 = rho2 + v * v;
      }
      tt[e] = (T)((2.0 * rho2 - u0 - u1) / (u1 - u0));
    }
  }
  for (int row = 0; row < S; ++row) {
    const int L = q_len[row];
    const T* cf = coef + q_off[row];
    T b1[PPT], b2[PPT], val[PPT];
#pragma unroll
    for (int e = 0; e < PPT; ++e) { b1[e] = 0; b2[e] = 0; }
    for (int a = L - 1; a >= 1; --a) {
      const T c = cf[a];
#pragma unroll
      for (int e = 0; e < PPT; ++e) {
        const T b0 = 2 * tt[e] * b1[e] - b2[e] + c;
        b2[e] = b1[e];
        b1[e] = b0;
      }
    }
#pragma unroll
    for (int e = 0; e < PPT; ++e) val[e] = scale * (tt[e] * b1[e] - b2[e] + cf[0]);
    store_row<T, PPT>(out + (int64_t)row * ld_out + i0, val);
  }
}

hipError_t launch_radial(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                         double u0, double u1, const int32_t* q_len, const int32_t* q_off, const void* coef,
                         int S, double scale, int prec, void* out, int64_t ld_out, hipStream_t s) {
  if (S <= 0 || n <= 0) return hipSuccess;
#define HDF_RAD(TIN, T)                                                                                      \
  do {                                                                                                       \
    constexpr int PPT = 16 / sizeof(T);                                                                      \
    const unsigned nb = (unsigned)((n + 256 * PPT - 1) / (256 * PPT));                                      \
    k_radial<TIN, T, PPT><<<nb, 256, 0, s>>>((const TIN*)x_soa, ldx, n, d, geo, u0, u1, q_len, q_off,       \
                                             (const T*)coef, S, (T)scale, (T*)out, ld_out);                  \
  } while (0)
  if (prec == 1 && dtype == 0) HDF_RAD(float, float);
  else if (prec == 0 && dtype == 1) HDF_RAD(double, double);
  else if (prec == 0 && dtype == 0) HDF_RAD(float, double);
  else return hipErrorInvalidValue;
#undef HDF_RAD
  return hipGetLastError();
}

// dX[i][j] = (1/R) [ sum_c w_ic KS[i][j 2m + c] + v_ic KS[i][j 2m + m + c]
//                    + 2 xt_ij (sum_c w_ic K2[i][c] + v_ic K2[i][m + c]) ]
// KS: n x ldks (the shifted-factor products, 2m columns per direction), K2: n x ldk2.
template <typename Tin, typename T, typename TIO>
__global__ void __launch_bounds__(256) k_adj_combine(const Tin* __restrict__ x_soa, int64_t ldx, int64_t n, int d,
                                                      const GeoDev* __restrict__ geo, const T* __restrict__ KS,
                                                      int64_t ldks, const T* __restrict__ K2, int64_t ldk2,
                                                      const TIO* __restrict__ Wm, const TIO* __restrict__ Vm,
                                                      int64_t ld, int m, TIO* __restrict__ dX, int64_t lddx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double Reff = geo->Reff;
  double s2 = 0.0;
  for (int c = 0; c < m; ++c)
    s2 += (double)Wm[i * ld + c] * (double)K2[i * ldk2 + c] + (double)Vm[i * ld + c] * (double)K2[i * ldk2 + m + c];
  for (int j = 0; j < d; ++j) {
    double sj = 0.0;
    const T* ks = KS + i * ldks + (int64_t)j * 2 * m;
    for (int c = 0; c < m; ++c) sj += (double)Wm[i * ld + c] * (double)ks[c] + (double)Vm[i * ld + c] * (double)ks[m + c];
    const double xt = ((double)x_soa[(int64_t)j * ldx + i] - geo->c[j]) / Reff;
    dX[i * lddx + j] = (TIO)((sj + 2.0 * xt * s2) / Reff);
  }
}

hipError_t launch_adj_combine(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                              const void* KS, int64_t ldks, const void* K2, int64_t ldk2, const void* Wm,
                              const void* Vm, int64_t ld, int m, void* dX, int64_t lddx, int prec, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = (unsigned)((n + 255) / 256);
#define HDF_COMB(TIN, T)                                                                                     \
  k_adj_combine<TIN, T, TIN><<<nb, 256, 0, s>>>((const TIN*)x_soa, ldx, n, d, geo, (const T*)KS, ldks,      \
                                                (const T*)K2, ldk2, (const TIN*)Wm, (const TIN*)Vm, ld, m,   \
                                                (TIN*)dX, lddx)
  if (prec == 1 && dtype == 0) HDF_COMB(float, float);
  else if (prec == 0 && dtype == 1) HDF_COMB(double, double);
  else if (prec == 0 && dtype == 0) HDF_COMB(float, double);
  else return hipErrorInvalidValue;
#undef HDF_COMB
  return hipGetLastError();
}

// ------------------------------------------------------------------ matvec
// Vector load of 8 consecutive values of a harmonic / radial row starting at
// p (a multiple of 8, p < N + 56).  Rows are padded by 64 points past N, so
// the 16-byte loads never leave the row; values at or past `end` (or of an
// invalid row) are replaced by zero with selects, never by branches, so all
// loads of an iteration issue back to back.
template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ row, int64_t p, int64_t end, bool ok, T (&a)[8]) {
  T v[8];
  if constexpr (sizeof(T) == 4) {
    const floatx4 v0 = *reinterpret_cast<const floatx4*>(row + p);
    const floatx4 v1 = *reinterpret_cast<const floatx4*>(row + p + 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) { v[e] = v0[e]; v[4 + e] = v1[e]; }
  } else {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const doublex2 w = *reinterpret_cast<const doublex2*>(row + p + 2 * h);
      v[2 * h] = w[0];
      v[2 * h + 1] = w[1];
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) a[e] = (ok && p + e < end) ? v[e] : (T)0;
}

// Pass 1, W = U^T V.  Per degree k this is the product Phi_k (Q_k o V)
// (Khatri-Rao: column (k,h,l) of U is phi_h * q_{k,l}).  One wavefront owns
// a block of 32 harmonics of one degree (two 16-row MFMA tiles, so every B
// operand q_{k,l}(i) V[i][c] is reused twice) and a contiguous range of
// points; output columns j = l * m16 + c are produced NCT 16-wide tiles at a
// time.  The reduction index (points) is assigned so that lane group g reads
// 8 consecutive points of each harmonic row (two 16-byte loads per row).
constexpr int kMvtRowTiles = 2;

template <typename T, int NCT, typename TV>
__global__ void __launch_bounds__(64) k_mv_t(const T* __restrict__ phi, int64_t ld_phi,
                                              const T* __restrict__ q, int64_t ld_q,
                                              const DegDev* __restrict__ degs,
                                              const TileDev* __restrict__ tiles,
                                              const TV* __restrict__ V, int64_t ldv, int64_t n,
                                              int m, int m16, int64_t split_len, int64_t rank,
                                              double* __restrict__ part) {
  typedef typename Mfma<T>::V Acc;
  const TileDev tile = tiles[blockIdx.x];
  const DegDev dg = degs[tile.deg];
  const int split = blockIdx.y;
  const int cpl = m16 / 16;                      // column tiles per radial function
  const int nct_all = dg.s * cpl;
  const int ct0 = tile.ct0;
  const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
  const T* prow[kMvtRowTiles];
  bool rowv[kMvtRowTiles];
#pragma unroll
  for (int rt = 0; rt < kMvtRowTiles; ++rt) {
    const int row = tile.h0 + rt * 16 + li;
    rowv[rt] = row < dg.nh;
    prow[rt] = phi + (int64_t)(dg.hoff + (rowv[rt] ? row : 0)) * ld_phi;
  }
  const T* qrow[NCT];
  int cc[NCT];
  bool cv[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int tix = ct0 + ct;
    const int l = tix / cpl;
    cc[ct] = (tix % cpl) * 16 + li;
    cv[ct] = (tix < nct_all) && (cc[ct] < m);
    qrow[ct] = q + (int64_t)(dg.qoff + (tix < nct_all ? l : 0)) * ld_q;
  }
  Acc acc[kMvtRowTiles][NCT];
#pragma unroll
  for (int rt = 0; rt < kMvtRowTiles; ++rt)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[rt][ct] = Acc{0, 0, 0, 0};
  const int64_t p_begin = (int64_t)split * split_len;
  const int64_t p_end = (p_begin + split_len < n) ? p_begin + split_len : n;
  // software pipeline: the Phi tiles of the next 32 points are loaded while
  // the MFMAs of the current ones run
  T a_nxt[kMvtRowTiles][8];
#pragma unroll
  for (int rt = 0; rt < kMvtRowTiles; ++rt) load8(prow[rt], p_begin + 8 * g, p_end, rowv[rt], a_nxt[rt]);
  for (int64_t p = p_begin; p < p_end; p += 32) {
    const int64_t pb = p + 8 * g;
    T a[kMvtRowTiles][8];
#pragma unroll
    for (int rt = 0; rt < kMvtRowTiles; ++rt)
#pragma unroll
      for (int e = 0; e < 8; ++e) a[rt][e] = a_nxt[rt][e];
    if (p + 32 < p_end) {
#pragma unroll
      for (int rt = 0; rt < kMvtRowTiles; ++rt) load8(prow[rt], pb + 32, p_end, rowv[rt], a_nxt[rt]);
    }
    // B operands: unconditional in-bounds loads (clamped point / column),
    // invalid entries zeroed by selects
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t pt = pb + t;
      const bool pv = pt < p_end;
      const int64_t ptc = pv ? pt : p_begin;
      const TV* vrow = V + ptc * ldv;
      T b[NCT];
      // the clamped indices address valid (finite) data, so validity is
      // applied as a 0/1 factor; a select would be turned back into a branch
      const T pmask = pv ? (T)1 : (T)0;
      if (cpl == 1) {
        const T vv = (T)vrow[li < m ? li : 0] * (li < m ? pmask : (T)0);
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) b[ct] = qrow[ct][ptc] * vv;
      } else {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          b[ct] = qrow[ct][ptc] * (T)vrow[cc[ct] < m ? cc[ct] : 0] * (cv[ct] ? pmask : (T)0);
      }
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        if (ct0 + ct >= nct_all) break;          // uniform: live column tiles only
#pragma unroll
        for (int rt = 0; rt < kMvtRowTiles; ++rt) acc[rt][ct] = Mfma<T>::run(a[rt][t], b[ct], acc[rt][ct]);
      }
    }
  }
  double* out = part + (int64_t)split * rank * m16;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int tix = ct0 + ct;
    if (tix >= nct_all) continue;
    const int l = tix / cpl;
    const int c = (tix % cpl) * 16 + li;
#pragma unroll
    for (int rt = 0; rt < kMvtRowTiles; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int h = tile.h0 + rt * 16 + Mfma<T>::row(g, e);
        if (h < dg.nh) out[(int64_t)(dg.roff + h * dg.s + l) * m16 + c] = (double)acc[rt][ct][e];
      }
  }
}

// Pass 1, tile-major.  Per degree k, W_k = Phi_k (Q_k o V): every wave item
// owns one 16-row tile of Phi_k and up to eight accumulator tiles (radial
// function l, column tile ct), so one pair of 16-byte loads of the tile's
// values per lane and 32-point chunk feeds 8 * nl * nct MFMAs.  MFMA K-step t
// of a chunk takes the four points p + 8 g + t (lane group g) with
//   A[r][g] = phi_{row0 + r}(p + 8 g + t) q_l(p + 8 g + t),
//   B[g][c] = V[p + 8 g + t][16 ct + c],
// A formed from the tile's values and the staged radial rows, B from V^T in LDS.  A rank-row item
// (MvtRankRow) takes row r's harmonic and radial row from its own table entry.  The tile's values are
// prefetched PF chunks ahead into registers; the staged operands (V^T and the
// radial rows) are staged for two chunks at a time into double-buffered LDS,
// with one barrier per such unit.  Every load is unconditional and in
// bounds: chunk and unit starts are clamped to the split's last chunk and
// unit, Phi and Q rows are padded by at least 63 points past n (zeros), V rows
// are clamped to n - 1 and the values of points past the split multiplied by
// zero.
// Prefetch depth (chunks of the tile in flight) and occupancy per type and column tiles, chosen so
// that the registers fit without spills: binary32 with one column tile 4 chunks deep at four
// wavefronts per SIMD (<= 128 registers), otherwise 2 deep (binary32: four wavefronts, three with
// four column tiles; binary64: two with one column tile, three with more).
// Without the occupancy hint the scheduler hoists the operands of all radial functions and
// overflows the registers.
template <typename T, int NCT> struct MvtPF { static constexpr int value = sizeof(T) == 4 && NCT == 1 ? 4 : 2; };
template <typename T, int NCT> struct MvtWaves {
  static constexpr int value = sizeof(T) == 4 ? (NCT < 4 ? 4 : 3) : (NCT == 1 ? 2 : 3);
};
// radial functions per wave item (accumulator tiles per wavefront: NL * NCT); binary32 with two
// column tiles keeps three, the registers of four spill
template <typename T, int NCT> struct MvtNL {
  static constexpr int value = sizeof(T) == 4 ? (NCT == 2 ? 3 : 8 / NCT) : 4 / NCT;
};
constexpr int kMvtCH = 32;                 // points per chunk (MFMA K-steps of one tile load)
constexpr int kMvtSP = 2;                  // chunks per staged unit (one barrier per unit)
constexpr int kMvtSpan = kMvtSP * kMvtCH;  // points per staged unit
constexpr int kMvtThreads = 64 * kMvtWavesPerGroup;
constexpr int kMvtVS = kMvtSpan + 4;       // padded staged row (LDS bank spread)


template <typename T, typename TV, int NCT>
__global__ void __launch_bounds__(kMvtThreads) __attribute__((amdgpu_waves_per_eu(MvtWaves<T, NCT>::value, 8)))
k_mv_t_tile(const T* __restrict__ phi, int64_t ld_phi,
                                                    const T* __restrict__ q, int64_t ld_q,
                                                    const MvtWave* __restrict__ waves,
                                                    const MvtRankRow* __restrict__ rrows,
                                                    const MvtGroup* __restrict__ groups, int n_groups,
                                                    int n_splits, int64_t split_len,
                                                    const TV* __restrict__ V, int64_t ldv, int64_t n, int m,
                                                    int m16, int64_t rank, double* __restrict__ part) {
  typedef typename Mfma<T>::V Acc;
  constexpr int PF = MvtPF<T, NCT>::value;
  static_assert(PF % 2 == 0, "the LDS buffer of a chunk is its slot's parity");
  constexpr int NL = MvtNL<T, NCT>::value;
  constexpr int CH = kMvtCH, VS = kMvtVS, SP = kMvtSP, SPAN = kMvtSpan;
  static_assert(PF % SP == 0, "whole staged units in flight");
  constexpr int PS = PF / SP;                       // staged units in flight
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  // block b runs group gi over split sp with b = 8 (G (sp / 8) + gi) + sp % 8: the workgroups of
  // all groups over one range of points land on one XCD (dispatch is round robin over the eight),
  // close together in time, so V and the radial rows of the range are fetched into its L2 once
  const int b = blockIdx.x;
  const int rest = b >> 3;
  const int gi = rest % n_groups;
  const int split = ((rest / n_groups) << 3) + (b & 7);
  if (split >= n_splits) return;                    // whole workgroup, before any barrier
  const MvtGroup gd = groups[gi];
  const int tid = threadIdx.x, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const bool active = wave < gd.nw;                 // uniform
  const MvtWave wi = waves[gd.w0 + (active ? wave : 0)];
  const int64_t p_begin = (int64_t)split * split_len;
  const int64_t p_end = (p_begin + split_len < n) ? p_begin + split_len : n;
  const int64_t p_last = p_begin + (p_end - 1 - p_begin) / CH * CH;   // start of the split's last chunk
  const int64_t u_last = p_begin + (p_end - 1 - p_begin) / SPAN * SPAN;   // ... and of its last unit
  const int half = (m16 + kMvtMaxNq + 1) * VS;      // one buffer: V^T (m16 rows), radial rows, a pad row
  // this lane's Phi row and first staged radial row (rows past the tile repeat its first row; their
  // outputs are not written); a rank-row item gives each lane its own pair
  const bool rank_item = wi.qrow < 0;               // uniform
  int hrow = wi.row0 + (li < wi.nr ? li : 0), qlane = wi.qrow - gd.q_lo;
  if (rank_item) {
    const MvtRankRow rr = rrows[wi.row0 + (li < wi.nr ? li : 0)];
    hrow = rr.hrow;
    qlane = rr.qrow - gd.q_lo;
  }
  const T* prow = phi + (int64_t)hrow * ld_phi + 8 * g;

  auto load_tile = [&](int64_t p, T (&a)[8]) {
    const int64_t pc = p < p_last ? p : p_last;
    const T* r = prow + pc;
    if constexpr (sizeof(T) == 4) {
      const floatx4 v0 = *reinterpret_cast<const floatx4*>(r);
      const floatx4 v1 = *reinterpret_cast<const floatx4*>(r + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) { a[e] = v0[e]; a[4 + e] = v1[e]; }
    } else {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const doublex2 w = *reinterpret_cast<const doublex2*>(r + 2 * h);
        a[2 * h] = w[0];
        a[2 * h + 1] = w[1];
      }
    }
  };
  // staging of a unit (SPAN = 64 points, two chunks) by all threads (TPB of them): V entries
  // e = tid + TPB j < 64 m16 (point e / m16, column e % m16) and the group's radial entries, SQ
  // consecutive points of one row per thread (row SQ tid / 64; rows past nq repeat the last one and
  // are never read).  The loads are unconditional and in bounds and keep the raw values; the masks
  // (points past the split, columns past m) and the choice of slot are applied when the values are
  // written to LDS, so the compiler's load-counter waits stay exact (a select right after a load,
  // or a branch around it, makes it wait for every load in flight).
  constexpr int TPB = kMvtThreads;
  constexpr int SV = (SPAN * 16 * NCT + TPB - 1) / TPB, SQ = SPAN * kMvtMaxNq / TPB;
  static_assert(SQ == 2 || SQ == 4, "radial staging: two or four consecutive points per thread");
  typedef T T2 __attribute__((ext_vector_type(2)));
  const int sv_n = SPAN * m16;                       // staged V entries per unit
  // e / m16 for the staged entries e < 4096 as (e * inv16) >> 20: exact for m16 <= 64 (the error
  // of the rounded-up reciprocal stays below 2^-8 < 1 / m16)
  const uint32_t inv16 = ((1u << 20) + (uint32_t)m16 - 1) / (uint32_t)m16;
  static_assert(TPB * SV <= 4096, "staged entry index range of the reciprocal division");
  // staged values are loaded with the same look-ahead as the tile (PF chunks = PS units, rotating
  // register slots): the load counter completes in issue order, so values loaded after the tile
  // prefetch could only be waited for together with it
  TV sv[PS][SV];
  T sq[PS][SQ];
  auto stage_load = [&](int64_t p0, TV (&sv)[SV], T (&sq)[SQ]) {
    const int64_t p = p0 < u_last ? p0 : u_last;
#pragma unroll
    for (int j = 0; j < SV; ++j) {
      const int e = tid + TPB * j;
      const int pp = (int)(((uint32_t)e * inv16) >> 20), c = e - pp * m16;
      const int64_t pt = p + pp;
      const int64_t ptc = pt < n ? pt : n - 1;
      sv[j] = V[ptc * ldv + (c < m ? c : 0)];
    }
    const int e = SQ * tid;
    const int r = e / SPAN, pq = e % SPAN;
    const int rc = r < gd.nq ? r : gd.nq - 1;
    const T* src = q + (int64_t)(gd.q_lo + rc) * ld_q + p + pq;
#pragma unroll
    for (int h = 0; h < SQ / 2; ++h) {
      const T2 w = *reinterpret_cast<const T2*>(src + 2 * h);
      sq[2 * h] = w[0];
      sq[2 * h + 1] = w[1];
    }
  };
  // values of the unit starting at p into buf; entries past the staged area go to the pad row
  auto stage_store = [&](T* buf, int64_t p, const TV (&sv)[SV], const T (&sq)[SQ]) {
#pragma unroll
    for (int j = 0; j < SV; ++j) {
      const int e = tid + TPB * j;
      const int pp = (int)(((uint32_t)e * inv16) >> 20), c = e - pp * m16;
      const bool ok = p + pp < p_end && c < m;
      const int at = e < sv_n ? c * VS + pp : (m16 + kMvtMaxNq) * VS + (tid & 63);
      buf[at] = ok ? (T)sv[j] : (T)0;
    }
    const int e = SQ * tid;
    T* dst = buf + m16 * VS + (e / SPAN) * VS + e % SPAN;
#pragma unroll
    for (int h = 0; h < SQ / 2; ++h) {
      T2 w;
      w[0] = sq[2 * h];
      w[1] = sq[2 * h + 1];
      *reinterpret_cast<T2*>(dst + 2 * h) = w;
    }
  };
  auto lds8 = [&](const T* p, T (&v)[8]) {
    if constexpr (sizeof(T) == 4) {
      const floatx4 a = *reinterpret_cast<const floatx4*>(p), b = *reinterpret_cast<const floatx4*>(p + 4);
#pragma unroll
      for (int t = 0; t < 4; ++t) { v[t] = a[t]; v[4 + t] = b[t]; }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 a = *reinterpret_cast<const double2*>(p + 2 * t);
        v[2 * t] = a[0];
        v[2 * t + 1] = a[1];
      }
    }
  };

  Acc acc[NL][NCT];
#pragma unroll
  for (int j = 0; j < NL; ++j)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[j][ct] = Acc{0, 0, 0, 0};
  // tile slot j holds chunk c = j (mod PF); staged slot u holds unit U = u (mod PS).  The chunk loop
  // runs in whole groups of PF chunks; chunks past the split load clamped, in-bounds data and meet
  // zero V values, so they add nothing.
  T a[PF][8];
#pragma unroll
  for (int j = 0; j < PF; ++j) load_tile(p_begin + j * CH, a[j]);
#pragma unroll
  for (int u = 0; u < PS; ++u) stage_load(p_begin + u * SPAN, sv[u], sq[u]);
  stage_store(lds, p_begin, sv[0], sq[0]);
  stage_load(p_begin + PS * SPAN, sv[0], sq[0]);    // slot 0 next holds unit PS
  __syncthreads();
  const int64_t n_chunks = (p_end - p_begin + CH - 1) / CH;
  const int64_t n_rounds = (n_chunks + PF - 1) / PF;
  for (int64_t it = 0; it < n_rounds; ++it) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int64_t pc = p_begin + (it * PF + j) * CH;
      const int buf = (int)((it * PS + j / SP) & 1);  // the unit's LDS buffer: its parity
      const T* cur = lds + buf * half + (j % SP) * CH;
      if (active) {                                 // uniform
        // radial function outermost: the A operands (tile values times the radial row) are formed
        // once and serve every column tile
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          if (l < wi.nl) {                          // uniform
            T av[8];
            lds8(cur + m16 * VS + (qlane + l) * VS + 8 * g, av);
#pragma unroll
            for (int t = 0; t < 8; ++t) av[t] *= a[j][t];
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
              if (ct < wi.nct) {                    // uniform
                T v[8];
                lds8(cur + (16 * (wi.ct0 + ct) + li) * VS + 8 * g, v);
#pragma unroll
                for (int t = 0; t < 8; ++t) acc[l][ct] = Mfma<T>::run(av[t], v[t], acc[l][ct]);
              }
              // column tiles one after the other: hoisting the operands of all of them overflows
              // the registers of the binary64 shapes and of binary32 with two column tiles
              if constexpr (sizeof(T) == 8 || NCT == 2) __builtin_amdgcn_sched_barrier(0);
            }
          }
        }
      }
      load_tile(pc + PF * CH, a[j]);
      if (j % SP == SP - 1) {
        // end of unit U: unit U + 1 (slot (U + 1) mod PS) goes to the other buffer, and the slot
        // is refilled with unit U + 1 + PS
        const int slot = (j / SP + 1) % PS;
        stage_store(lds + (buf ^ 1) * half, pc + CH, sv[slot], sq[slot]);
        stage_load(pc + CH + PS * SPAN, sv[slot], sq[slot]);
        __syncthreads();
      }
    }
  }
  if (!active) return;
  double* out = part + (int64_t)split * rank * m16;
  if (rank_item) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      if (ct < wi.nct) {
        const int c = 16 * (wi.ct0 + ct) + li;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = Mfma<T>::row(g, e);
          if (r < wi.nr) out[(int64_t)rrows[wi.row0 + r].out * m16 + c] = (double)acc[0][ct][e];
        }
      }
    }
    return;
  }
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    if (l < wi.nl) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        if (ct < wi.nct) {
          const int c = 16 * (wi.ct0 + ct) + li;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int h = Mfma<T>::row(g, e);
            if (h < wi.nr) out[(int64_t)(wi.out0 + h * wi.s + l) * m16 + c] = (double)acc[l][ct][e];
          }
        }
      }
    }
  }
}

int matvec_tile_nl(int prec, int nct) {
  if (prec == 1) return nct == 1 ? MvtNL<float, 1>::value : (nct == 2 ? MvtNL<float, 2>::value : MvtNL<float, 4>::value);
  return nct == 1 ? MvtNL<double, 1>::value : (nct == 2 ? MvtNL<double, 2>::value : MvtNL<double, 4>::value);
}

size_t matvec_tile_lds_bytes(int m16, int prec) {
  return 2 * (size_t)(m16 + kMvtMaxNq + 1) * kMvtVS * (prec == 1 ? 4 : 8);
}

hipError_t launch_matvec_t_tile(const void* phi, int64_t ld_phi, const void* q, int64_t ld_q,
                                const MvtWave* waves, const MvtRankRow* rank_rows, const MvtGroup* groups,
                                int n_groups, int n_splits,
                                int64_t split_len, const void* V, int64_t ldv, int64_t n, int m, int m16,
                                int64_t rank, double* partials, int prec, int io, hipStream_t s) {
  if (m16 < 16 || m16 > 64 || m16 % 16 || n_groups < 1 || n_splits < 1 || split_len % kMvtCH)
    return hipErrorInvalidValue;
  if ((int64_t)(n_splits - 1) * split_len >= n || (int64_t)n_splits * split_len < n) return hipErrorInvalidValue;
  const int cpl = m16 / 16;
  const size_t lds = matvec_tile_lds_bytes(m16, prec);
  const unsigned n_blocks = (unsigned)(((n_splits + 7) / 8) * 8 * n_groups);
#define HDF_MVTT(T, TV, NC)                                                                                   \
  k_mv_t_tile<T, TV, NC><<<n_blocks, kMvtThreads, lds, s>>>((const T*)phi, ld_phi, (const T*)q, ld_q, waves,          \
                                                    rank_rows, groups,                                        \
                                                    n_groups, n_splits, split_len, (const TV*)V, ldv, n, m,   \
                                                    m16, rank, partials)
#define HDF_MVTT_NCT(T, TV)                                                                                   \
  do {                                                                                                        \
    if (cpl == 1) HDF_MVTT(T, TV, 1);                                                                         \
    else if (cpl == 2) HDF_MVTT(T, TV, 2);                                                                    \
    else HDF_MVTT(T, TV, 4);                                                                                  \
  } while (0)
  if (prec == 1 && io == 0) HDF_MVTT_NCT(float, float);
  else if (prec == 0 && io == 1) HDF_MVTT_NCT(double, double);
  else if (prec == 0 && io == 0) HDF_MVTT_NCT(double, float);
  else return hipErrorInvalidValue;
#undef HDF_MVTT_NCT
#undef HDF_MVTT
  return hipGetLastError();
}

// Fixed-order reduction over the pass-1 splits (eight independent partial
// sums combined pairwise, so the order is fixed and the loads pipelined).
template <typename T>
__global__ void k_mv_reduce(const double* __restrict__ part, int n_splits, int64_t total, int m16,
                            const double* __restrict__ lam_row, double* __restrict__ W,
                            T* __restrict__ Wd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int sp = 0;
  for (; sp + 8 <= n_splits; sp += 8)
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += part[(int64_t)(sp + u) * total + e];
  for (int u = 0; sp + u < n_splits; ++u) acc[u] += part[(int64_t)(sp + u) * total + e];
  const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  W[e] = s;
  Wd[e] = (T)(lam_row[e / m16] * s);
}

// Pass 2, KV = U (D W).  One wavefront owns 64 points and one 16-column
// chunk of the right-hand sides.  The reduction runs over the rank columns
// (k, h, l) directly: the MFMA A operand is U[i, (k,h,l)] = phi_h(i) q_{k,l}(i),
// formed in registers from one load of each harmonic row and the point's
// radial values, and B is row (k,h,l) of D W.  Each harmonic row is read
// once, and the four accumulators (one per point tile) are the output itself.
// MFMA row i of point tile u is point p0 + 4 i + u, so each lane reads 4
// consecutive points of a harmonic (or radial) row with one 16-byte load.
// With hchunk > 0 (few points, many harmonics) blockIdx.z takes the harmonic
// rows [z hchunk, (z+1) hchunk) only and writes its share of KV to
// part[z][n][m]; k_mv_n_sum adds the shares in z order.
// With Wb (and hchunk == 0) the rows of D W come from its batch-major copy (k_wd_batches): the four
// values a lane needs for one radial function of a batch are one 16-byte (32-byte) load.
template <typename T, typename TO>
__global__ void __launch_bounds__(64) k_mv_n(const T* __restrict__ phi, int64_t ld_phi,
                                              const T* __restrict__ q, int64_t ld_q,
                                              const DegDev* __restrict__ degs, int n_deg,
                                              const T* __restrict__ Wd, const T* __restrict__ Wb, int m16,
                                              TO* __restrict__ KV, int64_t ldkv, int64_t n, int m,
                                              int hchunk, T* __restrict__ part) {
  typedef typename Mfma<T>::V Acc;
  const int lane = threadIdx.x, li = lane & 15, g = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 16;
  const int64_t pa = p0 + 4 * li;                // this lane's four A points
  const int zlo = hchunk > 0 ? (int)blockIdx.z * hchunk : 0;
  const int zhi = hchunk > 0 ? zlo + hchunk : 0x7fffffff;
  Acc acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = Acc{0, 0, 0, 0};
  // four consecutive points of a padded row (in bounds up to 63 points past n)
  auto load4 = [&](const T* row, T (&o)[4]) {
    if constexpr (sizeof(T) == 4) {
      const floatx4 w = *reinterpret_cast<const floatx4*>(row + pa);
#pragma unroll
      for (int u = 0; u < 4; ++u) o[u] = w[u];
    } else {
      const doublex2 w0 = *reinterpret_cast<const doublex2*>(row + pa);
      const doublex2 w1 = *reinterpret_cast<const doublex2*>(row + pa + 2);
      o[0] = w0[0]; o[1] = w0[1]; o[2] = w1[0]; o[3] = w1[1];
    }
  };
  constexpr int KB = 4;                          // K-steps per batch: 16 harmonics
  for (int di = 0; di < n_deg; ++di) {
    const DegDev dg = degs[di];
    // this workgroup's harmonics of the degree: [hlo, hhi)
    const int hlo = zlo > dg.hoff ? zlo - dg.hoff : 0;
    const int hhi = (zhi - dg.hoff) < dg.nh ? zhi - dg.hoff : dg.nh;
    if (hlo >= hhi) continue;
    // harmonic rows of a batch (clamped rows, masked values), the next batch in flight
    auto load_batch = [&](int hb, T (&vv)[KB][4]) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int hh = hb + 4 * kb + g;
        load4(phi + (int64_t)(dg.hoff + (hh < hhi ? hh : hlo)) * ld_phi, vv[kb]);
#pragma unroll
        for (int u = 0; u < 4; ++u) vv[kb][u] = (hh < hhi && pa + u < n) ? vv[kb][u] : (T)0;
      }
    };
    // radial values of function l at this lane's points and the batch's rows of D W for l
    auto load_l = [&](int hb, int l, T (&ql)[4], T (&bw)[KB]) {
      load4(q + (int64_t)(dg.qoff + l) * ld_q, ql);
      if (Wb) {                                     // uniform
        // block (batch hb / 16, radial function l) of the degree, column tile blockIdx.y
        const T* src = Wb + (((int64_t)dg.boff + (hb >> 4) * dg.s + l) * (m16 >> 4) + blockIdx.y) * 256 +
                       (g * 16 + li) * KB;
        if constexpr (sizeof(T) == 4) {
          const floatx4 w = *reinterpret_cast<const floatx4*>(src);
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) bw[kb] = w[kb];
        } else {
          const doublex2 w0 = *reinterpret_cast<const doublex2*>(src);
          const doublex2 w1 = *reinterpret_cast<const doublex2*>(src + 2);
          bw[0] = w0[0]; bw[1] = w0[1]; bw[2] = w1[0]; bw[3] = w1[1];
        }
        return;
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const int hh = hb + 4 * kb + g;
        bw[kb] = Wd[(int64_t)(dg.roff + (hh < hhi ? hh : hlo) * dg.s + l) * m16 + c0 + li];
      }
    };
    // binary32 issue order per batch: the operands of l = 0, then the next batch's rows, then
    // those of l + 1 ahead of l's MFMAs, so no wait of this batch covers the next batch's rows.
    // binary64 loads l's operands at l (the extra registers would cost a wavefront per SIMD).
    constexpr bool ahead = sizeof(T) == 4;
    T v_nxt[KB][4];
    load_batch(hlo, v_nxt);
    for (int hb = hlo; hb < hhi; hb += 4 * KB) {
      T v[KB][4];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int u = 0; u < 4; ++u) v[kb][u] = v_nxt[kb][u];
      T ql[4], bw[KB];
      if constexpr (ahead) load_l(hb, 0, ql, bw);
      if (hb + 4 * KB < hhi) load_batch(hb + 4 * KB, v_nxt);
      for (int l = 0; l < dg.s; ++l) {
        T qn[4], bn[KB];
        if constexpr (ahead) {
          if (l + 1 < dg.s) load_l(hb, l + 1, qn, bn);
        } else {
          load_l(hb, l, ql, bw);
        }
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = Mfma<T>::run(v[kb][u] * ql[u], bw[kb], acc[u]);
        if constexpr (ahead) {
#pragma unroll
          for (int u = 0; u < 4; ++u) ql[u] = qn[u];
#pragma unroll
          for (int kb = 0; kb < KB; ++kb) bw[kb] = bn[kb];
        }
      }
    }
  }
  const int c = c0 + li;
  if (c < m) {
    T* dpart = part ? part + (int64_t)blockIdx.z * n * m : nullptr;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t pt = p0 + 4 * Mfma<T>::row(g, e) + u;
        if (pt < n) {
          if (dpart) dpart[pt * m + c] = acc[u][e];
          else KV[pt * ldkv + c] = (TO)acc[u][e];
        }
      }
  }
}

template <typename T, typename TO>
__global__ void __launch_bounds__(256) k_mv_n_sum(const T* __restrict__ part, int nz, int64_t n, int m,
                                                  TO* __restrict__ KV, int64_t ldkv) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * m) return;
  const int64_t pt = e / m;
  const int c = (int)(e - pt * m);
  T s = 0;
  for (int z = 0; z < nz; ++z) s += part[((int64_t)z * n + pt) * m + c];
  KV[pt * ldkv + c] = (TO)s;
}

constexpr int kMvNctF = 4;   // column tiles per item of k_mv_t, binary32
constexpr int kMvNctD = 2;   // column tiles per item of k_mv_t, binary64

int matvec_row_block() { return 16 * kMvtRowTiles; }
int matvec_col_tiles(int prec) { return prec == 1 ? kMvNctF : kMvNctD; }

hipError_t launch_matvec_t(const void* phi, int64_t ld_phi, const void* q, int64_t ld_q,
                           const DegDev* degs, const TileDev* tiles, int n_tiles, int max_nct,
                           const void* V, int64_t ldv, int64_t n, int m, int m16, int n_splits,
                           int64_t split_len, int64_t rank, double* partials, int prec, int io,
                           hipStream_t s) {
  (void)max_nct;
  const dim3 grid(n_tiles, n_splits);
  if (prec == 1 && io == 0)
    k_mv_t<float, kMvNctF, float><<<grid, 64, 0, s>>>((const float*)phi, ld_phi, (const float*)q, ld_q, degs,
                                                     tiles, (const float*)V, ldv, n, m, m16, split_len, rank,
                                                     partials);
  else if (prec == 0 && io == 1)
    k_mv_t<double, kMvNctD, double><<<grid, 64, 0, s>>>((const double*)phi, ld_phi, (const double*)q, ld_q,
                                                       degs, tiles, (const double*)V, ldv, n, m, m16,
                                                       split_len, rank, partials);
  else if (prec == 0 && io == 0)
    k_mv_t<double, kMvNctD, float><<<grid, 64, 0, s>>>((const double*)phi, ld_phi, (const double*)q, ld_q,
                                                      degs, tiles, (const float*)V, ldv, n, m, m16,
                                                      split_len, rank, partials);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_matvec_reduce(const double* partials, int n_splits, int64_t rank, int m16,
                                const double* lam_row, double* W, void* Wd, int prec,
                                hipStream_t s) {
  const int64_t total = rank * m16;
  const unsigned nb = (unsigned)((total + 255) / 256);
  if (prec == 1)
    k_mv_reduce<float><<<nb, 256, 0, s>>>(partials, n_splits, total, m16, lam_row, W, (float*)Wd);
  else
    k_mv_reduce<double><<<nb, 256, 0, s>>>(partials, n_splits, total, m16, lam_row, W, (double*)Wd);
  return hipGetLastError();
}

// Batch-major copy of D W for pass 2: block B = boff_k + b s_k + l of degree k holds, for batch b
// (harmonics 16 b .. 16 b + 15) and radial function l, every 16-column tile ct as 256 values in
// the order (lane g 16 + c, K-step kb) with harmonic 16 b + 4 kb + g and column 16 ct + c; rows past
// the degree's harmonics are zero.  boff_k is DegDev::boff.
template <typename T>
__global__ void __launch_bounds__(256) k_wd_batches(const DegDev* __restrict__ degs, int n_deg,
                                                     const T* __restrict__ Wd, int m16, int64_t n_blocks,
                                                     T* __restrict__ Wb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int ncts = m16 >> 4;
  if (e >= n_blocks * ncts * 256) return;
  const int64_t blk = e / (ncts * 256);
  const int rest = (int)(e - blk * ncts * 256);
  const int ct = rest >> 8, lane = (rest >> 2) & 63, kb = rest & 3;
  const int g = lane >> 4, c = lane & 15;
  int di = 0;
  while (di + 1 < n_deg && degs[di + 1].boff <= blk) ++di;
  const DegDev dg = degs[di];
  const int64_t rel = blk - dg.boff;
  const int b = (int)(rel / dg.s), l = (int)(rel - (int64_t)b * dg.s);
  const int hh = 16 * b + 4 * kb + g;
  Wb[e] = hh < dg.nh ? Wd[(int64_t)(dg.roff + hh * dg.s + l) * m16 + 16 * ct + c] : (T)0;
}

hipError_t launch_wd_batches(const DegDev* degs, int n_deg, const void* Wd, int m16, int64_t n_blocks, void* Wb,
                             int prec, hipStream_t s) {
  if (m16 < 16 || m16 % 16 || n_blocks < 1 || n_deg < 1) return hipErrorInvalidValue;
  const int64_t total = n_blocks * (m16 / 16) * 256;
  const unsigned nb = (unsigned)((total + 255) / 256);
  if (prec == 1) k_wd_batches<float><<<nb, 256, 0, s>>>(degs, n_deg, (const float*)Wd, m16, n_blocks, (float*)Wb);
  else k_wd_batches<double><<<nb, 256, 0, s>>>(degs, n_deg, (const double*)Wd, m16, n_blocks, (double*)Wb);
  return hipGetLastError();
}

hipError_t launch_matvec_n(const void* phi, int64_t ld_phi, const void* q, int64_t ld_q,
                           const DegDev* degs, int n_deg, int max_s, const void* Wd, const void* Wb, int m16,
                           void* KV, int64_t ldkv, int64_t n, int m, int prec, int io, int hchunk, int nz,
                           void* part, hipStream_t s) {
  (void)max_s;
  if (nz < 1 || (nz > 1 && (hchunk <= 0 || !part))) return hipErrorInvalidValue;
  if (Wb && nz > 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((n + 63) / 64), (unsigned)(m16 / 16), (unsigned)nz);
  const int hc = nz > 1 ? hchunk : 0;
  const unsigned nb = (unsigned)((n * m + 255) / 256);
#define HDF_MVN(T, TO)                                                                                       \
  do {                                                                                                       \
    T* dst = nz > 1 ? (T*)part : nullptr;                                                                    \
    k_mv_n<T, TO><<<grid, 64, 0, s>>>((const T*)phi, ld_phi, (const T*)q, ld_q, degs, n_deg, (const T*)Wd,  \
                                      (const T*)Wb, m16, (TO*)KV, ldkv, n, m, hc, dst);                      \
    if (nz > 1) k_mv_n_sum<T, TO><<<nb, 256, 0, s>>>((const T*)part, nz, n, m, (TO*)KV, ldkv);               \
  } while (0)
  if (prec == 1 && io == 0) HDF_MVN(float, float);
  else if (prec == 0 && io == 1) HDF_MVN(double, double);
  else if (prec == 0 && io == 0) HDF_MVN(double, float);
  else return hipErrorInvalidValue;
#undef HDF_MVN
  return hipGetLastError();
}

}  // namespace hdf
