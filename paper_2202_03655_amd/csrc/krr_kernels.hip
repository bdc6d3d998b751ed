// Kernels of the kernel-ridge-regression consumer (Sec. 4.2), binary64:
// k-means, the exact dense kernel matvec (off-diagonal blocks, predictions),
// the block-diagonal preconditioner (dense blocks, Cholesky, inverse, batched
// GEMV) and the conjugate-gradient vector and scalar updates.  Every
// reduction runs in a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "krr_kernels.hpp"

namespace hdf {
namespace krr {

namespace {

constexpr int kMaxK = 256;

template <int KIND>
__device__ __forceinline__ double kval(double r2, double a) {
  // a: 1/(2 l^2) Gaussian, 1/l^2 Cauchy, sqrt(3)/l Matern-3/2, sqrt(5)/l Matern-5/2
  if constexpr (KIND == 0) {
    return exp(-r2 * a);
  } else if constexpr (KIND == 1) {
    return 1.0 / (1.0 + r2 * a);
  } else if constexpr (KIND == 2) {
    const double z = sqrt(r2) * a;
    return (1.0 + z) * exp(-z);
  } else {
    const double z = sqrt(r2) * a;
    return (1.0 + z + z * z / 3.0) * exp(-z);
  }
}

double kernel_param(int kind, double l) {
  switch (kind) {
    case 0: return 1.0 / (2.0 * l * l);
    case 1: return 1.0 / (l * l);
    case 2: return 1.7320508075688772 / l;
    default: return 2.23606797749979 / l;
  }
}

// Sum of part[0..np) in a fixed order over one 256-thread block; every
// thread gets the result.
__device__ double block_sum(const double* part, int np, double* sh) {
  double s = 0.0;
  for (int t = threadIdx.x; t < np; t += 256) s += part[t];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Tree sum of one value per thread of a 256-thread block, written by thread 0.
__device__ void block_store(double v, double* sh, double* out) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// ---------------------------------------------------------------- k-means

__global__ __launch_bounds__(256) void k_gather_rows(const double* __restrict__ x, int64_t ld,
                                                     const int64_t* __restrict__ idx, int64_t m, int d,
                                                     double* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= m * d) return;
  const int64_t i = e / d;
  const int t = (int)(e % d);
  out[i * ldo + t] = x[idx[i] * ld + t];
}

template <int D>
__global__ __launch_bounds__(256) void k_km_assign(const double* __restrict__ x, int64_t ld, int64_t n,
                                                   const double* __restrict__ centres, int k,
                                                   int32_t* __restrict__ labels, int32_t* __restrict__ changed,
                                                   int first) {
#pragma clang fp contract(off)
  __shared__ double sc[kMaxK * D];
  for (int t = threadIdx.x; t < k * D; t += 256) sc[t] = centres[t];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int moved = 0;
  if (i < n) {
    double xi[D];
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = x[i * ld + t];
    int best = 0;
    double bd = 0.0;
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < D; ++t) {
        const double u = xi[t] - sc[c * D + t];
        const double u2 = u * u;
        s = s + u2;
      }
      if (c == 0 || s < bd) {
        bd = s;
        best = c;
      }
    }
    moved = first ? 1 : (labels[i] != best);
    labels[i] = best;
  }
  const int cnt = __syncthreads_count(moved);
  if (threadIdx.x == 0) changed[blockIdx.x] = cnt;
}

constexpr int kKmChunk = 4096;

// part[(c * chunks + b) * (D + 1) + t]: sum of coordinate t (t = D: count) of
// the members of c among points [b * kKmChunk, (b + 1) * kKmChunk)
template <int D>
__global__ __launch_bounds__(256) void k_km_partial(const double* __restrict__ x, int64_t ld, int64_t n,
                                                    const int32_t* __restrict__ labels, double* __restrict__ part) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  const int b = blockIdx.y;
  const int64_t i0 = (int64_t)b * kKmChunk;
  const int64_t i1 = min(n, i0 + kKmChunk);
  double acc[D + 1];
#pragma unroll
  for (int t = 0; t <= D; ++t) acc[t] = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
    if (labels[i] == c) {
#pragma unroll
      for (int t = 0; t < D; ++t) acc[t] += x[i * ld + t];
      acc[D] += 1.0;
    }
  }
  double* out = part + ((int64_t)c * gridDim.y + b) * (D + 1);
#pragma unroll
  for (int t = 0; t <= D; ++t) {
    block_store(acc[t], sh, out + t);
    __syncthreads();
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_km_finish(const double* __restrict__ part, int chunks, int k,
                                                   double* __restrict__ centres) {
  const int c = threadIdx.x;
  if (c >= k) return;
  double acc[D + 1];
#pragma unroll
  for (int t = 0; t <= D; ++t) acc[t] = 0.0;
  for (int b = 0; b < chunks; ++b) {
    const double* p = part + ((int64_t)c * chunks + b) * (D + 1);
#pragma unroll
    for (int t = 0; t <= D; ++t) acc[t] += p[t];
  }
  if (acc[D] > 0.0) {
#pragma unroll
    for (int t = 0; t < D; ++t) centres[c * D + t] = acc[t] / acc[D];
  }
}

// ------------------------------------------------------ dense kernel matvec

template <int D, int KIND, bool MASK>
__global__ __launch_bounds__(256) void k_kmv(const double* __restrict__ x, int64_t ldx, int nx,
                                             const double* __restrict__ y, int64_t ldy, int ny,
                                             const double* __restrict__ w, const int32_t* __restrict__ lohi,
                                             double ka, int chunk, double* __restrict__ part) {
  __shared__ double sy[D][256];
  __shared__ double sw[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j0 = (int)min((int64_t)ny, (int64_t)blockIdx.y * chunk);
  const int j1 = (int)min((int64_t)ny, (int64_t)j0 + chunk);
  double xi[D];
  int lo = 0, hi = 0;
  if (i < nx) {
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = x[(int64_t)i * ldx + t];
    if (MASK) {
      lo = lohi[2 * i];
      hi = lohi[2 * i + 1];
    }
  } else {
#pragma unroll
    for (int t = 0; t < D; ++t) xi[t] = 0.0;
  }
  double acc = 0.0;
  for (int jb = j0; jb < j1; jb += 256) {
    const int j = jb + threadIdx.x;
    __syncthreads();
    if (j < j1) {
#pragma unroll
      for (int t = 0; t < D; ++t) sy[t][threadIdx.x] = y[(int64_t)j * ldy + t];
      sw[threadIdx.x] = w[j];
    }
    __syncthreads();
    const int cnt = min(256, j1 - jb);
#pragma unroll 4
    for (int jj = 0; jj < cnt; ++jj) {
      double r2 = 0.0;
#pragma unroll
      for (int t = 0; t < D; ++t) {
        const double u = xi[t] - sy[t][jj];
        r2 = fma(u, u, r2);
      }
      const double kv = kval<KIND>(r2, ka);
      double c = sw[jj];
      if (MASK) c = (jb + jj >= lo && jb + jj < hi) ? 0.0 : c;
      acc = fma(kv, c, acc);
    }
  }
  if (i < nx) part[(int64_t)blockIdx.y * nx + i] = acc;
}

__global__ __launch_bounds__(256) void k_kmv_finish(const double* __restrict__ part, int splits, int64_t n,
                                                    const double* __restrict__ base, const double* __restrict__ v,
                                                    double lam, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = base ? base[i] : 0.0;
  if (v) s = fma(lam, v[i], s);
  for (int k = 0; k < splits; ++k) s += part[(int64_t)k * n + i];
  out[i] = s;
}

__global__ __launch_bounds__(256) void k_pack_rows(const double* __restrict__ x, int64_t n, int d, int64_t ld,
                                                   double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * d) return;
  out[e] = x[(e / d) * ld + e % d];
}

__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ v, const int32_t* __restrict__ perm,
                                                int64_t n, double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p < n) out[p] = v[perm[p]];
}

__global__ __launch_bounds__(256) void k_scatter(const double* __restrict__ v, const int32_t* __restrict__ perm,
                                                 int64_t n, double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p < n) out[perm[p]] = v[p];
}

// ---------------------------------------------------- preconditioner blocks

template <int D, int KIND>
__global__ __launch_bounds__(256) void k_dense_blocks(const double* __restrict__ xs, const Block* __restrict__ blocks,
                                                      double ka, double lam, double* __restrict__ A) {
  const Block B = blocks[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t nn = (int64_t)B.n * B.n;
  if (e >= nn) return;
  const int64_t i = e / B.n, j = e % B.n;
  const double* xi = xs + (B.pos + i) * D;
  const double* xj = xs + (B.pos + j) * D;
  double r2 = 0.0;
#pragma unroll
  for (int t = 0; t < D; ++t) {
    const double u = xi[t] - xj[t];
    r2 = fma(u, u, r2);
  }
  A[B.aoff + e] = kval<KIND>(r2, ka) + (i == j ? lam : 0.0);
}

// Right-looking Cholesky A = U^T U of each block in place, on the upper
// triangle (row-major): row j of U is finished at step j, then the trailing
// rows c > j lose U[j][c] * U[j][c..n).  One workgroup per block; the lower
// triangle is left untouched.  status[b] = 0, or the 1-based step whose pivot
// was not positive and finite.
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, const Block* __restrict__ blocks,
                                                   int32_t* __restrict__ status) {
  __shared__ double piv;
  __shared__ int bad;
  const Block B = blocks[blockIdx.x];
  const int n = B.n;
  double* U = A + B.aoff;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) bad = 0;
  for (int j = 0; j < n; ++j) {
    __syncthreads();
    if (tid == 0) {
      const double a = U[(int64_t)j * n + j];
      const bool ok = a > 0.0 && a < INFINITY;
      if (!ok && bad == 0) bad = j + 1;
      piv = ok ? sqrt(a) : 1.0;
    }
    __syncthreads();
    const double pj = piv;
    for (int i = j + tid; i < n; i += blockDim.x) {
      double* u = U + (int64_t)j * n + i;
      *u = (i == j) ? pj : *u / pj;
    }
    __syncthreads();
    for (int c = j + 1 + wave; c < n; c += nw) {
      const double f = U[(int64_t)j * n + c];
      double* row = U + (int64_t)c * n;
      const double* rj = U + (int64_t)j * n;
      for (int i = c + lane; i < n; i += 64) row[i] = fma(-f, rj[i], row[i]);
    }
  }
  __syncthreads();
  if (tid == 0) status[blockIdx.x] = bad;
}

// X = A^{-1} = U^{-1} U^{-T} column by column: one thread per column col
// solves U^T y = e_col, then U x = y, in place in X (row-major, the same
// layout as A).  Threads are independent: each reads U (the same entry across
// a wavefront) and its own column of X.
__global__ __launch_bounds__(256) void k_chol_inverse(const double* __restrict__ Uall, const Block* __restrict__ blocks,
                                                      double* __restrict__ Xall) {
  const Block B = blocks[blockIdx.y];
  const int n = B.n;
  if ((int)blockIdx.x * 256 >= n) return;
  const int col = blockIdx.x * 256 + threadIdx.x;
  const bool act = col < n;
  const double* U = Uall + B.aoff;
  double* X = Xall + B.aoff;
  // lanes past the last column read the first column of U (valid, read-only) and store nothing
  const double* xc = act ? X + col : U;
  for (int i = 0; i < n; ++i) {
    double s = (i == col) ? 1.0 : 0.0;
    for (int k = 0; k < i; ++k) s = fma(-U[(int64_t)k * n + i], xc[(int64_t)k * n], s);
    if (act) X[(int64_t)i * n + col] = s / U[(int64_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = xc[(int64_t)i * n];
    for (int k = i + 1; k < n; ++k) s = fma(-U[(int64_t)i * n + k], xc[(int64_t)k * n], s);
    if (act) X[(int64_t)i * n + col] = s / U[(int64_t)i * n + i];
  }
}

// One wavefront per row position p of the cluster order.
__global__ __launch_bounds__(256) void k_block_gemv(const double* __restrict__ Ainv, const Block* __restrict__ blocks,
                                                    const int32_t* __restrict__ row_block, int64_t n,
                                                    const double* __restrict__ r, double* __restrict__ z,
                                                    double* __restrict__ part_rz, const CGState* __restrict__ st) {
  if (st && st->done) return;
  __shared__ double sh[4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + wave;
  double contrib = 0.0;
  if (p < n) {
    const Block B = blocks[row_block[p]];
    const int64_t i = p - B.pos;
    const double* row = Ainv + B.aoff + i * B.n;
    const double* rc = r + B.pos;
    double s = 0.0;
    for (int j = lane; j < B.n; j += 64) s = fma(row[j], rc[j], s);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) z[p] = s;
    contrib = r[p] * s;
  }
  if (part_rz) {
    if (lane == 0) sh[wave] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) part_rz[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  }
}

// ------------------------------------------------------ conjugate gradients

__global__ __launch_bounds__(256) void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                     int64_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) s = fma(a[i], b[i], s);
  block_store(s, sh, part + blockIdx.x);
}

__global__ __launch_bounds__(256) void k_cg_start(const double* __restrict__ y, int64_t n, double* __restrict__ x,
                                                  double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  x[i] = 0.0;
  r[i] = y[i];
}

__global__ __launch_bounds__(256) void k_cg_init(CGState* __restrict__ st, const double* __restrict__ part_bb,
                                                 const double* __restrict__ part_rz, int nrz, double rtol2, int max_it) {
  __shared__ double sh[256];
  const double bb = block_sum(part_bb, kDotBlocks, sh);
  const double rz = block_sum(part_rz, nrz, sh);
  if (threadIdx.x == 0) {
    st->bb = bb;
    st->rz = rz;
    st->rr = bb;
    st->rtol2 = rtol2;
    st->alpha = st->beta = st->pq = 0.0;
    st->it = 0;
    st->max_it = max_it;
    st->done = bb == 0.0 ? 1 : (max_it <= 0 ? 2 : 0);
  }
}

__global__ __launch_bounds__(256) void k_cg_alpha(CGState* __restrict__ st, const double* __restrict__ part_pq) {
  if (st->done) return;
  __shared__ double sh[256];
  const double pq = block_sum(part_pq, kDotBlocks, sh);
  if (threadIdx.x == 0) {
    st->pq = pq;
    st->alpha = st->rz / pq;
  }
}

__global__ __launch_bounds__(256) void k_cg_xr(double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ p, const double* __restrict__ q, int64_t n,
                                               const CGState* __restrict__ st, double* __restrict__ part_rr) {
  if (st->done) return;
  __shared__ double sh[256];
  const double a = st->alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)kDotBlocks * 256) {
    x[i] = fma(a, p[i], x[i]);
    const double ri = fma(-a, q[i], r[i]);
    r[i] = ri;
    s = fma(ri, ri, s);
  }
  block_store(s, sh, part_rr + blockIdx.x);
}

__global__ __launch_bounds__(256) void k_cg_check(CGState* __restrict__ st, const double* __restrict__ part_rr) {
  if (st->done) return;
  __shared__ double sh[256];
  const double rr = block_sum(part_rr, kDotBlocks, sh);
  if (threadIdx.x == 0) {
    st->rr = rr;
    const int it = st->it + 1;
    st->it = it;
    if (rr <= st->rtol2 * st->bb) st->done = 1;
    else if (it >= st->max_it) st->done = 2;
  }
}

__global__ __launch_bounds__(256) void k_cg_beta(CGState* __restrict__ st, const double* __restrict__ part_rz, int nrz) {
  if (st->done) return;
  __shared__ double sh[256];
  const double rz = block_sum(part_rz, nrz, sh);
  if (threadIdx.x == 0) {
    st->beta = rz / st->rz;
    st->rz = rz;
  }
}

__global__ __launch_bounds__(256) void k_cg_p(double* __restrict__ p, const double* __restrict__ z, int64_t n,
                                              const CGState* __restrict__ st) {
  if (st->done) return;
  const double b = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = fma(b, p[i], z[i]);
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_gather_rows(const double* x, int64_t ld, const int64_t* idx, int64_t m, int d, double* out,
                              int64_t ldo, hipStream_t s) {
  k_gather_rows<<<blocks_for(m * d), 256, 0, s>>>(x, ld, idx, m, d, out, ldo);
  return hipGetLastError();
}

#define KRR_DISPATCH_D(d, MACRO) \
  switch (d) {                   \
    case 1: MACRO(1); break;     \
    case 2: MACRO(2); break;     \
    case 3: MACRO(3); break;     \
    case 4: MACRO(4); break;     \
    case 5: MACRO(5); break;     \
    case 6: MACRO(6); break;     \
    case 7: MACRO(7); break;     \
    case 8: MACRO(8); break;     \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_km_assign(const double* x, int64_t ld, int64_t n, int d, const double* centres, int k,
                            int32_t* labels, int32_t* changed_per_block, int* n_blocks, hipStream_t s) {
  // first call on a labels array: n_blocks < 0 on entry (labels not read)
  const int first = *n_blocks < 0 ? 1 : 0;
  const unsigned g = blocks_for(n);
  *n_blocks = (int)g;
#define KM_A(D) k_km_assign<D><<<g, 256, 0, s>>>(x, ld, n, centres, k, labels, changed_per_block, first)
  KRR_DISPATCH_D(d, KM_A)
#undef KM_A
  return hipGetLastError();
}

int km_update_chunks(int64_t n) { return (int)std::max<int64_t>(1, (n + kKmChunk - 1) / kKmChunk); }

hipError_t launch_km_update(const double* x, int64_t ld, int64_t n, int d, const int32_t* labels, int k,
                            double* part, double* centres, hipStream_t s) {
  const int chunks = km_update_chunks(n);
  const dim3 g((unsigned)k, (unsigned)chunks);
#define KM_U(D)                                                      \
  k_km_partial<D><<<g, 256, 0, s>>>(x, ld, n, labels, part);         \
  k_km_finish<D><<<1, 256, 0, s>>>(part, chunks, k, centres)
  KRR_DISPATCH_D(d, KM_U)
#undef KM_U
  return hipGetLastError();
}

int kmv_splits(int64_t nx, int64_t ny) {
  // enough workgroups to fill the chip, at least 512 columns per split
  const int64_t rows = (nx + 255) / 256;
  int64_t s = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, rows));
  s = std::min<int64_t>(s, std::max<int64_t>(1, ny / 512));
  return (int)std::min<int64_t>(s, 1024);
}

hipError_t launch_kmv(const double* x, int64_t ldx, int64_t nx, const double* y, int64_t ldy, int64_t ny, int d,
                      int kernel, double l, const double* w, const int32_t* lohi, double* part, int splits,
                      hipStream_t s) {
  if (kernel < 0 || kernel > 3 || splits < 1) return hipErrorInvalidValue;
  const int64_t per = (ny + splits - 1) / splits;
  const int chunk = (int)std::max<int64_t>(256, (per + 255) / 256 * 256);
  const dim3 g(blocks_for(nx), (unsigned)splits);
  const double ka = kernel_param(kernel, l);
  const int ix = (int)nx, iy = (int)ny;
#define KMV_K(D, K)                                                                                        \
  do {                                                                                                     \
    if (lohi) k_kmv<D, K, true><<<g, 256, 0, s>>>(x, ldx, ix, y, ldy, iy, w, lohi, ka, chunk, part);       \
    else k_kmv<D, K, false><<<g, 256, 0, s>>>(x, ldx, ix, y, ldy, iy, w, lohi, ka, chunk, part);           \
  } while (0)
#define KMV_D(D)                         \
  switch (kernel) {                      \
    case 0: KMV_K(D, 0); break;          \
    case 1: KMV_K(D, 1); break;          \
    case 2: KMV_K(D, 2); break;          \
    default: KMV_K(D, 3); break;         \
  }
  KRR_DISPATCH_D(d, KMV_D)
#undef KMV_D
#undef KMV_K
  return hipGetLastError();
}

hipError_t launch_kmv_finish(const double* part, int splits, int64_t n, const double* base, const double* v,
                             double lam, double* out, hipStream_t s) {
  k_kmv_finish<<<blocks_for(n), 256, 0, s>>>(part, splits, n, base, v, lam, out);
  return hipGetLastError();
}

hipError_t launch_pack_rows(const double* x, int64_t n, int d, int64_t ld, double* out, hipStream_t s) {
  k_pack_rows<<<blocks_for(n * d), 256, 0, s>>>(x, n, d, ld, out);
  return hipGetLastError();
}

hipError_t launch_gather(const double* v, const int32_t* perm, int64_t n, double* out, hipStream_t s) {
  k_gather<<<blocks_for(n), 256, 0, s>>>(v, perm, n, out);
  return hipGetLastError();
}

hipError_t launch_scatter(const double* v, const int32_t* perm, int64_t n, double* out, hipStream_t s) {
  k_scatter<<<blocks_for(n), 256, 0, s>>>(v, perm, n, out);
  return hipGetLastError();
}

hipError_t launch_dense_blocks(const double* xs, int d, const Block* blocks, int nb, int max_n, int kernel,
                               double l, double lam, double* A, hipStream_t s) {
  if (kernel < 0 || kernel > 3 || nb < 1) return hipErrorInvalidValue;
  const dim3 g(blocks_for((int64_t)max_n * max_n), (unsigned)nb);
  const double ka = kernel_param(kernel, l);
#define DB_K(D, K) k_dense_blocks<D, K><<<g, 256, 0, s>>>(xs, blocks, ka, lam, A)
#define DB_D(D)                        \
  switch (kernel) {                    \
    case 0: DB_K(D, 0); break;         \
    case 1: DB_K(D, 1); break;         \
    case 2: DB_K(D, 2); break;         \
    default: DB_K(D, 3); break;        \
  }
  KRR_DISPATCH_D(d, DB_D)
#undef DB_D
#undef DB_K
  return hipGetLastError();
}

hipError_t launch_cholesky(double* A, const Block* blocks, int nb, int32_t* status, hipStream_t s) {
  k_cholesky<<<(unsigned)nb, 1024, 0, s>>>(A, blocks, status);
  return hipGetLastError();
}

hipError_t launch_chol_inverse(const double* U, const Block* blocks, int nb, int max_n, double* X, hipStream_t s) {
  const dim3 g(blocks_for(max_n), (unsigned)nb);
  k_chol_inverse<<<g, 256, 0, s>>>(U, blocks, X);
  return hipGetLastError();
}

int block_gemv_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + 3) / 4); }

hipError_t launch_block_gemv(const double* Ainv, const Block* blocks, const int32_t* row_block, int64_t n,
                             const double* r, double* z, double* part_rz, const CGState* st, hipStream_t s) {
  k_block_gemv<<<(unsigned)block_gemv_blocks(n), 256, 0, s>>>(Ainv, blocks, row_block, n, r, z, part_rz, st);
  return hipGetLastError();
}

hipError_t launch_dot_partial(const double* a, const double* b, int64_t n, double* part, hipStream_t s) {
  k_dot_partial<<<kDotBlocks, 256, 0, s>>>(a, b, n, part);
  return hipGetLastError();
}

hipError_t launch_cg_start(const double* y, int64_t n, double* x, double* r, hipStream_t s) {
  k_cg_start<<<blocks_for(n), 256, 0, s>>>(y, n, x, r);
  return hipGetLastError();
}

hipError_t launch_cg_init(CGState* st, const double* part_bb, const double* part_rz, int nrz, double rtol2,
                          int max_it, const double* z, double* p, int64_t n, hipStream_t s) {
  k_cg_init<<<1, 256, 0, s>>>(st, part_bb, part_rz, nrz, rtol2, max_it);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(p, z, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
}

hipError_t launch_cg_alpha(CGState* st, const double* part_pq, hipStream_t s) {
  k_cg_alpha<<<1, 256, 0, s>>>(st, part_pq);
  return hipGetLastError();
}

hipError_t launch_cg_xr(double* x, double* r, const double* p, const double* q, int64_t n, const CGState* st,
                        double* part_rr, hipStream_t s) {
  k_cg_xr<<<kDotBlocks, 256, 0, s>>>(x, r, p, q, n, st, part_rr);
  return hipGetLastError();
}

hipError_t launch_cg_check(CGState* st, const double* part_rr, hipStream_t s) {
  k_cg_check<<<1, 256, 0, s>>>(st, part_rr);
  return hipGetLastError();
}

hipError_t launch_cg_beta(CGState* st, const double* part_rz, int nrz, hipStream_t s) {
  k_cg_beta<<<1, 256, 0, s>>>(st, part_rz, nrz);
  return hipGetLastError();
}

hipError_t launch_cg_p(double* p, const double* z, int64_t n, const CGState* st, hipStream_t s) {
  k_cg_p<<<(unsigned)std::min<int64_t>(blocks_for(n), 1024), 256, 0, s>>>(p, z, n, st);
  return hipGetLastError();
}

}  // namespace krr
}  // namespace hdf
