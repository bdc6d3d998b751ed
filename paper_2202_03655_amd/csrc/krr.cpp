// C ABI of the kernel-ridge-regression consumer (Sec. 4.2): k-means, the
// exact dense kernel matvec, the KRR system with HDF diagonal blocks, its
// block-diagonal preconditioner and the device-resident conjugate-gradient
// loop.  All device work is binary64.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hdf.h"
#include "krr_kernels.hpp"
#include "status.hpp"

using hdf::krr::Block;
using hdf::krr::CGState;

namespace {

constexpr int kMaxBlock = 16384;   // largest cluster: its dense block is 2 GiB
constexpr int kBatch = 8;          // CG iterations enqueued per convergence check
constexpr int kSide = 4;           // streams the per-cluster factor products are spread over

struct Buf {
  void* p = nullptr;
  ~Buf() {
    if (p) hipFree(p);
  }
  hipError_t alloc(size_t bytes) {
    if (p) hipFree(p);
    p = nullptr;
    return hipMalloc(&p, std::max<size_t>(bytes, 256));
  }
  template <class T>
  T* as() const {
    return (T*)p;
  }
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

uint64_t splitmix64(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char *a0 = (const char*)a, *b0 = (const char*)b;
  return a0 < b0 + nb && b0 < a0 + na;
}

}  // namespace

#define KCHK(expr)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return hdf::set_error(e_ == hipErrorOutOfMemory ? HDF_E_OOM : HDF_E_HIP,                  \
                            std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

struct hdf_krr {
  int64_t n = 0;
  int d = 0, k = 0, kernel = 0;
  double l = 0, tol = 0, lam = 0;
  std::vector<hdf_handle> fac;            // per cluster, NULL when empty
  std::vector<int> block_cluster;         // non-empty block -> cluster
  std::vector<Block> blocks;              // non-empty blocks in cluster order
  int max_n = 0, splits = 1, nrz = 1;
  int64_t precond_elems = 0;
  double t_factor = 0, t_precond = 0;
  int last_it = 0;
  double last_relres = 0;
  bool od_timed = false, s_timed = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // off-diagonal kernel, solve
  // the cluster factors are small (few points, many harmonics): their products run on side streams,
  // concurrently with each other and with the off-diagonal kernel
  hipStream_t side[kSide] = {};
  hipEvent_t fork = nullptr, join[kSide] = {};
  // device: points in cluster order, permutation, exclusion ranges, row -> block, descriptors
  Buf xs, perm, lohi, row_block, blocks_dev, ainv;
  // work vectors (cluster order), partial sums, CG state
  Buf vs, outs, qb, part, x, r, z, p, q, st, part_pq, part_rr, part_bb, part_rz;
  ~hdf_krr() {
    for (hdf_handle h : fac)
      if (h) hdf_free(h);
    for (auto& e : ev)
      if (e) hipEventDestroy(e);
    for (auto& e : join)
      if (e) hipEventDestroy(e);
    if (fork) hipEventDestroy(fork);
    for (auto& t : side)
      if (t) hipStreamDestroy(t);
  }
};

// ------------------------------------------------------------------ k-means

hdf_status hdf_kmeans(const double* points, int64_t n, int d, int64_t ld, int k, int max_iter, uint64_t seed,
                      int32_t* labels, double* centres, int* iterations, void* hip_stream) {
  hdf::clear_error();
  if (!points || !labels || !centres) return hdf::set_error(HDF_E_ARG, "points, labels or centres is NULL");
  if (n < 1 || n > INT32_MAX) return hdf::set_error(HDF_E_ARG, "n must be in [1, 2^31)");
  if (d < 1 || d > HDF_MAX_DIM) return hdf::set_error(HDF_E_DIM, "d must be in [1, 8] for k-means");
  if (ld < d) return hdf::set_error(HDF_E_ARG, "ld must be >= d");
  if (k < 1 || k > HDF_MAX_CLUSTERS || k > n) return hdf::set_error(HDF_E_ARG, "k must be in [1, min(n, 256)]");
  if (max_iter < 1) return hdf::set_error(HDF_E_ARG, "max_iter must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<int64_t> idx;
  uint64_t state = seed;
  while ((int)idx.size() < k) {
    const int64_t i = (int64_t)((splitmix64(state) >> 11) % (uint64_t)n);
    if (std::find(idx.begin(), idx.end(), i) == idx.end()) idx.push_back(i);
  }
  const int nblk = (int)((n + 255) / 256);
  const int chunks = hdf::krr::km_update_chunks(n);
  Buf didx, changed, part;
  KCHK(didx.alloc(idx.size() * sizeof(int64_t)));
  KCHK(changed.alloc((size_t)nblk * sizeof(int32_t)));
  KCHK(part.alloc((size_t)k * chunks * (d + 1) * sizeof(double)));
  KCHK(hipMemcpyAsync(didx.p, idx.data(), idx.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  KCHK(hdf::krr::launch_gather_rows(points, ld, didx.as<int64_t>(), k, d, centres, d, s));
  std::vector<int32_t> ch(nblk);
  int its = 0, nb = -1;
  for (int it = 0; it < max_iter; ++it) {
    KCHK(hdf::krr::launch_km_assign(points, ld, n, d, centres, k, labels, changed.as<int32_t>(), &nb, s));
    ++its;
    if (it > 0) {
      KCHK(hipMemcpyAsync(ch.data(), changed.p, (size_t)nblk * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      KCHK(hipStreamSynchronize(s));
      int64_t moved = 0;
      for (int32_t c : ch) moved += c;
      if (moved == 0) break;
    }
    KCHK(hdf::krr::launch_km_update(points, ld, n, d, labels, k, part.as<double>(), centres, s));
  }
  KCHK(hipStreamSynchronize(s));
  if (iterations) *iterations = its;
  return HDF_OK;
}

// -------------------------------------------------------- dense kernel matvec

hdf_status hdf_kernel_matvec(const double* x, int64_t nx, int64_t ldx, const double* y, int64_t ny, int64_t ldy,
                             int d, hdf_kernel kernel, double lengthscale, const double* w, double* out,
                             void* hip_stream) {
  hdf::clear_error();
  if (!x || !y || !w || !out) return hdf::set_error(HDF_E_ARG, "a pointer is NULL");
  if (nx < 1 || ny < 1 || nx > INT32_MAX || ny > INT32_MAX) return hdf::set_error(HDF_E_ARG, "nx, ny must be in [1, 2^31)");
  if (d < 1 || d > HDF_MAX_DIM) return hdf::set_error(HDF_E_DIM, "d must be in [1, 8]");
  if (ldx < d || ldy < d) return hdf::set_error(HDF_E_ARG, "leading dimensions must be >= d");
  if ((int)kernel < 0 || (int)kernel > 3) return hdf::set_error(HDF_E_ARG, "unknown kernel");
  if (!(lengthscale > 0) || !std::isfinite(lengthscale)) return hdf::set_error(HDF_E_ARG, "lengthscale must be > 0");
  if (overlap(w, ny * 8, out, nx * 8)) return hdf::set_error(HDF_E_ARG, "w and out overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  const int splits = hdf::krr::kmv_splits(nx, ny);
  Buf part;
  KCHK(part.alloc((size_t)splits * nx * sizeof(double)));
  KCHK(hdf::krr::launch_kmv(x, ldx, nx, y, ldy, ny, d, (int)kernel, lengthscale, w, nullptr, part.as<double>(),
                            splits, s));
  KCHK(hdf::krr::launch_kmv_finish(part.as<double>(), splits, nx, nullptr, nullptr, 0.0, out, s));
  // the workspace is released on return
  KCHK(hipStreamSynchronize(s));
  return HDF_OK;
}

// ------------------------------------------------------------ KRR system

// out = lam v + blockdiag(factors) v + offdiag(K) v.  The cluster factors' products (into qb) run on the
// side streams after a fork from s; the off-diagonal kernel runs on s meanwhile; s waits for every side
// stream before the final sum.
static hdf_status krr_operator(hdf_krr* h, const double* v, double* out, hipStream_t s, bool timed) {
  KCHK(hipEventRecord(h->fork, s));
  for (int j = 0; j < kSide; ++j) KCHK(hipStreamWaitEvent(h->side[j], h->fork, 0));
  for (size_t b = 0; b < h->blocks.size(); ++b) {
    const Block& B = h->blocks[b];
    hdf_status st = hdf_matvec(h->fac[h->block_cluster[b]], v + B.pos, 1, 1, h->qb.as<double>() + B.pos, 1,
                               h->side[b % kSide]);
    if (st != HDF_OK) return st;
  }
  if (timed) KCHK(hipEventRecord(h->ev[0], s));
  KCHK(hdf::krr::launch_kmv(h->xs.as<double>(), h->d, h->n, h->xs.as<double>(), h->d, h->n, h->d, h->kernel, h->l,
                            v, h->lohi.as<int32_t>(), h->part.as<double>(), h->splits, s));
  if (timed) {
    KCHK(hipEventRecord(h->ev[1], s));
    h->od_timed = true;
  }
  for (int j = 0; j < kSide; ++j) {
    KCHK(hipEventRecord(h->join[j], h->side[j]));
    KCHK(hipStreamWaitEvent(s, h->join[j], 0));
  }
  KCHK(hdf::krr::launch_kmv_finish(h->part.as<double>(), h->splits, h->n, h->qb.as<double>(), v, h->lam, out, s));
  return HDF_OK;
}

hdf_status hdf_krr_create(const double* points, int64_t n, int d, int64_t ld, const int32_t* labels, int k,
                          hdf_kernel kernel, double lengthscale, double tol, double lambda, void* hip_stream,
                          hdf_krr_handle* out) {
  hdf::clear_error();
  if (!points || !labels || !out) return hdf::set_error(HDF_E_ARG, "points, labels or out is NULL");
  if (n < 1 || n > INT32_MAX) return hdf::set_error(HDF_E_ARG, "n must be in [1, 2^31)");
  if (d < 3 || d > HDF_MAX_DIM) return hdf::set_error(HDF_E_DIM, "d must be in [3, 8]");
  if (ld < d) return hdf::set_error(HDF_E_ARG, "ld must be >= d");
  if (k < 1 || k > HDF_MAX_CLUSTERS) return hdf::set_error(HDF_E_ARG, "k must be in [1, 256]");
  if ((int)kernel < 0 || (int)kernel > 3) return hdf::set_error(HDF_E_ARG, "unknown kernel");
  if (!(lengthscale > 0) || !std::isfinite(lengthscale)) return hdf::set_error(HDF_E_ARG, "lengthscale must be > 0");
  if (!(tol > 0 && tol < 1)) return hdf::set_error(HDF_E_ARG, "tol must be in (0, 1)");
  if (!(lambda > 0) || !std::isfinite(lambda)) return hdf::set_error(HDF_E_ARG, "lambda must be > 0");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<int32_t> lab(n);
  KCHK(hipMemcpyAsync(lab.data(), labels, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  KCHK(hipStreamSynchronize(s));
  std::vector<int64_t> count(k, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (lab[i] < 0 || lab[i] >= k)
      return hdf::set_error(HDF_E_ARG, "label " + std::to_string(lab[i]) + " of point " + std::to_string(i) +
                                           " is outside [0, k)");
    ++count[lab[i]];
  }
  for (int c = 0; c < k; ++c)
    if (count[c] > kMaxBlock)
      return hdf::set_error(HDF_E_ARG, "cluster " + std::to_string(c) + " has more than 16384 points");
  std::unique_ptr<hdf_krr> h(new hdf_krr);
  h->n = n;
  h->d = d;
  h->k = k;
  h->kernel = (int)kernel;
  h->l = lengthscale;
  h->tol = tol;
  h->lam = lambda;
  h->fac.assign(k, nullptr);
  // stable counting sort by cluster
  std::vector<int64_t> start(k + 1, 0);
  for (int c = 0; c < k; ++c) start[c + 1] = start[c] + count[c];
  std::vector<int32_t> perm(n), lohi(2 * n), row_block(n);
  std::vector<int64_t> perm64(n);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i) perm[fill[lab[i]]++] = (int32_t)i;
  }
  int64_t aoff = 0;
  for (int c = 0; c < k; ++c) {
    if (count[c] == 0) continue;
    const int b = (int)h->blocks.size();
    h->blocks.push_back(Block{start[c], aoff, (int32_t)count[c], 0});
    h->block_cluster.push_back(c);
    aoff += count[c] * count[c];
    h->max_n = std::max<int>(h->max_n, (int)count[c]);
    for (int64_t p = start[c]; p < start[c + 1]; ++p) {
      lohi[2 * p] = (int32_t)start[c];
      lohi[2 * p + 1] = (int32_t)start[c + 1];
      row_block[p] = b;
    }
  }
  h->precond_elems = aoff;
  for (int64_t p = 0; p < n; ++p) perm64[p] = perm[p];
  const int nb = (int)h->blocks.size();
  KCHK(h->xs.alloc((size_t)n * d * sizeof(double)));
  KCHK(h->perm.alloc((size_t)n * sizeof(int32_t)));
  KCHK(h->lohi.alloc((size_t)2 * n * sizeof(int32_t)));
  KCHK(h->row_block.alloc((size_t)n * sizeof(int32_t)));
  KCHK(h->blocks_dev.alloc((size_t)nb * sizeof(Block)));
  {
    Buf p64;
    KCHK(p64.alloc((size_t)n * sizeof(int64_t)));
    KCHK(hipMemcpyAsync(p64.p, perm64.data(), (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    KCHK(hipMemcpyAsync(h->perm.p, perm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KCHK(hipMemcpyAsync(h->lohi.p, lohi.data(), (size_t)2 * n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KCHK(hipMemcpyAsync(h->row_block.p, row_block.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KCHK(hipMemcpyAsync(h->blocks_dev.p, h->blocks.data(), (size_t)nb * sizeof(Block), hipMemcpyHostToDevice, s));
    KCHK(hdf::krr::launch_gather_rows(points, ld, p64.as<int64_t>(), n, d, h->xs.as<double>(), d, s));
    KCHK(hipStreamSynchronize(s));
  }
  // diagonal-block factors
  double t0 = now_ms();
  for (int b = 0; b < nb; ++b) {
    const Block& B = h->blocks[b];
    const int c = h->block_cluster[b];
    hdf_status st = hdf_build(h->xs.as<double>() + B.pos * d, 1, B.n, d, d, kernel, lengthscale, tol, HDF_FP64,
                              hip_stream, &h->fac[c]);
    if (st != HDF_OK)
      return hdf::set_error(st, "factor of cluster " + std::to_string(c) + ": " + hdf_last_error());
    hdf::set_product_timing(h->fac[c], false);
  }
  h->t_factor = now_ms() - t0;
  // preconditioner: dense blocks, Cholesky, inverses
  t0 = now_ms();
  {
    Buf A, status;
    KCHK(A.alloc((size_t)aoff * sizeof(double)));
    KCHK(h->ainv.alloc((size_t)aoff * sizeof(double)));
    KCHK(status.alloc((size_t)nb * sizeof(int32_t)));
    KCHK(hdf::krr::launch_dense_blocks(h->xs.as<double>(), d, h->blocks_dev.as<Block>(), nb, h->max_n, h->kernel,
                                       lengthscale, lambda, A.as<double>(), s));
    KCHK(hdf::krr::launch_cholesky(A.as<double>(), h->blocks_dev.as<Block>(), nb, status.as<int32_t>(), s));
    KCHK(hdf::krr::launch_chol_inverse(A.as<double>(), h->blocks_dev.as<Block>(), nb, h->max_n,
                                       h->ainv.as<double>(), s));
    std::vector<int32_t> stat(nb);
    KCHK(hipMemcpyAsync(stat.data(), status.p, (size_t)nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    KCHK(hipStreamSynchronize(s));
    for (int b = 0; b < nb; ++b)
      if (stat[b] != 0)
        return hdf::set_error(HDF_E_INFEASIBLE, "preconditioner block of cluster " +
                                                    std::to_string(h->block_cluster[b]) +
                                                    " is not positive definite (pivot " + std::to_string(stat[b]) + ")");
  }
  h->t_precond = now_ms() - t0;
  // workspace
  h->splits = hdf::krr::kmv_splits(n, n);
  h->nrz = hdf::krr::block_gemv_blocks(n);
  for (Buf* b : {&h->vs, &h->outs, &h->qb, &h->x, &h->r, &h->z, &h->p, &h->q}) KCHK(b->alloc((size_t)n * 8));
  KCHK(h->part.alloc((size_t)h->splits * n * 8));
  KCHK(h->st.alloc(sizeof(CGState)));
  for (Buf* b : {&h->part_pq, &h->part_rr, &h->part_bb}) KCHK(b->alloc((size_t)hdf::krr::kDotBlocks * 8));
  KCHK(h->part_rz.alloc((size_t)h->nrz * 8));
  for (auto& e : h->ev) KCHK(hipEventCreate(&e));
  KCHK(hipEventCreateWithFlags(&h->fork, hipEventDisableTiming));
  for (auto& e : h->join) KCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& t : h->side) KCHK(hipStreamCreateWithFlags(&t, hipStreamNonBlocking));
  *out = h.release();
  return HDF_OK;
}

hdf_status hdf_krr_apply(hdf_krr_handle h, const double* v, double* out, void* hip_stream) {
  hdf::clear_error();
  if (!h || !v || !out) return hdf::set_error(HDF_E_ARG, "handle, v or out is NULL");
  if (overlap(v, h->n * 8, out, h->n * 8)) return hdf::set_error(HDF_E_ARG, "v and out overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  KCHK(hdf::krr::launch_gather(v, h->perm.as<int32_t>(), h->n, h->vs.as<double>(), s));
  hdf_status st = krr_operator(h, h->vs.as<double>(), h->outs.as<double>(), s, true);
  if (st != HDF_OK) return st;
  KCHK(hdf::krr::launch_scatter(h->outs.as<double>(), h->perm.as<int32_t>(), h->n, out, s));
  return HDF_OK;
}

hdf_status hdf_krr_precond(hdf_krr_handle h, const double* r, double* z, void* hip_stream) {
  hdf::clear_error();
  if (!h || !r || !z) return hdf::set_error(HDF_E_ARG, "handle, r or z is NULL");
  if (overlap(r, h->n * 8, z, h->n * 8)) return hdf::set_error(HDF_E_ARG, "r and z overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  KCHK(hdf::krr::launch_gather(r, h->perm.as<int32_t>(), h->n, h->vs.as<double>(), s));
  KCHK(hdf::krr::launch_block_gemv(h->ainv.as<double>(), h->blocks_dev.as<Block>(), h->row_block.as<int32_t>(), h->n,
                                   h->vs.as<double>(), h->outs.as<double>(), nullptr, nullptr, s));
  KCHK(hdf::krr::launch_scatter(h->outs.as<double>(), h->perm.as<int32_t>(), h->n, z, s));
  return HDF_OK;
}

hdf_status hdf_krr_solve(hdf_krr_handle h, const double* y, double* w, int max_iter, double rtol, int* iterations,
                         double* relres, void* hip_stream) {
  hdf::clear_error();
  if (!h || !y || !w) return hdf::set_error(HDF_E_ARG, "handle, y or w is NULL");
  if (max_iter < 0) return hdf::set_error(HDF_E_ARG, "max_iter must be >= 0");
  if (!(rtol >= 0) || !std::isfinite(rtol)) return hdf::set_error(HDF_E_ARG, "rtol must be finite and >= 0");
  if (overlap(y, h->n * 8, w, h->n * 8)) return hdf::set_error(HDF_E_ARG, "y and w overlap");
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t n = h->n;
  double *b = h->vs.as<double>(), *x = h->x.as<double>(), *r = h->r.as<double>(), *z = h->z.as<double>(),
         *p = h->p.as<double>(), *q = h->q.as<double>();
  CGState* st = h->st.as<CGState>();
  const Block* blocks = h->blocks_dev.as<Block>();
  const int32_t* rb = h->row_block.as<int32_t>();
  KCHK(hipEventRecord(h->ev[2], s));
  KCHK(hdf::krr::launch_gather(y, h->perm.as<int32_t>(), n, b, s));
  KCHK(hdf::krr::launch_cg_start(b, n, x, r, s));
  KCHK(hdf::krr::launch_dot_partial(b, b, n, h->part_bb.as<double>(), s));
  KCHK(hdf::krr::launch_block_gemv(h->ainv.as<double>(), blocks, rb, n, r, z, h->part_rz.as<double>(), nullptr, s));
  KCHK(hdf::krr::launch_cg_init(st, h->part_bb.as<double>(), h->part_rz.as<double>(), h->nrz, rtol * rtol, max_iter,
                                z, p, n, s));
  CGState hs{};
  bool first = true;
  for (int it0 = 0;; it0 += kBatch) {
    const int cnt = std::min(kBatch, max_iter - it0);
    for (int i = 0; i < cnt; ++i) {
      hdf_status e = krr_operator(h, p, q, s, first);
      if (e != HDF_OK) return e;
      first = false;
      KCHK(hdf::krr::launch_dot_partial(p, q, n, h->part_pq.as<double>(), s));
      KCHK(hdf::krr::launch_cg_alpha(st, h->part_pq.as<double>(), s));
      KCHK(hdf::krr::launch_cg_xr(x, r, p, q, n, st, h->part_rr.as<double>(), s));
      KCHK(hdf::krr::launch_cg_check(st, h->part_rr.as<double>(), s));
      KCHK(hdf::krr::launch_block_gemv(h->ainv.as<double>(), blocks, rb, n, r, z, h->part_rz.as<double>(), st, s));
      KCHK(hdf::krr::launch_cg_beta(st, h->part_rz.as<double>(), h->nrz, s));
      KCHK(hdf::krr::launch_cg_p(p, z, n, st, s));
    }
    KCHK(hipMemcpyAsync(&hs, st, sizeof(CGState), hipMemcpyDeviceToHost, s));
    KCHK(hipStreamSynchronize(s));
    if (hs.done || cnt <= 0) break;
  }
  KCHK(hdf::krr::launch_scatter(x, h->perm.as<int32_t>(), n, w, s));
  KCHK(hipEventRecord(h->ev[3], s));
  h->s_timed = true;
  h->last_it = hs.it;
  h->last_relres = hs.bb > 0 ? std::sqrt(hs.rr / hs.bb) : 0.0;
  if (iterations) *iterations = h->last_it;
  if (relres) *relres = h->last_relres;
  return HDF_OK;
}

hdf_status hdf_krr_info(hdf_krr_handle h, hdf_krr_info_t* info) {
  hdf::clear_error();
  if (!h || !info) return hdf::set_error(HDF_E_ARG, "handle or info is NULL");
  std::memset(info, 0, sizeof(*info));
  info->n_points = h->n;
  info->n_dim = h->d;
  info->n_clusters = h->k;
  info->n_blocks = (int32_t)h->blocks.size();
  info->max_block = h->max_n;
  for (hdf_handle f : h->fac) {
    if (!f) continue;
    hdf_info_t fi;
    hdf_status st = hdf_info(f, &fi);
    if (st != HDF_OK) return st;
    info->max_degree = std::max(info->max_degree, fi.degree_p);
    info->sum_rank += fi.rank;
    info->factor_bytes += fi.factor_bytes;
  }
  info->precond_bytes = h->precond_elems * 8;
  info->t_factor_ms = h->t_factor;
  info->t_precond_ms = h->t_precond;
  info->t_offdiag_ms = -1;
  info->t_solve_ms = -1;
  float ms = 0;
  if (h->od_timed && hipEventSynchronize(h->ev[1]) == hipSuccess &&
      hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess)
    info->t_offdiag_ms = ms;
  if (h->s_timed && hipEventSynchronize(h->ev[3]) == hipSuccess &&
      hipEventElapsedTime(&ms, h->ev[2], h->ev[3]) == hipSuccess)
    info->t_solve_ms = ms;
  info->last_iterations = h->last_it;
  info->last_relres = h->last_relres;
  return HDF_OK;
}

hdf_status hdf_krr_block(hdf_krr_handle h, int c, hdf_handle* block) {
  hdf::clear_error();
  if (!h || !block) return hdf::set_error(HDF_E_ARG, "handle or block is NULL");
  if (c < 0 || c >= h->k) return hdf::set_error(HDF_E_ARG, "cluster index out of range");
  *block = h->fac[c];
  return HDF_OK;
}

void hdf_krr_free(hdf_krr_handle h) { delete h; }
