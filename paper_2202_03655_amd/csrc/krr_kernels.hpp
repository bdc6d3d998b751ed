// Launchers of the kernel-ridge-regression kernels (binary64 throughout).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace hdf {
namespace krr {

// Device-resident conjugate-gradient scalars.  done: 0 running, 1 converged,
// 2 iteration limit reached.
struct CGState {
  double rz, pq, rr, bb, alpha, beta, rtol2;
  int32_t it, done, max_it, pad;
};

constexpr int kDotBlocks = 256;    // partial sums per dot product

// per-cluster descriptors in cluster order
struct Block {
  int64_t pos;    // first position of the cluster
  int64_t aoff;   // offset of its n x n matrix in the block storage
  int32_t n;      // members
  int32_t pad;
};

// k-means
hipError_t launch_gather_rows(const double* x, int64_t ld, const int64_t* idx, int64_t m, int d, double* out,
                              int64_t ldo, hipStream_t s);
hipError_t launch_km_assign(const double* x, int64_t ld, int64_t n, int d, const double* centres, int k,
                            int32_t* labels, int32_t* changed_per_block, int* n_blocks, hipStream_t s);
hipError_t launch_km_update(const double* x, int64_t ld, int64_t n, int d, const int32_t* labels, int k,
                            double* part, double* centres, hipStream_t s);
int km_update_chunks(int64_t n);

// dense kernel matvec: part[s][i] = sum over the s-th column range of k(|x_i - y_j|) w_j, skipping
// j in [lohi[2i], lohi[2i+1]) when lohi != NULL
int kmv_splits(int64_t nx, int64_t ny);
hipError_t launch_kmv(const double* x, int64_t ldx, int64_t nx, const double* y, int64_t ldy, int64_t ny, int d,
                      int kernel, double l, const double* w, const int32_t* lohi, double* part, int splits,
                      hipStream_t s);
// out[i] = (base ? base[i] : 0) + lam * (v ? v[i] : 0) + sum_s part[s][i]
hipError_t launch_kmv_finish(const double* part, int splits, int64_t n, const double* base, const double* v,
                             double lam, double* out, hipStream_t s);
// contiguous n x d copy of a strided array
hipError_t launch_pack_rows(const double* x, int64_t n, int d, int64_t ld, double* out, hipStream_t s);

// vectors
hipError_t launch_gather(const double* v, const int32_t* perm, int64_t n, double* out, hipStream_t s);
hipError_t launch_scatter(const double* v, const int32_t* perm, int64_t n, double* out, hipStream_t s);

// preconditioner blocks
hipError_t launch_dense_blocks(const double* xs, int d, const Block* blocks, int nb, int max_n, int kernel,
                               double l, double lam, double* A, hipStream_t s);
hipError_t launch_cholesky(double* A, const Block* blocks, int nb, int32_t* status, hipStream_t s);
hipError_t launch_chol_inverse(const double* U, const Block* blocks, int nb, int max_n, double* X, hipStream_t s);
// z = blockdiag(Ainv) r; part_rz[b] (if not NULL) = block b's share of r . z; skipped when st->done
hipError_t launch_block_gemv(const double* Ainv, const Block* blocks, const int32_t* row_block, int64_t n,
                             const double* r, double* z, double* part_rz, const CGState* st, hipStream_t s);
int block_gemv_blocks(int64_t n);

// conjugate gradients (fixed-order reductions)
hipError_t launch_dot_partial(const double* a, const double* b, int64_t n, double* part, hipStream_t s);
hipError_t launch_cg_start(const double* y, int64_t n, double* x, double* r, hipStream_t s);
hipError_t launch_cg_init(CGState* st, const double* part_bb, const double* part_rz, int nrz, double rtol2,
                          int max_it, const double* z, double* p, int64_t n, hipStream_t s);
hipError_t launch_cg_alpha(CGState* st, const double* part_pq, hipStream_t s);
hipError_t launch_cg_xr(double* x, double* r, const double* p, const double* q, int64_t n, const CGState* st,
                        double* part_rr, hipStream_t s);
hipError_t launch_cg_check(CGState* st, const double* part_rr, hipStream_t s);
hipError_t launch_cg_beta(CGState* st, const double* part_rz, int nrz, hipStream_t s);
hipError_t launch_cg_p(double* p, const double* z, int64_t n, const CGState* st, hipStream_t s);

}  // namespace krr
}  // namespace hdf
