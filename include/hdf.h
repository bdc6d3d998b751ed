/*
 * hdf.h -- C ABI of the MI355X (gfx950) Harmonic Decomposition Factorization.
 *
 * The library builds, for an isotropic kernel k(||x_i - x_j||; l) on N points
 * in R^d (d >= 3), a low-rank factor K ~ U D U^T whose rank is chosen from an
 * error tolerance, not given by the caller (Ryan & Damle, "Linear Time Kernel
 * Matrix Approximation via Hyperspherical Harmonics", ICML 2022: abstract,
 * Sec. 3.2, Algorithm 1, and Remark 1 for the symmetric X = Y case with the
 * diagonal eigenvalue matrix D).  It then applies the factor (Sec. 3.6,
 * O(N r) matvec) and differentiates w^T K v with respect to the lengthscale
 * and the points (not in the paper).
 *
 * Conventions shared by every entry point:
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  Ownership stays with the caller
 *     unless stated.
 *   - Dense arrays are row-major with an explicit leading dimension (in
 *     elements): element (i, j) of an n x m array A with leading dimension
 *     lda is A[i * lda + j], lda >= m.
 *   - dtype 0 = float32, 1 = float64.  Precision HDF_MIXED requires float32
 *     points / vectors, HDF_FP64 requires float64.
 *   - All device work is enqueued on the caller's HIP stream (NULL = the
 *     default stream).  A handle must not be used concurrently from two
 *     streams or threads.
 *   - On error an entry point returns a negative hdf_status, writes no
 *     output, and leaves a human-readable reason in hdf_last_error()
 *     (thread-local).  Argument errors are detected on the host before any
 *     device work.
 */
#ifndef HDF_H
#define HDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdf_factor* hdf_handle;      /* opaque, owned by the library */

/* Kernels of Sec. 4.1 (Fig. 3 paragraph).  The Gaussian uses the lengthscale
 * convention exp(-r^2 / (2 l^2)) (the paper writes exp(-(r/sigma)^2)). */
typedef enum {
  HDF_GAUSSIAN = 0,   /* exp(-r^2/(2 l^2))                       */
  HDF_CAUCHY   = 1,   /* 1 / (1 + r^2/l^2)                       */
  HDF_MATERN32 = 2,   /* (1 + z) e^-z,         z = sqrt(3) r / l */
  HDF_MATERN52 = 3    /* (1 + z + z^2/3) e^-z, z = sqrt(5) r / l */
} hdf_kernel;

typedef enum {
  HDF_FP64  = 0,      /* every device step in binary64                        */
  HDF_MIXED = 1       /* binary32 data (points, V, KV); binary32 factor,
                         harmonics and MFMA contractions with binary64
                         geometry, reductions and compression, split (hi/lo)
                         binary32 Gram.  For tol <= HDF_SPLIT_TOL the factor
                         is stored and contracted in binary64 instead (its
                         binary32 rounding alone exceeds such tolerances, and
                         binary64 MFMA costs less than a three-product hi/lo
                         binary32 split): see hdf_info_t.factor_precision  */
} hdf_precision;

#define HDF_SPLIT_TOL 1e-6   /* HDF_MIXED: tolerances at or below use a binary64 factor */

typedef enum {
  HDF_OK           =  0,
  HDF_E_ARG        = -1,  /* invalid argument (NULL, size, dtype/precision)  */
  HDF_E_DIM        = -2,  /* d < 3 or d > HDF_MAX_DIM                         */
  HDF_E_NONFINITE  = -3,  /* a point coordinate is NaN or infinite           */
  HDF_E_INFEASIBLE = -4,  /* degree above HDF_MAX_DEGREE, or the factor would
                             exceed the memory budget (see hdf_build)        */
  HDF_E_OOM        = -5,  /* device allocation failed                        */
  HDF_E_HIP        = -6,  /* a HIP runtime call failed                       */
  HDF_E_DISABLED   = -7   /* reserved: an operation switched off at compile
                             time (none is, in this version)                 */
} hdf_status;

#define HDF_MAX_DIM     8
#define HDF_MAX_DEGREE  60   /* largest Chebyshev degree p accepted */
#define HDF_MAX_RHS     256  /* largest number of right-hand sides per call */

/* Summary of a built factor (hdf_info).  Sizes follow Sec. 3.6: H harmonics
 * of the kept degrees, S = sum_k s_k radial functions, rank r = sum_k
 * |H_k| s_k. */
typedef struct {
  int32_t  n_dim;          /* d                                            */
  int32_t  precision;      /* hdf_precision                                */
  int64_t  n_points;       /* N                                            */
  int64_t  n_points_y;     /* general factor K(X, Y): N_y (0: symmetric)     */
  int32_t  degree_p;       /* Chebyshev degree p (even)                    */
  int32_t  n_degrees;      /* p/2 + 1 harmonic degrees k = 0..p/2          */
  int64_t  n_harmonics;    /* H, harmonics of kept degrees (s_k > 0)       */
  int64_t  n_radial;       /* S = sum_k s_k                                */
  int64_t  rank;           /* r = sum_k |H_k| s_k                          */
  double   tau;            /* eigenvalue threshold (Sec. 3.5)              */
  double   nu;             /* estimate of ||K||_F / N                      */
  double   cheb_tail;      /* sum_{i>p} |a_i|                              */
  double   center_radius;  /* R = max_i ||x_i - c||                        */
  double   rho2_min, rho2_max;  /* interval of the radial basis           */
  int64_t  factor_bytes;   /* device bytes of the stored factor            */
  double   t_prep_ms;        /* host wall: geometry pass incl. its sync       */
  double   t_plan_ms;        /* host work of the planner (degree, cores, tau) */
  double   t_gram_ms;        /* host wall waiting on the Gram pass beyond the
                                planner work that overlaps it                */
  double   t_compress_ms;    /* host wall: compression incl. refinement pass */
  double   t_finish_ms;      /* host wall: tables, allocation, factor launch  */
  double   t_build_ms;       /* factor-evaluation kernel (HIP events)        */
  double   t_mv_t_ms;        /* last hdf_matvec: pass 1 kernel (U^T V)       */
  double   t_mv_reduce_ms;   /* last hdf_matvec: split reduction + scaling   */
  double   t_mv_n_ms;        /* last hdf_matvec: pass 2 kernel (U (D W))     */
  double   t_adjoint_ms;     /* last hdf_backward with dX: adjoint kernels   */
  int32_t  n_refined;        /* degrees refined by the second Gram pass      */
  int32_t  s_k[HDF_MAX_DEGREE / 2 + 1];   /* kept radial rank per degree   */
  int32_t  rank_rule;        /* hdf_rank_rule the factor was built with      */
  double   tau_bound;        /* threshold of the error budget at degree_p    */
  double   est_error;        /* HDF_RULE_SAMPLED: sampled relative Frobenius
                                error of the factor; -1 otherwise           */
  int32_t  degree_bound;     /* degree the budget rule picks (may differ from
                                degree_p under HDF_RULE_SAMPLED; -1 if above
                                HDF_MAX_DEGREE)                             */
  int32_t  storage;          /* hdf_storage                                  */
  int64_t  chunk_points;     /* HDF_STORE_NONE: points per chunk; 0 otherwise */
  int32_t  factor_precision; /* storage and arithmetic of the factor and its
                                contractions: HDF_MIXED = binary32,
                                HDF_FP64 = binary64 (HDF_MIXED builds with
                                tol <= HDF_SPLIT_TOL report HDF_FP64)        */
  int32_t  mf_fused;         /* HDF_STORE_NONE: 1 if the products run the
                                fused kernels (factor_bytes is then 0: no
                                scratch per point), 2 if they run their
                                double-buffered form (half of the
                                wavefronts evaluate the next 16 points while
                                the others contract the current ones);
                                0 otherwise                                 */
} hdf_info_t;

/* Build the factor (Algorithm 1, symmetric case, Remark 1).
 *   points  device, n x d, leading dimension ld (>= d), dtype 0/1.
 *   kernel, lengthscale (> 0), tol in (0, 1): target relative Frobenius
 *           error ||K - U D U^T||_F <= tol ||K||_F (Sec. 3.5 bound, restated
 *           in Frobenius form).
 *   prec    HDF_MIXED (dtype must be 0) or HDF_FP64 (dtype must be 1).
 *   out     receives the handle; untouched on error.
 * The handle keeps its own copy of the points.  Blocking device-to-host
 * synchronisations happen on `hip_stream` after the geometry pass and after
 * the radial Gram pass (the degree and the ranks depend on the data), and
 * after a second, binary64 Gram pass when a degree's first-pass Gram is too
 * ill-conditioned for the target accuracy.
 * HDF_E_INFEASIBLE when p > HDF_MAX_DEGREE or the factor would need more than
 * max(1 GiB, 60% of the free device memory). */
hdf_status hdf_build(const void* points, int dtype, int64_t n, int d, int64_t ld,
                     hdf_kernel kernel, double lengthscale, double tol,
                     hdf_precision prec, void* hip_stream, hdf_handle* out);

/* How p and tau are chosen. */
typedef enum {
  HDF_RULE_BOUND   = 0,  /* a-priori: Chebyshev tail <= tol nu / 2 and the
                            Frobenius budget threshold (Sec. 3.5, Eq. bound) */
  HDF_RULE_SAMPLED = 1   /* tighter (remark after Eq. bound): smallest even p
                            whose sampled Chebyshev truncation error is
                            <= tol / 2, then tau raised from the budget value,
                            dropping eigenpairs in increasing |lambda| while
                            the sampled error of U D U^T stays <= margin tol */
} hdf_rank_rule;

/* Where the factor lives between products. */
typedef enum {
  HDF_STORE_FACTOR = 0,  /* harmonics and radial functions of all N points
                            stored once at build, (H + S) x N values        */
  HDF_STORE_NONE   = 1   /* matrix-free: nothing per point is stored; every
                            pass re-evaluates the harmonics and radial
                            functions (Sec. 3.6 cost O(N r) per product,
                            plus the evaluation O(N H) twice): 16 points at
                            a time inside the contraction kernels (fused),
                            or chunk by chunk into a scratch of (H + S) x
                            chunk values (see hdf_build_options.chunked)   */
} hdf_storage;

/* Options of hdf_build_ex; zero-initialised fields take the defaults. */
typedef struct {
  int32_t rank_rule;     /* hdf_rank_rule (default HDF_RULE_BOUND)          */
  int32_t n_pairs;       /* sampled pairs, 1 .. 1048576 (default 16384)      */
  double  margin;        /* share of tol the sampled error may use, (0, 1]
                            (default 0.8)                                    */
  int32_t storage;       /* hdf_storage (default HDF_STORE_FACTOR)          */
  int32_t chunked;       /* HDF_STORE_NONE: 0 (default) uses the fused
                            evaluate-and-contract kernels when the harmonics
                            of 16 points fit in one workgroup's LDS, else
                            the chunk scratch; 1 always uses the chunk
                            scratch                                          */
  int64_t chunk;         /* HDF_STORE_NONE: points per chunk, >= 64
                            (default 262144)                                 */
} hdf_build_options;

/* hdf_build with options (NULL: defaults, identical to hdf_build).  Under
 * HDF_RULE_SAMPLED the relative Frobenius error is estimated from n_pairs
 * SplitMix64 pairs (seed 0x48444601, outputs 2t+1 and 2t+2 of pair t),
 * stratified into the off-diagonal pairs and the diagonal at the pairs'
 * first points, ||E||^2 ~ N(N-1) mean_off e^2 + N mean_diag e^2 (likewise
 * ||K||^2).  The estimate is not a bound: the result meets tol up to the
 * sampling error that the margin absorbs.  No additional synchronisation.
 * Under HDF_STORE_NONE the build stops before the factor evaluation and
 * factor_bytes (hdf_info) is the size of the chunk scratch (0 when the
 * fused kernels serve it); hdf_matvec and hdf_backward (dF/dl) re-evaluate
 * the factor in every pass, hdf_copy_factor returns HDF_E_ARG.  The memory budget of hdf_build applies to the
 * scratch. */
hdf_status hdf_build_ex(const void* points, int dtype, int64_t n, int d, int64_t ld,
                        hdf_kernel kernel, double lengthscale, double tol, hdf_precision prec,
                        const hdf_build_options* opts, void* hip_stream, hdf_handle* out);

/* General case X != Y (Algorithm 1 with two point sets): K(X, Y) ~ U V^T.
 *   x       device, nx x d (leading dimension ldx >= d); y device, ny x d
 *           (ldy >= d); both of the dtype matching prec, as for hdf_build.
 * One normalisation (centre, radius, radial interval) covers X u Y; ||K||_F
 * is estimated over sampled pairs (x_a, y_b), and the threshold uses
 * sqrt(nx ny) in place of N (Sec. 3.5 budget).  Per degree the two radial
 * matrices are factorised from their Gram blocks and the core R_x M R_y^T is
 * truncated by its singular values (Sec. 3.4, Eq. svd / Eq. rapprox).  The
 * handle then serves hdf_matvec (KV = K(X, Y) V, V of ny rows, KV of nx rows),
 * hdf_info (n_points = nx, n_points_y = ny, lambda = singular values),
 * hdf_get_plan (radial coefficients of the X side), hdf_copy_factor (X side)
 * and hdf_copy_factor_y (Y side); hdf_backward returns HDF_E_ARG.  Errors and
 * synchronisations as hdf_build. */
hdf_status hdf_build_cross(const void* x, int64_t nx, int64_t ldx, const void* y, int64_t ny,
                           int64_t ldy, int dtype, int d, hdf_kernel kernel, double lengthscale,
                           double tol, hdf_precision prec, void* hip_stream, hdf_handle* out);

/* KV = U D U^T V (Sec. 3.6, two passes over the factor, no host sync); for a
 * handle from hdf_build_cross, KV = U (V_y^T V) with V of ny rows.
 *   V   device, n x m (ldv >= m), KV device, n x m (ldkv >= m); same dtype as
 *       the points; 1 <= m <= HDF_MAX_RHS.  V and KV must not overlap. */
hdf_status hdf_matvec(hdf_handle h, const void* V, int64_t m, int64_t ldv,
                      void* KV, int64_t ldkv, void* hip_stream);

/* hdf_matvec for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and result as hdf_matvec, with 1 <= m <= 64 and a stored factor
 * (HDF_STORE_FACTOR; else HDF_E_ARG).  It calls no hipMalloc / hipFree and no
 * allocating routine, copies nothing from the host and records no events:
 * its work buffers (split partials, U^T V, D U^T V) live in a fixed 32 MiB
 * array per GPU inside the library, held until the process ends.  A factor
 * whose rank r needs more than that (at least 20 r m16 bytes with m16 =
 * 16 ceil(m / 16) for a binary32 factor, 24 r m16 for binary64) is rejected
 * with HDF_E_INFEASIBLE (r up to about 100,000 at m <= 16, binary32); large
 * ranks run pass 1 over fewer point splits than hdf_matvec does, so that the
 * split partials fit.  Every call on one GPU shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (different streams or host threads) race and must be serialised by the
 * caller. */
hdf_status hdf_matvec_noalloc(hdf_handle h, const void* V, int64_t m, int64_t ldv,
                              void* KV, int64_t ldkv, void* hip_stream);

/* Adjoint of F = sum_c w_c^T (U D U^T) v_c with the structure frozen at the
 * build (centre, radius, degree, radial basis and coefficients, ranks).
 *   Wm, Vm   device, n x m each with leading dimension ld (>= m).
 *   dlength  host, receives dF/dl (NULL: not computed).
 *   dX       device, n x d with leading dimension lddx (>= d), receives dF/dX
 *            (NULL: not computed); same dtype as the points.
 * One blocking synchronisation (U^T V and U^T W come to the host), two the
 * first time dF/dX is asked of a handle.  dF/dX needs a stored factor
 * (HDF_STORE_FACTOR) whose kept degrees are 0..K; otherwise HDF_E_ARG before
 * any device work.  It is formed from the stored factor: the stored harmonic
 * rows are solid harmonics, homogeneous harmonic polynomials of the scaled
 * point (Sec. 3.3 and Appendix A), and the gradient of one of degree k is a
 * fixed linear combination of those of degree k - 1, so dF/dx_i is a product
 * of stored rows with small coefficient matrices, plus a term in the radial
 * derivative dq/d(rho^2), whose Chebyshev series is the derivative of the
 * stored one.  Work space of n (2 m (d + 1)) elements of the factor's type is
 * kept with the handle. */
hdf_status hdf_backward(hdf_handle h, const void* Wm, const void* Vm, int64_t m, int64_t ld,
                        double* dlength, void* dX, int64_t lddx, void* hip_stream);

/* Fill `info` (host) from the handle. */
hdf_status hdf_info(hdf_handle h, hdf_info_t* info);

/* Copy host-side parts of the factor.  Any pointer may be NULL.
 *   index_table  int32, H x (d-1): (k, mu_1, ..., mu_{d-2}) per kept harmonic
 *                in the enumeration order (k ascending, then lexicographic).
 *   lambda       float64, S: eigenvalues, degree-major (k ascending, l).
 *   radial_coef  float64, sum_k L_k s_k: E_k column-major per degree
 *                (coefficient a of radial function l at [offset + l*L_k + a]).
 *   a_cheb       float64, p+1 Chebyshev coefficients used. */
hdf_status hdf_get_plan(hdf_handle h, int32_t* index_table, double* lambda,
                        double* radial_coef, double* a_cheb);

/* Copy the stored factor into caller buffers (device to device, enqueued on
 * hip_stream).  phi_out: H x n (harmonic-major, leading dimension ld_phi >= n),
 * q_out: S x n (radial functions, leading dimension ld_q >= n); element type
 * = the factor's (hdf_info_t.factor_precision: float32 for HDF_MIXED,
 * float64 for HDF_FP64).  Either may be NULL.
 * Column (k,h,l) of U is phi[row of h] * q[row of (k,l)] elementwise
 * (Algorithm 1: Xbar^(k)[:, l] times the harmonic). */
hdf_status hdf_copy_factor(hdf_handle h, void* phi_out, int64_t ld_phi, void* q_out, int64_t ld_q,
                           void* hip_stream);
/* As hdf_copy_factor for the Y side of a handle from hdf_build_cross
 * (harmonics and radial functions at the ny points y; ld >= ny).
 * HDF_E_ARG for a symmetric handle. */
hdf_status hdf_copy_factor_y(hdf_handle h, void* phi_out, int64_t ld_phi, void* q_out, int64_t ld_q,
                             void* hip_stream);

void        hdf_free(hdf_handle h);
const char* hdf_status_string(hdf_status s);
const char* hdf_last_error(void);

/* ---- Host-only planner entry points (no device work; usable without a GPU).
 * They expose the data-free steps of the build so they can be checked on the
 * host. ---- */

/* Chebyshev coefficients of f(s) = k(D |s|; l) on [-1, 1] (Sec. 3.3,
 * Eq. chebtrunc) from the DCT at n_nodes first-kind nodes (n_nodes a power of
 * two, >= 16); odd coefficients are exactly zero.  derivative != 0 gives the
 * coefficients of d f / d l instead.  a: host, n_nodes doubles. */
hdf_status hdf_plan_chebyshev(hdf_kernel kernel, double D, double lengthscale,
                              int n_nodes, int derivative, double* a);

/* Smallest even p <= p_max with sum_{i>p} |a_i| <= eps * nu / 2 (the degree
 * rule standing in for ChebDegreeNeeded, Algorithm 1 / Remark 3).  Writes
 * p and the tail; HDF_E_INFEASIBLE if none. */
hdf_status hdf_plan_degree(const double* a, int n, double eps, double nu, int p_max,
                           int* p, double* tail);

/* Radial cores M_k, k = 0..p/2, of the degree-p expansion (Eq. preharm,
 * Eq. preeigen, with Z_k folded in) in the basis T_a(t),
 * t = (2 rho^2 - u0 - u1) / (u1 - u0): kernel(x, y) ~ sum_k sum_h
 * S_k^h(xt) S_k^h(yt) sum_{a,b} M_k[a,b] T_a(t_x) T_b(t_y).  cores: host,
 * sum_k L_k^2 doubles, L_k = p/2 - k + 1, each core row-major, k ascending. */
hdf_status hdf_plan_cores(const double* a, int p, int d, double u0, double u1, double* cores);

/* Index set H_k (Sec. 3.3) in the enumeration order: count = |H_k|
 * (App. B); table (may be NULL) receives count x (d-2) int32. */
hdf_status hdf_plan_index_set(int d, int k, int32_t* table, int64_t* count);

/* Cross compression of one degree from its two radial Gram blocks (single
 * pass): Gx, Gy, M are L x L row-major (1 <= L <= 32); the eigenvalues of Gx,
 * Gy at or below null_rel times their largest are treated as null.  Writes
 * s = the number of singular values of R_x M R_y^T above tau, sig (s values,
 * descending) and the radial coefficients Ex, Ey (L x s, column-major by
 * column: Ex[l * L + a]).  Sec. 3.4 (Eq. svd, Eq. rapprox); host only. */
hdf_status hdf_plan_compress_cross(int L, const double* Gx, const double* Gy, const double* M, double tau,
                                   double null_rel, int32_t* s, double* sig, double* Ex, double* Ey);

/* ---- Kernel ridge regression consumer (Sec. 4.2).  All binary64.  The
 * weights solve (lambda I + K) w = y (Eq. opt) by preconditioned conjugate
 * gradients; the diagonal blocks of K, one per k-means cluster, are HDF
 * factors (hdf_build, HDF_FP64), the off-diagonal blocks are exact kernel
 * values, and the preconditioner is block diagonal with the exact inverses
 * of the blocks lambda I + K_{C_i C_i}.  Predictions are K(x*, x) w
 * (hdf_kernel_matvec). ---- */

typedef struct hdf_krr* hdf_krr_handle;     /* opaque, owned by the library */

#define HDF_MAX_CLUSTERS 256

/* Lloyd's k-means (the clustering of Sec. 4.2).
 *   points    device float64, n x d (ld >= d), 1 <= d <= HDF_MAX_DIM.
 *   k         1 <= k <= min(n, HDF_MAX_CLUSTERS); max_iter >= 1.
 *   seed      the k initial centres are distinct points, index
 *             (u >> 11) mod n of successive SplitMix64 outputs u from this
 *             seed, a repeated index skipped.
 *   labels    device int32, n: the cluster of every point.
 *   centres   device float64, k x d (row-major, leading dimension d).
 *   iterations host (may be NULL): assignments made.
 * A point goes to the centre of smallest sum_j (x_j - c_j)^2 (no fused
 * multiply-add, coordinates in order), ties to the lower index; a centre
 * becomes the mean of its members, an empty cluster keeps its centre; the
 * iteration stops at the first assignment that changes no label, or after
 * max_iter assignments.  One blocking synchronisation per assignment. */
hdf_status hdf_kmeans(const double* points, int64_t n, int d, int64_t ld, int k, int max_iter,
                      uint64_t seed, int32_t* labels, double* centres, int* iterations,
                      void* hip_stream);

/* out = K(X, Y) w with exact kernel values (the prediction K(x*, x) w of
 * Sec. 4.2).  x device nx x d (ldx >= d), y device ny x d (ldy >= d),
 * 1 <= d <= HDF_MAX_DIM, w device ny, out device nx (must not overlap w).
 * Fixed summation order: the same inputs give the same bits. */
hdf_status hdf_kernel_matvec(const double* x, int64_t nx, int64_t ldx, const double* y, int64_t ny,
                             int64_t ldy, int d, hdf_kernel kernel, double lengthscale,
                             const double* w, double* out, void* hip_stream);

/* Build the KRR system for points with cluster labels (e.g. from
 * hdf_kmeans).
 *   points  device float64, n x d (ld >= d), 3 <= d <= HDF_MAX_DIM.
 *   labels  device int32, n, each in [0, k); 1 <= k <= HDF_MAX_CLUSTERS.
 *   tol     tolerance of every diagonal-block factor (hdf_build).
 *   lambda  regularisation, > 0.
 * Blocking: labels are read back, and each block factor synchronises as
 * hdf_build does.  HDF_E_ARG for a label out of range or a cluster larger
 * than 16384 points; HDF_E_INFEASIBLE when a block factor is, or when a
 * preconditioner block is not numerically positive definite. */
hdf_status hdf_krr_create(const double* points, int64_t n, int d, int64_t ld, const int32_t* labels,
                          int k, hdf_kernel kernel, double lengthscale, double tol, double lambda,
                          void* hip_stream, hdf_krr_handle* out);

/* out = (lambda I + blockdiag(U_i D_i U_i^T) + offdiag(K)) v: the system
 * operator.  v, out device float64, n, in the caller's point order; they
 * must not overlap.  No host synchronisation. */
hdf_status hdf_krr_apply(hdf_krr_handle h, const double* v, double* out, void* hip_stream);

/* z = blockdiag((lambda I + K_{C_i C_i})^{-1}) r: the preconditioner.  r, z
 * device float64, n, caller's order, not overlapping.  No synchronisation. */
hdf_status hdf_krr_precond(hdf_krr_handle h, const double* r, double* z, void* hip_stream);

/* Preconditioned CG from w = 0 (Saad, Alg. 9.1), stopped at the first
 * iteration whose recursive residual satisfies ||r|| <= rtol ||y||, or after
 * max_iter iterations.
 *   y, w       device float64, n, caller's order, not overlapping.
 *   iterations host (may be NULL): iterations made (0 when y = 0).
 *   relres     host (may be NULL): ||r|| / ||y|| at the end.
 * The iterations run on the device, scalars included; the host reads the
 * convergence flag once per batch of 8 iterations (one synchronisation per
 * batch).  Iterations enqueued after convergence leave w unchanged. */
hdf_status hdf_krr_solve(hdf_krr_handle h, const double* y, double* w, int max_iter, double rtol,
                         int* iterations, double* relres, void* hip_stream);

typedef struct {
  int64_t n_points;
  int32_t n_dim, n_clusters;       /* k as given                               */
  int32_t n_blocks;                /* non-empty clusters                       */
  int32_t max_block;               /* largest cluster                          */
  int32_t max_degree;              /* largest Chebyshev degree over the blocks */
  int64_t sum_rank;                /* sum of the block ranks                   */
  int64_t factor_bytes;            /* device bytes of the block factors        */
  int64_t precond_bytes;           /* device bytes of the inverse blocks       */
  double  t_factor_ms;             /* host wall: block factors (hdf_build)     */
  double  t_precond_ms;            /* host wall: dense blocks, Cholesky,
                                      inverses (incl. their synchronisation)  */
  double  t_offdiag_ms;            /* last operator application: off-diagonal
                                      kernel (HIP events)                      */
  double  t_solve_ms;              /* last hdf_krr_solve (HIP events)          */
  int32_t last_iterations;
  double  last_relres;
} hdf_krr_info_t;

hdf_status hdf_krr_info(hdf_krr_handle h, hdf_krr_info_t* info);

/* The factor of cluster c (NULL for an empty cluster), owned by the KRR
 * handle; usable with hdf_info, hdf_get_plan, hdf_copy_factor and
 * hdf_matvec (its points are the members of c in increasing caller index).
 * Its products are not timed: hdf_info reports -1 for their kernel times. */
hdf_status hdf_krr_block(hdf_krr_handle h, int c, hdf_handle* block);

void hdf_krr_free(hdf_krr_handle h);

#ifdef __cplusplus
}
#endif
#endif /* HDF_H */
