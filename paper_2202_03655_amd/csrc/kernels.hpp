// Launchers of the gfx950 kernels of the HDF hot path (host-callable).
#pragma once
#include <hip/hip_runtime_api.h>
#include <cstdint>

namespace hdf {

// Device geometry record written by the prep pass (binary64).
struct GeoDev {
  double c[8];
  double R2, R, Reff, inv_unused;
  double nu2_sum;
  double rho2_min, rho2_max;
  double nonfinite;
};

constexpr int kPrepBlocks = 512;
constexpr int kNuPairs = 65536;
constexpr uint64_t kNuSeed = 0x48444600ull;

// Geometry: SoA copy of the points, bounding-box centre, radius, rho^2 range
// and the ||K||_F sample.  dtype 0 = float32, 1 = float64.
hipError_t launch_prep(const void* pts, int dtype, int64_t n, int d, int64_t ld, void* x_soa,
                       int64_t ldx, int kernel, double l, double* partials, GeoDev* geo,
                       hipStream_t s);

// Geometry of two sets (X u Y) with the cross-pair ||K(X, Y)||_F sample.
// partials: at least 2 * kPrepBlocks * 18 doubles.
hipError_t launch_prep_cross(const void* ptsx, int64_t nx, int64_t ldx, const void* ptsy, int64_t ny,
                             int64_t ldy, int dtype, int d, void* soax, int64_t ldsx, void* soay,
                             int64_t ldsy, int kernel, double l, double* partials, GeoDev* geo,
                             hipStream_t s);

// Sampled pairs of the tighter degree and rank rules: pair t uses SplitMix64
// outputs 2t+1 and 2t+2 of the stream `seed` (a = out >> 11 mod n, likewise
// b).  out[0..M) = ||x_a - x_b||, out[M..2M) = rho_a^2, out[2M..3M) = rho_b^2,
// out[3M..4M) = dot of the normalised points (x - c) / Reff; idx[0..M) = a,
// idx[M..2M) = b.  Needs the geometry of launch_prep.
constexpr uint64_t kPairSeed = 0x48444601ull;
hipError_t launch_pairs(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                        uint64_t seed, int M, double* out, int32_t* idx, hipStream_t s);

// Weighted Chebyshev moments mu[k][c] = sum_i rho_i^{2k} T_c(t_i), k <= K,
// c <= 2K, written to `moments` (rows 16*nrt x cols 16*nct, binary64).
// mode 0: binary64 MFMA; 1: binary32 MFMA; 2: binary32 hi/lo split MFMA.
int gram_blocks(int64_t n);
hipError_t launch_gram(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d,
                       const GeoDev* geo, double u0, double u1, int K, int mode,
                       double* partials, double* moments, hipStream_t s);

// Refinement Gram: G2_k = (Y_k T1_k)^T (Y_k T1_k) for the selected degrees
// k = sel[0..n_sel) (binary64), written to out[i][32][32]; T1 packed per degree
// at t1_off[k] (L_k x L_k).
int gram2_blocks(int64_t n, int n_sel);
hipError_t launch_gram2(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d,
                        const GeoDev* geo, double u0, double u1, int K, const double* T1,
                        const int32_t* t1_off, const int32_t* sel, int n_sel, double* partials,
                        double* out, hipStream_t s);

// Tables of the factor-evaluation kernel.
struct BuildTables {
  const int32_t* col_of;     // loop-order iteration -> harmonic row (or -1)
  const void* chain;         // (level, b, n) -> (A, B) pairs, storage type
  const int32_t* q_len;      // per radial row: L
  const int32_t* q_off;      // per radial row: offset into q_coef
  const void* q_coef;        // radial coefficients, storage type
  int K;                     // largest kept degree: depth of the harmonic recurrences
  int S;                     // radial rows
};
hipError_t launch_build(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d,
                        const GeoDev* geo, double u0, double u1, const BuildTables& tb,
                        int prec, void* phi, int64_t ld_phi, void* q, int64_t ld_q,
                        hipStream_t s);

// Per-degree description for the contraction kernels.
struct DegDev {
  int32_t hoff;   // first harmonic row of the degree in phi
  int32_t nh;     // |H_k|
  int32_t qoff;   // first radial row in q
  int32_t s;      // s_k
  int32_t roff;   // first rank row (k, h=0, l=0)
  int32_t boff;   // first block of the degree in pass 2's batch-major copy of D W
  int32_t pad[2];
};
struct TileDev {
  int32_t deg;    // index into DegDev
  int32_t h0;     // first harmonic of the row block
  int32_t ct0;    // first 16-wide output column tile of the slice
  int32_t pad;
};
// Contraction launchers: prec is the factor's storage and arithmetic type (1 = binary32,
// 0 = binary64), io the type of V and KV (0 = float32, 1 = float64).  Supported pairs:
// (1, 0), (0, 1) and (0, 0), the last for a binary64 factor of binary32 data.
int matvec_row_block();          // harmonic rows per pass-1 row block
int matvec_col_tiles(int prec);  // 16-wide column tiles per pass-1 launch slice

// Pass 1: partial[split][row][c] = sum_{i in split} U[i,row] V[i,c]
// (row = (k,h,l), c < m16, binary64 partials).
hipError_t launch_matvec_t(const void* phi, int64_t ld_phi, const void* q, int64_t ld_q,
                           const DegDev* degs, const TileDev* tiles, int n_tiles, int max_nct,
                           const void* V, int64_t ldv, int64_t n, int m, int m16, int n_splits,
                           int64_t split_len, int64_t rank, double* partials, int prec, int io,
                           hipStream_t s);
// Pass 1, tile-major (m16 <= 64).  A wave item is one 16-row tile of one
// degree's harmonics with a range of nl <= matvec_tile_nl(prec, NCT) of its
// radial functions and the column tiles [ct0, ct0 + nct) (NCT = 1, 2 or 4
// column tiles per launch); one load of the tile's harmonic values feeds the
// MFMAs of all its (l, column) slots.  A workgroup runs one group (up to kMvtWavesPerGroup wave items whose
// radial rows lie in [q_lo, q_lo + nq), nq <= kMvtMaxNq) over one split of
// split_len points (a multiple of 32; n_splits * split_len >= n >
// (n_splits - 1) * split_len) and writes partial[split][row][c] (binary64)
// for the rank rows of its wave items, every row once per split.
struct MvtWave {
  int32_t row0;   // first harmonic row of the tile (harmonic offset of the degree + h0)
  int32_t nr;     // harmonic rows in the tile (<= 16)
  int32_t qrow;   // radial row of the first radial function
  int32_t nl;     // radial functions
  int32_t ct0;    // first column tile
  int32_t nct;    // column tiles (<= 4)
  int32_t out0;   // rank row of (h0, first radial function)
  int32_t s;      // s_k: rank-row stride between consecutive harmonics
};
// A wave item with qrow < 0 is a rank-row item (nl = 1): its rows are the rank rows
// [row0, row0 + nr) of the rank-row table (nr <= 16), each a (harmonic row, radial row, output
// row) triple, so rows of different degrees and radial functions share one tile.  Row r of its
// tile is phi_{hrow}(x) q_{qrow}(x), its output row out.
struct MvtRankRow {
  int32_t hrow;   // harmonic row in phi
  int32_t qrow;   // radial row in q
  int32_t out;    // rank row of the result
  int32_t pad;
};
constexpr int kMvtWavesPerGroup = 8;   // wavefronts per workgroup
struct MvtGroup {
  int32_t w0, nw;     // wave items [w0, w0 + nw), nw <= kMvtWavesPerGroup
  int32_t q_lo, nq;   // radial rows staged in LDS
};
// radial functions per wave item for column-tile count nct (1, 2 or 4) of the launch
int matvec_tile_nl(int prec, int nct);
constexpr int kMvtMaxNq = 32;      // staged radial rows per workgroup
size_t matvec_tile_lds_bytes(int m16, int prec);
hipError_t launch_matvec_t_tile(const void* phi, int64_t ld_phi, const void* q, int64_t ld_q,
                                const MvtWave* waves, const MvtRankRow* rank_rows, const MvtGroup* groups,
                                int n_groups, int n_splits,
                                int64_t split_len, const void* V, int64_t ldv, int64_t n, int m, int m16,
                                int64_t rank, double* partials, int prec, int io, hipStream_t s);
// Batch-major copy Wb of Wd for pass 2 (n_blocks = sum over degrees of ceil(nh / 16) s; the
// degrees' block offsets in DegDev::boff): 16 m16 values per block.
hipError_t launch_wd_batches(const DegDev* degs, int n_deg, const void* Wd, int m16, int64_t n_blocks, void* Wb,
                             int prec, hipStream_t s);
// Reduce over splits: W[row][c] = sum_split partial (binary64) and
// Wd[row][c] = lambda_row * W (storage type) for pass 2.
hipError_t launch_matvec_reduce(const double* partials, int n_splits, int64_t rank, int m16,
                                const double* lam_row, double* W, void* Wd, int prec,
                                hipStream_t s);
// Pass 2: KV[i][c] = sum_rows U[i,row] Wd[row][c].
// nz > 1: harmonic rows split into nz chunks of hchunk rows, each chunk's share
// of KV in part (nz x n x m, storage type), summed in chunk order into KV
// Wb: optional batch-major copy of Wd (launch_wd_batches; nz == 1 only), read instead of Wd.
hipError_t launch_matvec_n(const void* phi, int64_t ld_phi, const void* q, int64_t ld_q,
                           const DegDev* degs, int n_deg, int max_s, const void* Wd, const void* Wb, int m16,
                           void* KV, int64_t ldkv, int64_t n, int m, int prec, int io, int hchunk, int nz,
                           void* part, hipStream_t s);

// Adjoint by contractions (see hdf_backward).  launch_radial evaluates S
// Chebyshev series of t(rho^2) at every point: out[row][i] = scale * sum_a
// coef[q_off[row] + a] T_a(t_i), a < q_len[row] (rows padded: the launch
// writes up to the next multiple of 2 or 4 points past n).  launch_adj_combine
// forms dX[i][j] = (1/R) [sum_c w_ic KS[i][2mj + c] + v_ic KS[i][2mj + m + c]
// + 2 xt_ij (sum_c w_ic K2[i][c] + v_ic K2[i][m + c])].  prec: factor type
// (1 binary32, 0 binary64); dtype: points, W, V and dX (0 float32, 1 float64).
hipError_t launch_radial(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                         double u0, double u1, const int32_t* q_len, const int32_t* q_off, const void* coef,
                         int S, double scale, int prec, void* out, int64_t ld_out, hipStream_t s);
hipError_t launch_adj_combine(const void* x_soa, int dtype, int64_t ldx, int64_t n, int d, const GeoDev* geo,
                              const void* KS, int64_t ldks, const void* K2, int64_t ldk2, const void* Wm,
                              const void* Vm, int64_t ld, int m, void* dX, int64_t lddx, int prec, hipStream_t s);

// Fused matrix-free passes (mf_kernels.hip).  A workgroup of kMfWaves
// wavefronts takes kMfP points at a time: it evaluates their harmonics (the
// factor-evaluation recurrences, split into subtrees run by 16-lane groups)
// and radial functions into LDS and contracts them there with MFMA, so no
// factor value reaches HBM.
constexpr int kMfP = 16;                 // points per chunk
constexpr int kMfWaves = 8;              // wavefronts per workgroup
// One evaluation job of a wavefront.  A subtree of the harmonic recursion
// fixes the azimuthal index m (cosine or sine branch) and, for d >= 4, the
// index of chain level d - 2; its base b is their sum.  Subtrees of one base
// share every value below their prefixes, so a job runs the shared levels of
// base b once per point (lane = point) and writes the harmonics of a list of
// its subtrees (16-lane group g takes every fourth).  For d >= 5 a job covers
// the level d - 3 indices [n_lo, n_hi] only.
struct MfJob {
  int32_t b;        // base
  int32_t n_lo, n_hi;
  int32_t off;      // loop-order offset of the job's first harmonic within each of its subtrees
  int32_t task0;    // first entry of the job's subtrees in the per-base list (btab)
  int32_t ntask;    // subtrees of the job
  int32_t pad[2];
};
// Pass 1: one accumulator tile of a wavefront, 16 harmonics of one degree with one radial function
// (slot i: loop-order rows rows[17 i .. 17 i + 15], radial row rows[17 i + 16]): rank rows
// out0 + j s for j < nr.
struct MfSlot1 {
  int32_t row0, qrow, out0, s, nr;
  int32_t pad[3];
};
// Pass 2: one MFMA step of a wavefront, harmonics j < nv <= 4 of one degree with one radial function
// (slot i: loop-order rows rows[5 i .. 5 i + 3], radial row rows[5 i + 4]): rank rows rank0 + j s.
struct MfSlot2 {
  int32_t row0, qrow, rank0, s, nv;
  int32_t pad[3];
};
// LDS layout (byte offsets) of a fused pass: harmonic rows in loop order ((n_loop + 1) x kMfP,
// the last row zero), radial rows, V^T of the chunk (pass 1) or the per-wavefront partial
// products (pass 2), the slots' row table (n_rows 16-bit indices), the radial coefficients, the
// level d-2 recurrence pairs, two buffers of subtree prefixes (n_tasks x kMfP each) and the
// per-base subtree list.
struct MfLayout {
  int32_t phc, qc, aux, rtab, qcoef, ctop, ptab, ptab_len, btab, total;
  int32_t phc_len, qc_len, aux_len;   // values per buffer of the chunk data (two buffers when spec)
};
// spec: the wavefront-specialised kernels (2 kMfWaves wavefronts, the chunk data double-buffered)
MfLayout mf_layout(int64_t n_loop, int S, int64_t n_rows, int64_t n_qcoef, int64_t n_tasks, int d, int K, int prec,
                   int pass, bool spec);
constexpr int kMfSlots1 = 16;            // pass-1 accumulator tiles per wavefront
constexpr int kMfSlots2 = 64;            // pass-2 steps per wavefront (their D W operands stay in registers)
// A wavefront's slot list is padded to whole blocks (pass 1: padding slots have out0 = -1; pass 2:
// nv = 0) so that the kernels test the list length once per block.
constexpr int kMfBlock1 = 4;
constexpr int kMfBlock2 = 8;
constexpr int kMfMaxKs = 8;              // radial coefficients per row <= 4 kMfMaxKs (p / 2 + 1 <= 31)
struct MfArgs {
  const void* x_soa; int64_t ldx; int64_t n; int dtype; int d;
  const GeoDev* geo; double u0, u1;
  const MfJob* jobs; const int32_t* job_off;          // jobs of wavefront w: [job_off[w], job_off[w + 1])
  const int32_t* btab; int n_tasks;                   // subtrees by base: (subtree index, first harmonic)
  int64_t n_loop;                                     // harmonics of the recursion (degrees <= K)
  const void* chain; int K;                           // recurrence pairs, as for the factor evaluation
  const void* qmat; int S, S_pad, L_pad; int64_t H;   // radial coefficients, S_pad x L_pad (factor type)
  int prec;                                           // factor type: 1 binary32, 0 binary64
};
// Workgroups of one fused pass that fit on a CU at once (occupancy of the kernel with its LDS).
int mf_blocks_per_cu(const MfArgs& a, int pass, const MfLayout& lay, bool spec);
// Pass 1: partial[split][row][c] for splits of split_len points (a multiple of kMfP), rank rows of
// slot group g (slots of wavefront w: [slot_off[9 g + w], slot_off[9 g + w + 1])), columns of tile ct;
// grid n_splits x (n_groups cpl).  rows: the slots' loop-order rows (n_rows entries).
hipError_t launch_mf_t(const MfArgs& a, const MfLayout& lay, bool spec, const MfSlot1* slots, const int32_t* slot_off,
                       const int32_t* rows, int n_rows, int n_groups, int cpl, int n_splits, int64_t split_len,
                       const void* V, int64_t ldv, int m, int m16, int64_t rank, double* partials, hipStream_t s);
// Pass 2: KV = U Wd over ranges of range_len points; with n_groups > 1 each slot group writes its
// share to part (n_groups x n x m, factor type), summed in group order into KV.
hipError_t launch_mf_n(const MfArgs& a, const MfLayout& lay, bool spec, const MfSlot2* slots, const int32_t* slot_off,
                       const int32_t* rows, int n_rows, int n_groups, int cpl, int n_ranges, int64_t range_len,
                       const void* Wd, int m16, void* KV, int64_t ldkv, int m, void* part, hipStream_t s);

// Scratch of hdf_matvec_noalloc: a fixed device array per GPU (scratch.hip).
// scratch_address returns its device address on the current device (resolved
// once per device); hipErrorInvalidDevice for device ordinals >= 64.
constexpr size_t kScratchBytes = (size_t)32 << 20;
hipError_t scratch_address(void** p);

}  // namespace hdf
