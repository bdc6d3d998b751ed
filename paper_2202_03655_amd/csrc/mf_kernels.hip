// Fused matrix-free passes of the factor product (Sec. 3.6 applied to a factor that is never
// stored).  K~V = U (D (U^T V)) costs O(N r) per pass; a stored factor costs (H + S) values per
// point of HBM traffic in each pass, while its evaluation (the harmonic recurrences of Sec. 3.3
// and App. A, the radial Chebyshev series) costs O(H) arithmetic per point.  Here a workgroup
// evaluates the harmonics and radial functions of kMfP = 16 points into LDS and contracts them
// there with MFMA, chunk after chunk: the only HBM traffic is the points, V (pass 1) or KV
// (pass 2), and the split partial sums.
//
// Evaluation: the loop nest of the factor-evaluation kernel (azimuthal index outermost, then the
// chain levels d-2 .. 1, one harmonic per innermost iteration) is cut into subtrees that fix the
// azimuthal index and, for d >= 4, the index of level d-2.  Subtrees with the same remaining loop
// bound have the same shape and the same base index; a wavefront runs four of them at once, one
// per 16-lane group with one point per lane, so every lane executes the same loop trip counts and
// reads the same recurrence pairs.  Each subtree first rebuilds its prefix (the azimuthal power
// and the level d-2 recurrence up to its index) with the operations of the factor-evaluation
// kernel, in the same order, then writes its harmonics to LDS in loop order; the contraction
// reads the rows of its slots through a small table of loop-order indices.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.hpp"

namespace hdf {
namespace {

typedef float mf_floatx4 __attribute__((ext_vector_type(4)));
typedef double mf_doublex4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA.  Operands: lane r + 16 q supplies A[r][q] and B[q][r].  Accumulator element e
// of lane j + 16 g holds D[row(g, e)][j] (f32: row = 4 g + e, f64: row = g + 4 e on gfx950).
template <typename T> struct MfMma;
template <> struct MfMma<float> {
  typedef mf_floatx4 V;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return 4 * g + e; }
};
template <> struct MfMma<double> {
  typedef mf_doublex4 V;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int e) { return g + 4 * e; }
};
// The recurrence pairs are read at wave-uniform addresses from a table no kernel writes; in the
// constant address space the compiler reads them with scalar loads (the scalar cache) instead of
// vector loads whose latency every harmonic of the innermost loop would wait for.
#ifndef EMU_DEVICE_CODE
#define HDF_MF_CONST __attribute__((address_space(4)))
#else
#define HDF_MF_CONST
#endif

constexpr int kMfThreads = 64 * kMfWaves;
static_assert(kMfSlots1 % kMfBlock1 == 0 && kMfSlots2 % kMfBlock2 == 0, "slot lists are whole blocks");
// wavefronts per SIMD the register budget targets: binary32 two workgroups per CU, binary64 one
template <typename T> struct MfWavesPerEu { static constexpr int value = sizeof(T) == 4 ? 4 : 2; };

// Four consecutive LDS values (one 16-byte read in binary32, two in binary64).
template <typename T>
__device__ __forceinline__ void mf_lds4(const T* p, T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    const mf_floatx4 a = *reinterpret_cast<const mf_floatx4*>(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = a[e];
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p), b = *reinterpret_cast<const double2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
}

// Shared levels below the prefixes.  The subtrees of one base b (all azimuthal indices and level
// d-2 indices with the same sum) have identical values below their prefixes, so those levels run
// once per point and every harmonic is written for NB subtrees at once: value pre[k] * s * p with
// s the product of the shared levels above.  The recurrences and their operation order are those
// of the factor-evaluation kernel; b and rem = K - b are the same for every lane, so the
// recurrence pairs are wave-uniform loads.  Harmonic t of the loop order goes to LDS row t
// (out[k]: the element offset of subtree k's next harmonic in phc).
template <typename T, int D, int LEVEL, int NB>
struct MfChainS {
  static __device__ __forceinline__ void run(const T (&xt)[D], const T (&r2)[D], int b, int rem, T s, int K,
                                             const HDF_MF_CONST T* __restrict__ chain, T* __restrict__ phc,
                                             int (&out)[NB], const T (&pre)[NB]) {
    const HDF_MF_CONST T* cf = chain + 2 * ((LEVEL - 1) * (K + 1) + b) * (K + 1);   // (A, B) pairs
    // the pair of index nn + 1 is loaded before the levels below index nn run, so that its wait
    // is the one those levels take for their own first block of pairs
    T pm1 = 0, p = cf[0], ca = cf[2], cb = cf[3];
    MfChainS<T, D, LEVEL - 1, NB>::run(xt, r2, b, rem, s * p, K, chain, phc, out, pre);
    for (int nn = 1; nn <= rem; ++nn) {
      if (nn == 1) {
        pm1 = p;
        p = ca * xt[LEVEL - 1];
      } else {
        const T pn = ca * xt[LEVEL - 1] * p - cb * r2[LEVEL - 1] * pm1;
        pm1 = p;
        p = pn;
      }
      ca = cf[2 * nn + 2];
      cb = cf[2 * nn + 3];
      MfChainS<T, D, LEVEL - 1, NB>::run(xt, r2, b + nn, rem - nn, s * p, K, chain, phc, out, pre);
    }
  }
};
// The innermost level: one harmonic per step for each of the NB subtrees.  When it is the first
// shared level, s is exactly 1 and s * p == p, so the values equal the factor-evaluation kernel's.
template <typename T, int D, int NB>
struct MfChainS<T, D, 1, NB> {
  static __device__ __forceinline__ void emit(T* __restrict__ phc, const int (&out)[NB], const T (&pre)[NB], T v,
                                              int u) {
#pragma unroll
    for (int k = 0; k < NB; ++k) phc[out[k] + u * kMfP] = pre[k] * v;
  }
  static __device__ __forceinline__ void step(int (&out)[NB], int n) {
#pragma unroll
    for (int k = 0; k < NB; ++k) out[k] += n * kMfP;
  }
  // pairs of the chain read in blocks of kMfPairs (one scalar load and one wait per block; the
  // table is padded so that a block may run past the last row)
  static constexpr int kMfPairs = sizeof(T) == 4 ? 8 : 4;
  static __device__ __forceinline__ void load(const HDF_MF_CONST T* __restrict__ cf, T (&c)[2 * kMfPairs]) {
#pragma unroll
    for (int i = 0; i < 2 * kMfPairs; ++i) c[i] = cf[i];
  }
  static __device__ __forceinline__ void run(const T (&xt)[D], const T (&r2)[D], int b, int rem, T s, int K,
                                             const HDF_MF_CONST T* __restrict__ chain, T* __restrict__ phc,
                                             int (&out)[NB], const T (&pre)[NB]) {
    const HDF_MF_CONST T* cf = chain + 2 * b * (K + 1);
    const T x = xt[0], rr = r2[0];
    T c[2 * kMfPairs];
    load(cf, c);
    // harmonics 0 and 1; p and pm1 are read below only when rem >= 2
    T pm1 = c[0], p = c[2] * x;
    emit(phc, out, pre, s * pm1, 0);
    if (rem >= 1) emit(phc, out, pre, s * p, 1);
#pragma unroll
    for (int u = 2; u < kMfPairs; ++u) {
      if (u <= rem) {
        const T pn = c[2 * u] * x * p - c[2 * u + 1] * rr * pm1;
        pm1 = p;
        p = pn;
        emit(phc, out, pre, s * p, u);
      }
    }
    step(out, rem + 1 < kMfPairs ? rem + 1 : kMfPairs);
    for (int n0 = kMfPairs; n0 <= rem; n0 += kMfPairs) {
      load(cf + 2 * n0, c);
#pragma unroll
      for (int u = 0; u < kMfPairs; ++u) {
        if (n0 + u <= rem) {
          const T pn = c[2 * u] * x * p - c[2 * u + 1] * rr * pm1;
          pm1 = p;
          p = pn;
          emit(phc, out, pre, s * p, u);
        }
      }
      step(out, rem + 1 - n0 < kMfPairs ? rem + 1 - n0 : kMfPairs);
    }
  }
};

// Scaled coordinates of the lane's point (points past n repeat point n - 1: finite values; their V
// entries are zero and their KV rows unwritten), with the same operations as the factor-evaluation
// kernel.  fetch issues the loads of a chunk's coordinates into raw, finish turns raw into xt, r2
// and t, so the loads of the next chunk can be in flight during a chunk's work.  The specialised
// kernels fetch into rawn instead, at the start of a chunk's evaluation, and advance moves rawn to
// raw at its end: no branch separates the two, so the registers need no copies that would wait for
// the loads before the barrier.
template <typename Tin, typename T, int D>
struct MfPoint {
  T xt[D], r2[D], tt;
  Tin raw[D], rawn[D];
  __device__ __forceinline__ void fetch(const MfArgs& a, int64_t c0, int pt) {
    const Tin* __restrict__ x_soa = (const Tin*)a.x_soa;
    const int64_t i = (c0 + pt < a.n) ? c0 + pt : a.n - 1;
#pragma unroll
    for (int j = 0; j < D; ++j) raw[j] = x_soa[(int64_t)j * a.ldx + i];
  }
  __device__ __forceinline__ void fetch_next(const MfArgs& a, int64_t c0, int pt) {
    const Tin* __restrict__ x_soa = (const Tin*)a.x_soa;
    const int64_t i = (c0 + pt < a.n) ? c0 + pt : a.n - 1;
#pragma unroll
    for (int j = 0; j < D; ++j) rawn[j] = x_soa[(int64_t)j * a.ldx + i];
  }
  __device__ __forceinline__ void advance() {
#pragma unroll
    for (int j = 0; j < D; ++j) raw[j] = rawn[j];
  }
  __device__ __forceinline__ void finish(const MfArgs& a) {
    {
#pragma clang fp contract(off)
      const HDF_MF_CONST GeoDev* geo = (const HDF_MF_CONST GeoDev*)a.geo;   // scalar loads
      const double Reff = geo->Reff;
      double rho2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double v = ((double)raw[j] - geo->c[j]) / Reff;
        xt[j] = (T)v;
        rho2 = rho2 + v * v;
      }
      tt = (T)((2.0 * rho2 - a.u0 - a.u1) / (a.u1 - a.u0));
    }
    T acc = 0;
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
      acc += xt[j] * xt[j];
      r2[j] = acc;
    }
  }
};

// First subtree index of azimuthal index mm and branch sg (0 cosine, 1 sine) in the enumeration
// (mm ascending, cosine before sine, then the level d-2 index): for d >= 4 each (mm, sg) has
// K - mm + 1 subtrees, for d = 3 one.
template <int D>
__device__ __forceinline__ int mf_task_off(int mm, int sg, int K) {
  if (mm == 0) return 0;
  if constexpr (D >= 4) return (K + 1) + 2 * ((mm - 1) * (K + 1) - (mm - 1) * mm / 2) + sg * (K - mm + 1);
  else return 2 * mm - 1 + sg;
}

// Prefix of every subtree at the lane's point: cm (x_{d-1} + i x_d)^mm (real or imaginary part)
// times, for d >= 4, the level d-2 recurrence value at the subtree's index; the operations of the
// factor-evaluation kernel in its order.  Entry e = 16 mm + point; ctop holds the level d-2 pairs.
template <typename T, int D>
__device__ __forceinline__ void mf_prefix(const T (&xt)[D], const T (&r2)[D], int K, const T* __restrict__ ctop,
                                          T* __restrict__ ptab, int tid) {
  const int pt = tid & 15;
  const T inv_sqrt_2pi = (T)0.39894228040143267794, inv_sqrt_pi = (T)0.56418958354775628695;
  for (int e = tid; e < 16 * (K + 1); e += kMfThreads) {
    const int mm = e >> 4;
    T cr = 1, ci = 0;
    for (int s = 0; s < mm; ++s) {
      const T ax = xt[D - 2], ay = xt[D - 1];
      const T ncr = ax * cr - ay * ci;
      ci = ay * cr + ax * ci;
      cr = ncr;
    }
    const T cm = (mm == 0) ? inv_sqrt_2pi : inv_sqrt_pi;
    const T pc = cm * cr, ps = cm * ci;
    T* oc = ptab + mf_task_off<D>(mm, 0, K) * kMfP + pt;
    T* os = ptab + mf_task_off<D>(mm, 1, K) * kMfP + pt;
    if constexpr (D >= 4) {
      const T* cf = ctop + 2 * mm * (K + 1);
      T pm1 = 0, p = cf[0];
      oc[0] = pc * p;
      if (mm > 0) os[0] = ps * p;
      for (int nn = 1; nn <= K - mm; ++nn) {
        if (nn == 1) {
          pm1 = p;
          p = cf[2] * xt[D - 3];
        } else {
          const T ca = cf[2 * nn], cb = cf[2 * nn + 1];
          const T pn = ca * xt[D - 3] * p - cb * r2[D - 3] * pm1;
          pm1 = p;
          p = pn;
        }
        oc[nn * kMfP] = pc * p;
        if (mm > 0) os[nn * kMfP] = ps * p;
      }
    } else {
      oc[0] = pc;
      if (mm > 0) os[0] = ps;
    }
  }
}

// One pass of a job over its shared levels for NB subtrees per 16-lane group: group g takes the
// subtrees task0 + g + 4 (kb + k), k < NB, of the per-base list (clamped to the last one: repeated
// subtrees write the same values to the same rows).
template <typename T, int D, int NB>
__device__ __forceinline__ void mf_job_pass(const MfJob& jb, int kb, const T (&xt)[D], const T (&r2)[D], int K,
                                            const HDF_MF_CONST T* __restrict__ chain,
                                            const int32_t* __restrict__ btab, const T* __restrict__ ptab,
                                            T* __restrict__ phc, int pt, int grp) {
  T pre[NB];
  int out[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    int e = grp + 4 * (kb + k);
    e = e < jb.ntask ? e : jb.ntask - 1;
    const int id = btab[2 * (jb.task0 + e)], t0 = btab[2 * (jb.task0 + e) + 1];
    pre[k] = ptab[id * kMfP + pt];
    out[k] = (t0 + jb.off) * kMfP + pt;
  }
  if constexpr (D >= 5) {
    // level d-3 with base b, indices [n_lo, n_hi]; below each, the d - 4 shared levels
    // the pair of index n + 1 is loaded before the levels below index n run (one wait for both)
    const HDF_MF_CONST T* cf = chain + 2 * ((D - 4) * (K + 1) + jb.b) * (K + 1);
    T pm1 = 0, p = cf[0], ca = cf[2], cb = cf[3];
    for (int n = 0; n <= jb.n_hi; ++n) {
      if (n == 1) {
        pm1 = p;
        p = ca * xt[D - 4];
      } else if (n >= 2) {
        const T pn = ca * xt[D - 4] * p - cb * r2[D - 4] * pm1;
        pm1 = p;
        p = pn;
      }
      if (n >= 1) {
        ca = cf[2 * n + 2];
        cb = cf[2 * n + 3];
      }
      if (n >= jb.n_lo) {
        T x[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) x[k] = pre[k] * p;
        MfChainS<T, D, D - 4, NB>::run(xt, r2, jb.b + n, K - jb.b - n, (T)1, K, chain, phc, out, x);
      }
    }
  } else {
    MfChainS<T, D, 1, NB>::run(xt, r2, jb.b, K - jb.b, (T)1, K, chain, phc, out, pre);
  }
}

// Harmonics of the chunk (loop order, row t at phc + t kMfP).  A job is one base b with a range of
// level d-3 indices (d >= 5) and a list of subtrees of that base, taken in passes of up to four
// subtrees per 16-lane group (a three-subtree pass repeats one).
template <typename T, int D>
__device__ __forceinline__ void mf_jobs(const MfArgs& a, const T (&xt)[D], const T (&r2)[D],
                                        const HDF_MF_CONST MfJob* __restrict__ jobs, int j_lo, int j_hi,
                                        const int32_t* __restrict__ btab, const T* __restrict__ ptab,
                                        T* __restrict__ phc, int tid) {
  const HDF_MF_CONST T* __restrict__ chain = (const HDF_MF_CONST T*)a.chain;
  const int pt = tid & 15, grp = (tid & 63) >> 4;
  const int K = a.K;
  for (int j = j_lo; j < j_hi; ++j) {
    MfJob jb;                                                  // uniform: scalar loads
    {
      const HDF_MF_CONST MfJob* jp = jobs + j;
      jb.b = jp->b; jb.n_lo = jp->n_lo; jb.n_hi = jp->n_hi;
      jb.off = jp->off; jb.task0 = jp->task0; jb.ntask = jp->ntask;
    }
    const int per_grp = (jb.ntask + 3) >> 2;
    for (int kb = 0; kb < per_grp; kb += 4) {
      const int nb = per_grp - kb;
      if (nb >= 3) mf_job_pass<T, D, 4>(jb, kb, xt, r2, K, chain, btab, ptab, phc, pt, grp);
      else if (nb == 2) mf_job_pass<T, D, 2>(jb, kb, xt, r2, K, chain, btab, ptab, phc, pt, grp);
      else mf_job_pass<T, D, 1>(jb, kb, xt, r2, K, chain, btab, ptab, phc, pt, grp);
    }
  }
}

// Radial functions of the chunk as a small product: Q[row][point] = sum_a C[row][a] T_a(t_point),
// C the rows' Chebyshev coefficients (qmat in LDS: S_pad x L_pad, zero-padded).  Wavefront w takes
// the 16-row tiles w, w + 8, ...; its lanes form T_a(t) of their point by the three-term recurrence
// (lane r + 16 q supplies B[q][r] = T_{4 ks + q}(t_r) of k-step ks) and L_pad / 4 MFMAs give the tile.
template <typename T>
__device__ __forceinline__ void mf_radial(const MfArgs& a, T tt, const T* __restrict__ qmat, T* __restrict__ qc,
                                          int tid) {
  const int lane = tid & 63, r = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int RT = a.S_pad >> 4, KS = a.L_pad >> 2;
  if (wave >= RT) return;                                    // uniform
  T bv[kMfMaxKs];
  {
    T t0 = 1, t1 = tt;
#pragma unroll
    for (int ks = 0; ks < kMfMaxKs; ++ks) {
      if (ks < KS) {
        const T v2 = 2 * tt * t1 - t0, v3 = 2 * tt * v2 - t1;
        bv[ks] = q == 0 ? t0 : (q == 1 ? t1 : (q == 2 ? v2 : v3));
        t0 = 2 * tt * v3 - v2;
        t1 = 2 * tt * t0 - v3;
      }
    }
  }
  for (int tl = wave; tl < RT; tl += kMfWaves) {
    typename MfMma<T>::V acc = {0, 0, 0, 0};
    const T* crow = qmat + (tl * 16 + r) * a.L_pad + q;
#pragma unroll
    for (int ks = 0; ks < kMfMaxKs; ++ks)
      if (ks < KS) acc = MfMma<T>::run(crow[4 * ks], bv[ks], acc);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = tl * 16 + MfMma<T>::row(q, e);
      if (row < a.S) qc[row * kMfP + r] = acc[e];
    }
  }
}

// The evaluation of one chunk, software-pipelined: on entry pnt holds the chunk's points, its raw
// coordinates the next chunk's (if any), and ptab_cur the chunk's subtree prefixes (written before
// the last barrier).  The harmonics and radial functions go to phc and qc; pnt advances to the next
// chunk, the loads of the chunk after it (at c_next2) are issued, and the next chunk's prefixes go
// to ptab_next (read after the next barrier).  With PIPE (the specialised kernels) the loads are
// issued first, for every chunk (past the points they read point n - 1).  Run by the kMfThreads
// threads of the evaluating wavefronts.
template <typename Tin, typename T, int D, bool PIPE>
__device__ __forceinline__ void mf_eval(const MfArgs& a, MfPoint<Tin, T, D>& pnt, bool has_next, int64_t c_next2,
                                        bool has_next2, int j_lo, int j_hi, const T* __restrict__ ctop,
                                        const T* __restrict__ ptab_cur, T* __restrict__ ptab_next,
                                        T* __restrict__ phc, T* __restrict__ qc, const T* __restrict__ qcoef,
                                        const int32_t* __restrict__ btab, int tid) {
  if constexpr (PIPE) pnt.fetch_next(a, c_next2, tid & 15);
  mf_jobs<T, D>(a, pnt.xt, pnt.r2, (const HDF_MF_CONST MfJob*)a.jobs, j_lo, j_hi, btab, ptab_cur, phc, tid);
  mf_radial<T>(a, pnt.tt, qcoef, qc, tid);
  if constexpr (PIPE) {
    pnt.finish(a);
    pnt.advance();
    if (has_next) mf_prefix<T, D>(pnt.xt, pnt.r2, a.K, ctop, ptab_next, tid);
  } else if (has_next) {
    pnt.finish(a);
    if (has_next2) pnt.fetch(a, c_next2, tid & 15);
    mf_prefix<T, D>(pnt.xt, pnt.r2, a.K, ctop, ptab_next, tid);
  }
}

// Tables every fused pass stages once per workgroup: the slots' harmonic rows (loop-order indices)
// and zeros in the 16 pad rows past the harmonics.
template <typename T>
__device__ __forceinline__ void mf_stage_tables(const MfArgs& a, int D, const int32_t* __restrict__ rows,
                                                int n_rows, uint16_t* rtab, T* phc, int n_phc, int phc_len,
                                                T* qcoef, T* ctop, int32_t* btab, int tid, int nthr) {
  for (int e = tid; e < n_rows; e += nthr) rtab[e] = (uint16_t)rows[e];
  for (int e = tid; e < 2 * a.n_tasks; e += nthr) btab[e] = a.btab[e];
  for (int e = tid; e < n_phc * kMfP; e += nthr) phc[(e / kMfP) * phc_len + a.n_loop * kMfP + e % kMfP] = 0;
  for (int e = tid; e < a.S_pad * a.L_pad; e += nthr) qcoef[e] = ((const T*)a.qmat)[e];
  if (D >= 4) {                                   // level d-2 recurrence pairs
    const T* src = (const T*)a.chain + (int64_t)2 * (D - 3) * (a.K + 1) * (a.K + 1);
    for (int e = tid; e < 2 * (a.K + 1) * (a.K + 1); e += nthr) ctop[e] = src[e];
  }
}

// Buffer sets of a fused pass: SPEC kernels double-buffer the chunk data (harmonics, radial rows,
// V^T or the partial products) so that half of the wavefronts evaluate chunk i + 1 while the other
// half contracts chunk i; the plain kernels alternate the two phases with all wavefronts.
template <bool SPEC> struct MfMode {
  static constexpr int threads = SPEC ? 2 * kMfThreads : kMfThreads;
  static constexpr int nbuf = SPEC ? 2 : 1;
};
template <typename T, bool SPEC> struct MfWaves {
  static constexpr int value = SPEC ? 4 : MfWavesPerEu<T>::value;
};
// In the specialised kernels the two roles run separate loops with the same number of barriers (on
// the device every s_barrier of a workgroup counts alike); the CPU emulation of the kernels is told
// that the two call sites are one barrier.
#ifndef EMU_DEVICE_CODE
#define HDF_MF_ROLE_BARRIER() __syncthreads()
#else
static int mf_role_barrier_site;
#define HDF_MF_ROLE_BARRIER() emu::syncthreads_at(&mf_role_barrier_site)
#endif

// One chunk of pass 1's contraction by wavefront w8: lane r + 16 q reads the four values of harmonic
// row rs[r] at points 4q .. 4q + 3 with one LDS read and feeds the four MFMA k-steps with them
// (k-step s takes point 4q + s as its k-index q; V^T is read the same way, so the sum over the
// chunk's points is complete).  Slots in blocks of kMfBlock1 (the host pads every wavefront's list
// to whole blocks), one uniform test per block so the block's LDS reads can be issued together.
template <typename T, int NS>
__device__ __forceinline__ void mf_mma1(typename MfMma<T>::V (&acc)[NS], const T* __restrict__ phc,
                                        const T* __restrict__ qc, const T* __restrict__ vc,
                                        const uint16_t* __restrict__ rtab, int s_lo, int ns, int r, int q) {
  T vb[4];
  mf_lds4<T>(vc + r * kMfP + 4 * q, vb);
#pragma unroll
  for (int tb = 0; tb < NS; tb += kMfBlock1) {
    if (tb < ns) {
#pragma unroll
      for (int u = 0; u < kMfBlock1; ++u) {
        const int t = tb + u;
        const uint16_t* rs = rtab + (s_lo + t) * 17;            // the slot's 16 rows, then its radial row
        T a4[4], q4[4];
        mf_lds4<T>(phc + rs[r] * kMfP + 4 * q, a4);
        mf_lds4<T>(qc + rs[16] * kMfP + 4 * q, q4);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[t] = MfMma<T>::run(a4[s] * q4[s], vb[s], acc[t]);
      }
    }
  }
}

// V^T of a chunk, columns of tile ct (threads tid < 256 of the evaluating wavefronts): fetch loads
// the thread's value of the chunk at c0 into a register one chunk ahead of its use, put writes it
// to LDS (zero past the range or past m), so the load's latency is hidden behind a chunk's evaluation.
template <typename Tin, typename T>
struct MfVStage {
  Tin v;
  __device__ __forceinline__ void fetch(const Tin* __restrict__ V, int64_t ldv, int64_t n, int m, int ct, int64_t c0,
                                        int tid) {
    if (tid < 16 * kMfP) {
      const int pp = tid >> 4, c = tid & 15, col = ct * 16 + c;
      const int64_t i = c0 + pp;
      const int64_t ic = i < n ? i : n - 1;
      v = V[ic * ldv + (col < m ? col : 0)];
    }
  }
  __device__ __forceinline__ void put(int64_t p_end, int m, int ct, int64_t c0, T* __restrict__ vc, int tid) const {
    if (tid < 16 * kMfP) {
      const int pp = tid >> 4, c = tid & 15, col = ct * 16 + c;
      vc[c * kMfP + pp] = (c0 + pp < p_end && col < m) ? (T)v : (T)0;
    }
  }
};

// Pass 1.  Block (split, y): slot group y / cpl, column tile y % cpl.  Each contracting wavefront
// keeps its slots' accumulator tiles for the whole split.
template <typename Tin, typename T, int D, bool SPEC>
__global__ void __launch_bounds__(MfMode<SPEC>::threads)
__attribute__((amdgpu_waves_per_eu(MfWaves<T, SPEC>::value, 8)))
k_mf_t(MfArgs a, MfLayout lay, const MfSlot1* __restrict__ slots, const int32_t* __restrict__ slot_off,
       const int32_t* __restrict__ rows, int n_rows, int cpl, int64_t split_len, const Tin* __restrict__ V,
       int64_t ldv, int m, int m16, int64_t rank, double* __restrict__ part) {
  typedef typename MfMma<T>::V Acc;
  constexpr int NS = kMfSlots1;
  extern __shared__ unsigned char smem_raw[];
  T* phc = reinterpret_cast<T*>(smem_raw + lay.phc);            // nbuf buffers of lay.phc_len values
  T* qc = reinterpret_cast<T*>(smem_raw + lay.qc);
  T* vc = reinterpret_cast<T*>(smem_raw + lay.aux);
  uint16_t* rtab = reinterpret_cast<uint16_t*>(smem_raw + lay.rtab);
  T* qcoef = reinterpret_cast<T*>(smem_raw + lay.qcoef);
  T* ctop = reinterpret_cast<T*>(smem_raw + lay.ctop);
  T* ptab = reinterpret_cast<T*>(smem_raw + lay.ptab);         // two buffers of lay.ptab_len values
  int32_t* btab = reinterpret_cast<int32_t*>(smem_raw + lay.btab);
  const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int w8 = wave & (kMfWaves - 1);
  const bool evalw = !SPEC || wave < kMfWaves;       // uniform
  const bool mmaw = !SPEC || wave >= kMfWaves;
  const int etid = tid & (kMfThreads - 1);
  const int split = blockIdx.x, gi = blockIdx.y / cpl, ct = blockIdx.y - gi * cpl;
  const int64_t p_begin = (int64_t)split * split_len;
  if (p_begin >= a.n) return;                     // whole workgroup, before any barrier
  const int64_t p_end = (p_begin + split_len < a.n) ? p_begin + split_len : a.n;
  const int nch = (int)((p_end - p_begin + kMfP - 1) / kMfP);
  mf_stage_tables<T>(a, D, rows, n_rows, rtab, phc, MfMode<SPEC>::nbuf, lay.phc_len, qcoef, ctop, btab, tid,
                     MfMode<SPEC>::threads);
  MfPoint<Tin, T, D> pnt;
  MfVStage<Tin, T> vs;
  if (evalw) {
    if constexpr (SPEC) {
      pnt.fetch_next(a, p_begin, etid & 15);
      pnt.advance();
      pnt.finish(a);
      pnt.fetch_next(a, p_begin + kMfP, etid & 15);
      pnt.advance();
    } else {
      pnt.fetch(a, p_begin, etid & 15);
      pnt.finish(a);
      if (nch > 1) pnt.fetch(a, p_begin + kMfP, etid & 15);
    }
    if constexpr (SPEC) vs.fetch(V, ldv, a.n, m, ct, p_begin, etid);
  }
  __syncthreads();                                // tables staged
  const int s_lo = slot_off[gi * (kMfWaves + 1) + w8];
  const int ns = slot_off[gi * (kMfWaves + 1) + w8 + 1] - s_lo;
  const int j_lo = a.job_off[w8], j_hi = a.job_off[w8 + 1];
  Acc acc[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) acc[t] = Acc{0, 0, 0, 0};
  if constexpr (SPEC) {
    // iteration it: the evaluating wavefronts fill buffer it & 1 with chunk it while the contracting
    // ones read chunk it - 1 from the other; nch + 1 barriers in either role
    if (evalw) {
      // no branch inside the loop body, so the prefetched registers need no copies at its end
      mf_prefix<T, D>(pnt.xt, pnt.r2, a.K, ctop, ptab, etid);
      for (int it = 0; it < nch; ++it) {
        HDF_MF_ROLE_BARRIER();
        const int b = it & 1;
        const int64_t c0 = p_begin + (int64_t)it * kMfP;
        mf_eval<Tin, T, D, true>(a, pnt, it + 1 < nch, c0 + 2 * kMfP, it + 2 < nch, j_lo, j_hi, ctop,
                                 ptab + b * lay.ptab_len, ptab + (b ^ 1) * lay.ptab_len, phc + b * lay.phc_len,
                                 qc + b * lay.qc_len, qcoef, btab, etid);
        vs.put(p_end, m, ct, c0, vc + b * lay.aux_len, etid);
        vs.fetch(V, ldv, a.n, m, ct, c0 + kMfP, etid);        // past the points: row n - 1, unused
      }
      HDF_MF_ROLE_BARRIER();
    } else {
      for (int it = 0; it <= nch; ++it) {
        HDF_MF_ROLE_BARRIER();
        if (it >= 1) {
          const int b = (it - 1) & 1;
          mf_mma1<T, NS>(acc, phc + b * lay.phc_len, qc + b * lay.qc_len, vc + b * lay.aux_len, rtab, s_lo, ns, r,
                         q);
        }
      }
    }
  } else {
    mf_prefix<T, D>(pnt.xt, pnt.r2, a.K, ctop, ptab, etid);
    for (int it = 0; it < nch; ++it) {
      const int64_t c0 = p_begin + (int64_t)it * kMfP;
      __syncthreads();                            // the previous chunk's reads are done
      mf_eval<Tin, T, D, false>(a, pnt, it + 1 < nch, c0 + 2 * kMfP, it + 2 < nch, j_lo, j_hi, ctop,
                                ptab + (it & 1) * lay.ptab_len, ptab + ((it & 1) ^ 1) * lay.ptab_len, phc, qc,
                                qcoef, btab, tid);
      vs.fetch(V, ldv, a.n, m, ct, c0, tid);
      vs.put(p_end, m, ct, c0, vc, tid);
      __syncthreads();
      mf_mma1<T, NS>(acc, phc, qc, vc, rtab, s_lo, ns, r, q);
    }
  }
  if (mmaw) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if (t < ns) {
        const MfSlot1 sd = slots[s_lo + t];
        if (sd.out0 < 0) continue;                   // padding slot
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = MfMma<T>::row(q, e);
          if (row < sd.nr)
            part[((int64_t)split * rank + sd.out0 + (int64_t)row * sd.s) * m16 + ct * 16 + r] = (double)acc[t][e];
        }
      }
    }
  }
}

// One chunk of pass 2's contraction by wavefront w8: U[point r][rank q] = phi_{rs[q]}(r) q_l(r)
// from LDS against the wavefront's D W operands, one 16 x 16 tile of KV, stored to red for the
// fixed-order sum over the eight wavefronts.  Slots in blocks of kMfBlock2 (padded lists; padding
// slots have zero D W operands).
template <typename T, int NS>
__device__ __forceinline__ void mf_mma2(const T (&wd)[NS], const T* __restrict__ phc, const T* __restrict__ qc,
                                        const uint16_t* __restrict__ rtab, int s_lo, int ns, int r, int q,
                                        T* __restrict__ red_w) {
  typename MfMma<T>::V acc = {0, 0, 0, 0};
#pragma unroll
  for (int tb = 0; tb < NS; tb += kMfBlock2) {
    if (tb < ns) {
#pragma unroll
      for (int u = 0; u < kMfBlock2; ++u) {
        const int t = tb + u;
        const uint16_t* rs = rtab + (s_lo + t) * 5;             // the slot's 4 rows, then its radial row
        const T v = phc[rs[q] * kMfP + r] * qc[rs[4] * kMfP + r];
        acc = MfMma<T>::run(v, wd[t], acc);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) red_w[MfMma<T>::row(q, e) * 16 + r] = acc[e];
}

// The eight wavefronts' tiles of the chunk at c0, added in a fixed order, into KV (or part).
template <typename Tin, typename T>
__device__ __forceinline__ void mf_reduce2(const T* __restrict__ red, int64_t c0, int64_t p_end, int m, int ct,
                                           int n_groups, int gi, int64_t n, Tin* __restrict__ KV, int64_t ldkv,
                                           T* __restrict__ part, int t) {
  if (t < 256) {
    const int pp = t >> 4, c = t & 15, col = ct * 16 + c;
    T sum = 0;
#pragma unroll
    for (int w = 0; w < kMfWaves; ++w) sum += red[w * 256 + pp * 16 + c];
    const int64_t i = c0 + pp;
    if (i < p_end && col < m) {
      if (n_groups == 1) KV[i * ldkv + col] = (Tin)sum;
      else part[((int64_t)gi * n + i) * m + col] = sum;
    }
  }
}

// Pass 2.  Block (range, y): slot group y / cpl, column tile y % cpl.  A contracting wavefront's
// D W operands (its slots' rank rows, this column tile) are loaded once into registers.
template <typename Tin, typename T, int D, bool SPEC>
__global__ void __launch_bounds__(MfMode<SPEC>::threads)
__attribute__((amdgpu_waves_per_eu(MfWaves<T, SPEC>::value, 8)))
k_mf_n(MfArgs a, MfLayout lay, const MfSlot2* __restrict__ slots, const int32_t* __restrict__ slot_off,
       const int32_t* __restrict__ rows, int n_rows, int cpl, int64_t range_len, const T* __restrict__ Wd, int m16,
       Tin* __restrict__ KV, int64_t ldkv, int m, int n_groups, T* __restrict__ part) {
  constexpr int NS = kMfSlots2;
  extern __shared__ unsigned char smem_raw[];
  T* phc = reinterpret_cast<T*>(smem_raw + lay.phc);
  T* qc = reinterpret_cast<T*>(smem_raw + lay.qc);
  T* red = reinterpret_cast<T*>(smem_raw + lay.aux);            // nbuf buffers of lay.aux_len values
  uint16_t* rtab = reinterpret_cast<uint16_t*>(smem_raw + lay.rtab);
  T* qcoef = reinterpret_cast<T*>(smem_raw + lay.qcoef);
  T* ctop = reinterpret_cast<T*>(smem_raw + lay.ctop);
  T* ptab = reinterpret_cast<T*>(smem_raw + lay.ptab);         // two buffers of lay.ptab_len values
  int32_t* btab = reinterpret_cast<int32_t*>(smem_raw + lay.btab);
  const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int w8 = wave & (kMfWaves - 1);
  const bool evalw = !SPEC || wave < kMfWaves;       // uniform
  const bool mmaw = !SPEC || wave >= kMfWaves;
  const int etid = tid & (kMfThreads - 1);
  const int range = blockIdx.x, gi = blockIdx.y / cpl, ct = blockIdx.y - gi * cpl;
  const int64_t p_begin = (int64_t)range * range_len;
  if (p_begin >= a.n) return;                     // whole workgroup, before any barrier
  const int64_t p_end = (p_begin + range_len < a.n) ? p_begin + range_len : a.n;
  const int nch = (int)((p_end - p_begin + kMfP - 1) / kMfP);
  mf_stage_tables<T>(a, D, rows, n_rows, rtab, phc, MfMode<SPEC>::nbuf, lay.phc_len, qcoef, ctop, btab, tid,
                     MfMode<SPEC>::threads);
  MfPoint<Tin, T, D> pnt;
  if (evalw) {
    if constexpr (SPEC) {
      pnt.fetch_next(a, p_begin, etid & 15);
      pnt.advance();
      pnt.finish(a);
      pnt.fetch_next(a, p_begin + kMfP, etid & 15);
      pnt.advance();
    } else {
      pnt.fetch(a, p_begin, etid & 15);
      pnt.finish(a);
      if (nch > 1) pnt.fetch(a, p_begin + kMfP, etid & 15);
    }
  }
  __syncthreads();                                // tables staged
  const int s_lo = slot_off[gi * (kMfWaves + 1) + w8];
  const int ns = slot_off[gi * (kMfWaves + 1) + w8 + 1] - s_lo;
  const int j_lo = a.job_off[w8], j_hi = a.job_off[w8 + 1];
  // B[q][r] = (D W)[rank0 + q s][ct 16 + r], zero for rows past the degree
  T wd[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    wd[t] = 0;
    if (mmaw && t < ns) {
      const MfSlot2 sd = slots[s_lo + t];
      if (q < sd.nv) wd[t] = Wd[((int64_t)sd.rank0 + (int64_t)q * sd.s) * m16 + ct * 16 + r];
    }
  }
  if constexpr (SPEC) {
    // iteration it: evaluate chunk it, contract chunk it - 1, add up chunk it - 2; nch + 2 barriers
    // in either role
    if (evalw) {
      mf_prefix<T, D>(pnt.xt, pnt.r2, a.K, ctop, ptab, etid);
      for (int it = 0; it < nch; ++it) {
        HDF_MF_ROLE_BARRIER();
        const int b = it & 1;
        mf_eval<Tin, T, D, true>(a, pnt, it + 1 < nch, p_begin + (int64_t)(it + 2) * kMfP, it + 2 < nch, j_lo,
                                 j_hi, ctop, ptab + b * lay.ptab_len, ptab + (b ^ 1) * lay.ptab_len,
                                 phc + b * lay.phc_len, qc + b * lay.qc_len, qcoef, btab, etid);
      }
      HDF_MF_ROLE_BARRIER();
      HDF_MF_ROLE_BARRIER();
    } else {
      for (int it = 0; it <= nch + 1; ++it) {
        HDF_MF_ROLE_BARRIER();
        if (it >= 2)
          mf_reduce2<Tin, T>(red + (it & 1) * lay.aux_len, p_begin + (int64_t)(it - 2) * kMfP, p_end, m, ct,
                             n_groups, gi, a.n, KV, ldkv, part, etid);
        if (it >= 1 && it <= nch) {
          const int b = (it - 1) & 1;
          mf_mma2<T, NS>(wd, phc + b * lay.phc_len, qc + b * lay.qc_len, rtab, s_lo, ns, r, q,
                         red + b * lay.aux_len + w8 * 256);
        }
      }
    }
  } else {
    mf_prefix<T, D>(pnt.xt, pnt.r2, a.K, ctop, ptab, etid);
    for (int it = 0; it < nch; ++it) {
      const int64_t c0 = p_begin + (int64_t)it * kMfP;
      __syncthreads();                            // the previous chunk's reads are done
      mf_eval<Tin, T, D, false>(a, pnt, it + 1 < nch, c0 + 2 * kMfP, it + 2 < nch, j_lo, j_hi, ctop,
                         ptab + (it & 1) * lay.ptab_len, ptab + ((it & 1) ^ 1) * lay.ptab_len, phc, qc, qcoef,
                         btab, tid);
      __syncthreads();
      mf_mma2<T, NS>(wd, phc, qc, rtab, s_lo, ns, r, q, red + wave * 256);
      __syncthreads();
      mf_reduce2<Tin, T>(red, c0, p_end, m, ct, n_groups, gi, a.n, KV, ldkv, part, tid);
    }
  }
}

// KV = sum over slot groups of part (fixed order).
template <typename T, typename Tin>
__global__ void __launch_bounds__(256) k_mf_sum(const T* __restrict__ part, int n_groups, int64_t n, int m,
                                                Tin* __restrict__ KV, int64_t ldkv) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m;
  const int c = (int)(e - i * m);
  T s = 0;
  for (int g = 0; g < n_groups; ++g) s += part[(int64_t)g * n * m + e];
  KV[i * ldkv + c] = (Tin)s;
}

int64_t mf_round16(int64_t b) { return (b + 15) / 16 * 16; }

}  // namespace

MfLayout mf_layout(int64_t n_loop, int S, int64_t n_rows, int64_t n_qcoef, int64_t n_tasks, int d, int K, int prec,
                   int pass, bool spec) {
  const int64_t el = prec == 1 ? 4 : 8;
  const int nbuf = spec ? 2 : 1;
  int64_t off = 0;
  MfLayout l{};
  l.phc_len = (int32_t)(mf_round16((n_loop + 1) * kMfP * el) / el);
  l.qc_len = (int32_t)(mf_round16((int64_t)S * kMfP * el) / el);
  l.aux_len = (int32_t)(mf_round16((pass == 1 ? 16 * kMfP : kMfWaves * 256) * el) / el);
  l.phc = (int32_t)off;
  off += nbuf * (int64_t)l.phc_len * el;
  l.qc = (int32_t)off;
  off += nbuf * (int64_t)l.qc_len * el;
  l.aux = (int32_t)off;
  off += nbuf * (int64_t)l.aux_len * el;
  l.rtab = (int32_t)off;
  off += mf_round16(n_rows * 2);
  l.qcoef = (int32_t)off;
  off += mf_round16(n_qcoef * el);                       // S_pad x L_pad radial coefficients
  l.ctop = (int32_t)off;
  off += mf_round16((d >= 4 ? 2 * (int64_t)(K + 1) * (K + 1) : 1) * el);
  l.ptab_len = (int32_t)(n_tasks * kMfP);
  l.ptab = (int32_t)off;
  off += mf_round16(2 * n_tasks * kMfP * el);
  l.btab = (int32_t)off;
  off += mf_round16(2 * n_tasks * 4);
  l.total = off > (int64_t)0x7fffffff ? 0x7fffffff : (int32_t)off;
  return l;
}

namespace {
// (points and product type, factor type, dimension) of a launch
template <typename TIN, typename T, int DD> struct MfTypes {
  typedef TIN Tin;
  typedef T Tf;
  static constexpr int D = DD;
};
template <int DD, typename F>
hipError_t mf_dispatch_types(const MfArgs& a, F& f) {
  if (a.prec == 1 && a.dtype == 0) return f(MfTypes<float, float, DD>{});
  if (a.prec == 0 && a.dtype == 1) return f(MfTypes<double, double, DD>{});
  if (a.prec == 0 && a.dtype == 0) return f(MfTypes<float, double, DD>{});
  return hipErrorInvalidValue;
}
// the wavefront-specialised kernels exist for binary32 factors (their registers allow four
// wavefronts per SIMD); binary64 factors use the plain ones
template <typename T, bool SPEC> struct MfSpecOk { static constexpr bool value = !SPEC || sizeof(T) == 4; };
template <typename F>
hipError_t mf_dispatch(const MfArgs& a, F&& f) {
  switch (a.d) {
    case 3: return mf_dispatch_types<3>(a, f);
    case 4: return mf_dispatch_types<4>(a, f);
    case 5: return mf_dispatch_types<5>(a, f);
    case 6: return mf_dispatch_types<6>(a, f);
    case 7: return mf_dispatch_types<7>(a, f);
    case 8: return mf_dispatch_types<8>(a, f);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace

int mf_blocks_per_cu(const MfArgs& a, int pass, const MfLayout& lay, bool spec) {
  int nb = 0;
  const hipError_t e = mf_dispatch(a, [&](auto ty) -> hipError_t {
    typedef typename decltype(ty)::Tin Tin;
    typedef typename decltype(ty)::Tf T;
    constexpr int D = decltype(ty)::D;
    if (spec) {
      if constexpr (MfSpecOk<T, true>::value) {
        const void* fn = pass == 1 ? reinterpret_cast<const void*>(&k_mf_t<Tin, T, D, true>)
                                   : reinterpret_cast<const void*>(&k_mf_n<Tin, T, D, true>);
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 2 * kMfThreads, (size_t)lay.total);
      }
      return hipErrorInvalidValue;
    }
    const void* fn = pass == 1 ? reinterpret_cast<const void*>(&k_mf_t<Tin, T, D, false>)
                               : reinterpret_cast<const void*>(&k_mf_n<Tin, T, D, false>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kMfThreads, (size_t)lay.total);
  });
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

hipError_t launch_mf_t(const MfArgs& a, const MfLayout& lay, bool spec, const MfSlot1* slots, const int32_t* slot_off,
                       const int32_t* rows, int n_rows, int n_groups, int cpl, int n_splits, int64_t split_len,
                       const void* V, int64_t ldv, int m, int m16, int64_t rank, double* partials, hipStream_t s) {
  if (split_len % kMfP != 0 || n_splits < 1 || (int64_t)(n_splits - 1) * split_len >= a.n ||
      (int64_t)n_splits * split_len < a.n || cpl < 1 || cpl * 16 != m16 || n_groups < 1 || a.H < 1)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_splits, (unsigned)(n_groups * cpl));
  return mf_dispatch(a, [&](auto ty) -> hipError_t {
    typedef typename decltype(ty)::Tin Tin;
    typedef typename decltype(ty)::Tf T;
    constexpr int D = decltype(ty)::D;
    if (spec) {
      if constexpr (MfSpecOk<T, true>::value) {
        k_mf_t<Tin, T, D, true><<<grid, 2 * kMfThreads, (size_t)lay.total, s>>>(
            a, lay, slots, slot_off, rows, n_rows, cpl, split_len, (const Tin*)V, ldv, m, m16, rank, partials);
        return hipGetLastError();
      }
      return hipErrorInvalidValue;
    }
    k_mf_t<Tin, T, D, false><<<grid, kMfThreads, (size_t)lay.total, s>>>(
        a, lay, slots, slot_off, rows, n_rows, cpl, split_len, (const Tin*)V, ldv, m, m16, rank, partials);
    return hipGetLastError();
  });
}

hipError_t launch_mf_n(const MfArgs& a, const MfLayout& lay, bool spec, const MfSlot2* slots, const int32_t* slot_off,
                       const int32_t* rows, int n_rows, int n_groups, int cpl, int n_ranges, int64_t range_len,
                       const void* Wd, int m16, void* KV, int64_t ldkv, int m, void* part, hipStream_t s) {
  if (range_len % kMfP != 0 || n_ranges < 1 || (int64_t)(n_ranges - 1) * range_len >= a.n ||
      (int64_t)n_ranges * range_len < a.n || cpl < 1 || cpl * 16 != m16 || n_groups < 1 || a.H < 1 ||
      (n_groups > 1 && !part))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_ranges, (unsigned)(n_groups * cpl));
  const unsigned nb = (unsigned)((a.n * m + 255) / 256);
  return mf_dispatch(a, [&](auto ty) -> hipError_t {
    typedef typename decltype(ty)::Tin Tin;
    typedef typename decltype(ty)::Tf T;
    constexpr int D = decltype(ty)::D;
    if (spec) {
      if constexpr (MfSpecOk<T, true>::value) {
        k_mf_n<Tin, T, D, true><<<grid, 2 * kMfThreads, (size_t)lay.total, s>>>(
            a, lay, slots, slot_off, rows, n_rows, cpl, range_len, (const T*)Wd, m16, (Tin*)KV, ldkv, m, n_groups,
            (T*)part);
      } else {
        return hipErrorInvalidValue;
      }
    } else {
      k_mf_n<Tin, T, D, false><<<grid, kMfThreads, (size_t)lay.total, s>>>(
          a, lay, slots, slot_off, rows, n_rows, cpl, range_len, (const T*)Wd, m16, (Tin*)KV, ldkv, m, n_groups,
          (T*)part);
    }
    if (n_groups > 1) k_mf_sum<T, Tin><<<nb, 256, 0, s>>>((const T*)part, n_groups, a.n, m, (Tin*)KV, ldkv);
    return hipGetLastError();
  });
}

}  // namespace hdf
