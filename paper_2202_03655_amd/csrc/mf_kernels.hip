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
// bound have the same shape; a wavefront runs four of them at once, one per 16-lane group with
// one point per lane, so every lane executes the same loop trip counts.  Each subtree first
// rebuilds its prefix (the azimuthal power and the level d-2 recurrence up to its index) with the
// operations of the factor-evaluation kernel, in the same order, then writes every harmonic of
// its subtree to the LDS row that the loop-order table names.
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
template <typename T> struct MfPair;
template <> struct MfPair<float> { typedef float2 type; };
template <> struct MfPair<double> { typedef double2 type; };

constexpr int kMfThreads = 64 * kMfWaves;
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

// Chain levels LEVEL .. 1 below a fixed prefix: the same two-term recurrences and operation order
// as the factor-evaluation kernel.  rem = K - b is the same for every lane of the wavefront.
template <typename T, int D, int LEVEL>
struct MfChain {
  typedef typename MfPair<T>::type P2;
  static __device__ __forceinline__ void run(const T (&xt)[D], const T (&r2)[D], int b, int rem, T prefix, int K,
                                             const P2* __restrict__ chain, const int32_t* __restrict__ cmap,
                                             int& t, T* __restrict__ phc, int pt, bool valid) {
    const P2* cf = chain + ((LEVEL - 1) * (K + 1) + b) * (K + 1);
    T pm1 = 0, p = cf[0].x;
    for (int nn = 0; nn <= rem; ++nn) {
      if (nn == 1) {
        pm1 = p;
        p = cf[1].x * xt[LEVEL - 1];
      } else if (nn >= 2) {
        const P2 c = cf[nn];
        const T pn = c.x * xt[LEVEL - 1] * p - c.y * r2[LEVEL - 1] * pm1;
        pm1 = p;
        p = pn;
      }
      MfChain<T, D, LEVEL - 1>::run(xt, r2, b + nn, rem - nn, prefix * p, K, chain, cmap, t, phc, pt, valid);
    }
  }
};
template <typename T, int D>
struct MfChain<T, D, 0> {
  typedef typename MfPair<T>::type P2;
  static __device__ __forceinline__ void run(const T (&)[D], const T (&)[D], int, int, T prefix, int,
                                             const P2* __restrict__, const int32_t* __restrict__ cmap, int& t,
                                             T* __restrict__ phc, int pt, bool valid) {
    const int row = cmap[t++];
    if (valid && row >= 0) phc[row * kMfP + pt] = prefix;
  }
};

// Harmonics and radial functions of points [c0, c0 + kMfP) into LDS (rows of kMfP values).  Points
// past n repeat point n - 1 (finite values; their V entries are zero and their KV rows unwritten).
template <typename Tin, typename T, int D>
__device__ __forceinline__ void mf_eval(const MfArgs& a, int64_t c0, const MfJob* __restrict__ jobs, int j_lo,
                                        int j_hi, const typename MfPair<T>::type* __restrict__ chain,
                                        const int32_t* __restrict__ cmap, T* __restrict__ phc, T* __restrict__ qc,
                                        int tid) {
  typedef typename MfPair<T>::type P2;
  const Tin* __restrict__ x_soa = (const Tin*)a.x_soa;
  const int lane = tid & 63, pt = lane & 15, grp = lane >> 4;
  const int K = a.K;
  T xt[D], r2[D], tt;
  {
#pragma clang fp contract(off)
    const GeoDev* geo = a.geo;
    const double Reff = geo->Reff;
    const int64_t i = (c0 + pt < a.n) ? c0 + pt : a.n - 1;
    double rho2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double v = ((double)x_soa[(int64_t)j * a.ldx + i] - geo->c[j]) / Reff;
      xt[j] = (T)v;
      rho2 = rho2 + v * v;
    }
    tt = (T)((2.0 * rho2 - a.u0 - a.u1) / (a.u1 - a.u0));
  }
  {
    T acc = 0;
#pragma unroll
    for (int j = D - 1; j >= 0; --j) {
      acc += xt[j] * xt[j];
      r2[j] = acc;
    }
  }
  const T inv_sqrt_2pi = (T)0.39894228040143267794, inv_sqrt_pi = (T)0.56418958354775628695;
  for (int j = j_lo; j < j_hi; ++j) {
    const int rem = jobs[j].rem, ntask = jobs[j].ntask;        // uniform
    const bool valid = grp < ntask;
    const int sl = valid ? grp : 0;
    const int32_t* jw = reinterpret_cast<const int32_t*>(jobs + j);
    const int ms = jw[4 + sl], ntop = jw[8 + sl];
    int t = jw[12 + sl];
    const int mm = ms < 0 ? -ms : ms;
    T cr = 1, ci = 0;
    for (int s = 0; s < mm; ++s) {
      const T ax = xt[D - 2], ay = xt[D - 1];
      const T ncr = ax * cr - ay * ci;
      ci = ay * cr + ax * ci;
      cr = ncr;
    }
    const T cm = (mm == 0) ? inv_sqrt_2pi : inv_sqrt_pi;
    const T pre = cm * (ms >= 0 ? cr : ci);
    if constexpr (D >= 4) {
      const P2* cf = chain + ((D - 3) * (K + 1) + mm) * (K + 1);
      T pm1 = 0, p = cf[0].x;
      for (int nn = 1; nn <= ntop; ++nn) {
        if (nn == 1) {
          pm1 = p;
          p = cf[1].x * xt[D - 3];
        } else {
          const P2 c = cf[nn];
          const T pn = c.x * xt[D - 3] * p - c.y * r2[D - 3] * pm1;
          pm1 = p;
          p = pn;
        }
      }
      MfChain<T, D, D - 3>::run(xt, r2, mm + ntop, rem, pre * p, K, chain, cmap, t, phc, pt, valid);
    } else {
      MfChain<T, D, 1>::run(xt, r2, mm, rem, pre, K, chain, cmap, t, phc, pt, valid);
    }
  }
  // radial functions: Clenshaw in T_a(t); entry e = row * kMfP + point, point e % 16 == pt
  const T* __restrict__ q_coef = (const T*)a.q_coef;
  for (int e = tid; e < a.S * kMfP; e += kMfThreads) {
    const int row = e >> 4;
    const int L = a.q_len[row];
    const T* cf = q_coef + a.q_off[row];
    T b1 = 0, b2 = 0;
    for (int s = L - 1; s >= 1; --s) {
      const T c = cf[s];
      const T b0 = 2 * tt * b1 - b2 + c;
      b2 = b1;
      b1 = b0;
    }
    qc[row * kMfP + pt] = tt * b1 - b2 + cf[0];
  }
}

// Tables every fused pass stages once per workgroup: the loop-order row table, the recurrence
// pairs, and zeros in the 16 pad rows past the harmonics.
template <typename T>
__device__ __forceinline__ void mf_stage_tables(const MfArgs& a, int D, typename MfPair<T>::type* chain,
                                                int32_t* cmap, T* phc, int tid) {
  typedef typename MfPair<T>::type P2;
  for (int64_t e = tid; e < a.n_loop; e += kMfThreads) cmap[e] = a.col_of[e];
  const int npair = (D - 2) * (a.K + 1) * (a.K + 1);
  for (int e = tid; e < npair; e += kMfThreads) chain[e] = ((const P2*)a.chain)[e];
  for (int e = tid; e < 16 * kMfP; e += kMfThreads) phc[a.H * kMfP + e] = 0;
}

// Pass 1.  Block (split, y): slot group y / cpl, column tile y % cpl.  Each wavefront keeps its
// slots' accumulator tiles for the whole split; per chunk, lane r + 16 q reads the four values of
// harmonic row row0 + r at points 4q .. 4q + 3 with one LDS read and feeds the four MFMA k-steps
// with them (k-step s takes point 4q + s as its k-index q; V^T is read the same way, so the sum
// over the chunk's points is complete).
template <typename Tin, typename T, int D>
__global__ void __launch_bounds__(kMfThreads) __attribute__((amdgpu_waves_per_eu(MfWavesPerEu<T>::value, 8)))
k_mf_t(MfArgs a, MfLayout lay, const MfSlot1* __restrict__ slots, const int32_t* __restrict__ slot_off, int cpl,
       int64_t split_len, const Tin* __restrict__ V, int64_t ldv, int m, int m16, int64_t rank,
       double* __restrict__ part) {
  typedef typename MfMma<T>::V Acc;
  typedef typename MfPair<T>::type P2;
  constexpr int NS = kMfSlots1;
  extern __shared__ unsigned char smem_raw[];
  T* phc = reinterpret_cast<T*>(smem_raw + lay.phc);
  T* qc = reinterpret_cast<T*>(smem_raw + lay.qc);
  T* vc = reinterpret_cast<T*>(smem_raw + lay.aux);
  int32_t* cmap = reinterpret_cast<int32_t*>(smem_raw + lay.cmap);
  P2* chain = reinterpret_cast<P2*>(smem_raw + lay.chain);
  const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int split = blockIdx.x, gi = blockIdx.y / cpl, ct = blockIdx.y - gi * cpl;
  const int64_t p_begin = (int64_t)split * split_len;
  if (p_begin >= a.n) return;                     // whole workgroup, before any barrier
  const int64_t p_end = (p_begin + split_len < a.n) ? p_begin + split_len : a.n;
  mf_stage_tables<T>(a, D, chain, cmap, phc, tid);
  const int s_lo = slot_off[gi * (kMfWaves + 1) + wave];
  const int ns = slot_off[gi * (kMfWaves + 1) + wave + 1] - s_lo;
  const int j_lo = a.job_off[wave], j_hi = a.job_off[wave + 1];
  Acc acc[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) acc[t] = Acc{0, 0, 0, 0};
  for (int64_t c0 = p_begin; c0 < p_end; c0 += kMfP) {
    __syncthreads();                              // the previous chunk's reads are done
    mf_eval<Tin, T, D>(a, c0, a.jobs, j_lo, j_hi, chain, cmap, phc, qc, tid);
    if (tid < 16 * kMfP) {                        // V^T of the chunk, columns of tile ct
      const int pp = tid >> 4, c = tid & 15, col = ct * 16 + c;
      const int64_t i = c0 + pp;
      const int64_t ic = i < a.n ? i : a.n - 1;
      const Tin v = V[ic * ldv + (col < m ? col : 0)];
      vc[c * kMfP + pp] = (i < p_end && col < m) ? (T)v : (T)0;
    }
    __syncthreads();
    T vb[4];
    mf_lds4<T>(vc + r * kMfP + 4 * q, vb);
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if (t < ns) {
        const MfSlot1 sd = slots[s_lo + t];
        T a4[4], q4[4];
        mf_lds4<T>(phc + (sd.row0 + r) * kMfP + 4 * q, a4);
        mf_lds4<T>(qc + sd.qrow * kMfP + 4 * q, q4);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[t] = MfMma<T>::run(a4[s] * q4[s], vb[s], acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    if (t < ns) {
      const MfSlot1 sd = slots[s_lo + t];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = MfMma<T>::row(q, e);
        if (row < sd.nr)
          part[((int64_t)split * rank + sd.out0 + (int64_t)row * sd.s) * m16 + ct * 16 + r] = (double)acc[t][e];
      }
    }
  }
}

// Pass 2.  Block (range, y): slot group y / cpl, column tile y % cpl.  A wavefront's D W operands
// (its slots' rank rows, this column tile) are loaded once into registers; per chunk it forms the
// A operand U[point r][rank q] = phi_{row0 + q}(r) q_l(r) from LDS and accumulates one 16 x 16
// tile of KV over its slots; the eight wavefronts' tiles are added in a fixed order.
template <typename Tin, typename T, int D>
__global__ void __launch_bounds__(kMfThreads) __attribute__((amdgpu_waves_per_eu(MfWavesPerEu<T>::value, 8)))
k_mf_n(MfArgs a, MfLayout lay, const MfSlot2* __restrict__ slots, const int32_t* __restrict__ slot_off, int cpl,
       int64_t range_len, const T* __restrict__ Wd, int m16, Tin* __restrict__ KV, int64_t ldkv, int m, int n_groups,
       T* __restrict__ part) {
  typedef typename MfMma<T>::V Acc;
  typedef typename MfPair<T>::type P2;
  constexpr int NS = kMfSlots2;
  extern __shared__ unsigned char smem_raw[];
  T* phc = reinterpret_cast<T*>(smem_raw + lay.phc);
  T* qc = reinterpret_cast<T*>(smem_raw + lay.qc);
  T* red = reinterpret_cast<T*>(smem_raw + lay.aux);
  int32_t* cmap = reinterpret_cast<int32_t*>(smem_raw + lay.cmap);
  P2* chain = reinterpret_cast<P2*>(smem_raw + lay.chain);
  const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, q = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int range = blockIdx.x, gi = blockIdx.y / cpl, ct = blockIdx.y - gi * cpl;
  const int64_t p_begin = (int64_t)range * range_len;
  if (p_begin >= a.n) return;                     // whole workgroup, before any barrier
  const int64_t p_end = (p_begin + range_len < a.n) ? p_begin + range_len : a.n;
  mf_stage_tables<T>(a, D, chain, cmap, phc, tid);
  const int s_lo = slot_off[gi * (kMfWaves + 1) + wave];
  const int ns = slot_off[gi * (kMfWaves + 1) + wave + 1] - s_lo;
  const int j_lo = a.job_off[wave], j_hi = a.job_off[wave + 1];
  // B[q][r] = (D W)[rank0 + q s][ct 16 + r], zero for rows past the degree
  T wd[NS];
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    wd[t] = 0;
    if (t < ns) {
      const MfSlot2 sd = slots[s_lo + t];
      if (q < sd.nv) wd[t] = Wd[((int64_t)sd.rank0 + (int64_t)q * sd.s) * m16 + ct * 16 + r];
    }
  }
  for (int64_t c0 = p_begin; c0 < p_end; c0 += kMfP) {
    __syncthreads();                              // the previous chunk's reads are done
    mf_eval<Tin, T, D>(a, c0, a.jobs, j_lo, j_hi, chain, cmap, phc, qc, tid);
    __syncthreads();
    Acc acc = Acc{0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      if (t < ns) {
        const MfSlot2 sd = slots[s_lo + t];
        const T u = phc[(sd.row0 + q) * kMfP + r] * qc[sd.qrow * kMfP + r];
        acc = MfMma<T>::run(u, wd[t], acc);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wave * 256 + MfMma<T>::row(q, e) * 16 + r] = acc[e];
    __syncthreads();
    if (tid < 256) {
      const int pp = tid >> 4, c = tid & 15, col = ct * 16 + c;
      T sum = 0;
#pragma unroll
      for (int w = 0; w < kMfWaves; ++w) sum += red[w * 256 + pp * 16 + c];
      const int64_t i = c0 + pp;
      if (i < p_end && col < m) {
        if (n_groups == 1) KV[i * ldkv + col] = (Tin)sum;
        else part[((int64_t)gi * a.n + i) * m + col] = sum;
      }
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

MfLayout mf_layout(int64_t H, int S, int64_t n_loop, int d, int K, int prec, int pass) {
  const int64_t el = prec == 1 ? 4 : 8;
  int64_t off = 0;
  MfLayout l{};
  l.phc = (int32_t)off;
  off += mf_round16((H + 16) * kMfP * el);
  l.qc = (int32_t)off;
  off += mf_round16((int64_t)S * kMfP * el);
  l.aux = (int32_t)off;
  off += mf_round16((pass == 1 ? 16 * kMfP : kMfWaves * 256) * el);
  l.cmap = (int32_t)off;
  off += mf_round16(n_loop * 4);
  l.chain = (int32_t)off;
  off += mf_round16((int64_t)(d - 2) * (K + 1) * (K + 1) * 2 * el);
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

int mf_blocks_per_cu(const MfArgs& a, int pass, const MfLayout& lay) {
  int nb = 0;
  const hipError_t e = mf_dispatch(a, [&](auto ty) -> hipError_t {
    typedef typename decltype(ty)::Tin Tin;
    typedef typename decltype(ty)::Tf T;
    constexpr int D = decltype(ty)::D;
    const void* fn = pass == 1 ? reinterpret_cast<const void*>(&k_mf_t<Tin, T, D>)
                               : reinterpret_cast<const void*>(&k_mf_n<Tin, T, D>);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, kMfThreads, (size_t)lay.total);
  });
  return (e != hipSuccess || nb < 1) ? 1 : nb;
}

hipError_t launch_mf_t(const MfArgs& a, const MfLayout& lay, const MfSlot1* slots, const int32_t* slot_off,
                       int n_groups, int cpl, int n_splits, int64_t split_len, const void* V, int64_t ldv, int m,
                       int m16, int64_t rank, double* partials, hipStream_t s) {
  if (split_len % kMfP != 0 || n_splits < 1 || (int64_t)(n_splits - 1) * split_len >= a.n ||
      (int64_t)n_splits * split_len < a.n || cpl < 1 || cpl * 16 != m16 || n_groups < 1 || a.H < 1)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_splits, (unsigned)(n_groups * cpl));
  return mf_dispatch(a, [&](auto ty) -> hipError_t {
    typedef typename decltype(ty)::Tin Tin;
    typedef typename decltype(ty)::Tf T;
    constexpr int D = decltype(ty)::D;
    k_mf_t<Tin, T, D><<<grid, kMfThreads, (size_t)lay.total, s>>>(a, lay, slots, slot_off, cpl, split_len,
                                                                    (const Tin*)V, ldv, m, m16, rank, partials);
    return hipGetLastError();
  });
}

hipError_t launch_mf_n(const MfArgs& a, const MfLayout& lay, const MfSlot2* slots, const int32_t* slot_off,
                       int n_groups, int cpl, int n_ranges, int64_t range_len, const void* Wd, int m16, void* KV,
                       int64_t ldkv, int m, void* part, hipStream_t s) {
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
    k_mf_n<Tin, T, D><<<grid, kMfThreads, (size_t)lay.total, s>>>(a, lay, slots, slot_off, cpl, range_len,
                                                                    (const T*)Wd, m16, (Tin*)KV, ldkv, m, n_groups,
                                                                    (T*)part);
    if (n_groups > 1) k_mf_sum<T, Tin><<<nb, 256, 0, s>>>((const T*)part, n_groups, a.n, m, (Tin*)KV, ldkv);
    return hipGetLastError();
  });
}

}  // namespace hdf
