// C ABI of the HDF library: argument checks, the build pipeline (device
// geometry -> host planner -> device radial Gram -> host compression ->
// device factor evaluation) and the matvec / adjoint drivers.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/hdf.h"
#include "kernels.hpp"
#include "planner.hpp"
#include "status.hpp"

namespace {

thread_local std::string g_err;

hdf_status fail(hdf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

// Caching device allocator.  A build allocates gigabytes (the stored factor)
// and hipMalloc / hipFree of that size cost about a millisecond each, so freed
// blocks are kept per device and reused for requests of the same size class
// (a block serves requests down to 80 % of its size).  Blocks are returned
// only when no enqueued work can still use them: the handle destructor waits
// for the device first, and a buffer that grows waits before giving back its
// old block.  When hipMalloc fails, the device's cached blocks are released
// and the allocation is tried again.  The cache holds at most a quarter of
// the device memory; it lives until the process ends.
#ifndef HDF_ALLOC_CACHE
#define HDF_ALLOC_CACHE 1      // 0: exact-size hipMalloc / hipFree (the CPU emulation's memory checks)
#endif
namespace pool {
struct Block {
  void* p;
  int dev;
};
std::mutex& mu() {
  static std::mutex* m = new std::mutex;
  return *m;
}
std::multimap<size_t, Block>& blocks() {
  static auto* b = new std::multimap<size_t, Block>;
  return *b;
}
std::map<int, size_t>& cached() {
  static auto* c = new std::map<int, size_t>;
  return *c;
}
size_t size_class(size_t b) {
  const size_t g = (size_t)2 << 20;
  return b < g ? (b + 255) / 256 * 256 : (b + g - 1) / g * g;
}
void trim(int dev) {
  std::lock_guard<std::mutex> lk(mu());
  for (auto it = blocks().begin(); it != blocks().end();) {
    if (it->second.dev == dev) {
      hipFree(it->second.p);
      cached()[dev] -= it->first;
      it = blocks().erase(it);
    } else {
      ++it;
    }
  }
}
hipError_t alloc(void** p, size_t b, size_t* got, int* dev_out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (!HDF_ALLOC_CACHE) {
    e = hipMalloc(p, b);
    *got = e == hipSuccess ? b : 0;
    *dev_out = dev;
    if (e != hipSuccess) *p = nullptr;
    return e;
  }
  const size_t want = size_class(b);
  {
    std::lock_guard<std::mutex> lk(mu());
    for (auto it = blocks().lower_bound(want); it != blocks().end() && it->first <= want + want / 4; ++it) {
      if (it->second.dev != dev) continue;
      *p = it->second.p;
      *got = it->first;
      *dev_out = dev;
      cached()[dev] -= it->first;
      blocks().erase(it);
      return hipSuccess;
    }
  }
  e = hipMalloc(p, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    trim(dev);
    e = hipMalloc(p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return e;
  }
  *got = want;
  *dev_out = dev;
  return hipSuccess;
}
void release(void* p, size_t bytes, int dev) {
  if (!HDF_ALLOC_CACHE) {
    hipFree(p);
    return;
  }
  static size_t cap = 0;
  std::lock_guard<std::mutex> lk(mu());
  if (!cap) {
    size_t f = 0, t = 0;
    cap = (hipMemGetInfo(&f, &t) == hipSuccess && t) ? t / 4 : ((size_t)16 << 30);
  }
  if (cached()[dev] + bytes > cap) {
    hipFree(p);
    return;
  }
  blocks().insert({bytes, Block{p, dev}});
  cached()[dev] += bytes;
}
size_t cached_bytes(int dev) {
  std::lock_guard<std::mutex> lk(mu());
  return cached()[dev];
}
}  // namespace pool

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int dev = 0;
  ~DevBuf() { release(); }
  void release() {
    if (p) pool::release(p, bytes, dev);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    if (p) {
      // work enqueued on the old block may still run
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      release();
    }
    return pool::alloc(&p, std::max<size_t>(b, 256), &bytes, &dev);
  }
};

// A table inside a shared device buffer (the buffer owns the memory).
struct DevView {
  void* p = nullptr;
};

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

namespace hdf {
hdf_status set_error(hdf_status s, const std::string& msg) { return fail(s, msg); }
void clear_error() { g_err.clear(); }
}  // namespace hdf


struct hdf_factor {
  int d = 0, prec = 0, dtype = 0, kernel = 0;
  int64_t N = 0, ldN = 0;
  double l = 0, tol = 0;
  hdf::GeoDev geo{};
  double u0 = 0, u1 = 1, nu = 0, tail = 0, tau = 0;
  int p = 0, K = 0;
  int rank_rule = HDF_RULE_BOUND, p_bound = -1;
  // HDF_STORE_NONE: the factor is re-evaluated in every pass, either by the fused kernels (16
  // points at a time in LDS, mf_fused) or per chunk of points into cphi / cq
  int storage = HDF_STORE_FACTOR;
  int64_t chunk = 0, ldC = 0;
  int mf_chunked = 0;                             // option: never use the fused kernels
  bool mf_fused = false;
  DevBuf mf_tabs;                                 // jobs | job_off | slots1 | slot_off1 | slots2 | slot_off2
  size_t mf_o_joff = 0, mf_o_s1 = 0, mf_o_so1 = 0, mf_o_s2 = 0, mf_o_so2 = 0, mf_o_r1 = 0, mf_o_r2 = 0, mf_o_bt = 0;
  int mf_ntasks = 0;
  int mf_g1 = 1, mf_g2 = 1, mf_nb1 = 0, mf_nb2 = 0, n_cu = 0, mf_nr1 = 0, mf_nr2 = 0;
  int64_t mf_nloop = 0, mf_nqc = 0, mf_t1 = 0, mf_t2 = 0;
  int mf_spad = 0, mf_lpad = 0;
  bool mf_spec = false;
  size_t mf_o_qm = 0;
  hdf::MfLayout mf_lay1{}, mf_lay2{};
  double tau0 = 0, est_error = -1.0;             // budget threshold, sampled estimate
  std::vector<double> a;                          // p+1 coefficients
  std::vector<std::vector<double>> cores;
  std::vector<hdf::DegreeFactor> deg;             // k = 0..K
  std::vector<std::vector<double>> dC;            // per kept degree: E'^T (dM/dl) E' (s x s), lazily
  // general factor K(X, Y) ~ U V^T: the X side is the fields above (N, ldN,
  // x_soa, phi, q, tables, deg[].E = Ex, deg[].lam = singular values), the Y
  // side these
  bool cross = false;
  int64_t N2 = 0, ldN2 = 0;
  std::vector<hdf::DegreeFactor> degy;            // deg[].E = Ey
  DevBuf x_soa2, phi2, q2;
  DevView q_coef2;
  hdf::BuildTables tables2{};
  std::vector<hdf::DegDev> degs;                  // kept degrees
  std::vector<int> kept_k;
  std::vector<int32_t> index_table;               // H x (d-1)
  int64_t H = 0, S = 0, r = 0;
  int64_t n_wblocks = 0;                          // blocks of pass 2's batch-major copy of D W
  int max_s = 0;
  int n_refined = 0;                              // degrees refined by the second Gram pass
  double t_prep = 0, t_plan = 0, t_gram = 0, t_compress = 0, t_finish = 0, t_build = -1;
  hipEvent_t ev_b0 = nullptr, ev_b1 = nullptr;
  hipEvent_t ev_mv[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_adj[2] = {nullptr, nullptr};
  bool mv_timed = false, adj_timed = false;
  bool time_products = true;                      // HIP events around the product's kernels
  // device storage
  DevBuf x_soa, geo_dev, part, phi, q, tiles_dev, moments;
  // tables of the factor evaluation (in build_tabs) and of the products (in prod_tabs), each
  // set uploaded in one copy
  DevBuf build_tabs, prod_tabs;
  DevView col_of, chain, q_len, q_off, q_coef, degs_dev, lam_row, tile_tabs, degs_by_k;
  int n_tiles = 0, tiles_cpl = 0;                 // pass-1 work items for cpl = m16/16
  // tile-major pass 1 (m16 <= 64): wave items and their workgroup groups for each cpl = m16 / 16
  // in 1..4, built with the factor; tile_tabs holds all wave items, then all groups, then the
  // rank-row table
  int tw_off[5] = {0, 0, 0, 0, 0}, tg_off[5] = {0, 0, 0, 0, 0}, n_tgroups[5] = {0, 0, 0, 0, 0};
  size_t tg_base = 0;                             // byte offset of the groups in tile_tabs
  size_t rr_base = 0;                             // byte offset of the rank-row table in tile_tabs
  // host copies of uploaded build tables: they outlive their asynchronous uploads
  std::vector<std::vector<char>> host_keep;
  // host copies of the pass-1 tables: they outlive their asynchronous uploads
  std::vector<hdf::TileDev> tiles_host;
  // matvec / adjoint workspace
  DevBuf ws_part, ws_W, ws_Wd, ws_Wb, ws_n, bw_GV, bw_GVd, bw_GW, bw_GWd, bw_VW;
  DevBuf cphi, cq;                                // matrix-free chunk scratch
  // adjoint (dF/dX by contractions): the loop-order row table, q' = dq/d(rho^2) rows and their
  // coefficients, the shifted-factor degree table (harmonics of k - 1 with radial rows of k), the
  // contraction coefficients and products; host copies outlive their asynchronous uploads
  std::vector<int32_t> col_of_host;
  DevBuf dq, dq_coef, adj_degs, adj_c2, adj_cs, adj_kv2, adj_kvs;
  std::vector<hdf::DegDev> adj_degs_host;
  int64_t r_shift = 0;
  std::vector<char> adj_c2_host, adj_cs_host;
  hdf::BuildTables tables{};
  ~hdf_factor() {
    // the device buffers go back to the allocator cache once no enqueued work can use them
    (void)hipDeviceSynchronize();
    if (ev_b0) hipEventDestroy(ev_b0);
    if (ev_b1) hipEventDestroy(ev_b1);
    for (auto& e : ev_mv)
      if (e) hipEventDestroy(e);
    for (auto& e : ev_adj)
      if (e) hipEventDestroy(e);
  }
  // factor storage and arithmetic (1 = binary32, 0 = binary64) and its element size; the
  // caller's data (points, V, KV, W, dX) is in the points' type (dtype) throughout
  int fprec = 1;
  size_t felem() const { return fprec == 1 ? 4 : 8; }
  size_t ioel() const { return dtype == 0 ? 4 : 8; }
};

void hdf::set_product_timing(hdf_factor* h, bool on) { h->time_products = on; }


#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? HDF_E_OOM : HDF_E_HIP,                   \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

namespace {

// Loop order of the factor-evaluation kernel: azimuthal index outermost (|m|
// ascending, +m then -m), then the chain levels from d-2 down to 1; each
// innermost iteration is one harmonic.  Returns its canonical row or -1 for a
// dropped degree.
// A harmonic's index (k, mu_1 .. mu_{d-3}, m) packed one byte per entry (d <= 8,
// k and mu <= 30, m + 128 in [98, 158]).
static uint64_t harmonic_key(int k, const int32_t* mu, int nmu, int m) {
  uint64_t key = (uint64_t)k;
  for (int j = 0; j < nmu; ++j) key = key << 8 | (uint64_t)mu[j];
  return key << 8 | (uint64_t)(m + 128);
}

void loop_order_columns(int d, int K, const std::unordered_map<uint64_t, int>& canon,
                        std::vector<int32_t>& col_of) {
  col_of.clear();
  std::vector<int32_t> path, mus;   // upper indices from level d-2 down to level 1
  std::function<void(int, int, int)> rec = [&](int level, int b, int msigned) {
    for (int nn = 0; nn <= K - b; ++nn) {
      const int a = b + nn;
      path.push_back(a);
      if (level == 1) {
        // path = [mu_{d-3}, ..., mu_1, k] (for d = 3: [k])
        mus.clear();
        for (int j = (int)path.size() - 2; j >= 0; --j) mus.push_back(path[j]);   // mu_1..mu_{d-3}
        auto it = canon.find(harmonic_key(path.back(), mus.data(), (int)mus.size(), msigned));
        col_of.push_back(it == canon.end() ? -1 : it->second);
      } else {
        rec(level - 1, a, msigned);
      }
      path.pop_back();
    }
  };
  for (int mm = 0; mm <= K; ++mm) {
    rec(d - 2, mm, mm);
    if (mm > 0) rec(d - 2, mm, -mm);
  }
}


}  // namespace

// Kept degrees, harmonic tables, memory budget and the factor evaluation,
// common to the symmetric and the general (X != Y) build.  A general factor
// evaluates its Y side too, with the Y-side radial coefficients; its diagonal
// is the identity (sqrt of the singular values is folded into both sides).
// Zero columns [n, ld) of a rows x ld matrix (the padding of the factor rows).
static hipError_t clear_padding(void* base, int64_t rows, int64_t n, int64_t ld, size_t el, hipStream_t s) {
  if (rows <= 0 || ld <= n) return hipSuccess;
  return hipMemset2DAsync((char*)base + n * el, ld * el, 0, (ld - n) * el, rows, s);
}

// Wave items of the tile-major pass 1 for cpl = m16 / 16 (1..4): one per 16 harmonics of a kept
// degree and range of its radial functions (nl * nct accumulator tiles at most), then groups of up
// to kMvtWavesPerGroup items whose radial rows span at most kMvtMaxNq rows.
//
// Every item loads the same bytes (its 16 rows of the harmonics) while its MFMA work grows with its
// radial functions, and the low degrees have the most of them.  The waves of a group synchronise
// once per chunk and waves w and w + 4 share a SIMD, so the busiest SIMD of a group sets the pace
// of its chunk loop.
//  - The harmonics of a degree that do not fill a 16-row tile (a degree's last rows, or all of a
//    degree with fewer than 16) are not padded: their rank rows (harmonic, radial function) are
//    pooled over the degrees and cut into rank-row items of up to 16 rows (MvtRankRow) whose
//    radial rows span at most kMvtMaxNq rows, one accumulator tile per column tile, instead of a
//    partly empty tile per radial function.
//  - When all radial rows fit one group's staging, items of one column tile are cut to at most
//    kMvtSplitAcc radial functions and hdf::place_wave_items places the items so that the waves of
//    each SIMD and the groups carry about equal numbers of accumulator tiles.  Otherwise the items,
//    ordered by their first radial row, form runs of consecutive items.
// rr receives the rank-row table (the same for every cpl).
constexpr int kMvtSplitAcc = 3;
static void tile_tables(const std::vector<hdf::DegDev>& degs, int fprec, int cpl, std::vector<hdf::MvtWave>& tw,
                        std::vector<hdf::MvtGroup>& tg, std::vector<hdf::MvtRankRow>& rr) {
  const int nct_t = cpl == 1 ? 1 : (cpl == 2 ? 2 : 4);
  const int nlmax = hdf::matvec_tile_nl(fprec, nct_t);
  int q_min = 1 << 30, q_max = 0;
  for (const hdf::DegDev& dg : degs)
    if (dg.nh > 0 && dg.s > 0) {
      q_min = std::min(q_min, dg.qoff);
      q_max = std::max(q_max, dg.qoff + dg.s);
    }
  const bool spread = q_max - q_min <= hdf::kMvtMaxNq;
  const int nl_cap = spread && nct_t == 1 ? std::min(nlmax, kMvtSplitAcc) : nlmax;
  const int w_base = (int)tw.size();
  std::vector<hdf::MvtRankRow> pool;
  std::vector<std::pair<int, int>> qr;            // radial rows [lo, hi) of each item (host only)
  for (const hdf::DegDev& dg : degs)
    for (int h0 = 0; h0 < dg.nh; h0 += 16) {
      const int nr = std::min(16, dg.nh - h0);
      if (nr < 16) {
        for (int h = h0; h < dg.nh; ++h)
          for (int l = 0; l < dg.s; ++l) pool.push_back(hdf::MvtRankRow{dg.hoff + h, dg.qoff + l, dg.roff + h * dg.s + l, 0});
        continue;
      }
      for (int l0 = 0; l0 < dg.s; l0 += nl_cap) {
        hdf::MvtWave w{};
        w.row0 = dg.hoff + h0;
        w.nr = nr;
        w.qrow = dg.qoff + l0;
        w.nl = std::min(nl_cap, dg.s - l0);
        w.ct0 = 0;
        w.nct = cpl;
        w.out0 = dg.roff + h0 * dg.s + l0;
        w.s = dg.s;
        tw.push_back(w);
        qr.push_back({w.qrow, w.qrow + w.nl});
      }
    }
  if (!pool.empty()) {
    if (rr.empty()) rr = pool;
    // items of up to 16 consecutive pooled rows whose radial rows span at most kMvtMaxNq
    for (size_t r0 = 0; r0 < pool.size();) {
      int lo = pool[r0].qrow, hi = pool[r0].qrow + 1;
      size_t r1 = r0 + 1;
      while (r1 < pool.size() && r1 - r0 < 16) {
        const int lo2 = std::min(lo, pool[r1].qrow), hi2 = std::max(hi, pool[r1].qrow + 1);
        if (hi2 - lo2 > hdf::kMvtMaxNq) break;
        lo = lo2;
        hi = hi2;
        ++r1;
      }
      hdf::MvtWave w{};
      w.row0 = (int32_t)r0;
      w.nr = (int32_t)(r1 - r0);
      w.qrow = -1;
      w.nl = 1;
      w.ct0 = 0;
      w.nct = cpl;
      tw.push_back(w);
      qr.push_back({lo, hi});
      r0 = r1;
    }
  }
  const int n_items = (int)tw.size() - w_base;
  std::vector<int> loads(n_items), order, nw;
  for (int i = 0; i < n_items; ++i) loads[i] = std::max(1, tw[w_base + i].nl) * cpl;
  if (spread) {
    // every group stages all radial rows (rank-row items draw on any of them)
    if (!hdf::place_wave_items(loads, hdf::kMvtWavesPerGroup, 4, order, nw)) {
      order.resize(n_items);
      for (int i = 0; i < n_items; ++i) order[i] = i;
      nw.clear();
      for (int i = 0; i < n_items; i += hdf::kMvtWavesPerGroup) nw.push_back(std::min(hdf::kMvtWavesPerGroup, n_items - i));
    }
    std::vector<hdf::MvtWave> placed;
    for (int i : order) placed.push_back(tw[w_base + i]);
    std::copy(placed.begin(), placed.end(), tw.begin() + w_base);
    int w0 = 0;
    for (int g : nw) {
      hdf::MvtGroup gr{};
      gr.w0 = w0;
      gr.nw = g;
      gr.q_lo = q_min;
      gr.nq = q_max - q_min;
      tg.push_back(gr);
      w0 += g;
    }
    return;
  }
  // items in order of their first radial row (the rank-row items join the tiles of their degrees),
  // then runs of consecutive items whose radial rows span at most kMvtMaxNq rows
  std::vector<int> by_q(n_items);
  for (int i = 0; i < n_items; ++i) by_q[i] = i;
  std::stable_sort(by_q.begin(), by_q.end(), [&](int a, int b) { return qr[a].first < qr[b].first; });
  std::vector<hdf::MvtWave> sorted;
  std::vector<std::pair<int, int>> sorted_qr;
  for (int i : by_q) {
    sorted.push_back(tw[w_base + i]);
    sorted_qr.push_back(qr[i]);
  }
  std::copy(sorted.begin(), sorted.end(), tw.begin() + w_base);
  for (int i = 0; i < n_items;) {
    hdf::MvtGroup gr{};
    gr.w0 = i;
    int lo = sorted_qr[i].first, hi = sorted_qr[i].second;
    int j = i + 1;
    while (j < n_items && j - i < hdf::kMvtWavesPerGroup) {
      const int lo2 = std::min(lo, sorted_qr[j].first), hi2 = std::max(hi, sorted_qr[j].second);
      if (hi2 - lo2 > hdf::kMvtMaxNq) break;
      lo = lo2;
      hi = hi2;
      ++j;
    }
    gr.nw = j - i;
    gr.q_lo = lo;
    gr.nq = hi - lo;
    tg.push_back(gr);
    i = j;
  }
}

// Tables of the fused matrix-free passes, packed into one upload (see MfJob, MfSlot1, MfSlot2):
// evaluation jobs per wavefront (subtrees of one shape, four per job, spread over the wavefronts
// by longest-first assignment of their leaf counts), then the pass-1 accumulator tiles and the
// pass-2 steps, each cut into groups of at most kMfWaves x kMfSlots wavefront shares.
static bool mf_tables(hdf_factor* f, const std::vector<int32_t>& col_of, std::vector<char>& out) {
  const int d = f->d, K = f->kept_k.back();
  auto binom = [](int64_t nn, int64_t kk) {
    double v = 1.0;
    for (int64_t i = 1; i <= kk; ++i) v = v * (double)(nn - kk + i) / (double)i;
    return (int64_t)std::llround(v);
  };
  const int TL = d == 3 ? 1 : d - 3;              // levels below a subtree's prefix
  // subtrees (enumeration order: m ascending, cosine before sine, then the level d-2 index), listed
  // by base b = m + (level d-2 index) with their first loop-order harmonic
  std::vector<std::vector<std::pair<int, int>>> by_b(K + 1);
  int64_t t = 0;
  int id = 0;
  for (int mm = 0; mm <= K; ++mm)
    for (int sg = 0; sg < (mm > 0 ? 2 : 1); ++sg) {
      const int top = d == 3 ? 0 : K - mm;
      for (int ntop = 0; ntop <= top; ++ntop, ++id) {
        const int b = mm + ntop;
        by_b[b].push_back({id, (int)t});
        t += binom(K - b + TL, TL);
      }
    }
  if (t != f->mf_nloop || id != (d == 3 ? 2 * K + 1 : (K + 1) * (K + 1))) return false;
  std::vector<int32_t> btab;
  std::vector<int> bstart(K + 1);
  for (int b = 0; b <= K; ++b) {
    bstart[b] = (int)btab.size() / 2;
    for (auto& e : by_b[b]) { btab.push_back(e.first); btab.push_back(e.second); }
  }
  // jobs: one per base, split (level d-3 ranges, then subtree lists in multiples of four) while the
  // largest exceeds an eighth of the total; cost = per pass over the shared levels, the harmonics
  // below times (recurrence + one product and store per subtree in the lane group), plus the level
  // d-3 steps
  auto below = [&](int b, int n) -> int64_t { return d >= 5 ? binom(K - b - n + d - 4, d - 4) : (int64_t)(K - b + 1); };
  auto cost = [&](const hdf::MfJob& j) {
    int64_t leaves = 0;
    const int nhi = d >= 5 ? j.n_hi : 0;
    for (int n = d >= 5 ? j.n_lo : 0; n <= nhi; ++n) leaves += below(j.b, n);
    const int per_grp = (j.ntask + 3) / 4;
    double c = 0.0;
    for (int kb = 0; kb < per_grp; kb += 4) {
      const int nb = std::min(4, per_grp - kb);
      c += (double)leaves * (5.0 + 2.0 * nb) + (d >= 5 ? 5.0 * (nhi + 1) : 0.0) + 8.0;
    }
    return c;
  };
  std::vector<hdf::MfJob> jl;
  for (int b = 0; b <= K; ++b) {
    hdf::MfJob j{};
    j.b = b; j.n_lo = 0; j.n_hi = d >= 5 ? K - b : 0; j.off = 0;
    j.task0 = bstart[b]; j.ntask = (int)by_b[b].size();
    jl.push_back(j);
  }
  for (int guard = 0; guard < 256 && (int)jl.size() < 128; ++guard) {
    double total = 0.0;
    size_t imax = 0;
    for (size_t i = 0; i < jl.size(); ++i) {
      total += cost(jl[i]);
      if (cost(jl[i]) > cost(jl[imax])) imax = i;
    }
    hdf::MfJob j = jl[imax];
    if (cost(j) <= 1.05 * total / hdf::kMfWaves) break;
    hdf::MfJob a2 = j, b2 = j;
    if (d >= 5 && j.n_hi > j.n_lo) {
      int64_t all = 0, acc = 0;
      for (int n = j.n_lo; n <= j.n_hi; ++n) all += below(j.b, n);
      int cut = j.n_lo;
      while (cut < j.n_hi && 2 * (acc + below(j.b, cut)) <= all) acc += below(j.b, cut++);
      if (cut == j.n_lo) acc += below(j.b, cut++);
      a2.n_hi = cut - 1;
      b2.n_lo = cut;
      b2.off = j.off + (int32_t)acc;
    } else if (j.ntask > 4) {
      const int first = std::max(4, (j.ntask / 2 + 3) / 4 * 4);
      if (first >= j.ntask) break;
      a2.ntask = first;
      b2.task0 = j.task0 + first;
      b2.ntask = j.ntask - first;
    } else {
      break;
    }
    jl[imax] = a2;
    jl.push_back(b2);
  }
  std::vector<std::pair<double, hdf::MfJob>> jc;
  for (auto& j : jl) jc.push_back({cost(j), j});
  std::stable_sort(jc.begin(), jc.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  std::vector<std::vector<hdf::MfJob>> per(hdf::kMfWaves);
  // besides its jobs, evaluating wavefront w forms the radial tiles w, w + 8, ... (one MFMA chain of
  // L_pad / 4 steps each) and the subtree prefixes of the entries 64 w + 512 i < 16 (K + 1) (one
  // serial recurrence of about K + 1 steps each), all before the same barrier: their latencies
  // enter its load, in the cost units above (measured on the headline workload: a radial tile
  // about 6 units per step, a prefix entry about 3.5 units per recurrence step)
  std::vector<double> load(hdf::kMfWaves, 0.0);
  for (int w = 0; w < hdf::kMfWaves; ++w) {
    for (int tl = w; tl < f->mf_spad / 16; tl += hdf::kMfWaves) load[w] += 6.0 * (f->mf_lpad / 4) + 2.0;
    for (int e = 64 * w; e < 16 * (K + 1); e += 64 * hdf::kMfWaves) load[w] += 3.5 * (K + 1);
  }
  for (auto& e : jc) {
    const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    per[w].push_back(e.second);
    load[w] += e.first;
  }
  std::vector<hdf::MfJob> jobs;
  std::vector<int32_t> joff;
  for (int w = 0; w < hdf::kMfWaves; ++w) {
    joff.push_back((int32_t)jobs.size());
    jobs.insert(jobs.end(), per[w].begin(), per[w].end());
  }
  joff.push_back((int32_t)jobs.size());
  // contraction slots; their harmonics by loop-order row (rows past a degree's end: the zero pad row)
  std::vector<int32_t> loop_row((size_t)f->H, -1);
  for (size_t tt = 0; tt < col_of.size(); ++tt)
    if (col_of[tt] >= 0) loop_row[(size_t)col_of[tt]] = (int32_t)tt;
  for (int32_t v : loop_row)
    if (v < 0) return false;
  const int32_t zero_row = (int32_t)f->mf_nloop;
  std::vector<hdf::MfSlot1> s1;
  std::vector<hdf::MfSlot2> s2;
  std::vector<int32_t> r1, r2;
  for (const hdf::DegDev& dg : f->degs) {
    for (int h0 = 0; h0 < dg.nh; h0 += 16)
      for (int l = 0; l < dg.s; ++l) {
        hdf::MfSlot1 x{};
        x.row0 = (int32_t)r1.size(); x.qrow = dg.qoff + l; x.out0 = dg.roff + h0 * dg.s + l; x.s = dg.s;
        x.nr = std::min(16, dg.nh - h0);
        for (int j = 0; j < 16; ++j) r1.push_back(j < x.nr ? loop_row[(size_t)(dg.hoff + h0 + j)] : zero_row);
        r1.push_back(x.qrow);
        s1.push_back(x);
      }
    for (int h0 = 0; h0 < dg.nh; h0 += 4)
      for (int l = 0; l < dg.s; ++l) {
        hdf::MfSlot2 x{};
        x.row0 = (int32_t)r2.size(); x.qrow = dg.qoff + l; x.rank0 = dg.roff + h0 * dg.s + l; x.s = dg.s;
        x.nv = std::min(4, dg.nh - h0);
        for (int j = 0; j < 4; ++j) r2.push_back(j < x.nv ? loop_row[(size_t)(dg.hoff + h0 + j)] : zero_row);
        r2.push_back(x.qrow);
        s2.push_back(x);
      }
  }
  if ((int64_t)s1.size() != f->mf_t1 || (int64_t)s2.size() != f->mf_t2) return false;
  // groups of kMfWaves wavefront lists; each list is padded to whole blocks with slots that add
  // nothing (rows: the zero row; pass 1: out0 = -1; pass 2: nv = 0)
  auto groups = [&](auto& slots, std::vector<int32_t>& rows, int stride, int per_wave, int block, auto pad_slot,
                    std::vector<int32_t>& off) {
    using S = typename std::decay<decltype(slots)>::type::value_type;
    const int64_t total = (int64_t)slots.size();
    const int64_t cap = (int64_t)hdf::kMfWaves * (per_wave - block + 1);   // room for the padding
    const int g = (int)std::max<int64_t>(1, (total + cap - 1) / cap);
    std::vector<S> ps;
    std::vector<int32_t> pr;
    off.clear();
    for (int gi = 0; gi < g; ++gi) {
      const int64_t lo = total * gi / g, hi = total * (gi + 1) / g;
      for (int w = 0; w < hdf::kMfWaves; ++w) {
        off.push_back((int32_t)ps.size());
        const int64_t a = lo + (hi - lo) * w / hdf::kMfWaves, b = lo + (hi - lo) * (w + 1) / hdf::kMfWaves;
        for (int64_t i = a; i < b; ++i) {
          ps.push_back(slots[(size_t)i]);
          pr.insert(pr.end(), rows.begin() + i * stride, rows.begin() + (i + 1) * stride);
        }
        while ((ps.size() - (size_t)off.back()) % (size_t)block) {
          ps.push_back(pad_slot());
          for (int e = 0; e < stride; ++e) pr.push_back(e + 1 < stride ? zero_row : 0);
        }
      }
      off.push_back((int32_t)ps.size());
    }
    slots.swap(ps);
    rows.swap(pr);
    return g;
  };
  std::vector<int32_t> so1, so2;
  f->mf_g1 = groups(s1, r1, 17, hdf::kMfSlots1, hdf::kMfBlock1, [] { hdf::MfSlot1 x{}; x.out0 = -1; return x; }, so1);
  f->mf_g2 = groups(s2, r2, 5, hdf::kMfSlots2, hdf::kMfBlock2, [] { hdf::MfSlot2 x{}; x.nv = 0; return x; }, so2);
  if ((int64_t)r1.size() > f->mf_nr1 || (int64_t)r2.size() > f->mf_nr2) return false;   // the LDS layout's room
  f->mf_nr1 = (int)r1.size();
  f->mf_nr2 = (int)r2.size();
  auto put = [&](const void* p, size_t bytes) {
    const size_t at = (out.size() + 255) / 256 * 256;
    out.resize(at + bytes);
    if (bytes) std::memcpy(out.data() + at, p, bytes);
    return at;
  };
  out.clear();
  put(jobs.data(), jobs.size() * sizeof(hdf::MfJob));
  f->mf_o_joff = put(joff.data(), joff.size() * 4);
  f->mf_o_s1 = put(s1.data(), s1.size() * sizeof(hdf::MfSlot1));
  f->mf_o_so1 = put(so1.data(), so1.size() * 4);
  f->mf_o_s2 = put(s2.data(), s2.size() * sizeof(hdf::MfSlot2));
  f->mf_o_so2 = put(so2.data(), so2.size() * 4);
  f->mf_o_r1 = put(r1.data(), r1.size() * 4);
  f->mf_o_r2 = put(r2.data(), r2.size() * 4);
  f->mf_o_bt = put(btab.data(), btab.size() * 4);
  {
    // radial coefficient matrix S_pad x L_pad in the factor's type
    std::vector<double> qm((size_t)f->mf_spad * f->mf_lpad, 0.0);
    int row = 0;
    for (size_t di = 0; di < f->kept_k.size(); ++di) {
      const hdf::DegreeFactor& df = f->deg[f->kept_k[di]];
      for (int l = 0; l < df.s; ++l, ++row)
        for (int aa = 0; aa < df.L; ++aa) qm[(size_t)row * f->mf_lpad + aa] = df.E[(size_t)l * df.L + aa];
    }
    if (f->fprec == 1) {
      std::vector<float> qf(qm.begin(), qm.end());
      f->mf_o_qm = put(qf.data(), qf.size() * 4);
    } else {
      f->mf_o_qm = put(qm.data(), qm.size() * 8);
    }
  }
  f->mf_ntasks = id;
  return true;
}

static hdf_status finish_build(hdf_factor* f, double t0, hipStream_t s) {
  struct FinishTimer {
    hdf_factor* f;
    double t;
    ~FinishTimer() { f->t_finish = now_ms() - t; }
  } timer{f, 0.0};
  const int K = f->K, d = f->d, dtype = f->dtype;
  const int prec = f->fprec;
  const int64_t n = f->N;
  // kept degrees, offsets, tables
  int64_t hoff = 0, qoff = 0, roff = 0, boff = 0;
  std::unordered_map<uint64_t, int> canon;
  for (int k = 0; k <= K; ++k) {
    const hdf::DegreeFactor& df = f->deg[k];
    if (df.s == 0) continue;
    const int64_t nh = hdf::index_count(d, k);
    hdf::DegDev dd{};
    dd.hoff = (int32_t)hoff; dd.nh = (int32_t)nh; dd.qoff = (int32_t)qoff; dd.s = df.s; dd.roff = (int32_t)roff;
    dd.boff = (int32_t)boff;
    boff += (nh + 15) / 16 * df.s;
    f->degs.push_back(dd);
    f->kept_k.push_back(k);
    std::vector<int32_t> tab;
    hdf::index_set(d, k, tab);
    canon.reserve(canon.size() + (size_t)nh);
    for (int64_t h = 0; h < nh; ++h) {
      const int32_t* t = &tab[(size_t)h * (d - 2)];
      f->index_table.push_back(k);
      for (int j = 0; j < d - 2; ++j) f->index_table.push_back(t[j]);
      canon[harmonic_key(k, t, d - 3, t[d - 3])] = (int)(hoff + h);
    }
    hoff += nh;
    qoff += df.s;
    roff += nh * df.s;
    f->max_s = std::max(f->max_s, df.s);
  }
  f->H = hoff; f->S = qoff; f->r = roff; f->n_wblocks = boff;
  f->t_compress = now_ms() - t0;
  timer.t = now_ms();

  // 5. memory budget, then the factor evaluation
  const bool mfree = f->storage == HDF_STORE_NONE;
  if (mfree && f->H > 0 && !f->mf_chunked) {
    // fused passes when the harmonics of 16 points fit in one workgroup's LDS
    const int Kh = f->kept_k.back();
    f->mf_nloop = 0;
    for (int k = 0; k <= Kh; ++k) f->mf_nloop += hdf::index_count(d, k);
    int64_t t1 = 0, t2 = 0;
    for (const hdf::DegDev& dg : f->degs) {
      t1 += (int64_t)((dg.nh + 15) / 16) * dg.s;
      t2 += (int64_t)((dg.nh + 3) / 4) * dg.s;
    }
    // row-table entries, with room for the padding of every wavefront list to whole blocks
    auto padded = [](int64_t t, int per_wave, int block) {
      const int64_t cap = (int64_t)hdf::kMfWaves * (per_wave - block + 1);
      const int64_t g = std::max<int64_t>(1, (t + cap - 1) / cap);
      return t + g * hdf::kMfWaves * (block - 1);
    };
    f->mf_nr1 = (int)(17 * padded(t1, hdf::kMfSlots1, hdf::kMfBlock1));
    f->mf_nr2 = (int)(5 * padded(t2, hdf::kMfSlots2, hdf::kMfBlock2));
    f->mf_t1 = t1;
    f->mf_t2 = t2;
    int lmax = 1;
    for (size_t di = 0; di < f->kept_k.size(); ++di) lmax = std::max(lmax, f->deg[f->kept_k[di]].L);
    f->mf_spad = (int)((f->S + 15) / 16 * 16);
    f->mf_lpad = (lmax + 3) / 4 * 4;
    f->mf_nqc = (int64_t)f->mf_spad * f->mf_lpad;
    const int64_t ntasks = d == 3 ? 2 * Kh + 1 : (int64_t)(Kh + 1) * (Kh + 1);
    auto lays = [&](bool spec) {
      f->mf_lay1 = hdf::mf_layout(f->mf_nloop, (int)f->S, f->mf_nr1, f->mf_nqc, ntasks, d, Kh, f->fprec, 1, spec);
      f->mf_lay2 = hdf::mf_layout(f->mf_nloop, (int)f->S, f->mf_nr2, f->mf_nqc, ntasks, d, Kh, f->fprec, 2, spec);
    };
    int dev = 0, max_lds = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    HIPCHK(hipDeviceGetAttribute(&f->n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    // the wavefront-specialised kernels (binary32) when their double buffers fit, else the plain ones
    lays(true);
    f->mf_spec = f->fprec == 1 && std::max(f->mf_lay1.total, f->mf_lay2.total) <= max_lds;
    if (!f->mf_spec) lays(false);
    f->mf_fused = std::max(f->mf_lay1.total, f->mf_lay2.total) <= max_lds && f->mf_nloop < 65535 &&
                  f->mf_lpad <= 4 * hdf::kMfMaxKs;
  }
  const size_t fbytes = f->mf_fused ? 0
                        : (size_t)(f->H + f->S) * (mfree ? f->ldC : f->ldN + (f->cross ? f->ldN2 : 0)) * f->felem();
  size_t freeb = 0, totb = 0;
  HIPCHK(hipMemGetInfo(&freeb, &totb));
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) freeb += pool::cached_bytes(dev);   // reusable blocks
  }
  const size_t budget = std::max<size_t>((size_t)1 << 30, (size_t)(0.6 * (double)freeb));
  if (fbytes > budget) {
    char buf[200];
    snprintf(buf, sizeof buf, "factor needs %.3g GB (H=%lld, S=%lld), budget %.3g GB",
             fbytes / 1e9, (long long)f->H, (long long)f->S, budget / 1e9);
    return fail(HDF_E_INFEASIBLE, buf);
  }
  if (f->H > 0) {
    if (mfree) {
      if (!f->mf_fused) {
        HIPCHK(f->cphi.ensure((size_t)f->H * f->ldC * f->felem()));
        HIPCHK(f->cq.ensure((size_t)f->S * f->ldC * f->felem()));
      }
    } else {
      HIPCHK(f->phi.ensure((size_t)f->H * f->ldN * f->felem()));
      HIPCHK(f->q.ensure((size_t)f->S * f->ldN * f->felem()));
    }
    if (f->cross) {
      HIPCHK(f->phi2.ensure((size_t)f->H * f->ldN2 * f->felem()));
      HIPCHK(f->q2.ensure((size_t)f->S * f->ldN2 * f->felem()));
    }
    // The harmonic recurrences run up to the largest kept degree only:
    // dropped top degrees would be evaluated and discarded.
    const int Kh = f->kept_k.back();
    // loop-order column table
    std::vector<int32_t> col_of;
    loop_order_columns(d, Kh, canon, col_of);
    f->col_of_host = col_of;                      // the adjoint's host-side harmonic evaluation
    // uploads from copies the handle keeps, so no synchronisation is needed before the
    // host vectors below go out of scope
    auto upload = [&](DevBuf& b, const void* src, size_t bytes) -> hipError_t {
      hipError_t e = b.ensure(bytes);
      if (e != hipSuccess) return e;
      f->host_keep.emplace_back((const char*)src, (const char*)src + bytes);
      return hipMemcpyAsync(b.p, f->host_keep.back().data(), bytes, hipMemcpyHostToDevice, s);
    };
    // several tables packed (256-byte aligned) into one device buffer with one copy
    struct Batch {
      std::vector<char> host;
      std::vector<std::pair<DevView*, size_t>> parts;
      void add(DevView& v, const void* src, size_t bytes) {
        const size_t off = (host.size() + 255) / 256 * 256;
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, src, bytes);
        parts.push_back({&v, off});
      }
    };
    auto upload_batch = [&](DevBuf& b, Batch& batch) -> hipError_t {
      hipError_t e = b.ensure(std::max<size_t>(batch.host.size(), 256));
      if (e != hipSuccess) return e;
      for (auto& pr : batch.parts) pr.first->p = (char*)b.p + pr.second;
      f->host_keep.emplace_back(std::move(batch.host));
      return hipMemcpyAsync(b.p, f->host_keep.back().data(), f->host_keep.back().size(), hipMemcpyHostToDevice, s);
    };
    Batch bt;
    bt.add(f->col_of, col_of.data(), col_of.size() * sizeof(int32_t));
    // recurrence coefficients as (A, B) pairs in the storage type
    hdf::ChainCoeffs cc;
    hdf::chain_coeffs(d, Kh, cc);
    const size_t npair = cc.A.size();
    // eight pad pairs: the adjoint reads one pair ahead, the fused passes whole blocks of pairs
    std::vector<double> pd(2 * npair + 16, 0.0);
    for (size_t i = 0; i < npair; ++i) { pd[2 * i] = cc.A[i]; pd[2 * i + 1] = cc.B[i]; }
    std::vector<int32_t> ql, qo;
    std::vector<double> qc, qc2;
    for (size_t di = 0; di < f->kept_k.size(); ++di) {
      const hdf::DegreeFactor& df = f->deg[f->kept_k[di]];
      for (int l = 0; l < df.s; ++l) {
        ql.push_back(df.L);
        qo.push_back((int32_t)qc.size());
        qc.insert(qc.end(), df.E.begin() + (size_t)l * df.L, df.E.begin() + (size_t)(l + 1) * df.L);
        if (f->cross) {
          const hdf::DegreeFactor& dy = f->degy[f->kept_k[di]];
          qc2.insert(qc2.end(), dy.E.begin() + (size_t)l * dy.L, dy.E.begin() + (size_t)(l + 1) * dy.L);
        }
      }
    }
    auto add_typed = [&](DevView& v, const std::vector<double>& x) {
      if (f->fprec == 1) {
        std::vector<float> tmp(x.begin(), x.end());
        bt.add(v, tmp.data(), tmp.size() * 4);
      } else {
        bt.add(v, x.data(), x.size() * 8);
      }
    };
    add_typed(f->chain, pd);
    add_typed(f->q_coef, qc);
    if (f->cross) add_typed(f->q_coef2, qc2);
    bt.add(f->q_len, ql.data(), ql.size() * 4);
    bt.add(f->q_off, qo.data(), qo.size() * 4);
    HIPCHK(upload_batch(f->build_tabs, bt));
    hdf::BuildTables tb{};
    tb.col_of = (const int32_t*)f->col_of.p;
    tb.chain = f->chain.p;
    tb.q_len = (const int32_t*)f->q_len.p;
    tb.q_off = (const int32_t*)f->q_off.p;
    tb.q_coef = f->q_coef.p;
    tb.K = Kh;
    tb.S = (int)f->S;
    f->tables = tb;
    // tables of the products (not read by the factor evaluation): built and uploaded after its
    // launch in the stored case, so the host work overlaps the evaluation on the device
    auto product_tables = [&]() -> hdf_status {
      // host tables first, then the uploads: an upload from pageable memory may wait for the
      // stream (the evaluation just launched) before it returns
      std::vector<hdf::MvtWave> tw;
      std::vector<hdf::MvtGroup> tg;
      std::vector<hdf::MvtRankRow> rr;
      for (int cpl = 1; cpl <= 4; ++cpl) {
        f->tw_off[cpl] = (int)tw.size();
        f->tg_off[cpl] = (int)tg.size();
        tile_tables(f->degs, f->fprec, cpl, tw, tg, rr);
        f->n_tgroups[cpl] = (int)tg.size() - f->tg_off[cpl];
      }
      if (rr.empty()) rr.push_back(hdf::MvtRankRow{0, 0, 0, 0});   // never read: no rank-row items
      const size_t wb = tw.size() * sizeof(hdf::MvtWave);
      f->tg_base = (wb + 255) / 256 * 256;
      const size_t gb = tg.size() * sizeof(hdf::MvtGroup);
      f->rr_base = (f->tg_base + gb + 255) / 256 * 256;
      std::vector<char> tabs(f->rr_base + rr.size() * sizeof(hdf::MvtRankRow), 0);
      std::memcpy(tabs.data(), tw.data(), wb);
      std::memcpy(tabs.data() + f->tg_base, tg.data(), gb);
      std::memcpy(tabs.data() + f->rr_base, rr.data(), rr.size() * sizeof(hdf::MvtRankRow));
      std::vector<double> lr;
      lr.reserve(f->r);
      for (size_t di = 0; di < f->degs.size(); ++di) {
        const hdf::DegreeFactor& df = f->deg[f->kept_k[di]];
        for (int h = 0; h < f->degs[di].nh; ++h)
          for (int l = 0; l < df.s; ++l) lr.push_back(f->cross ? 1.0 : df.lam[l]);
      }
      std::vector<hdf::DegDev> dbk(K + 1);
      for (int k = 0; k <= K; ++k) { dbk[k] = hdf::DegDev{}; }
      for (size_t di = 0; di < f->degs.size(); ++di) dbk[f->kept_k[di]] = f->degs[di];
      Batch bp;
      bp.add(f->degs_dev, f->degs.data(), f->degs.size() * sizeof(hdf::DegDev));
      bp.add(f->tile_tabs, tabs.data(), tabs.size());
      bp.add(f->lam_row, lr.data(), lr.size() * 8);
      bp.add(f->degs_by_k, dbk.data(), dbk.size() * sizeof(hdf::DegDev));
      HIPCHK(upload_batch(f->prod_tabs, bp));
      return HDF_OK;
    };
    if (mfree) {                                // evaluated in every product
      const hdf_status pst = product_tables();
      if (pst != HDF_OK) return pst;
      if (f->mf_fused) {
        std::vector<char> tabs;
        if (!mf_tables(f, col_of, tabs)) return fail(HDF_E_ARG, "internal: inconsistent fused-pass tables");
        HIPCHK(upload(f->mf_tabs, tabs.data(), tabs.size()));
      }
      return HDF_OK;
    }
    HIPCHK(hipEventCreate(&f->ev_b0));
    HIPCHK(hipEventCreate(&f->ev_b1));
    HIPCHK(hipEventRecord(f->ev_b0, s));
    HIPCHK(hdf::launch_build(f->x_soa.p, dtype, f->ldN, n, d, (const hdf::GeoDev*)f->geo_dev.p,
                             f->u0, f->u1, tb, prec, f->phi.p, f->ldN, f->q.p, f->ldN, s));
    // rows are padded past N: clear the padding so contraction kernels may
    // read whole 8-point groups without masking
    HIPCHK(clear_padding(f->phi.p, f->H, n, f->ldN, f->felem(), s));
    HIPCHK(clear_padding(f->q.p, f->S, n, f->ldN, f->felem(), s));
    if (f->cross) {
      f->tables2 = tb;
      f->tables2.q_coef = f->q_coef2.p;
      HIPCHK(hdf::launch_build(f->x_soa2.p, dtype, f->ldN2, f->N2, d, (const hdf::GeoDev*)f->geo_dev.p,
                               f->u0, f->u1, f->tables2, prec, f->phi2.p, f->ldN2, f->q2.p, f->ldN2, s));
      HIPCHK(clear_padding(f->phi2.p, f->H, f->N2, f->ldN2, f->felem(), s));
      HIPCHK(clear_padding(f->q2.p, f->S, f->N2, f->ldN2, f->felem(), s));
    }
    HIPCHK(hipEventRecord(f->ev_b1, s));
    const hdf_status pst = product_tables();
    if (pst != HDF_OK) return pst;
  }
  return HDF_OK;
}

extern "C" {

const char* hdf_status_string(hdf_status s) {
  switch (s) {
    case HDF_OK: return "ok";
    case HDF_E_ARG: return "invalid argument";
    case HDF_E_DIM: return "dimension not supported (need 3 <= d <= 8)";
    case HDF_E_NONFINITE: return "non-finite point coordinate";
    case HDF_E_INFEASIBLE: return "infeasible: degree or factor size above the limits";
    case HDF_E_OOM: return "device out of memory";
    case HDF_E_HIP: return "HIP runtime error";
    case HDF_E_DISABLED: return "operation switched off in this library";
  }
  return "unknown status";
}

const char* hdf_last_error(void) { return g_err.c_str(); }

void hdf_free(hdf_handle h) { delete h; }

// ------------------------------------------------------------------ build
hdf_status hdf_build(const void* points, int dtype, int64_t n, int d, int64_t ld,
                     hdf_kernel kernel, double lengthscale, double tol, hdf_precision prec,
                     void* hip_stream, hdf_handle* out) {
  return hdf_build_ex(points, dtype, n, d, ld, kernel, lengthscale, tol, prec, nullptr, hip_stream, out);
}

hdf_status hdf_build_ex(const void* points, int dtype, int64_t n, int d, int64_t ld,
                        hdf_kernel kernel, double lengthscale, double tol, hdf_precision prec,
                        const hdf_build_options* opts, void* hip_stream, hdf_handle* out) {
  g_err.clear();
  if (!out) return fail(HDF_E_ARG, "out is NULL");
  if (!points) return fail(HDF_E_ARG, "points is NULL");
  if (d < 3 || d > HDF_MAX_DIM) return fail(HDF_E_DIM, "d must be in [3, 8]");
  if (n < 1) return fail(HDF_E_ARG, "n must be >= 1");
  if (ld < d) return fail(HDF_E_ARG, "ld must be >= d");
  if (dtype != 0 && dtype != 1) return fail(HDF_E_ARG, "dtype must be 0 (f32) or 1 (f64)");
  if (prec != HDF_FP64 && prec != HDF_MIXED) return fail(HDF_E_ARG, "unknown precision");
  if ((prec == HDF_MIXED) != (dtype == 0))
    return fail(HDF_E_ARG, "HDF_MIXED needs float32 points, HDF_FP64 needs float64 points");
  if ((int)kernel < 0 || (int)kernel > 3) return fail(HDF_E_ARG, "unknown kernel");
  if (!(lengthscale > 0) || !std::isfinite(lengthscale)) return fail(HDF_E_ARG, "lengthscale must be > 0");
  if (!(tol > 0 && tol < 1)) return fail(HDF_E_ARG, "tol must be in (0, 1)");
  const int rule = opts ? opts->rank_rule : HDF_RULE_BOUND;
  if (rule != HDF_RULE_BOUND && rule != HDF_RULE_SAMPLED) return fail(HDF_E_ARG, "unknown rank_rule");
  const int n_pairs = (opts && opts->n_pairs) ? opts->n_pairs : 16384;
  const double margin = (opts && opts->margin != 0.0) ? opts->margin : 0.8;
  if (n_pairs < 1 || n_pairs > (1 << 20)) return fail(HDF_E_ARG, "n_pairs must be in [1, 1048576]");
  if (!(margin > 0.0 && margin <= 1.0)) return fail(HDF_E_ARG, "margin must be in (0, 1]");
  const int storage = opts ? opts->storage : HDF_STORE_FACTOR;
  if (storage != HDF_STORE_FACTOR && storage != HDF_STORE_NONE) return fail(HDF_E_ARG, "unknown storage");
  const int64_t chunk = (opts && opts->chunk) ? opts->chunk : 262144;
  if (storage == HDF_STORE_NONE && chunk < 64) return fail(HDF_E_ARG, "chunk must be >= 64");
  const int mf_chunked = opts ? opts->chunked : 0;
  if (mf_chunked != 0 && mf_chunked != 1) return fail(HDF_E_ARG, "chunked must be 0 or 1");
  hipStream_t s = (hipStream_t)hip_stream;

  std::unique_ptr<hdf_factor> f(new hdf_factor());
  f->rank_rule = rule;
  if (storage == HDF_STORE_NONE) {
    f->storage = HDF_STORE_NONE;
    f->mf_chunked = mf_chunked;
    f->chunk = std::min<int64_t>(chunk, n);
    f->ldC = (f->chunk + 63) / 64 * 64 + 64;
  }
  f->d = d; f->prec = prec; f->dtype = dtype; f->kernel = kernel;
  f->fprec = (prec == HDF_MIXED && tol > HDF_SPLIT_TOL) ? 1 : 0;
  f->N = n; f->l = lengthscale; f->tol = tol;
  // rows of the factor are padded by at least 64 points: the streaming kernels
  // issue unconditional 16-byte loads up to 63 points past the last point
  f->ldN = (n + 63) / 64 * 64 + 64;
  const size_t in_elem = dtype == 0 ? 4 : 8;

  // 1. geometry on the device, one sync
  double t0 = now_ms();
  HIPCHK(f->x_soa.ensure((size_t)d * f->ldN * in_elem));
  HIPCHK(f->geo_dev.ensure(sizeof(hdf::GeoDev)));
  HIPCHK(f->part.ensure((size_t)hdf::kPrepBlocks * 32 * sizeof(double)));
  HIPCHK(hdf::launch_prep(points, dtype, n, d, ld, f->x_soa.p, f->ldN, kernel, lengthscale,
                          (double*)f->part.p, (hdf::GeoDev*)f->geo_dev.p, s));
  HIPCHK(hipMemcpyAsync(&f->geo, f->geo_dev.p, sizeof(hdf::GeoDev), hipMemcpyDeviceToHost, s));
  hdf::PairSample ps;
  DevBuf pairs_dev;
  std::vector<double> pair_vals;
  std::vector<int32_t> pair_idx;
  if (rule == HDF_RULE_SAMPLED) {
    HIPCHK(pairs_dev.ensure((size_t)n_pairs * (4 * sizeof(double) + 2 * sizeof(int32_t))));
    double* pv = (double*)pairs_dev.p;
    int32_t* pi = (int32_t*)(pv + 4 * (size_t)n_pairs);
    HIPCHK(hdf::launch_pairs(f->x_soa.p, dtype, f->ldN, n, d, (const hdf::GeoDev*)f->geo_dev.p, hdf::kPairSeed,
                             n_pairs, pv, pi, s));
    pair_vals.resize(4 * (size_t)n_pairs);
    pair_idx.resize(2 * (size_t)n_pairs);
    HIPCHK(hipMemcpyAsync(pair_vals.data(), pv, pair_vals.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(pair_idx.data(), pi, pair_idx.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (rule == HDF_RULE_SAMPLED) {
    const size_t M = (size_t)n_pairs;
    ps.r.assign(pair_vals.begin(), pair_vals.begin() + M);
    ps.ra2.assign(pair_vals.begin() + M, pair_vals.begin() + 2 * M);
    ps.rb2.assign(pair_vals.begin() + 2 * M, pair_vals.begin() + 3 * M);
    ps.dot.assign(pair_vals.begin() + 3 * M, pair_vals.end());
    ps.a.assign(pair_idx.begin(), pair_idx.begin() + M);
    ps.b.assign(pair_idx.begin() + M, pair_idx.end());
  }
  f->t_prep = now_ms() - t0;
  if (f->geo.nonfinite > 0) return fail(HDF_E_NONFINITE, "points contain NaN or Inf");

  // 2. host planner
  t0 = now_ms();
  f->nu = std::sqrt(f->geo.nu2_sum / (double)hdf::kNuPairs);
  const double D = 2.0 * f->geo.R;
  std::vector<double> afull(hdf::kChebNodes);
  hdf::chebyshev_coeffs(kernel, D, lengthscale, hdf::kChebNodes, false, afull.data());
  f->p = hdf::choose_degree(afull.data(), hdf::kChebNodes, tol * f->nu / 2.0, HDF_MAX_DEGREE, &f->tail);
  f->p_bound = f->p;
  if (rule == HDF_RULE_SAMPLED) {
    f->p = hdf::choose_degree_sampled(kernel, lengthscale, afull.data(), hdf::kChebNodes, D, (double)n, ps, tol,
                                      HDF_MAX_DEGREE, f->p_bound);
    f->tail = -1.0;
  }
  if (f->p < 0) {
    int pp = hdf::choose_degree(afull.data(), hdf::kChebNodes, tol * f->nu / 2.0, hdf::kChebNodes - 2, nullptr);
    char buf[160];
    snprintf(buf, sizeof buf, "Chebyshev degree %d needed (> %d): diameter/lengthscale too large for tol",
             pp, HDF_MAX_DEGREE);
    return fail(HDF_E_INFEASIBLE, buf);
  }
  f->K = f->p / 2;
  f->a.assign(afull.begin(), afull.begin() + f->p + 1);
  hdf::radial_interval(f->geo.rho2_min, f->geo.rho2_max, &f->u0, &f->u1);
  f->t_plan = now_ms() - t0;

  // 3. radial Gram moments on the device, second sync; the radial cores and
  // the threshold are formed on the host while the device runs
  t0 = now_ms();
  const int K = f->K;
  const int nrt = (K + 1 + 15) / 16, nct = (2 * K + 1 + 15) / 16;
  // Mixed precision uses the split (hi/lo) product on every tolerance: the
  // radial Gram can be ill-conditioned (cond ~1e6 measured on uniform-cube
  // data), and a plain binary32 Gram then forces a null-space cut that drops
  // directions the tolerance needs.  Its cost is negligible.
  const int gram_mode = (prec == HDF_FP64) ? 0 : 2;
  const int gb = hdf::gram_blocks(n);
  HIPCHK(f->part.ensure((size_t)gb * nrt * 16 * nct * 16 * sizeof(double) + 4096));
  HIPCHK(f->moments.ensure((size_t)nrt * 16 * nct * 16 * sizeof(double)));
  HIPCHK(hdf::launch_gram(f->x_soa.p, dtype, f->ldN, n, d, (const hdf::GeoDev*)f->geo_dev.p,
                          f->u0, f->u1, K, gram_mode, (double*)f->part.p, (double*)f->moments.p, s));
  const int mcols = nct * 16;
  std::vector<double> mom((size_t)nrt * 16 * mcols);
  HIPCHK(hipMemcpyAsync(mom.data(), f->moments.p, mom.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  const double t_overlap = now_ms();
  hdf::radial_cores(f->a.data(), f->p, d, f->u0, f->u1, f->cores);
  f->tau = hdf::tau_threshold(tol, f->nu, n, d, f->p);
  const double t_cores = now_ms() - t_overlap;
  HIPCHK(hipStreamSynchronize(s));
  f->t_plan += t_cores;
  f->t_gram = now_ms() - t0 - t_cores;

  // 4. compression per degree.  The single-pass result from the first Gram
  // is accepted for a degree when its first-pass error stays below the
  // target: eta1 * cond(G_k) * tau / |lambda|_max,k <= target, with eta1 the
  // relative accuracy of the first Gram (binary64 1e-16, split binary32
  // 1e-9) and target 1e-14 (binary64) or 1e-3 tol (mixed).  The other
  // degrees are refined by a second, binary64 Gram pass over the
  // preconditioned radial columns (CholeskyQR2-style; one more sync).
  t0 = now_ms();
  const double eta1 = (gram_mode == 0) ? 1e-16 : (gram_mode == 2 ? 1e-9 : 1e-6);
  const double target = (prec == HDF_FP64) ? 1e-14 : 1e-3 * tol;
  const double floor_rel = (gram_mode == 0) ? 1e-15 : (gram_mode == 2 ? 1e-10 : 1e-6);
  f->deg.resize(K + 1);
  std::vector<hdf::Precond> pcs(K + 1);
  std::vector<double> t1_all;
  std::vector<int32_t> t1_off(K + 1, 0);
  std::vector<int> refine;
  std::vector<char> needs_refine(K + 1, 0);
  // the degrees are independent (host pool); the refinement list and the T1 table follow in
  // degree order
  hdf::parallel_for(K + 1, [&](int k) {
    const int L = K - k + 1;
    std::vector<double> G((size_t)L * L);
    for (int aa = 0; aa < L; ++aa)
      for (int bb = 0; bb < L; ++bb)
        G[(size_t)aa * L + bb] = 0.5 * (mom[(size_t)k * mcols + aa + bb] + mom[(size_t)k * mcols + std::abs(aa - bb)]);
    hdf::gram_precondition(L, G.data(), floor_rel, pcs[k]);
    double gmax = 0.0, gmin = INFINITY;
    for (double v : pcs[k].lam1c) { gmax = std::max(gmax, v); gmin = std::min(gmin, v); }
    const double cond = gmax / gmin;
    hdf::compress_degree_eig(k, L, pcs[k].w1.data(), pcs[k].V1.data(), f->cores[k].data(), f->tau, floor_rel,
                             f->deg[k]);
    double lmax = 0.0;
    for (double v : f->deg[k].lam) lmax = std::max(lmax, std::fabs(v));
    const double est = eta1 * cond * (lmax > 0 ? f->tau / lmax : 1.0);
    needs_refine[k] = est > target;
  });
  for (int k = 0; k <= K; ++k) {
    if (needs_refine[k]) refine.push_back(k);
    t1_off[k] = (int32_t)t1_all.size();
    t1_all.insert(t1_all.end(), pcs[k].T1.begin(), pcs[k].T1.end());
  }
  f->n_refined = (int)refine.size();
  if (!refine.empty()) {
    DevBuf t1d, t1o, g2, g2part, selk;
    const int gb2 = hdf::gram2_blocks(n, (int)refine.size());
    HIPCHK(t1d.ensure(t1_all.size() * 8));
    HIPCHK(t1o.ensure(t1_off.size() * 4));
    HIPCHK(selk.ensure(refine.size() * 4));
    HIPCHK(g2.ensure(refine.size() * 1024 * 8));
    HIPCHK(g2part.ensure((size_t)gb2 * refine.size() * 1024 * 8));
    std::vector<int32_t> sel(refine.begin(), refine.end());
    HIPCHK(hipMemcpyAsync(t1d.p, t1_all.data(), t1_all.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(t1o.p, t1_off.data(), t1_off.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(selk.p, sel.data(), sel.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hdf::launch_gram2(f->x_soa.p, dtype, f->ldN, n, d, (const hdf::GeoDev*)f->geo_dev.p, f->u0,
                             f->u1, K, (const double*)t1d.p, (const int32_t*)t1o.p,
                             (const int32_t*)selk.p, (int)sel.size(), (double*)g2part.p,
                             (double*)g2.p, s));
    std::vector<double> g2h(refine.size() * 1024);
    HIPCHK(hipMemcpyAsync(g2h.data(), g2.p, g2h.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t ri = 0; ri < refine.size(); ++ri) {
      const int k = refine[ri];
      const int L = K - k + 1;
      std::vector<double> G2((size_t)L * L);
      for (int aa = 0; aa < L; ++aa)
        for (int bb = 0; bb < L; ++bb) G2[(size_t)aa * L + bb] = g2h[ri * 1024 + aa * 32 + bb];
      hdf::compress_degree_refined(k, L, G2.data(), pcs[k], f->cores[k].data(), f->tau, 1e-14, f->deg[k]);
    }
  }
  f->tau0 = f->tau;
  if (rule == HDF_RULE_SAMPLED) {
    // raise tau from the budget value while the sampled error allows; the
    // kept eigenpairs of every degree are a prefix in |lambda| order
    f->tau = hdf::tune_threshold(kernel, lengthscale, d, (double)n, f->u0, f->u1, f->deg, ps, tol, margin, f->tau0,
                                 &f->est_error);
    for (int k = 0; k <= K; ++k) {
      hdf::DegreeFactor& df = f->deg[k];
      int sk = 0;
      while (sk < df.s && std::fabs(df.lam[sk]) > f->tau) ++sk;
      df.s = sk;
      df.lam.resize(sk);
      df.E.resize((size_t)sk * df.L);
      df.Ep.resize((size_t)sk * df.L);
    }
  }
  {
    const hdf_status st = finish_build(f.get(), t0, s);
    if (st != HDF_OK) return st;
  }
  *out = f.release();
  return HDF_OK;
}

// ------------------------------------------------------------------ general build
hdf_status hdf_build_cross(const void* x, int64_t nx, int64_t ldx, const void* y, int64_t ny, int64_t ldy,
                           int dtype, int d, hdf_kernel kernel, double lengthscale, double tol,
                           hdf_precision prec, void* hip_stream, hdf_handle* out) {
  g_err.clear();
  if (!out) return fail(HDF_E_ARG, "out is NULL");
  if (!x || !y) return fail(HDF_E_ARG, "x or y is NULL");
  if (d < 3 || d > HDF_MAX_DIM) return fail(HDF_E_DIM, "d must be in [3, 8]");
  if (nx < 1 || ny < 1) return fail(HDF_E_ARG, "nx and ny must be >= 1");
  if (ldx < d || ldy < d) return fail(HDF_E_ARG, "leading dimensions must be >= d");
  if (dtype != 0 && dtype != 1) return fail(HDF_E_ARG, "dtype must be 0 (f32) or 1 (f64)");
  if (prec != HDF_FP64 && prec != HDF_MIXED) return fail(HDF_E_ARG, "unknown precision");
  if ((prec == HDF_MIXED) != (dtype == 0))
    return fail(HDF_E_ARG, "HDF_MIXED needs float32 points, HDF_FP64 needs float64 points");
  if ((int)kernel < 0 || (int)kernel > 3) return fail(HDF_E_ARG, "unknown kernel");
  if (!(lengthscale > 0) || !std::isfinite(lengthscale)) return fail(HDF_E_ARG, "lengthscale must be > 0");
  if (!(tol > 0 && tol < 1)) return fail(HDF_E_ARG, "tol must be in (0, 1)");
  hipStream_t s = (hipStream_t)hip_stream;

  std::unique_ptr<hdf_factor> f(new hdf_factor());
  f->cross = true;
  f->d = d; f->prec = prec; f->dtype = dtype; f->kernel = kernel;
  f->fprec = (prec == HDF_MIXED && tol > HDF_SPLIT_TOL) ? 1 : 0;
  f->N = nx; f->N2 = ny; f->l = lengthscale; f->tol = tol;
  f->ldN = (nx + 63) / 64 * 64 + 64;
  f->ldN2 = (ny + 63) / 64 * 64 + 64;
  const size_t in_elem = dtype == 0 ? 4 : 8;

  // 1. geometry of X u Y and the cross-pair norm sample, one sync
  double t0 = now_ms();
  HIPCHK(f->x_soa.ensure((size_t)d * f->ldN * in_elem));
  HIPCHK(f->x_soa2.ensure((size_t)d * f->ldN2 * in_elem));
  HIPCHK(f->geo_dev.ensure(sizeof(hdf::GeoDev)));
  HIPCHK(f->part.ensure((size_t)hdf::kPrepBlocks * 64 * sizeof(double)));
  HIPCHK(hdf::launch_prep_cross(x, nx, ldx, y, ny, ldy, dtype, d, f->x_soa.p, f->ldN, f->x_soa2.p, f->ldN2,
                                kernel, lengthscale, (double*)f->part.p, (hdf::GeoDev*)f->geo_dev.p, s));
  HIPCHK(hipMemcpyAsync(&f->geo, f->geo_dev.p, sizeof(hdf::GeoDev), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  f->t_prep = now_ms() - t0;
  if (f->geo.nonfinite > 0) return fail(HDF_E_NONFINITE, "points contain NaN or Inf");

  // 2. host planner (degree rule as in the symmetric case)
  t0 = now_ms();
  f->nu = std::sqrt(f->geo.nu2_sum / (double)hdf::kNuPairs);
  const double D = 2.0 * f->geo.R;
  std::vector<double> afull(hdf::kChebNodes);
  hdf::chebyshev_coeffs(kernel, D, lengthscale, hdf::kChebNodes, false, afull.data());
  f->p = hdf::choose_degree(afull.data(), hdf::kChebNodes, tol * f->nu / 2.0, HDF_MAX_DEGREE, &f->tail);
  f->p_bound = f->p;
  if (f->p < 0) {
    int pp = hdf::choose_degree(afull.data(), hdf::kChebNodes, tol * f->nu / 2.0, hdf::kChebNodes - 2, nullptr);
    char buf[160];
    snprintf(buf, sizeof buf, "Chebyshev degree %d needed (> %d): diameter/lengthscale too large for tol",
             pp, HDF_MAX_DEGREE);
    return fail(HDF_E_INFEASIBLE, buf);
  }
  f->K = f->p / 2;
  f->a.assign(afull.begin(), afull.begin() + f->p + 1);
  hdf::radial_interval(f->geo.rho2_min, f->geo.rho2_max, &f->u0, &f->u1);
  f->t_plan = now_ms() - t0;

  // 3. radial Gram moments of both sets, one sync; cores and tau meanwhile
  t0 = now_ms();
  const int K = f->K;
  const int nrt = (K + 1 + 15) / 16, nct = (2 * K + 1 + 15) / 16;
  const int gram_mode = (prec == HDF_FP64) ? 0 : 2;
  const int gb = std::max(hdf::gram_blocks(nx), hdf::gram_blocks(ny));
  const size_t mom_n = (size_t)nrt * 16 * nct * 16;
  HIPCHK(f->part.ensure(std::max((size_t)gb * mom_n * sizeof(double) + 4096,
                                 (size_t)hdf::kPrepBlocks * 64 * sizeof(double))));
  HIPCHK(f->moments.ensure(2 * mom_n * sizeof(double)));
  HIPCHK(hdf::launch_gram(f->x_soa.p, dtype, f->ldN, nx, d, (const hdf::GeoDev*)f->geo_dev.p, f->u0, f->u1,
                          K, gram_mode, (double*)f->part.p, (double*)f->moments.p, s));
  HIPCHK(hdf::launch_gram(f->x_soa2.p, dtype, f->ldN2, ny, d, (const hdf::GeoDev*)f->geo_dev.p, f->u0, f->u1,
                          K, gram_mode, (double*)f->part.p, (double*)f->moments.p + mom_n, s));
  const int mcols = nct * 16;
  std::vector<double> mom(2 * mom_n);
  HIPCHK(hipMemcpyAsync(mom.data(), f->moments.p, mom.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  const double t_overlap = now_ms();
  hdf::radial_cores(f->a.data(), f->p, d, f->u0, f->u1, f->cores);
  f->tau = hdf::tau_threshold(tol, f->nu, std::sqrt((double)nx * (double)ny), d, f->p);
  f->tau0 = f->tau;
  const double t_cores = now_ms() - t_overlap;
  HIPCHK(hipStreamSynchronize(s));
  f->t_plan += t_cores;
  f->t_gram = now_ms() - t0 - t_cores;

  // 4. compression per degree (SVD of R_x M R_y^T); a degree whose first-pass
  // Gram error on either side exceeds the target is refined by a second,
  // binary64 Gram pass of both sets
  t0 = now_ms();
  const double eta1 = (gram_mode == 0) ? 1e-16 : 1e-9;
  const double target = (prec == HDF_FP64) ? 1e-14 : 1e-3 * tol;
  const double floor_rel = (gram_mode == 0) ? 1e-15 : 1e-10;
  f->deg.resize(K + 1);
  f->degy.resize(K + 1);
  std::vector<hdf::DegreeFactorCross> dc(K + 1);
  std::vector<hdf::Precond> pcx(K + 1), pcy(K + 1);
  std::vector<double> t1x, t1y;
  std::vector<int32_t> t1_off(K + 1, 0);
  std::vector<int> refine;
  auto gram_of = [&](const double* mm, int k, int L, std::vector<double>& G) {
    G.assign((size_t)L * L, 0.0);
    for (int aa = 0; aa < L; ++aa)
      for (int bb = 0; bb < L; ++bb)
        G[(size_t)aa * L + bb] = 0.5 * (mm[(size_t)k * mcols + aa + bb] + mm[(size_t)k * mcols + std::abs(aa - bb)]);
  };
  auto cond_of = [](const hdf::Precond& pc) {
    double gmax = 0.0, gmin = INFINITY;
    for (double v : pc.lam1c) { gmax = std::max(gmax, v); gmin = std::min(gmin, v); }
    return gmax / gmin;
  };
  for (int k = 0; k <= K; ++k) {
    const int L = K - k + 1;
    std::vector<double> Gx, Gy;
    gram_of(mom.data(), k, L, Gx);
    gram_of(mom.data() + mom_n, k, L, Gy);
    hdf::gram_precondition(L, Gx.data(), floor_rel, pcx[k]);
    hdf::gram_precondition(L, Gy.data(), floor_rel, pcy[k]);
    hdf::SqrtFactor fx, fy;
    hdf::sqrt_factor_single(L, Gx.data(), floor_rel, fx);
    hdf::sqrt_factor_single(L, Gy.data(), floor_rel, fy);
    hdf::compress_degree_cross(k, L, fx, fy, f->cores[k].data(), f->tau, dc[k]);
    double smax = 0.0;
    for (double v : dc[k].sig) smax = std::max(smax, v);
    const double est = eta1 * std::max(cond_of(pcx[k]), cond_of(pcy[k])) * (smax > 0 ? f->tau / smax : 1.0);
    if (est > target) refine.push_back(k);
    t1_off[k] = (int32_t)t1x.size();
    t1x.insert(t1x.end(), pcx[k].T1.begin(), pcx[k].T1.end());
    t1y.insert(t1y.end(), pcy[k].T1.begin(), pcy[k].T1.end());
  }
  f->n_refined = (int)refine.size();
  if (!refine.empty()) {
    DevBuf t1dx, t1dy, t1o, g2, g2part, selk;
    const int nsel = (int)refine.size();
    const int gb2 = std::max(hdf::gram2_blocks(nx, nsel), hdf::gram2_blocks(ny, nsel));
    HIPCHK(t1dx.ensure(t1x.size() * 8));
    HIPCHK(t1dy.ensure(t1y.size() * 8));
    HIPCHK(t1o.ensure(t1_off.size() * 4));
    HIPCHK(selk.ensure(refine.size() * 4));
    HIPCHK(g2.ensure(2 * refine.size() * 1024 * 8));
    HIPCHK(g2part.ensure((size_t)gb2 * refine.size() * 1024 * 8));
    std::vector<int32_t> sel(refine.begin(), refine.end());
    HIPCHK(hipMemcpyAsync(t1dx.p, t1x.data(), t1x.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(t1dy.p, t1y.data(), t1y.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(t1o.p, t1_off.data(), t1_off.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(selk.p, sel.data(), sel.size() * 4, hipMemcpyHostToDevice, s));
    HIPCHK(hdf::launch_gram2(f->x_soa.p, dtype, f->ldN, nx, d, (const hdf::GeoDev*)f->geo_dev.p, f->u0, f->u1,
                             K, (const double*)t1dx.p, (const int32_t*)t1o.p, (const int32_t*)selk.p, nsel,
                             (double*)g2part.p, (double*)g2.p, s));
    HIPCHK(hdf::launch_gram2(f->x_soa2.p, dtype, f->ldN2, ny, d, (const hdf::GeoDev*)f->geo_dev.p, f->u0,
                             f->u1, K, (const double*)t1dy.p, (const int32_t*)t1o.p, (const int32_t*)selk.p,
                             nsel, (double*)g2part.p, (double*)g2.p + refine.size() * 1024, s));
    std::vector<double> g2h(2 * refine.size() * 1024);
    HIPCHK(hipMemcpyAsync(g2h.data(), g2.p, g2h.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (size_t ri = 0; ri < refine.size(); ++ri) {
      const int k = refine[ri];
      const int L = K - k + 1;
      std::vector<double> G2x((size_t)L * L), G2y((size_t)L * L);
      for (int aa = 0; aa < L; ++aa)
        for (int bb = 0; bb < L; ++bb) {
          G2x[(size_t)aa * L + bb] = g2h[ri * 1024 + aa * 32 + bb];
          G2y[(size_t)aa * L + bb] = g2h[(refine.size() + ri) * 1024 + aa * 32 + bb];
        }
      hdf::SqrtFactor fx, fy;
      hdf::sqrt_factor_refined(L, G2x.data(), pcx[k], 1e-14, fx);
      hdf::sqrt_factor_refined(L, G2y.data(), pcy[k], 1e-14, fy);
      hdf::compress_degree_cross(k, L, fx, fy, f->cores[k].data(), f->tau, dc[k]);
    }
  }
  for (int k = 0; k <= K; ++k) {
    hdf::DegreeFactor& dx = f->deg[k];
    hdf::DegreeFactor& dy = f->degy[k];
    dx.k = dy.k = k;
    dx.L = dy.L = K - k + 1;
    dx.s = dy.s = dc[k].s;
    dx.lam = dy.lam = dc[k].sig;
    dx.E = dc[k].Ex;
    dy.E = dc[k].Ey;
  }
  {
    const hdf_status st = finish_build(f.get(), t0, s);
    if (st != HDF_OK) return st;
  }
  *out = f.release();
  return HDF_OK;
}

// ------------------------------------------------------------------ matvec
// Pass 1 (W = U^T V, binary64) and the scaled copy Wd = D W for pass 2.
// side 0: the factor's (X) rows; side 1: the Y rows of a general factor.
// Matrix-free factor: evaluate the harmonics and radial functions of points [c0, c0 + nc) into the
// chunk scratch (padding columns cleared, as for a stored factor).
static hdf_status eval_chunk(hdf_handle h, int64_t c0, int64_t nc, hipStream_t s) {
  const size_t in_el = h->dtype == 0 ? 4 : 8;
  HIPCHK(hdf::launch_build((const char*)h->x_soa.p + c0 * in_el, h->dtype, h->ldN, nc, h->d,
                           (const hdf::GeoDev*)h->geo_dev.p, h->u0, h->u1, h->tables, h->fprec, h->cphi.p, h->ldC,
                           h->cq.p, h->ldC, s));
  HIPCHK(clear_padding(h->cphi.p, h->H, nc, h->ldC, h->felem(), s));
  HIPCHK(clear_padding(h->cq.p, h->S, nc, h->ldC, h->felem(), s));
  return HDF_OK;
}

static hdf_status pass1(hdf_handle h, int side, const void* V, int64_t m, int64_t ldv, int m16, DevBuf& W,
                        DevBuf& Wd, hipStream_t s, bool timed);

// Pass 1 of a matrix-free factor: per chunk, evaluate the factor, then contract it into its own range
// of split partials; one fixed-order reduction over all chunks' partials gives W.
// Device tables of the tile-major pass 1 for cpl = m16 / 16 (1..4), built with the factor.
static const hdf::MvtWave* tile_waves(hdf_handle h, int cpl) {
  return (const hdf::MvtWave*)h->tile_tabs.p + h->tw_off[cpl];
}
static const hdf::MvtRankRow* tile_rank_rows(hdf_handle h) {
  return (const hdf::MvtRankRow*)((const char*)h->tile_tabs.p + h->rr_base);
}
static const hdf::MvtGroup* tile_groups(hdf_handle h, int cpl) {
  return (const hdf::MvtGroup*)((const char*)h->tile_tabs.p + h->tg_base) + h->tg_off[cpl];
}

// Splits of the tile-major pass 1 over n points: about 1024 workgroups (of G groups each; two run
// at once on a CU), splits a multiple of 128 points, partial records capped at about 96 MB.
static void tile_splits(int64_t n, int n_groups, size_t per_split, int* n_splits, int64_t* split_len) {
  int64_t ns = std::max<int64_t>(1, 1024 / std::max(1, n_groups));
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, (int64_t)(96e6 / (double)per_split)));
  ns = std::min<int64_t>(ns, (n + 127) / 128);
  ns = std::max<int64_t>(ns, 1);
  int64_t len = (n + ns - 1) / ns;
  len = (len + 127) / 128 * 128;                 // whole rounds of the kernel's four-chunk prefetch
  *split_len = len;
  *n_splits = (int)((n + len - 1) / len);
}

// Pass 1 of a matrix-free factor: per chunk, evaluate the factor, then contract it into its own range
// of split partials; one fixed-order reduction over all chunks' partials gives W.
static hdf_status pass1_chunked(hdf_handle h, const void* V, int64_t m, int64_t ldv, int m16, DevBuf& W,
                                DevBuf& Wd, hipStream_t s, bool timed) {
  const size_t el = h->felem();
  const int cpl = m16 / 16;
  const size_t per_split = (size_t)h->r * m16 * sizeof(double);
  // work items and groups as for a stored factor of chunk points
  hdf_status st = pass1(h, 2, V, m, ldv, m16, W, Wd, s, false);   // side 2: tables only
  if (st != HDF_OK) return st;
  const bool tile = m16 <= 64;
  std::vector<int> splits;
  std::vector<int64_t> slen;
  int total = 0;
  for (int64_t c0 = 0; c0 < h->N; c0 += h->chunk) {
    const int64_t nc = std::min(h->chunk, h->N - c0);
    int ns;
    int64_t len;
    if (tile) {
      tile_splits(nc, h->n_tgroups[cpl], per_split, &ns, &len);
    } else {
      ns = (int)std::max<int64_t>(1, 16384 / std::max<int64_t>(1, (int64_t)h->n_tiles));
      ns = (int)std::min<int64_t>(ns, (nc + 1023) / 1024);
      ns = std::max(ns, 1);
      len = ((nc + ns - 1) / ns + 15) / 16 * 16;
      ns = (int)((nc + len - 1) / len);
    }
    splits.push_back(ns);
    slen.push_back(len);
    total += ns;
  }
  if ((double)per_split * total > 1.5e9)
    return fail(HDF_E_INFEASIBLE, "matrix-free pass 1 needs more than 1.5 GB of partial sums: use a larger chunk");
  HIPCHK(h->ws_part.ensure(per_split * total));
  HIPCHK(W.ensure((size_t)h->r * m16 * sizeof(double)));
  HIPCHK(Wd.ensure((size_t)h->r * m16 * el));
  if (timed) {
    if (!h->ev_mv[0])
      for (auto& e : h->ev_mv) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(h->ev_mv[0], s));
  }
  int slot = 0;
  size_t ci = 0;
  for (int64_t c0 = 0; c0 < h->N; c0 += h->chunk, ++ci) {
    const int64_t nc = std::min(h->chunk, h->N - c0);
    st = eval_chunk(h, c0, nc, s);
    if (st != HDF_OK) return st;
    const void* Vc = (const char*)V + c0 * ldv * h->ioel();
    double* part = (double*)h->ws_part.p + (size_t)slot * h->r * m16;
    if (tile)
      HIPCHK(hdf::launch_matvec_t_tile(h->cphi.p, h->ldC, h->cq.p, h->ldC, tile_waves(h, cpl), tile_rank_rows(h),
                                       tile_groups(h, cpl), h->n_tgroups[cpl], splits[ci], slen[ci], Vc, ldv, nc,
                                       (int)m, m16, h->r, part,
                                       h->fprec, h->dtype, s));
    else
      HIPCHK(hdf::launch_matvec_t(h->cphi.p, h->ldC, h->cq.p, h->ldC, (const hdf::DegDev*)h->degs_dev.p,
                                  (const hdf::TileDev*)h->tiles_dev.p, h->n_tiles, h->max_s * cpl, Vc, ldv, nc,
                                  (int)m, m16, splits[ci], slen[ci], h->r, part, h->fprec, h->dtype, s));
    slot += splits[ci];
  }
  if (timed) HIPCHK(hipEventRecord(h->ev_mv[1], s));
  HIPCHK(hdf::launch_matvec_reduce((const double*)h->ws_part.p, total, h->r, m16, (const double*)h->lam_row.p,
                                   (double*)W.p, Wd.p, h->fprec, s));
  if (timed) HIPCHK(hipEventRecord(h->ev_mv[2], s));
  return HDF_OK;
}

// Arguments of the fused matrix-free kernels.
static hdf::MfArgs mf_args(hdf_handle h) {
  hdf::MfArgs a{};
  const char* base = (const char*)h->mf_tabs.p;
  a.x_soa = h->x_soa.p; a.ldx = h->ldN; a.n = h->N; a.dtype = h->dtype; a.d = h->d;
  a.geo = (const hdf::GeoDev*)h->geo_dev.p; a.u0 = h->u0; a.u1 = h->u1;
  a.jobs = (const hdf::MfJob*)base; a.job_off = (const int32_t*)(base + h->mf_o_joff);
  a.btab = (const int32_t*)(base + h->mf_o_bt); a.n_tasks = h->mf_ntasks;
  a.n_loop = h->mf_nloop;
  a.chain = h->chain.p; a.K = h->tables.K;
  a.qmat = base + h->mf_o_qm; a.S = (int)h->S; a.S_pad = h->mf_spad; a.L_pad = h->mf_lpad;
  a.H = h->H; a.prec = h->fprec;
  return a;
}

// Workgroups of one fused pass that run at once on the device (occupancy x CUs), queried once.
static int mf_resident(hdf_handle h, int pass) {
  int& nb = pass == 1 ? h->mf_nb1 : h->mf_nb2;
  if (!nb) nb = hdf::mf_blocks_per_cu(mf_args(h), pass, pass == 1 ? h->mf_lay1 : h->mf_lay2, h->mf_spec);
  return std::max(1, nb) * std::max(1, h->n_cu);
}

// Pass 1 of a fused matrix-free factor: one launch over splits of the points (one workgroup per
// resident slot), the split partials reduced as for a stored factor.
static hdf_status pass1_fused(hdf_handle h, const void* V, int64_t m, int64_t ldv, int m16, DevBuf& W, DevBuf& Wd,
                              hipStream_t s, bool timed) {
  const int cpl = m16 / 16;
  const int64_t n = h->N;
  const int ny = h->mf_g1 * cpl;
  int64_t ns = std::max<int64_t>(1, mf_resident(h, 1) / ny);
  const size_t per_split = (size_t)h->r * m16 * sizeof(double);
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, (int64_t)(256e6 / (double)per_split)));
  ns = std::min<int64_t>(ns, (n + hdf::kMfP - 1) / hdf::kMfP);
  const int64_t len = ((n + ns - 1) / ns + hdf::kMfP - 1) / hdf::kMfP * hdf::kMfP;
  const int n_splits = (int)((n + len - 1) / len);
  HIPCHK(h->ws_part.ensure(per_split * n_splits));
  HIPCHK(W.ensure((size_t)h->r * m16 * sizeof(double)));
  HIPCHK(Wd.ensure((size_t)h->r * m16 * h->felem()));
  if (timed) {
    if (!h->ev_mv[0])
      for (auto& e : h->ev_mv) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(h->ev_mv[0], s));
  }
  const char* base = (const char*)h->mf_tabs.p;
  HIPCHK(hdf::launch_mf_t(mf_args(h), h->mf_lay1, h->mf_spec, (const hdf::MfSlot1*)(base + h->mf_o_s1),
                          (const int32_t*)(base + h->mf_o_so1), (const int32_t*)(base + h->mf_o_r1), h->mf_nr1,
                          h->mf_g1, cpl, n_splits, len, V, ldv, (int)m, m16, h->r, (double*)h->ws_part.p, s));
  if (timed) HIPCHK(hipEventRecord(h->ev_mv[1], s));
  HIPCHK(hdf::launch_matvec_reduce((const double*)h->ws_part.p, n_splits, h->r, m16, (const double*)h->lam_row.p,
                                   (double*)W.p, Wd.p, h->fprec, s));
  if (timed) HIPCHK(hipEventRecord(h->ev_mv[2], s));
  return HDF_OK;
}

// Pass 2 of a fused matrix-free factor: KV = U (D W) over ranges of the points.
static hdf_status pass2_fused(hdf_handle h, int64_t m, int m16, void* KV, int64_t ldkv, hipStream_t s) {
  const int cpl = m16 / 16;
  const int64_t n = h->N;
  const int ny = h->mf_g2 * cpl;
  int64_t nr = std::max<int64_t>(1, mf_resident(h, 2) / ny);
  nr = std::min<int64_t>(nr, (n + hdf::kMfP - 1) / hdf::kMfP);
  const int64_t len = ((n + nr - 1) / nr + hdf::kMfP - 1) / hdf::kMfP * hdf::kMfP;
  const int n_ranges = (int)((n + len - 1) / len);
  if (h->mf_g2 > 1) HIPCHK(h->ws_n.ensure((size_t)h->mf_g2 * n * m * h->felem()));
  const char* base = (const char*)h->mf_tabs.p;
  HIPCHK(hdf::launch_mf_n(mf_args(h), h->mf_lay2, h->mf_spec, (const hdf::MfSlot2*)(base + h->mf_o_s2),
                          (const int32_t*)(base + h->mf_o_so2), (const int32_t*)(base + h->mf_o_r2), h->mf_nr2,
                          h->mf_g2, cpl, n_ranges, len, h->ws_Wd.p, m16, KV, ldkv, (int)m,
                          h->mf_g2 > 1 ? h->ws_n.p : nullptr, s));
  return HDF_OK;
}

// side 2 (matrix-free factors): build the work-item tables only.
static hdf_status pass1(hdf_handle h, int side, const void* V, int64_t m, int64_t ldv, int m16, DevBuf& W,
                        DevBuf& Wd, hipStream_t s, bool timed) {
  if (h->storage == HDF_STORE_NONE && side != 2)
    return h->mf_fused ? pass1_fused(h, V, m, ldv, m16, W, Wd, s, timed)
                       : pass1_chunked(h, V, m, ldv, m16, W, Wd, s, timed);
  const int64_t n = side == 1 ? h->N2 : (side == 2 ? h->chunk : h->N);
  const void* phi = side == 1 ? h->phi2.p : h->phi.p;
  const void* qv = side == 1 ? h->q2.p : h->q.p;
  const int64_t ldn = side == 1 ? h->ldN2 : h->ldN;
  const size_t el = h->felem();
  const int cpl = m16 / 16;
  const int max_nct = h->max_s * cpl;
  if (h->tiles_cpl != cpl) {
    // work items: (degree, row block, column slice), no empty slices
    std::vector<hdf::TileDev>& tiles = h->tiles_host;
    tiles.clear();
    const int nct = hdf::matvec_col_tiles(h->fprec);
    for (size_t di = 0; di < h->degs.size(); ++di)
      for (int h0 = 0; h0 < h->degs[di].nh; h0 += hdf::matvec_row_block())
        for (int ct0 = 0; ct0 < h->degs[di].s * cpl; ct0 += nct)
          tiles.push_back(hdf::TileDev{(int32_t)di, h0, ct0, 0});
    HIPCHK(h->tiles_dev.ensure(tiles.size() * sizeof(hdf::TileDev)));
    HIPCHK(hipMemcpyAsync(h->tiles_dev.p, tiles.data(), tiles.size() * sizeof(hdf::TileDev),
                          hipMemcpyHostToDevice, s));
    h->n_tiles = (int)tiles.size();
    h->tiles_cpl = cpl;
  }
  const size_t per_split = (size_t)h->r * m16 * sizeof(double);
  if (side == 2 && m16 > 64) return HDF_OK;
  if (m16 <= 64) {
    // tile-major variant: the wave items and groups of this cpl were built with the factor
    if (side == 2) return HDF_OK;
    int n_splits;
    int64_t split_len;
    tile_splits(n, h->n_tgroups[cpl], per_split, &n_splits, &split_len);
    HIPCHK(h->ws_part.ensure(per_split * n_splits));
    HIPCHK(W.ensure((size_t)h->r * m16 * sizeof(double)));
    HIPCHK(Wd.ensure((size_t)h->r * m16 * el));
    if (timed) {
      if (!h->ev_mv[0])
        for (auto& e : h->ev_mv) HIPCHK(hipEventCreate(&e));
      HIPCHK(hipEventRecord(h->ev_mv[0], s));
    }
    HIPCHK(hdf::launch_matvec_t_tile(phi, ldn, qv, ldn, tile_waves(h, cpl), tile_rank_rows(h), tile_groups(h, cpl),
                                     h->n_tgroups[cpl],
                                     n_splits, split_len, V, ldv, n, (int)m, m16, h->r, (double*)h->ws_part.p,
                                     h->fprec, h->dtype, s));
    if (timed) HIPCHK(hipEventRecord(h->ev_mv[1], s));
    HIPCHK(hdf::launch_matvec_reduce((const double*)h->ws_part.p, n_splits, h->r, m16,
                                     (const double*)h->lam_row.p, (double*)W.p, Wd.p, h->fprec, s));
    if (timed) HIPCHK(hipEventRecord(h->ev_mv[2], s));
    return HDF_OK;
  }
  if (side == 2) return HDF_OK;
  // about 16k wavefronts in pass 1, partial records capped at ~96 MB
  int n_splits = (int)std::max<int64_t>(1, 16384 / std::max<int64_t>(1, (int64_t)h->n_tiles));
  n_splits = (int)std::min<int64_t>(n_splits, std::max<int64_t>(1, (int64_t)(96e6 / (double)per_split)));
  n_splits = (int)std::min<int64_t>(n_splits, (n + 1023) / 1024);
  n_splits = std::max(n_splits, 1);
  int64_t split_len = (n + n_splits - 1) / n_splits;
  split_len = (split_len + 15) / 16 * 16;
  n_splits = (int)((n + split_len - 1) / split_len);
  HIPCHK(h->ws_part.ensure(per_split * n_splits));
  HIPCHK(W.ensure((size_t)h->r * m16 * sizeof(double)));
  HIPCHK(Wd.ensure((size_t)h->r * m16 * el));
  if (timed) {
    if (!h->ev_mv[0])
      for (auto& e : h->ev_mv) HIPCHK(hipEventCreate(&e));
    HIPCHK(hipEventRecord(h->ev_mv[0], s));
  }
  HIPCHK(hdf::launch_matvec_t(phi, ldn, qv, ldn, (const hdf::DegDev*)h->degs_dev.p,
                              (const hdf::TileDev*)h->tiles_dev.p, h->n_tiles, max_nct, V, ldv, n,
                              (int)m, m16, n_splits, split_len, h->r, (double*)h->ws_part.p,
                              h->fprec, h->dtype, s));
  if (timed) HIPCHK(hipEventRecord(h->ev_mv[1], s));
  HIPCHK(hdf::launch_matvec_reduce((const double*)h->ws_part.p, n_splits, h->r, m16,
                                   (const double*)h->lam_row.p, (double*)W.p, Wd.p, h->fprec, s));
  if (timed) HIPCHK(hipEventRecord(h->ev_mv[2], s));
  return HDF_OK;
}

// Pass 2 over n points of a factor (phi, q with leading dimension ld): KV = U (D W), W from pass 1.
static hdf_status pass2(hdf_handle h, const void* phi, const void* q, int64_t ld, int64_t n, int64_t m, int m16,
                        void* KV, int64_t ldkv, hipStream_t s) {
  const size_t el = h->felem();
  // few points: split the harmonic rows so that pass 2 still has >= 1024 wavefronts
  const int64_t waves = ((n + 63) / 64) * (m16 / 16);
  int nz = 1, hchunk = 0;
  if (waves < 1024 && h->H >= 32) {
    const int64_t want = std::min<int64_t>((1024 + waves - 1) / waves, h->H / 16);
    if (want > 1) {
      hchunk = (int)(((h->H + want - 1) / want + 15) / 16 * 16);
      nz = (int)((h->H + hchunk - 1) / hchunk);
    }
  }
  if (nz > 1) HIPCHK(h->ws_n.ensure((size_t)nz * n * m * el));
  // one pass over the points: D W in batch-major order, four rows per lane in one load
  const void* Wb = nullptr;
  if (nz == 1) {
    HIPCHK(h->ws_Wb.ensure((size_t)h->n_wblocks * 16 * m16 * el));
    HIPCHK(hdf::launch_wd_batches((const hdf::DegDev*)h->degs_dev.p, (int)h->degs.size(), h->ws_Wd.p, m16,
                                  h->n_wblocks, h->ws_Wb.p, h->fprec, s));
    Wb = h->ws_Wb.p;
  }
  HIPCHK(hdf::launch_matvec_n(phi, ld, q, ld, (const hdf::DegDev*)h->degs_dev.p, (int)h->degs.size(), h->max_s,
                              h->ws_Wd.p, Wb, m16, KV, ldkv, n, (int)m, h->fprec, h->dtype, nz > 1 ? hchunk : 0, nz,
                              nz > 1 ? h->ws_n.p : nullptr, s));
  return HDF_OK;
}

static hdf_status matvec_impl(hdf_handle h, const void* V, int64_t m, int64_t ldv, void* KV,
                              int64_t ldkv, hipStream_t s) {
  const int64_t n = h->N;
  const size_t el = h->ioel();
  if (h->r == 0) {
    HIPCHK(hipMemset2DAsync(KV, ldkv * el, 0, m * el, n, s));
    return HDF_OK;
  }
  const int m16 = (int)((m + 15) / 16 * 16);
  const bool timed = h->time_products;
  hdf_status st = pass1(h, h->cross ? 1 : 0, V, m, ldv, m16, h->ws_W, h->ws_Wd, s, timed);
  if (st != HDF_OK) return st;
  if (h->storage == HDF_STORE_NONE && h->mf_fused) {
    st = pass2_fused(h, m, m16, KV, ldkv, s);
    if (st != HDF_OK) return st;
  } else if (h->storage == HDF_STORE_NONE) {
    for (int64_t c0 = 0; c0 < n; c0 += h->chunk) {
      const int64_t nc = std::min(h->chunk, n - c0);
      st = eval_chunk(h, c0, nc, s);
      if (st != HDF_OK) return st;
      st = pass2(h, h->cphi.p, h->cq.p, h->ldC, nc, m, m16, (char*)KV + c0 * ldkv * el, ldkv, s);
      if (st != HDF_OK) return st;
    }
  } else {
    st = pass2(h, h->phi.p, h->q.p, h->ldN, n, m, m16, KV, ldkv, s);
    if (st != HDF_OK) return st;
  }
  if (timed) {
    HIPCHK(hipEventRecord(h->ev_mv[3], s));
    h->mv_timed = true;
  }
  return HDF_OK;
}

hdf_status hdf_matvec(hdf_handle h, const void* V, int64_t m, int64_t ldv, void* KV, int64_t ldkv,
                      void* hip_stream) {
  g_err.clear();
  if (!h) return fail(HDF_E_ARG, "handle is NULL");
  if (!V || !KV) return fail(HDF_E_ARG, "V or KV is NULL");
  if (m < 1 || m > HDF_MAX_RHS) return fail(HDF_E_ARG, "m must be in [1, 256]");
  if (ldv < m || ldkv < m) return fail(HDF_E_ARG, "leading dimensions must be >= m");
  const size_t el = h->ioel();
  const char* v0 = (const char*)V;
  const char* v1 = v0 + (((h->cross ? h->N2 : h->N) - 1) * ldv + m) * el;
  const char* k0 = (const char*)KV;
  const char* k1 = k0 + ((h->N - 1) * ldkv + m) * el;
  if (v0 < k1 && k0 < v1) return fail(HDF_E_ARG, "V and KV overlap");
  return matvec_impl(h, V, m, ldv, KV, ldkv, (hipStream_t)hip_stream);
}

// The product without allocation: every work buffer (split partials, W, D W) lives in the
// library's per-GPU scratch array, the pass-1 tables were built with the factor, and pass 2 runs
// unsplit, so nothing is allocated and nothing is copied from the host.
hdf_status hdf_matvec_noalloc(hdf_handle h, const void* V, int64_t m, int64_t ldv, void* KV, int64_t ldkv,
                              void* hip_stream) {
  g_err.clear();
  if (!h) return fail(HDF_E_ARG, "handle is NULL");
  if (!V || !KV) return fail(HDF_E_ARG, "V or KV is NULL");
  if (m < 1 || m > 64) return fail(HDF_E_ARG, "hdf_matvec_noalloc takes 1 <= m <= 64");
  if (ldv < m || ldkv < m) return fail(HDF_E_ARG, "leading dimensions must be >= m");
  if (h->storage != HDF_STORE_FACTOR)
    return fail(HDF_E_ARG, "hdf_matvec_noalloc needs a stored factor (HDF_STORE_FACTOR)");
  const size_t io = h->ioel();
  {
    const char* v0 = (const char*)V;
    const char* v1 = v0 + (((h->cross ? h->N2 : h->N) - 1) * ldv + m) * io;
    const char* k0 = (const char*)KV;
    const char* k1 = k0 + ((h->N - 1) * ldkv + m) * io;
    if (v0 < k1 && k0 < v1) return fail(HDF_E_ARG, "V and KV overlap");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  if (h->r == 0) {
    HIPCHK(hipMemset2DAsync(KV, ldkv * io, 0, m * io, h->N, s));
    return HDF_OK;
  }
  void* base = nullptr;
  HIPCHK(hdf::scratch_address(&base));
  const int m16 = (int)((m + 15) / 16 * 16), cpl = m16 / 16;
  const size_t per_split = (size_t)h->r * m16 * sizeof(double);
  auto round256 = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t w_bytes = round256((size_t)h->r * m16 * sizeof(double));
  const size_t wd_bytes = round256((size_t)h->r * m16 * h->felem());
  if (w_bytes + wd_bytes + per_split > hdf::kScratchBytes) {
    char buf[200];
    snprintf(buf, sizeof buf, "rank %lld x %d columns needs %.3g MB of work space, above the %.3g MB scratch",
             (long long)h->r, m16, (double)(w_bytes + wd_bytes + per_split) / 1e6, (double)hdf::kScratchBytes / 1e6);
    return fail(HDF_E_INFEASIBLE, buf);
  }
  const int side = h->cross ? 1 : 0;
  const int64_t n1 = side ? h->N2 : h->N;
  int n_splits;
  int64_t split_len;
  tile_splits(n1, h->n_tgroups[cpl], per_split, &n_splits, &split_len);
  const int max_splits = (int)((hdf::kScratchBytes - w_bytes - wd_bytes) / per_split);
  if (n_splits > max_splits) {
    split_len = ((n1 + max_splits - 1) / max_splits + 31) / 32 * 32;
    n_splits = (int)((n1 + split_len - 1) / split_len);
  }
  double* W = (double*)base;
  void* Wd = (char*)base + w_bytes;
  double* part = (double*)((char*)base + w_bytes + wd_bytes);
  HIPCHK(hdf::launch_matvec_t_tile(side ? h->phi2.p : h->phi.p, side ? h->ldN2 : h->ldN, side ? h->q2.p : h->q.p,
                                   side ? h->ldN2 : h->ldN, tile_waves(h, cpl), tile_rank_rows(h), tile_groups(h, cpl),
                                   h->n_tgroups[cpl], n_splits, split_len, V, ldv, n1, (int)m, m16, h->r, part,
                                   h->fprec, h->dtype, s));
  HIPCHK(hdf::launch_matvec_reduce(part, n_splits, h->r, m16, (const double*)h->lam_row.p, W, Wd, h->fprec, s));
  HIPCHK(hdf::launch_matvec_n(h->phi.p, h->ldN, h->q.p, h->ldN, (const hdf::DegDev*)h->degs_dev.p,
                              (int)h->degs.size(), h->max_s, Wd, nullptr, m16, KV, ldkv, h->N, (int)m, h->fprec,
                              h->dtype, 0, 1, nullptr, s));
  return HDF_OK;
}

// dF/dX by factor contractions (the formula above k_radial in kernels.hip): with Gv = C U^T V and
// Gw = C U^T W (binary64, rank rows with stride gstride), the product of U' = phi q' with [Gv | Gw]
// and of the shifted factor S_{k-1} q_k with [G^(j)T Gv | G^(j)T Gw] for every direction j, then the
// pointwise combination.  Needs the kept degrees to be 0..K (every degree-(k-1) harmonic stored).
static hdf_status adjoint_dx(hdf_handle h, const double* gv, const double* gw, int64_t gstride, int m,
                             const void* Wm, const void* Vm, int64_t ld, void* dX, int64_t lddx, hipStream_t s) {
  const int d = h->d, m2 = 2 * m, md2 = m2 * d;
  const int Kh = h->kept_k.back();
  const size_t fel = h->felem();
  const int io = h->fprec == 1 ? 0 : 1;          // contraction outputs in the factor's type
  // derivative maps of the harmonic basis: depend on d and the degrees only, kept per process
  static std::mutex maps_mu;
  static std::map<std::pair<int, int>, std::vector<std::vector<double>>> maps;
  const std::vector<std::vector<double>>* G = nullptr;
  {
    std::lock_guard<std::mutex> lk(maps_mu);
    auto it = maps.find({d, Kh});
    if (it == maps.end()) {
      hdf::ChainCoeffs cc;
      hdf::chain_coeffs(d, Kh, cc);
      std::vector<int> rows_k(Kh + 1);
      for (int k = 0; k <= Kh; ++k) rows_k[k] = h->degs[k].hoff;
      std::vector<std::vector<double>> g;
      hdf::harmonic_derivative_maps(d, Kh, cc, h->col_of_host.data(), (int)h->H, rows_k, g);
      it = maps.emplace(std::make_pair(d, Kh), std::move(g)).first;
    }
    G = &it->second;
  }
  // shifted-factor degrees: harmonics of k - 1 with the radial rows and rank of degree k
  if (h->adj_degs_host.empty() && Kh >= 1) {
    int64_t roff = 0;
    for (int k = 1; k <= Kh; ++k) {
      const hdf::DegDev& dg = h->degs[k];
      const hdf::DegDev& d1 = h->degs[k - 1];
      hdf::DegDev e{};
      e.hoff = d1.hoff; e.nh = d1.nh; e.qoff = dg.qoff; e.s = dg.s; e.roff = (int32_t)roff;
      h->adj_degs_host.push_back(e);
      roff += (int64_t)d1.nh * dg.s;
    }
    h->r_shift = roff;
    HIPCHK(h->adj_degs.ensure(h->adj_degs_host.size() * sizeof(hdf::DegDev)));
    HIPCHK(hipMemcpyAsync(h->adj_degs.p, h->adj_degs_host.data(), h->adj_degs_host.size() * sizeof(hdf::DegDev),
                          hipMemcpyHostToDevice, s));
  }
  // q' = dq/d(rho^2): the derivative Chebyshev series of every radial function, scaled by dt/d(rho^2)
  if (!h->dq.p) {
    std::vector<double> dc;
    for (size_t di = 0; di < h->kept_k.size(); ++di) {
      const hdf::DegreeFactor& df = h->deg[h->kept_k[di]];
      const int L = df.L;
      for (int l = 0; l < df.s; ++l) {
        const double* c = &df.E[(size_t)l * L];
        std::vector<double> b(L + 2, 0.0);      // b_{a-1} = b_{a+1} + 2 a c_a, then b_0 / 2
        for (int a = L - 1; a >= 1; --a) b[a - 1] = b[a + 1] + 2.0 * a * c[a];
        b[0] *= 0.5;
        dc.insert(dc.end(), b.begin(), b.begin() + L);
      }
    }
    std::vector<char>& keep = h->adj_c2_host;   // reused below; the coefficients go first
    keep.assign(dc.size() * fel, 0);
    if (fel == 4)
      for (size_t i = 0; i < dc.size(); ++i) ((float*)keep.data())[i] = (float)dc[i];
    else
      std::memcpy(keep.data(), dc.data(), dc.size() * 8);
    HIPCHK(h->dq_coef.ensure(keep.size()));
    HIPCHK(hipMemcpyAsync(h->dq_coef.p, keep.data(), keep.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h->dq.ensure((size_t)h->S * h->ldN * fel));
    HIPCHK(hdf::launch_radial(h->x_soa.p, h->dtype, h->ldN, h->N, d, (const hdf::GeoDev*)h->geo_dev.p, h->u0,
                              h->u1, h->tables.q_len, h->tables.q_off, h->dq_coef.p, (int)h->S, 2.0 / (h->u1 - h->u0),
                              h->fprec, h->dq.p, h->ldN, s));
    HIPCHK(clear_padding(h->dq.p, h->S, h->N, h->ldN, fel, s));
    HIPCHK(hipStreamSynchronize(s));             // the coefficient copy above is read before keep is reused
  }
  // coefficients: C2 = [lambda gv | lambda gw] (rank x 2m), Cs = [G^(j)T C2]_j (shifted rank x 2m d)
  const int c2s = (m2 + 15) / 16 * 16, css = (md2 + 15) / 16 * 16;
  std::vector<double> C2((size_t)h->r * m2), Cs((size_t)std::max<int64_t>(h->r_shift, 1) * md2, 0.0);
  for (size_t di = 0; di < h->degs.size(); ++di) {
    const hdf::DegDev& dg = h->degs[di];
    const hdf::DegreeFactor& df = h->deg[h->kept_k[di]];
    for (int hh = 0; hh < dg.nh; ++hh)
      for (int l = 0; l < dg.s; ++l) {
        const int64_t row = dg.roff + (int64_t)hh * dg.s + l;
        for (int c = 0; c < m; ++c) {
          C2[row * m2 + c] = df.lam[l] * gv[row * gstride + c];
          C2[row * m2 + m + c] = df.lam[l] * gw[row * gstride + c];
        }
      }
  }
  for (int k = 1; k <= Kh; ++k) {
    const hdf::DegDev& dg = h->degs[k];
    const hdf::DegDev& e = h->adj_degs_host[k - 1];
    const int n0 = dg.nh, n1 = e.nh, sk = dg.s;
    const std::vector<double>& gk = (*G)[k];
    for (int j = 0; j < d; ++j)
      for (int hp = 0; hp < n1; ++hp)
        for (int l = 0; l < sk; ++l) {
          double* out = &Cs[(e.roff + (int64_t)hp * sk + l) * md2 + (int64_t)j * m2];
          for (int hh = 0; hh < n0; ++hh) {
            const double gg = gk[((size_t)j * n0 + hh) * n1 + hp];
            if (gg == 0.0) continue;
            const double* in = &C2[(dg.roff + (int64_t)hh * sk + l) * m2];
            for (int c = 0; c < m2; ++c) out[c] += gg * in[c];
          }
        }
  }
  auto pack = [&](const std::vector<double>& v, int64_t rows, int cols, int stride, std::vector<char>& dst) {
    dst.assign((size_t)std::max<int64_t>(rows, 1) * stride * fel, 0);
    for (int64_t r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) {
        const double x = v[r * cols + c];
        if (fel == 4) ((float*)dst.data())[r * stride + c] = (float)x;
        else ((double*)dst.data())[r * stride + c] = x;
      }
  };
  pack(C2, h->r, m2, c2s, h->adj_c2_host);
  pack(Cs, h->r_shift, md2, css, h->adj_cs_host);
  HIPCHK(h->adj_c2.ensure(h->adj_c2_host.size()));
  HIPCHK(h->adj_cs.ensure(h->adj_cs_host.size()));
  HIPCHK(hipMemcpyAsync(h->adj_c2.p, h->adj_c2_host.data(), h->adj_c2_host.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(h->adj_cs.p, h->adj_cs_host.data(), h->adj_cs_host.size(), hipMemcpyHostToDevice, s));
  HIPCHK(h->adj_kv2.ensure((size_t)h->N * m2 * fel));
  HIPCHK(h->adj_kvs.ensure((size_t)h->N * md2 * fel));
  if (!h->ev_adj[0])
    for (auto& e : h->ev_adj) HIPCHK(hipEventCreate(&e));
  HIPCHK(hipEventRecord(h->ev_adj[0], s));
  // U' [Gv | Gw] and the shifted factor times [G^(j)T Gv | G^(j)T Gw] (pass-2 kernel, one chunk)
  HIPCHK(hdf::launch_matvec_n(h->phi.p, h->ldN, h->dq.p, h->ldN, (const hdf::DegDev*)h->degs_dev.p,
                              (int)h->degs.size(), h->max_s, h->adj_c2.p, nullptr, c2s, h->adj_kv2.p, m2, h->N, m2,
                              h->fprec, io, 0, 1, nullptr, s));
  HIPCHK(hdf::launch_matvec_n(h->phi.p, h->ldN, h->q.p, h->ldN, (const hdf::DegDev*)h->adj_degs.p, Kh, h->max_s,
                              h->adj_cs.p, nullptr, css, h->adj_kvs.p, md2, h->N, md2, h->fprec, io, 0, 1, nullptr,
                              s));
  HIPCHK(hdf::launch_adj_combine(h->x_soa.p, h->dtype, h->ldN, h->N, d, (const hdf::GeoDev*)h->geo_dev.p,
                                 h->adj_kvs.p, md2, h->adj_kv2.p, m2, Wm, Vm, ld, m, dX, lddx, h->fprec, s));
  HIPCHK(hipEventRecord(h->ev_adj[1], s));
  h->adj_timed = true;
  return HDF_OK;
}

hdf_status hdf_backward(hdf_handle h, const void* Wm, const void* Vm, int64_t m, int64_t ld,
                        double* dlength, void* dX, int64_t lddx, void* hip_stream) {
  g_err.clear();
  if (!h) return fail(HDF_E_ARG, "handle is NULL");
  if (!Wm || !Vm) return fail(HDF_E_ARG, "W or V is NULL");
  if (m < 1 || m > HDF_MAX_RHS) return fail(HDF_E_ARG, "m must be in [1, 256]");
  if (ld < m) return fail(HDF_E_ARG, "ld must be >= m");
  if (dX && lddx < h->d) return fail(HDF_E_ARG, "lddx must be >= d");
  if (h->cross) return fail(HDF_E_ARG, "hdf_backward needs a symmetric factor (hdf_build)");
  if (dX && h->storage != HDF_STORE_FACTOR)
    return fail(HDF_E_ARG, "dF/dX needs a stored factor (HDF_STORE_FACTOR): it contracts the stored harmonics");
  if (dX && h->r > 0)
    for (size_t i = 0; i < h->kept_k.size(); ++i)
      if (h->kept_k[i] != (int)i)
        return fail(HDF_E_ARG, "dF/dX needs the kept degrees to be 0..K (a degree below the largest kept one "
                               "was dropped, so its harmonics, the derivatives of the next degree's, are not stored)");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t el = h->ioel(), fel = h->felem();
  (void)fel;
  if (!dlength && !dX) return HDF_OK;
  if (h->r == 0) {
    if (dlength) *dlength = 0.0;
    if (dX) HIPCHK(hipMemset2DAsync(dX, lddx * el, 0, h->d * el, h->N, s));
    return HDF_OK;
  }
  // U^T V and U^T W: one pass 1 over [V | W] (2m columns; a pass costs the
  // same for any m up to 16), two passes when 2m exceeds the column limit
  const bool joint = 2 * m <= HDF_MAX_RHS;
  int m16;
  const DevBuf *gv_src, *gw_src;
  int64_t gw_col = 0;
  if (joint) {
    const int64_t m2 = 2 * m;
    m16 = (int)((m2 + 15) / 16 * 16);
    HIPCHK(h->bw_VW.ensure((size_t)h->N * m2 * el));
    HIPCHK(hipMemcpy2DAsync(h->bw_VW.p, m2 * el, Vm, ld * el, m * el, h->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpy2DAsync((char*)h->bw_VW.p + m * el, m2 * el, Wm, ld * el, m * el, h->N,
                            hipMemcpyDeviceToDevice, s));
    hdf_status st = pass1(h, 0, h->bw_VW.p, m2, m2, m16, h->bw_GV, h->bw_GVd, s, false);
    if (st != HDF_OK) return st;
    gv_src = gw_src = &h->bw_GV;
    gw_col = m;
  } else {
    m16 = (int)((m + 15) / 16 * 16);
    hdf_status st = pass1(h, 0, Vm, m, ld, m16, h->bw_GV, h->bw_GVd, s, false);
    if (st != HDF_OK) return st;
    st = pass1(h, 0, Wm, m, ld, m16, h->bw_GW, h->bw_GWd, s, false);
    if (st != HDF_OK) return st;
    gv_src = &h->bw_GV;
    gw_src = &h->bw_GW;
  }
  if (dlength) {
    // dF/dl = sum_{k,h,c} gw^T (E'_k^T dM_k/dl E'_k) gv, dM/dl from the Chebyshev
    // coefficients of dk/dl with the structure (degree, radius, basis) frozen.
    // The cores of dk/dl (host work) are formed while the device runs the
    // passes above, and kept with the factor for later calls.
    if (h->dC.empty()) {
      std::vector<double> da(hdf::kChebNodes);
      hdf::chebyshev_coeffs(h->kernel, 2.0 * h->geo.R, h->l, hdf::kChebNodes, true, da.data());
      std::vector<std::vector<double>> dM;
      hdf::radial_cores(da.data(), h->p, h->d, h->u0, h->u1, dM);
      h->dC.resize(h->degs.size());
      for (size_t dj = 0; dj < h->degs.size(); ++dj) {
        const hdf::DegreeFactor& df = h->deg[h->kept_k[dj]];
        const int L = df.L, sk = df.s;
        const std::vector<double>& M = dM[df.k];
        std::vector<double> MEp((size_t)L * sk, 0.0);
        std::vector<double>& dC = h->dC[dj];
        dC.assign((size_t)sk * sk, 0.0);
        for (int a = 0; a < L; ++a)
          for (int l = 0; l < sk; ++l) {
            double acc = 0.0;
            for (int b = 0; b < L; ++b) acc += M[(size_t)a * L + b] * df.Ep[(size_t)l * L + b];
            MEp[(size_t)a * sk + l] = acc;
          }
        for (int l = 0; l < sk; ++l)
          for (int l2 = 0; l2 < sk; ++l2) {
            double acc = 0.0;
            for (int a = 0; a < L; ++a) acc += df.Ep[(size_t)l * L + a] * MEp[(size_t)a * sk + l2];
            dC[(size_t)l * sk + l2] = acc;
          }
      }
    }
  }
  // U^T V and U^T W on the host (binary64), one synchronisation
  std::vector<double> gv((size_t)h->r * m16), gwbuf;
  HIPCHK(hipMemcpyAsync(gv.data(), gv_src->p, gv.size() * 8, hipMemcpyDeviceToHost, s));
  if (!joint) {
    gwbuf.resize((size_t)h->r * m16);
    HIPCHK(hipMemcpyAsync(gwbuf.data(), gw_src->p, gwbuf.size() * 8, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  const double* gw = joint ? gv.data() + gw_col : gwbuf.data();
  if (dlength) {
    double dl = 0.0;
    for (size_t dj = 0; dj < h->degs.size(); ++dj) {
      const hdf::DegDev& dg = h->degs[dj];
      const int sk = dg.s;
      const std::vector<double>& dC = h->dC[dj];
      for (int hh = 0; hh < dg.nh; ++hh)
        for (int c = 0; c < m; ++c)
          for (int l = 0; l < sk; ++l) {
            const double gwl = gw[(size_t)(dg.roff + hh * sk + l) * m16 + c];
            if (gwl == 0.0) continue;
            double acc = 0.0;
            for (int l2 = 0; l2 < sk; ++l2) acc += dC[(size_t)l * sk + l2] * gv[(size_t)(dg.roff + hh * sk + l2) * m16 + c];
            dl += gwl * acc;
          }
    }
    *dlength = dl;
  }
  if (dX) {
    const hdf_status st = adjoint_dx(h, gv.data(), gw, m16, (int)m, Wm, Vm, ld, dX, lddx, s);
    if (st != HDF_OK) return st;
  }
  return HDF_OK;
}

// ------------------------------------------------------------------ info
hdf_status hdf_info(hdf_handle h, hdf_info_t* info) {
  g_err.clear();
  if (!h || !info) return fail(HDF_E_ARG, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n_dim = h->d;
  info->precision = h->prec;
  info->n_points = h->N;
  info->n_points_y = h->cross ? h->N2 : 0;
  info->degree_p = h->p;
  info->n_degrees = h->K + 1;
  info->n_harmonics = h->H;
  info->n_radial = h->S;
  info->rank = h->r;
  info->tau = h->tau;
  info->nu = h->nu;
  info->cheb_tail = h->tail;
  info->center_radius = h->geo.R;
  info->rho2_min = h->u0;
  info->rho2_max = h->u1;
  info->factor_bytes = h->mf_fused ? 0
                       : (int64_t)((h->H + h->S) *
                                   (h->storage == HDF_STORE_NONE ? h->ldC : h->ldN + (h->cross ? h->ldN2 : 0)) *
                                   h->felem());
  info->mf_fused = h->mf_fused ? (h->mf_spec ? 2 : 1) : 0;
  info->storage = h->storage;
  info->factor_precision = h->fprec == 1 ? HDF_MIXED : HDF_FP64;
  info->chunk_points = h->storage == HDF_STORE_NONE ? h->chunk : 0;
  info->t_prep_ms = h->t_prep;
  info->t_plan_ms = h->t_plan;
  info->t_gram_ms = h->t_gram;
  info->t_compress_ms = h->t_compress;
  info->t_finish_ms = h->t_finish;
  if (h->ev_b0 && h->ev_b1 && h->t_build < 0) {
    float ms = 0.f;
    if (hipEventSynchronize(h->ev_b1) == hipSuccess && hipEventElapsedTime(&ms, h->ev_b0, h->ev_b1) == hipSuccess)
      h->t_build = ms;
  }
  info->t_build_ms = h->t_build;
  info->n_refined = h->n_refined;
  info->rank_rule = h->rank_rule;
  info->tau_bound = h->tau0;
  info->est_error = h->est_error;
  info->degree_bound = h->p_bound;
  info->t_mv_t_ms = info->t_mv_reduce_ms = info->t_mv_n_ms = info->t_adjoint_ms = -1.0;
  if (h->adj_timed && hipEventSynchronize(h->ev_adj[1]) == hipSuccess) {
    float a = 0;
    if (hipEventElapsedTime(&a, h->ev_adj[0], h->ev_adj[1]) == hipSuccess) info->t_adjoint_ms = a;
  }
  if (h->mv_timed && hipEventSynchronize(h->ev_mv[3]) == hipSuccess) {
    float a = 0.f, b = 0.f, c2 = 0.f;
    if (hipEventElapsedTime(&a, h->ev_mv[0], h->ev_mv[1]) == hipSuccess) info->t_mv_t_ms = a;
    if (hipEventElapsedTime(&b, h->ev_mv[1], h->ev_mv[2]) == hipSuccess) info->t_mv_reduce_ms = b;
    if (hipEventElapsedTime(&c2, h->ev_mv[2], h->ev_mv[3]) == hipSuccess) info->t_mv_n_ms = c2;
  }
  for (int k = 0; k <= h->K && k <= HDF_MAX_DEGREE / 2; ++k) info->s_k[k] = h->deg[k].s;
  return HDF_OK;
}

hdf_status hdf_get_plan(hdf_handle h, int32_t* index_table, double* lambda, double* radial_coef,
                        double* a_cheb) {
  g_err.clear();
  if (!h) return fail(HDF_E_ARG, "handle is NULL");
  if (index_table) std::copy(h->index_table.begin(), h->index_table.end(), index_table);
  if (lambda || radial_coef) {
    size_t li = 0, ci = 0;
    for (int k = 0; k <= h->K; ++k) {
      const hdf::DegreeFactor& df = h->deg[k];
      for (int l = 0; l < df.s; ++l) {
        if (lambda) lambda[li] = df.lam[l];
        ++li;
      }
      if (radial_coef) std::copy(df.E.begin(), df.E.end(), radial_coef + ci);
      ci += df.E.size();
    }
  }
  if (a_cheb) std::copy(h->a.begin(), h->a.end(), a_cheb);
  return HDF_OK;
}

hdf_status hdf_copy_factor(hdf_handle h, void* phi_out, int64_t ld_phi, void* q_out, int64_t ld_q,
                           void* hip_stream) {
  g_err.clear();
  if (!h) return fail(HDF_E_ARG, "handle is NULL");
  if (h->storage == HDF_STORE_NONE) return fail(HDF_E_ARG, "a matrix-free factor (HDF_STORE_NONE) stores no factor");
  if ((phi_out && ld_phi < h->N) || (q_out && ld_q < h->N)) return fail(HDF_E_ARG, "leading dimension < n");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t el = h->felem();
  if (phi_out && h->H > 0)
    HIPCHK(hipMemcpy2DAsync(phi_out, ld_phi * el, h->phi.p, h->ldN * el, h->N * el, h->H,
                            hipMemcpyDeviceToDevice, s));
  if (q_out && h->S > 0)
    HIPCHK(hipMemcpy2DAsync(q_out, ld_q * el, h->q.p, h->ldN * el, h->N * el, h->S,
                            hipMemcpyDeviceToDevice, s));
  return HDF_OK;
}

hdf_status hdf_copy_factor_y(hdf_handle h, void* phi_out, int64_t ld_phi, void* q_out, int64_t ld_q,
                             void* hip_stream) {
  g_err.clear();
  if (!h) return fail(HDF_E_ARG, "handle is NULL");
  if (!h->cross) return fail(HDF_E_ARG, "the handle is a symmetric factor (no Y side)");
  if ((phi_out && ld_phi < h->N2) || (q_out && ld_q < h->N2)) return fail(HDF_E_ARG, "leading dimension < n_y");
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t el = h->felem();
  if (phi_out && h->H > 0)
    HIPCHK(hipMemcpy2DAsync(phi_out, ld_phi * el, h->phi2.p, h->ldN2 * el, h->N2 * el, h->H,
                            hipMemcpyDeviceToDevice, s));
  if (q_out && h->S > 0)
    HIPCHK(hipMemcpy2DAsync(q_out, ld_q * el, h->q2.p, h->ldN2 * el, h->N2 * el, h->S,
                            hipMemcpyDeviceToDevice, s));
  return HDF_OK;
}

// ------------------------------------------------------------------ host planner
hdf_status hdf_plan_compress_cross(int L, const double* Gx, const double* Gy, const double* M, double tau,
                                   double null_rel, int32_t* s, double* sig, double* Ex, double* Ey) {
  g_err.clear();
  if (!Gx || !Gy || !M || !s) return fail(HDF_E_ARG, "NULL argument");
  if (L < 1 || L > 32) return fail(HDF_E_ARG, "L must be in [1, 32]");
  hdf::SqrtFactor fx, fy;
  hdf::sqrt_factor_single(L, Gx, null_rel, fx);
  hdf::sqrt_factor_single(L, Gy, null_rel, fy);
  hdf::DegreeFactorCross out;
  hdf::compress_degree_cross(0, L, fx, fy, M, tau, out);
  *s = out.s;
  if (sig) std::copy(out.sig.begin(), out.sig.end(), sig);
  if (Ex) std::copy(out.Ex.begin(), out.Ex.end(), Ex);
  if (Ey) std::copy(out.Ey.begin(), out.Ey.end(), Ey);
  return HDF_OK;
}

hdf_status hdf_plan_chebyshev(hdf_kernel kernel, double D, double lengthscale, int n_nodes,
                              int derivative, double* a) {
  g_err.clear();
  if (!a) return fail(HDF_E_ARG, "a is NULL");
  if (n_nodes < 16 || (n_nodes & (n_nodes - 1))) return fail(HDF_E_ARG, "n_nodes must be a power of two >= 16");
  if ((int)kernel < 0 || (int)kernel > 3) return fail(HDF_E_ARG, "unknown kernel");
  if (!(lengthscale > 0) || !(D >= 0)) return fail(HDF_E_ARG, "need D >= 0 and lengthscale > 0");
  hdf::chebyshev_coeffs(kernel, D, lengthscale, n_nodes, derivative != 0, a);
  return HDF_OK;
}

hdf_status hdf_plan_degree(const double* a, int n, double eps, double nu, int p_max, int* p,
                           double* tail) {
  g_err.clear();
  if (!a || !p) return fail(HDF_E_ARG, "NULL argument");
  if (n < 2) return fail(HDF_E_ARG, "n must be >= 2");
  double t = 0;
  const int pp = hdf::choose_degree(a, n, eps * nu / 2.0, p_max, &t);
  if (pp < 0) return fail(HDF_E_INFEASIBLE, "no even degree <= p_max meets the tail bound");
  *p = pp;
  if (tail) *tail = t;
  return HDF_OK;
}

hdf_status hdf_plan_cores(const double* a, int p, int d, double u0, double u1, double* cores) {
  g_err.clear();
  if (!a || !cores) return fail(HDF_E_ARG, "NULL argument");
  if (p < 0 || (p % 2) || p > HDF_MAX_DEGREE) return fail(HDF_E_ARG, "p must be even in [0, HDF_MAX_DEGREE]");
  if (d < 3 || d > HDF_MAX_DIM) return fail(HDF_E_DIM, "d must be in [3, 8]");
  if (!(u1 > u0) || u0 < 0) return fail(HDF_E_ARG, "need 0 <= u0 < u1");
  std::vector<std::vector<double>> c;
  hdf::radial_cores(a, p, d, u0, u1, c);
  size_t o = 0;
  for (auto& M : c) {
    std::copy(M.begin(), M.end(), cores + o);
    o += M.size();
  }
  return HDF_OK;
}

hdf_status hdf_plan_index_set(int d, int k, int32_t* table, int64_t* count) {
  g_err.clear();
  if (!count) return fail(HDF_E_ARG, "count is NULL");
  if (d < 3 || d > HDF_MAX_DIM) return fail(HDF_E_DIM, "d must be in [3, 8]");
  if (k < 0) return fail(HDF_E_ARG, "k must be >= 0");
  std::vector<int32_t> t;
  hdf::index_set(d, k, t);
  *count = (int64_t)(t.size() / (d - 2));
  if (table) std::copy(t.begin(), t.end(), table);
  return HDF_OK;
}

}  // extern "C"
