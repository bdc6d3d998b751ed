// Runtime of the CPU emulation of the HIP kernels (test infrastructure).
//
// Each HIP thread is a fiber with its own stack; a block runs to completion
// before the next one starts.  __syncthreads is a block-wide collective and the
// 16x16x4 MFMA a wave-wide one (operand and accumulator lane layouts of gfx950).
// Device memory is host memory: hipMalloc'd buffers are exact-size heap blocks
// (AddressSanitizer redzones) or, with EMU_GUARD, end flush against a
// PROT_NONE region.  Stream work (launches, copies, event records) is queued
// and runs at synchronisation points, so host buffers handed to an async copy
// must still be alive when the stream is synchronised.
//
// Environment switches:
//   EMU_FILL=0xNN      byte written into fresh device memory and LDS (0xbe)
//   EMU_GUARD=1        guard regions after every device buffer
//   EMU_STRICT=1       every pointer argument of a kernel and every device side
//                      of a copy must be library or registered user memory
//   EMU_ORDER=0..3     thread order between collectives: forward, reverse,
//                      random permutation, waves reversed
//   EMU_STACK_KB, EMU_VERBOSE, EMU_WARN_EXIT_BARRIER
// Faults it reports: out-of-bounds and use-after-free (ASan), misaligned
// vector accesses (UBSan), host memory passed to a kernel, divergent barriers,
// MFMA or a lane shuffle issued by part of a wave or from different call
// sites, deadlock.
#define EMU_DEVICE_CODE
#include "emu_hip.h"

#include <sys/mman.h>

#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <vector>
#include <chrono>

namespace emu {

enum { READY = 0, BARRIER = 1, MFMA32 = 2, MFMA64 = 3, DONE = 4, SHFL = 5 };

struct Fiber {
  void* sp = nullptr;
  char* stack = nullptr;
  size_t ssize = 0;
  dim3 tid;
  int state = READY;
  int lane = 0, wave = 0;
  double a = 0, b = 0, c[4] = {0, 0, 0, 0}, dout[4] = {0, 0, 0, 0};
  const void* site = nullptr;   // call site of the pending barrier / MFMA
  long long nbar = 0;           // barriers passed
  long long nmfma = 0;          // MFMAs issued
};

Fiber* cur = nullptr;
dim3 g_blockIdx, g_blockDim, g_gridDim;
static std::vector<Fiber> fibers;
static const std::function<void()>* g_body = nullptr;
static unsigned char* g_dyn = nullptr;
static long long g_block_serial = 0;
static std::map<const void*, long long> g_shared_filled;
static int g_garbage = getenv("EMU_FILL") ? (int)strtol(getenv("EMU_FILL"), nullptr, 0) : 0xbe;
static long long g_launches = 0;
static hipError_t g_last = hipSuccess;
const char* g_kernel_name = "";

const dim3& tidx() { return cur->tid; }
unsigned char* dyn_smem() { return g_dyn; }

void garbage_once(void* p, size_t n) {
  auto it = g_shared_filled.find(p);
  if (it != g_shared_filled.end() && it->second == g_block_serial) return;
  g_shared_filled[p] = g_block_serial;
  memset(p, g_garbage, n);
}

// context switches: a minimal callee-saved-register swap (x86-64 SysV)
extern "C" void emu_swap(void** save_sp, void* new_sp);
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
.size emu_swap,.-emu_swap
)");
static void* main_sp = nullptr;

static void to_main() { emu_swap(&cur->sp, main_sp); }

extern "C" void emu_entry() {
  (*g_body)();
  cur->state = DONE;
  emu_swap(&cur->sp, main_sp);
  abort();
}

static void resume(Fiber* f) {
  cur = f;
  emu_swap(&main_sp, f->sp);
  cur = nullptr;
}

static void init_fiber(Fiber& f) {
  // initial frame: 6 callee-saved slots, then the return address emu_entry;
  // at emu_entry's first instruction rsp + 8 must be 16-byte aligned
  uintptr_t top = ((uintptr_t)f.stack + f.ssize) & ~(uintptr_t)15;
  void** sp = (void**)top;
  *--sp = nullptr;                      // fake return address of emu_entry (alignment)
  *--sp = (void*)&emu_entry;
  for (int i = 0; i < 6; ++i) *--sp = nullptr;
  f.sp = sp;
}

__attribute__((noinline)) void syncthreads() {
  cur->site = __builtin_return_address(0);
  cur->state = BARRIER;
  to_main();
}

// A barrier reached from different call sites that the kernel declares to be one barrier (the two
// roles of a wavefront-specialised kernel): the site is the given tag; counts must still agree.
void syncthreads_at(const void* site) {
  cur->site = site;
  cur->state = BARRIER;
  to_main();
}

// __syncthreads_count: a barrier that also counts the threads with p != 0
static int g_count_acc = 0;
int syncthreads_count(int p) {
  g_count_acc += p != 0;
  syncthreads();
  const int r = g_count_acc;
  syncthreads();
  if (tidx().x == 0) g_count_acc = 0;
  syncthreads();
  return r;
}

// __shfl_xor: a wave-wide collective; lane L receives the value of lane L ^ mask
__attribute__((noinline)) double shfl_xor(double v, int mask) {
  Fiber* f = cur;
  f->site = __builtin_return_address(0);
  f->a = v;
  f->b = mask;
  f->state = SHFL;
  to_main();
  return f->dout[0];
}

template <int MODE, typename T>
__attribute__((noinline)) static void mfma_arrive(T a, T b, const T* c, T* d, const void* site) {
  Fiber* f = cur;
  f->site = site;
  f->a = a; f->b = b;
  for (int e = 0; e < 4; ++e) f->c[e] = (double)c[e];
  f->state = MODE;
  to_main();
  for (int e = 0; e < 4; ++e) d[e] = (T)f->dout[e];
}

__attribute__((noinline)) f4 mfma_f32(float a, float b, f4 c) {
  float cc[4] = {c[0], c[1], c[2], c[3]}, dd[4];
  mfma_arrive<MFMA32, float>(a, b, cc, dd, __builtin_return_address(0));
  return f4{dd[0], dd[1], dd[2], dd[3]};
}
__attribute__((noinline)) d4 mfma_f64(double a, double b, d4 c) {
  double cc[4] = {c[0], c[1], c[2], c[3]}, dd[4];
  mfma_arrive<MFMA64, double>(a, b, cc, dd, __builtin_return_address(0));
  return d4{dd[0], dd[1], dd[2], dd[3]};
}

static void resolve_mfma(Fiber* w, int mode) {
  // lane r + 16 q supplies A[r][q], B[q][r]; lane j + 16 g element e holds D[row][j]
  for (int L = 0; L < 64; ++L) {
    const int j = L & 15, g = L >> 4;
    for (int e = 0; e < 4; ++e) {
      const int i = mode == MFMA32 ? 4 * g + e : g + 4 * e;
      if (mode == MFMA32) {
        float acc = (float)w[L].c[e];
        for (int q = 0; q < 4; ++q) acc = fmaf((float)w[i + 16 * q].a, (float)w[j + 16 * q].b, acc);
        w[L].dout[e] = acc;
      } else {
        double acc = w[L].c[e];
        for (int q = 0; q < 4; ++q) acc = fma(w[i + 16 * q].a, w[j + 16 * q].b, acc);
        w[L].dout[e] = acc;
      }
    }
  }
  for (int L = 0; L < 64; ++L) w[L].state = READY;
}

static void die(const char* what) {
  fprintf(stderr, "EMU ERROR in %s block %u: %s\n", g_kernel_name, g_blockIdx.x, what);
  fflush(stderr);
  abort();
}

void check_launch(unsigned grid, unsigned block, size_t shm) {
  if (grid == 0 || block == 0 || block > 1024 || shm > 160 * 1024) {
    fprintf(stderr, "EMU launch config error: grid %u block %u shm %zu\n", grid, block, shm);
    g_last = hipErrorInvalidValue;
  }
  if (shm > 64 * 1024) fprintf(stderr, "EMU note: dynamic LDS %zu > 64 KiB\n", shm);
}

void run_grid(dim3 grid, unsigned block, size_t shm, const std::function<void()>& body) {
  ++g_launches;
  const size_t ss = (getenv("EMU_STACK_KB") ? atoi(getenv("EMU_STACK_KB")) : 128) * 1024;
  if (fibers.size() < block) {
    size_t old = fibers.size();
    fibers.resize(block);
    for (size_t i = old; i < block; ++i) {
      fibers[i].stack = (char*)mmap(nullptr, ss, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
      fibers[i].ssize = ss;
    }
  }
  g_gridDim = grid;
  g_blockDim = dim3(block, 1, 1);
  g_body = &body;
  const unsigned long long nblk = (unsigned long long)grid.x * grid.y * grid.z;
  static const bool verbose = getenv("EMU_VERBOSE") != nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  struct Rep { const char* nm; unsigned long long nb; unsigned blk; std::chrono::steady_clock::time_point t0; bool v;
    ~Rep() { if (v) fprintf(stderr, "EMU %s blocks %llu x %u: %.1f ms\n", nm, nb, blk,
               std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count()); } }
    rep{g_kernel_name, nblk, block, t0, verbose};
  for (unsigned long long bl = 0; bl < nblk; ++bl) {
    ++g_block_serial;
    g_blockIdx = dim3((unsigned)(bl % grid.x), (unsigned)((bl / grid.x) % grid.y), (unsigned)(bl / grid.x / grid.y));
    if (shm) {
      g_dyn = (unsigned char*)malloc(shm);
      memset(g_dyn, g_garbage, shm);
    }
    for (unsigned t = 0; t < block; ++t) {
      Fiber& f = fibers[t];
      f.tid = dim3(t, 0, 0);
      f.state = READY;
      f.nbar = 0;
      f.nmfma = 0;
      f.lane = t & 63;
      f.wave = t >> 6;
      init_fiber(f);
    }
    for (;;) {
      // schedule: 0 forward, 1 reverse, 2 random permutation per round, 3 waves reversed
      {
        static const int order = getenv("EMU_ORDER") ? atoi(getenv("EMU_ORDER")) : 0;
        static unsigned long long rng = 0x9E3779B97F4A7C15ull;
        static std::vector<unsigned> perm;
        perm.resize(block);
        for (unsigned t = 0; t < block; ++t) perm[t] = t;
        if (order == 1) std::reverse(perm.begin(), perm.end());
        else if (order == 2) {
          for (unsigned t = block - 1; t > 0; --t) {
            rng ^= rng << 13; rng ^= rng >> 7; rng ^= rng << 17;
            std::swap(perm[t], perm[rng % (t + 1)]);
          }
        } else if (order == 3) {
          for (unsigned t = 0; t < block; ++t) perm[t] = ((block / 64 - 1 - t / 64) * 64) + (t & 63);
        }
        for (unsigned i = 0; i < block; ++i)
          if (fibers[perm[i]].state == READY) resume(&fibers[perm[i]]);
      }
      int nd = 0, nb = 0, nm = 0;
      for (unsigned t = 0; t < block; ++t) {
        const int s = fibers[t].state;
        nd += s == DONE; nb += s == BARRIER; nm += s == MFMA32 || s == MFMA64 || s == SHFL;
      }
      if (nd == (int)block) break;
      bool any = false;
      for (unsigned w = 0; w * 64 < block; ++w) {
        Fiber* wf = &fibers[w * 64];
        const unsigned nl = std::min<unsigned>(64, block - w * 64);
        int c32 = 0, c64 = 0, csh = 0;
        for (unsigned L = 0; L < nl; ++L) {
          c32 += wf[L].state == MFMA32; c64 += wf[L].state == MFMA64; csh += wf[L].state == SHFL;
        }
        if (csh) {
          if (csh == 64) {
            const int mask = (int)wf[0].b;
            for (unsigned L = 1; L < 64; ++L)
              if (wf[L].site != wf[0].site || (int)wf[L].b != mask) die("shuffle lanes at different call sites or masks");
            if (mask < 0 || mask > 63) die("shuffle mask out of range");
            for (unsigned L = 0; L < 64; ++L) wf[L].dout[0] = wf[L ^ mask].a;
            for (unsigned L = 0; L < 64; ++L) wf[L].state = READY;
            any = true;
          } else {
            for (unsigned L = 0; L < nl; ++L)
              if (wf[L].state == DONE || wf[L].state == BARRIER || wf[L].state == MFMA32 || wf[L].state == MFMA64)
                die("shuffle issued by part of a wave");
          }
          continue;
        }
        if (c32 + c64 == 0) continue;
        if (nl != 64) die("MFMA in a partial wave");
        if (c32 == 64 || c64 == 64) {
          for (unsigned L = 1; L < 64; ++L)
            if (wf[L].site != wf[0].site || wf[L].nmfma != wf[0].nmfma)
              die("MFMA lanes of one wave at different call sites or counts");
          for (unsigned L = 0; L < 64; ++L) ++wf[L].nmfma;
        }
        if (c32 == 64) { resolve_mfma(wf, MFMA32); any = true; }
        else if (c64 == 64) { resolve_mfma(wf, MFMA64); any = true; }
        else {
          // some lanes of this wave are elsewhere: they must still arrive
          for (unsigned L = 0; L < nl; ++L)
            if (wf[L].state == DONE || wf[L].state == BARRIER) {
              char buf[160];
              snprintf(buf, sizeof buf, "wave %u: %d lanes at MFMA, lane %u %s", w, c32 + c64, L,
                       wf[L].state == DONE ? "exited" : "at barrier");
              die(buf);
            }
        }
      }
      if (any) continue;
      if (nm == 0 && nb > 0) {
        // barrier: every thread that has not exited is waiting
        {
          const void* site0 = nullptr; long long n0 = -1;
          for (unsigned t = 0; t < block; ++t)
            if (fibers[t].state == BARRIER) {
              if (n0 < 0) { site0 = fibers[t].site; n0 = fibers[t].nbar; }
              else if (fibers[t].site != site0 || fibers[t].nbar != n0) {
                char buf[200];
                snprintf(buf, sizeof buf, "divergent barrier: thread %u at site %p count %lld vs %p count %lld",
                         t, fibers[t].site, fibers[t].nbar, site0, n0);
                die(buf);
              }
            }
          if (nd > 0 && getenv("EMU_WARN_EXIT_BARRIER")) fprintf(stderr, "EMU note: %s barrier with %d exited threads\n", g_kernel_name, nd);
        }
        for (unsigned t = 0; t < block; ++t)
          if (fibers[t].state == BARRIER) { fibers[t].state = READY; ++fibers[t].nbar; }
        continue;
      }
      die("deadlock");
    }
    if (shm) { free(g_dyn); g_dyn = nullptr; }
  }
}

// ---- queue ----
static std::deque<std::function<void()>> q;
void enqueue(hipStream_t, std::function<void()> f) { q.push_back(std::move(f)); }
static void flush() {
  while (!q.empty()) {
    auto f = std::move(q.front());
    q.pop_front();
    f();
  }
}

static std::map<uintptr_t, size_t> user_regions;
static bool in_user(const void* p, size_t n) {
  auto it = user_regions.upper_bound((uintptr_t)p);
  if (it == user_regions.begin()) return false;
  --it;
  return (uintptr_t)p >= it->first && (uintptr_t)p + n <= it->first + it->second;
}
static bool strict();
static std::map<uintptr_t, size_t> allocs;
static bool in_dev(const void* p, size_t n) {
  auto it = allocs.upper_bound((uintptr_t)p);
  if (it == allocs.begin()) return false;
  --it;
  return (uintptr_t)p >= it->first && (uintptr_t)p + n <= it->first + it->second;
}
static void check_range(const void* p, size_t n, bool dev, const char* what) {
  if (n == 0) return;
  // user tensors are not library allocations: a range must lie inside one
  // allocation or touch none
  if (strict() && dev && !in_dev(p, n) && !in_user(p, n)) {
    fprintf(stderr, "EMU STRICT %s: %p+%zu is not device memory\n", what, p, n); abort(); }
  if (strict() && !dev && (in_dev(p, 1) || in_user(p, 1))) {
    fprintf(stderr, "EMU STRICT %s: host side %p is device memory\n", what, p); abort(); }
  if (dev && !in_dev(p, n) && (in_dev(p, 1) || in_dev((const char*)p + n - 1, 1))) {
    fprintf(stderr, "EMU %s: device range %p+%zu straddles an allocation\n", what, p, n); abort(); }
  if (!dev && in_dev(p, 1)) { fprintf(stderr, "EMU %s: host pointer %p is device memory\n", what, p); abort(); }
}

static bool strict() { static const bool s = getenv("EMU_STRICT") != nullptr; return s; }
void check_ptr(const char* kname, const char* what, int idx, const void* p) {
  if (!strict() || !p) return;
  if (in_dev(p, 1) || in_user(p, 1)) return;
  fprintf(stderr, "EMU STRICT: kernel %s %s #%d = %p is not device memory\n", kname, what, idx, p);
  fflush(stderr);
  abort();
}

}  // namespace emu

namespace emu {
// file-scope device arrays announce themselves during static initialisation, possibly before this
// file's globals exist: they wait in a function-local list until hipGetSymbolAddress turns them into
// device memory (garbage-filled, like an allocation)
static std::vector<std::pair<void*, size_t>>& pending_symbols() {
  static std::vector<std::pair<void*, size_t>> v;
  return v;
}
void register_symbol(void* p, size_t n) { pending_symbols().push_back({p, n}); }
}  // namespace emu

struct emu_event { bool done = false; long long t = 0; };
static long long g_tick = 0;

extern "C" {
static std::map<uintptr_t, std::pair<void*, size_t>> g_guarded;
hipError_t hipMalloc(void** p, size_t b) {
  void* m = nullptr;
  static const bool guard = getenv("EMU_GUARD") != nullptr;
  if (guard) {
    // data flush (within 256 B) against a trailing 1 MiB PROT_NONE region, 1 MiB before
    const size_t G = 1 << 20, pg = 4096;
    const size_t body = ((b + 255) / 256 * 256 + pg - 1) / pg * pg;
    char* base = (char*)mmap(nullptr, body + 2 * G, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (base == MAP_FAILED) return hipErrorOutOfMemory;
    mprotect(base, G, PROT_NONE);
    mprotect(base + G + body, G, PROT_NONE);
    m = base + G + body - (b + 255) / 256 * 256;
    g_guarded[(uintptr_t)m] = {base, body + 2 * G};
  } else if (posix_memalign(&m, 256, b ? b : 1)) return hipErrorOutOfMemory;
  memset(m, emu::g_garbage, b);
  emu::allocs[(uintptr_t)m] = b;
  *p = m;
  return hipSuccess;
}
hipError_t hipFree(void* p) {
  emu::flush();
  if (!p) return hipSuccess;
  if (!emu::allocs.erase((uintptr_t)p)) { fprintf(stderr, "EMU hipFree of unknown %p\n", p); abort(); }
  auto it = g_guarded.find((uintptr_t)p);
  if (it != g_guarded.end()) { munmap(it->second.first, it->second.second); g_guarded.erase(it); }
  else free(p);
  return hipSuccess;
}
static bool dev_dst(hipMemcpyKind k) { return k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice; }
static bool dev_src(hipMemcpyKind k) { return k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice; }
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t b, hipMemcpyKind k, hipStream_t s) {
  emu::check_range(dst, b, dev_dst(k), "memcpy dst");
  emu::check_range(src, b, dev_src(k), "memcpy src");
  emu::enqueue(s, [=]() { memcpy(dst, src, b); });
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dp, const void* src, size_t sp, size_t w, size_t h,
                            hipMemcpyKind k, hipStream_t s) {
  if (w > dp || w > sp) { fprintf(stderr, "EMU memcpy2D width > pitch\n"); return hipErrorInvalidValue; }
  if (h) {
    emu::check_range(dst, dp * (h - 1) + w, dev_dst(k), "memcpy2D dst");
    emu::check_range(src, sp * (h - 1) + w, dev_src(k), "memcpy2D src");
  }
  emu::enqueue(s, [=]() {
    for (size_t r = 0; r < h; ++r) memcpy((char*)dst + r * dp, (const char*)src + r * sp, w);
  });
  return hipSuccess;
}
hipError_t hipMemset2DAsync(void* dst, size_t pitch, int v, size_t w, size_t h, hipStream_t s) {
  if (h) emu::check_range(dst, pitch * (h - 1) + w, true, "memset2D");
  emu::enqueue(s, [=]() {
    for (size_t r = 0; r < h; ++r) memset((char*)dst + r * pitch, v, w);
  });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t b, hipStream_t s) {
  emu::check_range(dst, b, true, "memset");
  emu::enqueue(s, [=]() { memset(dst, v, b); });
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { emu::flush(); return hipSuccess; }
hipError_t hipDeviceSynchronize() { emu::flush(); return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = new emu_event; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new emu_event; return hipSuccess; }
// one queue runs all work in submission order: every stream wait is already satisfied
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { static char dummy[8]; *s = (hipStream_t)dummy; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  e->done = false;
  emu::enqueue(s, [e]() { e->done = true; e->t = ++g_tick; });
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { emu::flush(); return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  if (!a->done || !b->done) return hipErrorNotReady;
  *ms = 0.001f * (float)(b->t - a->t);
  return hipSuccess;
}
hipError_t hipMemGetInfo(size_t* f, size_t* t) { *f = (size_t)200 << 30; *t = (size_t)288 << 30; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
// a small device: 4 CUs, one workgroup of a kernel at a time, the gfx950 LDS limit
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int) {
  if (a == hipDeviceAttributeMaxSharedMemoryPerBlock) *v = 160 * 1024;
  else if (a == hipDeviceAttributeMultiprocessorCount) *v = 4;
  else return hipErrorInvalidValue;
  return hipSuccess;
}
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, const void*, int, size_t) { *nb = 1; return hipSuccess; }
hipError_t hipGetLastError() { hipError_t e = emu::g_last; emu::g_last = hipSuccess; return e; }
const char* hipGetErrorString(hipError_t e) { return e ? "emulated error" : "no error"; }
void emu_flush() { emu::flush(); }
void emu_register(void* p, size_t n) { emu::user_regions[(uintptr_t)p] = n; }
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
  if (!emu::allocs.count((uintptr_t)symbol)) {
    size_t n = 0;
    for (auto& e : emu::pending_symbols())
      if (e.first == symbol) n = e.second;
    if (!n) {
      fprintf(stderr, "EMU hipGetSymbolAddress of an unregistered symbol %p\n", symbol);
      abort();
    }
    memset(const_cast<void*>(symbol), emu::g_garbage, n);
    emu::allocs[(uintptr_t)symbol] = n;
  }
  *p = const_cast<void*>(symbol);
  return hipSuccess;
}
long long emu_launches() { return emu::g_launches; }
}
