// HIP subset used by the HDF kernels and the C ABI, emulated on the CPU for
// memory-safety tests (see emu_rt.cpp).  Included in place of
// <hip/hip_runtime.h> through shim/hip/.
#pragma once
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <cmath>
#include <math.h>
#include <functional>
#include <algorithm>
#include <type_traits>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1, hipErrorInvalidDevice = 101,
       hipErrorNotReady = 600 };
typedef struct emu_stream* hipStream_t;
typedef struct emu_event* hipEvent_t;
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };

extern "C" {
hipError_t hipMalloc(void** p, size_t b);
hipError_t hipFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t b, hipMemcpyKind k, hipStream_t s);
hipError_t hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch, size_t w, size_t h,
                            hipMemcpyKind k, hipStream_t s);
hipError_t hipMemset2DAsync(void* dst, size_t pitch, int v, size_t w, size_t h, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int v, size_t b, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipMemGetInfo(size_t* f, size_t* t);
hipError_t hipGetDevice(int* d);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
typedef enum { hipDeviceAttributeMaxSharedMemoryPerBlock = 74, hipDeviceAttributeMultiprocessorCount = 63 } hipDeviceAttribute_t;
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, const void* fn, int block, size_t shm);
void emu_flush();
}

#ifdef EMU_DEVICE_CODE
using std::isfinite;
using std::isnan;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))
namespace emu {
// a file-scope device array: device memory of its own size (garbage-filled), visible to
// hipGetSymbolAddress and to the kernels' pointer checks
void register_symbol(void* p, size_t n);
struct SymbolReg {
  SymbolReg(void* p, size_t n) { register_symbol(p, n); }
};
}  // namespace emu

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
typedef float float2 __attribute__((ext_vector_type(2)));
typedef double double2 __attribute__((ext_vector_type(2)));

namespace emu {
struct Fiber;
extern Fiber* cur;
extern dim3 g_blockIdx, g_blockDim, g_gridDim;
const dim3& tidx();
void syncthreads();
void syncthreads_at(const void* site);   // a barrier whose call sites count as one (see mf_kernels.hip)
unsigned char* dyn_smem();
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
f4 mfma_f32(float a, float b, f4 c);
d4 mfma_f64(double a, double b, d4 c);
void check_launch(unsigned grid, unsigned block, size_t shm);
int syncthreads_count(int p);
double shfl_xor(double v, int mask);
void enqueue(hipStream_t s, std::function<void()> f);
void run_grid(dim3 grid, unsigned block, size_t shm, const std::function<void()>& body);
extern const char* g_kernel_name;
void check_ptr(const char* kname, const char* what, int idx, const void* p);
template <typename T> struct StructCheck { static void run(const char*, int, const T&) {} };
template <typename T> inline void check_arg(const char* kname, int idx, const T& a) {
  if constexpr (std::is_pointer<T>::value) { if (a) check_ptr(kname, "arg", idx, (const void*)a); }
  else StructCheck<T>::run(kname, idx, a);
}
void garbage_once(void* p, size_t n);
template <typename K, typename... A>
void launch(const char* name, dim3 grid, dim3 block, size_t shm, hipStream_t s, K k, A... args) {
  check_launch(grid.x * grid.y * grid.z, block.x * block.y * block.z, shm);
  { int idx = 0; (check_arg(name, idx++, args), ...); }
  if (block.y != 1 || block.z != 1) abort();
  enqueue(s, [=]() { g_kernel_name = name; run_grid(grid, block.x, shm, [=]() { k(args...); }); });
}
}  // namespace emu

#define threadIdx (emu::tidx())
#define blockIdx (emu::g_blockIdx)
#define blockDim (emu::g_blockDim)
#define gridDim (emu::g_gridDim)
#define __syncthreads() emu::syncthreads()
#define __syncthreads_count(p) emu::syncthreads_count(p)
#define __shfl_xor(v, m) emu::shfl_xor(v, m)
// wavefront-level synchronisation point: a wave-wide collective (a shuffle of nothing)
#define __builtin_amdgcn_wave_barrier() ((void)emu::shfl_xor(0.0, 0))
using std::max;
using std::min;
#define __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, x, y, z) emu::mfma_f32(a, b, c)
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) emu::mfma_f64(a, b, c)
#define __builtin_nontemporal_store(v, p) (*(p) = (v))
// the kernels apply it only to wave-uniform values, which every lane already holds
#define __builtin_amdgcn_readfirstlane(x) (x)
// instruction-scheduling hints of the device compiler: nothing to emulate
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define amdgpu_waves_per_eu(...) unused

#endif
