// CPU stand-in for the part of the HIP runtime and device language that the
// library uses, for running its kernels on the host under AddressSanitizer
// (test infrastructure; the library itself is built with hipcc for gfx950).
//
// Every GPU thread of a workgroup runs as a fiber.  Workgroup barriers wait for
// every thread that has not returned.  Wavefront operations (shuffles,
// ballots, readfirstlane, wave barriers) act on the 64 consecutive threads of a
// wavefront, as on CDNA hardware: they complete once every live thread of the
// wavefront has arrived, and the run stops with a report when a shuffle reads a
// thread that has returned, when lanes of one wavefront wait at a wavefront
// operation and at a workgroup barrier at once, or when nothing can proceed.
// Device allocations sit flush against an inaccessible guard region (after the
// end, or before the start with CPU_HIP_GUARD=start) and start filled with 0xff
// bytes (NaN doubles).
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct cpu_hip_uint3 {
  unsigned x, y, z;
};

typedef enum hipError_t {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorInvalidConfiguration = 9,
  hipErrorLaunchFailure = 719,
} hipError_t;

typedef struct cpu_hip_stream* hipStream_t;
typedef struct cpu_hip_event* hipEvent_t;
typedef struct cpu_hip_graph* hipGraph_t;
typedef struct cpu_hip_graph* hipGraphExec_t;
typedef struct cpu_hip_graph_node* hipGraphNode_t;

enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice,
                     hipMemcpyDefault };
enum hipStreamCaptureStatus { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
                            hipStreamCaptureModeRelaxed = 2 };
enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 };
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

// ---- device-side built-ins ---------------------------------------------------
extern cpu_hip_uint3 threadIdx, blockIdx;
extern dim3 blockDim, gridDim;
constexpr int warpSize = 64;

namespace cpu_hip {
void syncthreads();
double shfl(double v, int src);
int shfl_i(int v, int src);
unsigned long long ballot(int pred);
int readfirstlane(int v);
void wave_barrier();
void launch(dim3 grid, dim3 block, std::function<void()> body);
}  // namespace cpu_hip

inline void __syncthreads() { cpu_hip::syncthreads(); }
inline double __shfl(double v, int src, int = 64) { return cpu_hip::shfl(v, src); }
inline int __shfl(int v, int src, int = 64) { return cpu_hip::shfl_i(v, src); }
inline unsigned long long __ballot(int pred) { return cpu_hip::ballot(pred); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __builtin_amdgcn_readfirstlane(int v) { return cpu_hip::readfirstlane(v); }
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
// the fibers of a workgroup never run at the same time: a plain read-modify-write is atomic
inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
  const unsigned long long o = *p;
  if (v > o) *p = v;
  return o;
}
inline unsigned long long atomicMin(unsigned long long* p, unsigned long long v) {
  const unsigned long long o = *p;
  if (v < o) *p = v;
  return o;
}
inline long long __double_as_longlong(double x) {
  long long r;
  __builtin_memcpy(&r, &x, sizeof r);
  return r;
}
inline double __longlong_as_double(long long x) {
  double r;
  __builtin_memcpy(&r, &x, sizeof r);
  return r;
}
#define __builtin_amdgcn_fence(order, scope) ((void)0)
inline void __builtin_amdgcn_wave_barrier() { cpu_hip::wave_barrier(); }

#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) \
  ::cpu_hip::launch(dim3(G), dim3(B), [=]() { K(__VA_ARGS__); })

// ---- host API ----------------------------------------------------------------
hipError_t hipMalloc(void** p, size_t n);
template <class T>
inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc(reinterpret_cast<void**>(p), n); }
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t n, unsigned flags = 0);
template <class T>
inline hipError_t hipHostMalloc(T** p, size_t n, unsigned flags = 0) {
  return hipHostMalloc(reinterpret_cast<void**>(p), n, flags);
}
hipError_t hipHostFree(void* p);
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind k, hipStream_t s = nullptr);
hipError_t hipMemset(void* dst, int v, size_t n);
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s = nullptr);
hipError_t hipDeviceSynchronize();
hipError_t hipGetDevice(int* d);
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t a, int dev);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipStreamIsCapturing(hipStream_t s, hipStreamCaptureStatus* st);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err, char* log, size_t n);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* n, const void* kernel, int block, size_t shmem);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);
#define HIP_SYMBOL(x) (&(x))
