// Host-only stand-in for the part of the HIP runtime API that the library's host code
// (runtime, loader, planning) calls, so that this code can be built with a plain host
// compiler and run under ThreadSanitizer on a machine without a GPU.  Test infrastructure:
// streams complete their work at once, device memory is zero-filled host memory, events are
// always complete, and a captured stream records one graph node per batch kernel launched
// on it.  Thread-safe (one lock) where the library may call it from several threads.
#ifndef DRT_FAKE_HIP_RUNTIME_H
#define DRT_FAKE_HIP_RUNTIME_H

#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (&(x))

typedef int hipError_t;
enum : int {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
  hipErrorStreamCaptureInvalidated = 901,
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
enum hipStreamCaptureStatus { hipStreamCaptureStatusNone, hipStreamCaptureStatusActive, hipStreamCaptureStatusInvalidated };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct float2 { float x, y; };
struct double2 { double x, y; };
struct float4 { float x, y, z, w; };
struct uint2 { unsigned x, y; };

struct fake_graph_node { int kind; };
struct fake_graph { std::vector<fake_graph_node*> nodes; };
struct ihipStream_t {
  bool capturing = false;
  fake_graph* graph = nullptr;
};
struct ihipEvent_t { int unused; };
struct hipGraphExec { fake_graph* graph; };
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef fake_graph* hipGraph_t;
typedef hipGraphExec* hipGraphExec_t;
typedef fake_graph_node* hipGraphNode_t;
struct hipKernelNodeParams {
  dim3 blockDim, gridDim;
  void** extra = nullptr;
  void* func = nullptr;
  void** kernelParams = nullptr;
  unsigned sharedMemBytes = 0;
};

inline std::mutex& fake_hip_mutex() {
  static std::mutex m;
  return m;
}
// the kernel function a batch node stands for (set by the stub of launch_batch)
void* fake_batch_kernel_of(int kind);

inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
inline hipError_t hipMemGetInfo(size_t* free_b, size_t* total) {
  *free_b = size_t(64) << 30;
  *total = size_t(64) << 30;
  return hipSuccess;
}
inline hipError_t hipMalloc(void** p, size_t n) {
  *p = std::calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <class T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc((void**)p, n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned = 0) { return hipMalloc(p, n); }
template <class T> inline hipError_t hipHostMalloc(T** p, size_t n, unsigned f = 0) { return hipHostMalloc((void**)p, n, f); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
  if (n) std::memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind k, hipStream_t) {
  return hipMemcpy(d, s, n, k);
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  std::memset(d, v, n);
  return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new ihipStream_t; return hipSuccess; }
inline hipError_t hipStreamCreate(hipStream_t* s) { return hipStreamCreateWithFlags(s, 0); }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new ihipEvent_t{0}; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }

inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  std::lock_guard<std::mutex> l(fake_hip_mutex());
  s->capturing = true;
  s->graph = new fake_graph;
  return hipSuccess;
}
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  std::lock_guard<std::mutex> l(fake_hip_mutex());
  s->capturing = false;
  *g = s->graph;
  s->graph = nullptr;
  return hipSuccess;
}
// records a batch kernel node when s is being captured (called by the launch stub)
inline void fake_capture_launch(hipStream_t s, int kind) {
  std::lock_guard<std::mutex> l(fake_hip_mutex());
  if (s && s->capturing) s->graph->nodes.push_back(new fake_graph_node{kind});
}
inline hipError_t hipStreamGetCaptureInfo_v2(hipStream_t s, hipStreamCaptureStatus* cs, unsigned long long* id,
                                             hipGraph_t* g, const hipGraphNode_t** deps, size_t* nd) {
  std::lock_guard<std::mutex> l(fake_hip_mutex());
  *cs = s->capturing ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
  if (id) *id = 0;
  if (g) *g = s->graph;
  const bool any = s->capturing && !s->graph->nodes.empty();
  if (deps) *deps = any ? &s->graph->nodes.back() : nullptr;
  if (nd) *nd = any ? 1 : 0;
  return hipSuccess;
}
inline hipError_t hipGraphKernelNodeGetParams(hipGraphNode_t n, hipKernelNodeParams* p) {
  *p = hipKernelNodeParams{};
  p->func = fake_batch_kernel_of(n->kind);
  p->blockDim = dim3(256);
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = new hipGraphExec{g};
  return hipSuccess;
}
inline hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t, hipGraphNode_t, const hipKernelNodeParams*) {
  return hipSuccess;
}
inline hipError_t hipGraphNodeSetEnabled(hipGraphExec_t, hipGraphNode_t, unsigned) { return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  if (g)
    for (auto* n : g->nodes) delete n;
  delete g;
  return hipSuccess;
}

#endif  // DRT_FAKE_HIP_RUNTIME_H
