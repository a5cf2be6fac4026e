// Host-runtime stand-in for the server's host code: device and pinned memory
// are heap blocks (filled with 0xCD, as uninitialised memory), operations on a
// stream run at once, a capture records them into a graph that a launch
// replays; kernel launchers are stubs defined by the driver.
#pragma once
#include "../../hip/hip_runtime.h"
#include <cstdlib>
#include <functional>
#include <mutex>
#include <vector>
enum { hipErrorOutOfMemory = 2 };
struct MockEvent { int x = 0; };
struct MockGraph { std::vector<std::function<void()>> ops; };
struct MockStream { int x = 0; };
typedef MockEvent *hipEvent_t;
typedef MockGraph *hipGraph_t;
typedef MockGraph *hipGraphExec_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2, hipHostMallocDefault = 0 };
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1 };
inline thread_local MockGraph *g_capture = nullptr;
inline void mock_do(std::function<void()> f) { if (g_capture) g_capture->ops.push_back(std::move(f)); else f(); }
inline void *mock_alloc(size_t n) { void *p = std::malloc(n ? n : 1); std::memset(p, 0xCD, n); return p; }
inline hipError_t hipMalloc(void **p, size_t n) { *p = mock_alloc(n); return hipSuccess; }
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { *p = mock_alloc(n); return hipSuccess; }
inline hipError_t hipHostFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t)
{ mock_do([=] { std::memcpy(d, s, n); }); return hipSuccess; }
inline hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { mock_do([=] { std::memset(d, v, n); }); return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new MockStream; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete static_cast<MockStream *>(s); return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { *e = new MockEvent; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { mock_do([e] { e->x++; }); return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { mock_do([e] { (void)e->x; }); return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { g_capture = new MockGraph; return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = g_capture; g_capture = nullptr; return hipSuccess; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, char *, size_t) { *x = new MockGraph(*g); return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) { for (auto &op : x->ops) op(); return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete x; return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
// event timing (the batch tuner) and pointer attributes (device checks)
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new MockEvent; return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{ *ms = 0.001f * (float)((a->x * 7 + b->x * 13) % 17 + 1); return hipSuccess; }
enum hipMemoryType { hipMemoryTypeHost = 1, hipMemoryTypeDevice = 2, hipMemoryTypeManaged = 4 };
struct hipPointerAttribute_t { hipMemoryType type = hipMemoryTypeDevice; int device = 0; };
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t *a, const void *) { *a = hipPointerAttribute_t{}; return hipSuccess; }
// the typed forms of the runtime's allocation calls
template <typename T> inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc(reinterpret_cast<void **>(p), n); }
template <typename T> inline hipError_t hipHostMalloc(T **p, size_t n, unsigned f) { return hipHostMalloc(reinterpret_cast<void **>(p), n, f); }
