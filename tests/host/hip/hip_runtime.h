// A host-only stand-in for the part of the HIP runtime API that the engine's
// batched-plan host code uses (rd_batch.hip, rd_host.cpp).  It lets that code
// run on a CPU, under AddressSanitizer, with every "device" buffer in host
// memory.  Work enqueued on a stream runs at once; work enqueued while a
// stream is being captured is recorded and runs when the instantiated graph
// is launched.  Every handle and pointer is checked against the live objects
// and allocations: a call on a destroyed stream, event or graph, a free of an
// unknown pointer, a copy outside a live allocation, a capture that ends with
// a forked stream not joined back, all abort with a message.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>

#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif

typedef int hipError_t;
enum : int {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorStreamCaptureUnjoined = 3,
    hipErrorStreamCaptureInvalidated = 4,
};

struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph_t;
struct ihipGraphExec_t;
typedef ihipStream_t *hipStream_t;
typedef ihipEvent_t *hipEvent_t;
typedef ihipGraph_t *hipGraph_t;
typedef ihipGraphExec_t *hipGraphExec_t;
typedef void *hipGraphNode_t;

enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
};
enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2
};

#define hipStreamNonBlocking 0x1u
#define hipEventDisableTiming 0x2u
#define hipEventDisableSystemFence 0x20000000u
#define hipHostMallocDefault 0x0u

const char *hipGetErrorString(hipError_t e);
hipError_t hipGetLastError();
hipError_t hipSetDevice(int device);
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *exec, hipGraph_t g, hipGraphNode_t *err_node, char *log,
                               size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t g);

// ---- stand-in only (not HIP API): used by the harness's kernel stand-ins ----
namespace hipstub {
// Runs `work` on stream s now, or records it when s is being captured.
void enqueue(hipStream_t s, const char *what, std::function<void()> work);
// True when [p, p + bytes) lies inside one live device allocation.
bool device_range_live(const void *p, size_t bytes);
// Counters of the stand-in's activity.
struct Counters {
    long captures, graph_launches, eager_ops, graph_ops, mallocs, frees;
};
Counters counters();
// Live device allocations and bytes (for leak checks at the end).
size_t live_device_allocations();
size_t live_device_bytes();
// The elapsed time that hipEventElapsedTime reports next (then reset to 1 ms).
void set_next_elapsed(float ms);
}  // namespace hipstub
