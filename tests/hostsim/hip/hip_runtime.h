// Host-only stand-in of the part of the HIP runtime API that libcsaw's host
// sources (runtime.hip, server.hip) use, so that they can be compiled by g++
// and run under AddressSanitizer / ThreadSanitizer on a machine without a
// GPU. Test infrastructure only.
//
// Model: "device" memory is host heap memory; each stream is a worker thread
// that runs its queued work in order (so host code that touches a buffer
// while work on it is pending is a data race the sanitizers can see); events
// mark positions in a stream's queue; a stream under capture records its
// work instead, and a graph replays the recording on the stream it is
// launched on. Kernel launches are the stand-in launchers of
// kernels_sim.cpp, which enqueue host functions.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>

#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) (reinterpret_cast<const void*>(&(x)))

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
    hipErrorLaunchFailure = 719,
    hipErrorStreamCaptureUnsupported = 900,
    hipErrorUnknown = 999
} hipError_t;

typedef struct ihipStream_t* hipStream_t;
typedef struct ihipEvent_t* hipEvent_t;
typedef struct ihipGraph_t* hipGraph_t;
typedef struct ihipGraphExec_t* hipGraphExec_t;
typedef struct ihipGraphNode_t* hipGraphNode_t;

typedef enum hipMemcpyKind {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
    hipMemcpyDefault = 4
} hipMemcpyKind;

typedef enum hipStreamCaptureMode {
    hipStreamCaptureModeGlobal = 0,
    hipStreamCaptureModeThreadLocal = 1,
    hipStreamCaptureModeRelaxed = 2
} hipStreamCaptureMode;

#define hipStreamDefault 0u
#define hipStreamNonBlocking 1u
#define hipEventDefault 0u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u
#define hipHostMallocMapped 2u
#define hipHostMallocCoherent 0x40000000u

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

// Launch macros: the host sources built here never launch a kernel
// themselves (their launchers are replaced by kernels_sim.cpp).
#define hipLaunchKernelGGL(...) ((void)0)
#define hipExtLaunchKernelGGL(...) ((void)0)

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void* p);
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned flags);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
hipError_t hipMemsetAsync(void* dst, int value, size_t bytes, hipStream_t s);
hipError_t hipGetSymbolAddress(void** p, const void* symbol);

hipError_t hipSetDevice(int device);
hipError_t hipGetDevice(int* device);
hipError_t hipGetLastError(void);
const char* hipGetErrorString(hipError_t e);

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* graph);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t* err_node, char* log,
                               size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);
hipError_t hipGraphDestroy(hipGraph_t graph);

// --- for the stand-in launchers and the driver
namespace hipsim {
// Runs fn on stream s in order, or records it while s is captured.
void enqueue(hipStream_t s, std::function<void()> fn);
// Device memory limit of the stand-in (bytes; 0 = none): hipMalloc beyond it fails.
void set_device_limit(size_t bytes);
size_t device_bytes_in_use();
}  // namespace hipsim
