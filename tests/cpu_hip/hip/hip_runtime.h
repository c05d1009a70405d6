// CPU stand-in for the part of the HIP runtime API that libmuca's host code
// (muca_runtime.cpp, muca_batch.cpp, muca_server.cpp) calls.  Test
// infrastructure only: it lets those files be built with a host compiler and
// run under the sanitizers with no GPU.  "Device" memory is host memory, each
// stream is a worker thread that runs its work in order, events mark points in
// a stream, and stream capture records a stream's work into a graph that a
// launch replays.  The kernels are stand-ins too (cpu_hip.cpp).
#pragma once

#include <stddef.h>
#include <stdint.h>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __shared__

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidResourceHandle = 400,
    hipErrorNotReady = 600,
    hipErrorStreamCaptureUnsupported = 900,
    hipErrorUnknown = 999
} hipError_t;

struct ihipStream_t;
struct ihipEvent_t;
struct ihipGraph;
struct hipGraphExec;
struct hipGraphNode;
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef ihipGraph* hipGraph_t;
typedef hipGraphExec* hipGraphExec_t;
typedef hipGraphNode* hipGraphNode_t;
typedef void (*hipHostFn_t)(void* user_data);

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

typedef enum hipDeviceAttribute_t { hipDeviceAttributeMultiprocessorCount = 1 } hipDeviceAttribute_t;

#define hipStreamDefault 0u
#define hipStreamNonBlocking 1u
#define hipEventDefault 0u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

hipError_t hipGetDevice(int* device);
hipError_t hipSetDevice(int device);
hipError_t hipDeviceGetAttribute(int* value, hipDeviceAttribute_t attr, int device);
hipError_t hipGetLastError(void);
const char* hipGetErrorName(hipError_t e);
const char* hipGetErrorString(hipError_t e);

hipError_t hipMalloc(void** p, size_t bytes);
hipError_t hipFree(void* p);
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int flags);
hipError_t hipHostFree(void* p);
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s);

hipError_t hipStreamCreate(hipStream_t* s);
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int flags);
hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* user_data);

hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t start, hipEvent_t stop);

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* graph);
hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t* error_node, char* log,
                               size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t graph);
hipError_t hipGraphExecDestroy(hipGraphExec_t exec);

#ifdef __cplusplus
template <class T>
inline hipError_t hipMalloc(T** p, size_t bytes)
{
    return hipMalloc(reinterpret_cast<void**>(p), bytes);
}
#endif
