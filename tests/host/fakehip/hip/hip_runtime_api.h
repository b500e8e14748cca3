// Host-only stand-in for the few HIP runtime declarations the serving engine uses, so that
// csrc/server.cpp can be compiled and exercised on a CPU against a simulated device
// (tests/host/serve_sim.cpp).  Not used by the library build.
#pragma once
#include <cstddef>

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorNotReady = 600,
    hipErrorLaunchFailure = 719
} hipError_t;

struct SimStream;
struct SimEvent;
typedef SimStream *hipStream_t;
typedef SimEvent *hipEvent_t;

enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
typedef enum { hipMemcpyDeviceToDevice = 3 } hipMemcpyKind;

hipError_t hipGetDevice(int *dev);
hipError_t hipSetDevice(int dev);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t s);
hipError_t hipDeviceSynchronize(void);
const char *hipGetErrorString(hipError_t e);
