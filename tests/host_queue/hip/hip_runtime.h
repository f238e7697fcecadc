// Host-only stand-in for the few HIP runtime types and calls that the serving queue's host
// code uses, so that csrc/queue.cpp can be built with g++ and the thread/address/undefined-
// behaviour sanitizers on a machine without a GPU (tests/test_queue_host.py).  Streams,
// events and device memory become host objects; copies are memcpy.  Test infrastructure
// only: the library itself is always built against the real runtime.
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>

typedef enum { hipSuccess = 0, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 } hipError_t;
typedef enum { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 } hipMemcpyKind;
struct MockStream {
    int id;
};
struct MockEvent {
    int id;
};
typedef MockStream *hipStream_t;
typedef MockEvent *hipEvent_t;
constexpr unsigned hipStreamNonBlocking = 1;

struct int2 {
    int x, y;
};
struct int4 {
    int x, y, z, w;
};
inline int2 make_int2(int x, int y) { return int2{x, y}; }
inline int4 make_int4(int x, int y, int z, int w) { return int4{x, y, z, w}; }

inline const char *hipGetErrorString(hipError_t) { return "mock"; }
inline hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipSetDevice(int) { return hipSuccess; }
template <typename T>
inline hipError_t hipMalloc(T **p, size_t n) {
    *p = static_cast<T *>(std::malloc(n ? n : 1));
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void *p) {
    std::free(p);
    return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new MockStream{0};
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new MockEvent{0};
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
    std::memcpy(d, s, n);
    return hipSuccess;
}
