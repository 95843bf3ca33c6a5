// A host-only stand-in for the part of the HIP runtime API that the streamed pipeline
// (csrc/pipeline.cpp) calls. It lets the pipeline's scheduler, locking and chunk
// bookkeeping be compiled with g++ and run under ThreadSanitizer and AddressSanitizer
// on a machine without a GPU. Semantics: "device" memory is host memory, and every
// operation enqueued on a stream runs at once on the calling thread, so each stream is
// trivially in order and every event has completed when its record returns. This
// models the ordering the pipeline requests (nothing it waits for is ever late); it
// does not model asynchrony. Test code only: the library never includes it.
#pragma once

#include <chrono>
#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
    hipErrorLaunchFailure = 719,
} hipError_t;

typedef enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice } hipMemcpyKind;

struct hipStubStream { int id; };
struct hipStubEvent { double t_ms; bool recorded; };
typedef hipStubStream* hipStream_t;
typedef hipStubEvent* hipEvent_t;

#define hipStreamNonBlocking 1u
#define hipEventDefault 0u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

inline double hip_stub_now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "hip stub error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) { *p = std::malloc(n ? n : 1); return *p ? hipSuccess : hipErrorOutOfMemory; }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned) { *d = h; return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new hipStubStream{0}; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) { *e = new hipStubEvent{0.0, false}; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->t_ms = hip_stub_now_ms(); e->recorded = true; return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t e) { return e && e->recorded ? hipSuccess : hipErrorNotReady; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = static_cast<float>(b->t_ms - a->t_ms);
    return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
    std::memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h, hipMemcpyKind,
                                   hipStream_t) {
    for (size_t r = 0; r < h; ++r)
        std::memmove(static_cast<uint8_t*>(d) + r * dp, static_cast<const uint8_t*>(s) + r * sp, w);
    return hipSuccess;
}
