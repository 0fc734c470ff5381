// CPU stand-in of the HIP host calls the serving runtime makes, for building its host
// logic under sanitizers in tests (no device code; never part of the library).

#pragma once
#include <cstddef>
#include <cstring>
#include <cstdlib>
#include <atomic>
typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1 };
typedef struct FakeStream* hipStream_t;
struct FakeStream { int id; };
enum { hipStreamNonBlocking = 1 };
enum hipMemcpyKind { hipMemcpyDeviceToHost = 2 };
enum { hipMemoryTypeHost = 0, hipMemoryTypeDevice = 1, hipMemoryTypeManaged = 2 };
struct hipPointerAttribute_t { int type; };
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new FakeStream{1}; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "fake"; }
inline hipError_t hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) { a->type = p ? hipMemoryTypeDevice : hipMemoryTypeHost; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
inline hipError_t hipMemGetInfo(size_t* f, size_t* t) { *f = (size_t)1 << 34; *t = *f; return hipSuccess; }
