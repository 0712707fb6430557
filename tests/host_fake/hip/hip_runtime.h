// A host-only stand-in for the HIP runtime header, for building the library's
// host files (api.cpp, serve.cpp) on the CPU with ThreadSanitizer: device
// memory is host memory, every copy and fill completes at once, streams and
// events are plain objects whose work is always finished.  Device-only
// helpers compile but are never called (the kernels are replaced by
// fake_kernels.cpp).
#pragma once

#include <cstddef>
#include <cstdint>
#include <cstdlib>
#include <cstring>

#define __device__
#define __host__
#define __global__
#define __shared__ static
#define __forceinline__ inline
#define __align__(n) __attribute__((aligned(n)))
#define HIP_SYMBOL(x) ((const void*)&(x))

struct uint2 { unsigned int x, y; };
struct uint4 { unsigned int x, y, z, w; };
inline uint2 make_uint2(unsigned int x, unsigned int y) { return uint2{x, y}; }
struct dim3 { unsigned int x = 1, y = 1, z = 1; };
static const dim3 threadIdx{}, blockIdx{}, blockDim{}, gridDim{};

// device intrinsics referenced by inline device helpers (never executed here)
inline unsigned int __umulhi(unsigned int a, unsigned int b) { return (unsigned int)(((uint64_t)a * b) >> 32); }
inline long long __float2ll_rn(float x) { return (long long)x; }
template <typename T> inline T __shfl_up(T v, int, int = 64) { return v; }
template <typename T> inline T __shfl_xor(T v, int, int = 64) { return v; }
template <typename T> inline T __shfl(T v, int, int = 64) { return v; }
inline unsigned long long __ballot(int p) { return p ? 1ull : 0ull; }
inline int __popcll(unsigned long long m) { return __builtin_popcountll(m); }
inline int __ffsll(long long m) { return __builtin_ffsll(m); }
inline void __syncthreads() {}
template <typename T> inline T min(T a, T b) { return b < a ? b : a; }
template <typename T> inline T max(T a, T b) { return a < b ? b : a; }

enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorNotReady = 600,
};
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost,
                     hipMemcpyDeviceToDevice, hipMemcpyDefault };
enum hipDeviceAttribute_t { hipDeviceAttributeMaxSharedMemoryPerBlock = 1 };
enum hipMemPoolAttr { hipMemPoolAttrReleaseThreshold = 1 };
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipHostMallocDefault 0u

struct ihipStream_t { int id; };
struct ihipEvent_t { int id; };
typedef ihipStream_t* hipStream_t;
typedef ihipEvent_t* hipEvent_t;
typedef void* hipGraphExec_t;
typedef void* hipMemPool_t;

inline const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 163840; return hipSuccess; }
inline hipError_t hipMemGetInfo(size_t* free_b, size_t* total) {
    *free_b = (size_t)16 << 30;
    *total = (size_t)32 << 30;
    return hipSuccess;
}
inline hipError_t hipMalloc(void** p, size_t bytes) {
    *p = std::calloc(1, bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMallocAsync(void** p, size_t bytes, hipStream_t) { return hipMalloc(p, bytes); }
inline hipError_t hipFreeAsync(void* p, hipStream_t) { return hipFree(p); }
inline hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) { return hipMalloc(p, bytes); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memmove(d, s, n); return hipSuccess; }
inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t = nullptr) {
    std::memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t = nullptr) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { *s = new ihipStream_t{1}; return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) { *e = new ihipEvent_t{1}; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = const_cast<void*>(sym); return hipSuccess; }
inline hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t* p, int) { *p = nullptr; return hipSuccess; }
inline hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void*) { return hipSuccess; }
inline hipError_t hipMemPoolTrimTo(hipMemPool_t, size_t) { return hipSuccess; }
