// Host stand-in for the HIP runtime header, used only to compile the
// library's device math with g++ for the CPU unit tests of its adjoints.
// Kernels and launchers are not compiled against it.
#pragma once
#include <cmath>
#include <cstring>
#define __device__
#define __host__
#define __forceinline__ inline
using std::fabs;
using std::fma;
using std::fmax;
using std::fmin;
using std::pow;
using std::sqrt;
typedef void* hipEvent_t;
typedef void* hipStream_t;
typedef int hipError_t;
enum { hipSuccess = 0 };
inline hipError_t hipEventCreate(hipEvent_t*) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float*, hipEvent_t, hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline long long __double_as_longlong(double x) { long long r; std::memcpy(&r, &x, 8); return r; }
inline double __longlong_as_double(long long x) { double r; std::memcpy(&r, &x, 8); return r; }
// the device reciprocal estimate; exact here, the Newton steps keep it so
inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
