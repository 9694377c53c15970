// Shared device/host helpers of libisdf (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/isdf.h"

#define ISDF_WAVE 64

// Host: turn a failed HIP enqueue into ISDF_E_HIP.
#define ISDF_TRY_HIP(expr)                        \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return ISDF_E_HIP;      \
  } while (0)

#define ISDF_TRY(expr)                            \
  do {                                            \
    int s_ = (expr);                              \
    if (s_ != ISDF_OK) return s_;                 \
  } while (0)

// Entry points take the enumerations as int32_t and check them before any
// conversion: a value outside an enumeration's range is undefined behaviour
// once loaded as the enum type.
static inline bool dtype_valid(int32_t v) { return v == ISDF_C128 || v == ISDF_C64; }
static inline bool prec_valid(int32_t v) { return v >= ISDF_P_FP64 && v <= ISDF_P_FP16X3; }

namespace isdf {

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carves aligned slices from the caller's workspace.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* b, size_t c) : base((char*)b), cap(c) {}
  template <class T>
  T* take(size_t count) {
    used = align_up(used, 256);
    T* p = base ? (T*)(base + used) : nullptr;
    used += count * sizeof(T);
    return p;
  }
  bool fits() const { return used <= cap; }
};

static inline bool launch_ok() { return hipGetLastError() == hipSuccess; }

// ---------------------------------------------------------------- device
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, ISDF_WAVE);
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, ISDF_WAVE);
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, ISDF_WAVE));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, ISDF_WAVE));
  return v;
}

// Fixed-order reductions of per-workgroup pairs (deterministic run to run).
constexpr int PAIR_THREADS = 256;

// Sums (a, b) over the workgroup (waves in order) into part[2 blockIdx.x + {0, 1}].
__device__ __forceinline__ void block_pair_store(double a, double b, double* part) {
  __shared__ double red[2][PAIR_THREADS / ISDF_WAVE];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / ISDF_WAVE;
  if ((threadIdx.x & (ISDF_WAVE - 1)) == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < (int)(blockDim.x / ISDF_WAVE); ++i) {
      sa += red[0][i];
      sb += red[1][i];
    }
    part[2 * blockIdx.x] = sa;
    part[2 * blockIdx.x + 1] = sb;
  }
}

// out[0] = sum_i part[2 i], out[1] = sum_i part[2 i + 1] (one workgroup).
static __global__ __launch_bounds__(PAIR_THREADS) void sum_pairs(const double* __restrict__ part, int n,
                                                           double* __restrict__ out) {
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < n; i += PAIR_THREADS) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  __shared__ double red[2][PAIR_THREADS / ISDF_WAVE];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / ISDF_WAVE;
  if ((threadIdx.x & (ISDF_WAVE - 1)) == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < PAIR_THREADS / ISDF_WAVE; ++i) {
      sa += red[0][i];
      sb += red[1][i];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

// Positive doubles order like their bit patterns: atomic min/max on them.
__device__ __forceinline__ void atomic_min_pos(double* p, double v) {
  atomicMin((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}
__device__ __forceinline__ void atomic_max_pos(double* p, double v) {
  atomicMax((unsigned long long*)p, (unsigned long long)__double_as_longlong(v));
}

// Complex element loaders: (re, im) as double from either storage type.
template <class T>
struct Cplx;
template <>
struct Cplx<double> {
  __device__ __forceinline__ static double2 load(const double* p) {
    return *reinterpret_cast<const double2*>(p);
  }
  __device__ __forceinline__ static void store(double* p, double re, double im) {
    *reinterpret_cast<double2*>(p) = make_double2(re, im);
  }
};
template <>
struct Cplx<float> {
  __device__ __forceinline__ static double2 load(const float* p) {
    float2 v = *reinterpret_cast<const float2*>(p);
    return make_double2((double)v.x, (double)v.y);
  }
  __device__ __forceinline__ static void store(float* p, double re, double im) {
    *reinterpret_cast<float2*>(p) = make_float2((float)re, (float)im);
  }
};

// Grid-stride fill (used instead of hipMemsetAsync so that captured graphs
// replay correctly).
template <class T>
__global__ void fill_kernel(T* __restrict__ p, int64_t n, T v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t s = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) p[i] = v;
}

template <class T>
static inline bool fill(T* p, int64_t n, T v, hipStream_t st) {
  if (n <= 0) return true;
  int64_t blocks = ceil_div(n, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return launch_ok();
}

}  // namespace isdf
