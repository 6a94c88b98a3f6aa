// Peak probes (libnnp_peaks.so): FP32/FP64 fused multiply-add and FP32
// exponential issue rates, FP32/FP64/BF16 matrix-core (MFMA) rates, and a
// streaming HBM copy.  Built with the same
// flags as the energy+force kernels, so the FP32 probe issues single
// v_fma_f32 instructions exactly as those kernels do.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "nnp_peaks.h"

namespace {

constexpr int LANES = 256;  // workgroup size of every probe
constexpr int CHAINS = 16;  // independent dependency chains per lane

__device__ inline float fma_t(float x, float a, float b) { return __builtin_fmaf(x, a, b); }
__device__ inline double fma_t(double x, double a, double b) { return __builtin_fma(x, a, b); }

template <class T>
__global__ __launch_bounds__(LANES) void k_fma(T* out, int iters, T a, T b) {
  T x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = (T)((threadIdx.x + 7 * c) & 255) * (T)(1.0 / 256);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = fma_t(x[c], a, b);
  }
  T s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += x[c];
  // never true for a, b in (0, 1): the store only keeps the chains live
  if (s == (T)-1) out[(int64_t)blockIdx.x * LANES + threadIdx.x] = s;
}

__global__ __launch_bounds__(LANES) void k_exp(float* out, int iters) {
  float x[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) x[c] = (float)((threadIdx.x + 7 * c) & 255) * (1.0f / 256);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = __builtin_amdgcn_exp2f(-x[c]);  // stays in [1/2, 1]
  }
  float s = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) s += x[c];
  if (s == -1.0f) out[(int64_t)blockIdx.x * LANES + threadIdx.x] = s;
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Matrix-core issue rates: every wave runs `iters` rounds of MCH independent
// accumulator chains of one 16x16 MFMA shape (the shapes the network kernel
// uses): 16x16x4 FP32 and FP64 (2 * 16 * 16 * 4 = 2048 operations each) and
// 16x16x32 BF16 with FP32 accumulation (16384 operations).
constexpr int MCH = 4;

__device__ inline v4f mfma_step(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline v4d mfma_step(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline v4f mfma_step(v8bf a, v8bf b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

template <class In, class Acc, class Out>
__global__ __launch_bounds__(LANES) void k_mfma(Out* out, int iters, In a, In b) {
  Acc acc[MCH];
#pragma unroll
  for (int c = 0; c < MCH; ++c) acc[c] = Acc{} + (Out)((threadIdx.x + c) & 7);
#pragma unroll 2
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < MCH; ++c) acc[c] = mfma_step(a, b, acc[c]);
  }
  Out s = 0;
#pragma unroll
  for (int c = 0; c < MCH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  // never true (the sums stay positive): the store only keeps the chains live
  if (s == (Out)-1) out[(int64_t)blockIdx.x * LANES + threadIdx.x] = s;
}

// Four independent 16-byte loads in flight per lane before the stores.
__global__ __launch_bounds__(LANES) void k_copy(const v4f* __restrict__ src, v4f* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * LANES;
  int64_t i = (int64_t)blockIdx.x * LANES + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const v4f a = __builtin_nontemporal_load(src + i);
    const v4f b = __builtin_nontemporal_load(src + i + stride);
    const v4f c = __builtin_nontemporal_load(src + i + 2 * stride);
    const v4f d = __builtin_nontemporal_load(src + i + 3 * stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
    __builtin_nontemporal_store(c, dst + i + 2 * stride);
    __builtin_nontemporal_store(d, dst + i + 3 * stride);
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

bool bad_shape(const void* out, int blocks, int iters) {
  return out == nullptr || blocks < 1 || blocks > (1 << 20) || iters < 1 || iters > (1 << 24);
}

int launched() { return hipGetLastError() == hipSuccess ? 0 : -4; }

}  // namespace

extern "C" int nnp_peak_fma_f32(float* out, int blocks, int iters, void* stream) {
  if (bad_shape(out, blocks, iters)) return -1;
  k_fma<float><<<blocks, LANES, 0, (hipStream_t)stream>>>(out, iters, 0.9999f, 1e-4f);
  return launched();
}

extern "C" int nnp_peak_fma_f64(double* out, int blocks, int iters, void* stream) {
  if (bad_shape(out, blocks, iters)) return -1;
  k_fma<double><<<blocks, LANES, 0, (hipStream_t)stream>>>(out, iters, 0.9999, 1e-4);
  return launched();
}

extern "C" int nnp_peak_exp_f32(float* out, int blocks, int iters, void* stream) {
  if (bad_shape(out, blocks, iters)) return -1;
  k_exp<<<blocks, LANES, 0, (hipStream_t)stream>>>(out, iters);
  return launched();
}

extern "C" int nnp_peak_mfma_f32(float* out, int blocks, int iters, void* stream) {
  if (bad_shape(out, blocks, iters)) return -1;
  k_mfma<float, v4f, float><<<blocks, LANES, 0, (hipStream_t)stream>>>(out, iters, 0.5f, 1e-4f);
  return launched();
}

extern "C" int nnp_peak_mfma_f64(double* out, int blocks, int iters, void* stream) {
  if (bad_shape(out, blocks, iters)) return -1;
  k_mfma<double, v4d, double><<<blocks, LANES, 0, (hipStream_t)stream>>>(out, iters, 0.5, 1e-4);
  return launched();
}

extern "C" int nnp_peak_mfma_bf16(float* out, int blocks, int iters, void* stream) {
  if (bad_shape(out, blocks, iters)) return -1;
  v8bf a, b;
  for (int k = 0; k < 8; ++k) {
    a[k] = (__bf16)0.5f;
    b[k] = (__bf16)1e-4f;
  }
  k_mfma<v8bf, v4f, float><<<blocks, LANES, 0, (hipStream_t)stream>>>(out, iters, a, b);
  return launched();
}

extern "C" int nnp_peak_copy(const void* src, void* dst, int64_t bytes, int blocks, void* stream) {
  if (src == nullptr || dst == nullptr || bytes <= 0 || bytes % 16 != 0 || blocks < 1 || blocks > (1 << 20) ||
      ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
    return -1;
  const char* s = (const char*)src;
  char* d = (char*)dst;
  if (s < d + bytes && d < s + bytes) return -1;
  k_copy<<<blocks, LANES, 0, (hipStream_t)stream>>>((const v4f*)src, (v4f*)dst, bytes / 16);
  return launched();
}
