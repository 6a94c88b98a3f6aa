// Fills, (un)permutation to the caller's atom order and the deterministic
// FP64 energy sums E_b = sum_i E_i (Fig. 1(b), the E_system loop).
#include "kernels.h"

namespace nnp {

template <class T>
__global__ void __launch_bounds__(256) k_fill(T* __restrict__ p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <class T>
void launch_fill(T* p, int64_t n, T v, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, v);
}
template void launch_fill<float>(float*, int64_t, float, hipStream_t);
template void launch_fill<double>(double*, int64_t, double, hipStream_t);
template void launch_fill<int>(int*, int64_t, int, hipStream_t);

void launch_fill_int(int* p, int64_t n, int v, hipStream_t stream) { launch_fill<int>(p, n, v, stream); }

template <class IO, class FAcc>
__global__ void __launch_bounds__(256) k_unpermute(int64_t n, const int* __restrict__ perm, const IO* __restrict__ Ei_s,
                                                   const FAcc* __restrict__ F_s, double* __restrict__ Ei_o,
                                                   IO* __restrict__ Ei_out, IO* __restrict__ F_out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t i = perm[s];
  const IO e = Ei_s[s];
  Ei_o[i] = (double)e;
  if (Ei_out) Ei_out[i] = e;
  if (F_out) {
    F_out[3 * i + 0] = (IO)F_s[s];  // sorted accumulator: component planes [3][n]
    F_out[3 * i + 1] = (IO)F_s[n + s];
    F_out[3 * i + 2] = (IO)F_s[2 * n + s];
  }
}

template <class IO, class FAcc>
void launch_unpermute(int64_t n, const int* perm, const IO* Ei_s, const FAcc* F_s, double* Ei_o, IO* Ei_out,
                      IO* F_out, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_unpermute<IO, FAcc>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, perm, Ei_s,
                     F_s, Ei_o, Ei_out, F_out);
}
template void launch_unpermute<double, double>(int64_t, const int*, const double*, const double*, double*, double*,
                                               double*, hipStream_t);
template void launch_unpermute<float, float>(int64_t, const int*, const float*, const float*, double*, float*, float*,
                                             hipStream_t);
template void launch_unpermute<float, double>(int64_t, const int*, const float*, const double*, double*, float*,
                                              float*, hipStream_t);

// out[s] = in[perm[s]] for rows of 3 (caller order -> sorted order).
template <class IO>
__global__ void __launch_bounds__(256) k_permute_rows3(int64_t n, const int* __restrict__ perm, const IO* __restrict__ in,
                                                       IO* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t i = perm[s];
  out[3 * s + 0] = in[3 * i + 0];
  out[3 * s + 1] = in[3 * i + 1];
  out[3 * s + 2] = in[3 * i + 2];
}

template <class IO>
void launch_permute_rows3(int64_t n, const int* perm, const IO* in, IO* out, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_permute_rows3<IO>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, perm, in, out);
}
template void launch_permute_rows3<float>(int64_t, const int*, const float*, float*, hipStream_t);
template void launch_permute_rows3<double>(int64_t, const int*, const double*, double*, hipStream_t);

// gE_atom[s] = gE[structure of caller atom perm[s]] (0 if gE is null).
__global__ void __launch_bounds__(256) k_gather_struct_grad(int64_t n, const int* __restrict__ perm,
                                                            const int64_t* __restrict__ soff, int n_struct,
                                                            const double* __restrict__ gE, double* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (!gE) {
    out[s] = 0.0;
    return;
  }
  const int64_t i = perm[s];
  int lo = 0, hi = n_struct - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (soff[mid] <= i) lo = mid; else hi = mid - 1;
  }
  out[s] = gE[lo];
}

void launch_gather_struct_grad(int64_t n, const int* perm, const int64_t* soff, int n_struct, const double* gE,
                               double* gE_atom, hipStream_t stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_struct_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, perm, soff,
                     n_struct, gE, gE_atom);
}

// Block tree sum of a range in a fixed order.
__device__ inline double block_sum_256(double v) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(256) k_chunk_sum(const double* __restrict__ x, const int64_t* __restrict__ lo,
                                                   const int64_t* __restrict__ hi, double* __restrict__ partial) {
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = lo[c] + threadIdx.x; i < hi[c]; i += 256) s += x[i];
  s = block_sum_256(s);
  if (threadIdx.x == 0) partial[c] = s;
}

__global__ void __launch_bounds__(256) k_struct_sum(const double* __restrict__ partial, const int* __restrict__ sc,
                                                    double* __restrict__ out) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int c = sc[b] + threadIdx.x; c < sc[b + 1]; c += 256) s += partial[c];
  s = block_sum_256(s);
  if (threadIdx.x == 0) out[b] = s;
}

void launch_energy(const double* Ei_o, const int64_t* chunk_lo, const int64_t* chunk_hi, int nchunk,
                   const int* struct_chunk, int n_struct, double* partial, double* energies, hipStream_t stream) {
  if (nchunk > 0)
    hipLaunchKernelGGL(k_chunk_sum, dim3(nchunk), dim3(256), 0, stream, Ei_o, chunk_lo, chunk_hi, partial);
  hipLaunchKernelGGL(k_struct_sum, dim3(n_struct), dim3(256), 0, stream, partial, struct_chunk, energies);
}

}  // namespace nnp
