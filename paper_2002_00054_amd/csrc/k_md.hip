// Velocity Verlet (constant N, V, E) around the energy+force path: the MD
// step the method is used in (Sec. 4, MD proxy application with energy
// conservation checks).  Per step, with a = F / m:
//   v <- v + (dt/2) a(t);  x <- x + dt v;  F <- F(x);  v <- v + (dt/2) a(t + dt).
// Units: A, fs, eV, amu; accel_conv turns eV/(A amu) into A/fs^2 and
// ke_conv turns amu A^2/fs^2 into eV.  Updates are done in FP64 and rounded
// once to the positions' type; positions are wrapped back into [0, L).
#include <algorithm>

#include "kernels.h"

namespace nnp {
namespace {

constexpr int MD_THREADS = 256;

__device__ inline int clamp_type(int t) { return t < 0 ? 0 : (t >= MAX_EL ? MAX_EL - 1 : t); }

template <class IO>
__global__ void __launch_bounds__(MD_THREADS) k_kick_drift(int64_t n, IO* pos, IO* vel, const IO* F,
                                                           const int32_t* types, MdArgs m) {
  const int64_t stride = (int64_t)gridDim.x * MD_THREADS;
  for (int64_t i = (int64_t)blockIdx.x * MD_THREADS + threadIdx.x; i < n; i += stride) {
    const double h = m.half_kick[clamp_type(types[i])];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const double v = (double)vel[3 * i + x] + h * (double)F[3 * i + x];
      double p = (double)pos[3 * i + x] + m.dt * v;
      p -= m.L[x] * floor(p * m.invL[x]);
      vel[3 * i + x] = (IO)v;
      pos[3 * i + x] = (IO)p;
    }
  }
}

// Second half-kick (h = 0: none) and the kinetic energy: one FP64 partial
// sum per block, combined in a fixed order by k_ke_total.
template <class IO>
__global__ void __launch_bounds__(MD_THREADS) k_kick_ke(int64_t n, IO* vel, const IO* F, const int32_t* types,
                                                        MdArgs m, int kick, double* partial) {
  __shared__ double red[MD_THREADS];
  const int64_t stride = (int64_t)gridDim.x * MD_THREADS;
  double ke = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MD_THREADS + threadIdx.x; i < n; i += stride) {
    const int t = clamp_type(types[i]);
    const double h = kick ? m.half_kick[t] : 0.0;
    double v2 = 0.0;
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      const double v = (double)vel[3 * i + x] + h * (double)F[3 * i + x];
      const IO vr = (IO)v;
      if (kick) vel[3 * i + x] = vr;
      v2 += (double)vr * (double)vr;
    }
    ke += m.half_mass[t] * v2;
  }
  red[threadIdx.x] = ke;
  __syncthreads();
  for (int s = MD_THREADS / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_ke_total(const double* partial, int nb, double conv, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[b];
    *out = s * conv;
  }
}

}  // namespace

int md_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + MD_THREADS - 1) / MD_THREADS, 1024)); }

template <class IO>
void launch_kick_drift(int64_t n, IO* pos, IO* vel, const IO* F, const int32_t* types, const MdArgs& m,
                       hipStream_t stream) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_kick_drift<IO>, dim3(md_blocks(n)), dim3(MD_THREADS), 0, stream, n, pos, vel, F, types, m);
}

template <class IO>
void launch_kick_ke(int64_t n, IO* vel, const IO* F, const int32_t* types, const MdArgs& m, bool kick,
                    double* partial, double* ke_out, hipStream_t stream) {
  const int nb = md_blocks(n);
  if (n > 0)
    hipLaunchKernelGGL(k_kick_ke<IO>, dim3(nb), dim3(MD_THREADS), 0, stream, n, vel, F, types, m, kick ? 1 : 0,
                       partial);
  hipLaunchKernelGGL(k_ke_total, dim3(1), dim3(64), 0, stream, partial, n > 0 ? nb : 0, m.ke_conv, ke_out);
}

template void launch_kick_drift<float>(int64_t, float*, float*, const float*, const int32_t*, const MdArgs&,
                                       hipStream_t);
template void launch_kick_drift<double>(int64_t, double*, double*, const double*, const int32_t*, const MdArgs&,
                                        hipStream_t);
template void launch_kick_ke<float>(int64_t, float*, const float*, const int32_t*, const MdArgs&, bool, double*,
                                    double*, hipStream_t);
template void launch_kick_ke<double>(int64_t, double*, const double*, const int32_t*, const MdArgs&, bool, double*,
                                     double*, hipStream_t);

}  // namespace nnp
