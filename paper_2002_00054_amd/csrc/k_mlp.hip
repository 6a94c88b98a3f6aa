// Per-element atomic networks (Sec. 3.1 step 2, Fig. 1(c)) and their
// derivatives:
//   forward   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), E_i = w3 . h2 + b3
//             on the scaled descriptors x = G~;
//   dE/dG     c = diag(1/scale) W1^T [(1 - h1^2) o W2^T [(1 - h2^2) o w3]]
//             (the network part of step 3, counted with the forces in the
//             paper's Fig. 5);
//   weights   differentiation form: gradient of sum_i [a_i E_i - <dE_i/dx_i, t_i>]
//             with a tangent t_i per atom (forward-over-reverse).
// Sorted atoms of one element are contiguous, so every workgroup works on
// rows of a single element and reads that element's weights with uniform
// loads.
#include <algorithm>

#include "kernels.h"

namespace nnp {

// Workgroup b -> (element, first row) for tiles of `rows` rows per element.
__device__ inline bool element_tile(int b, int rows, int n_el, const int* __restrict__ eoff, int& e, int64_t& r0,
                                    int64_t& r1) {
  int acc = 0;
  for (int f = 0; f < n_el; ++f) {
    const int64_t lo = eoff[f], hi = eoff[f + 1];
    const int nt = (int)((hi - lo + rows - 1) / rows);
    if (b < acc + nt) {
      e = f;
      r0 = lo + (int64_t)(b - acc) * rows;
      r1 = hi;
      return true;
    }
    acc += nt;
  }
  return false;
}

__device__ inline float tanh_t(float x) { return tanhf(x); }
__device__ inline double tanh_t(double x) { return tanh(x); }

// ------------------------------------------------------------------ MFMA
// Network forward + input gradient on the matrix cores, one 16-atom tile per
// wave step.  Activations are kept transposed (units x atoms) and used as the
// B operand, weights as the A operand, so the accumulator layout of one layer
// is directly the B operand of the next layer: no LDS transposes.  Each lane
// carries 8 values of a 32-wide vector; slot s = 4 t + r of lane group
// g = lane / 16 stands for unit kin_acc(g, s) (accumulator order: the FP32
// 16x16 accumulators hold rows 4 g + r of tile t, the FP64 ones rows g + 4 r,
// as measured on gfx950) or for unit 8 g + s (the input rows read from G~).
// Any bijection works for the reduction as long as the A operand uses the
// same one.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <class T>
__device__ inline int kin_acc(int g, int s) {
  if constexpr (sizeof(T) == 8) return 16 * (s >> 2) + g + 4 * (s & 3);
  else return 16 * (s >> 2) + 4 * g + (s & 3);
}
__device__ inline int kin_row(int g, int s) { return 8 * g + s; }

__device__ inline f32x4 mfma4(float a, float b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline f64x4 mfma4(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

template <class T> struct Acc4;
template <> struct Acc4<float> { using type = f32x4; };
template <> struct Acc4<double> { using type = f64x4; };

// y = W x for one tile with 16x16x4 MFMA (FP32 or FP64).  w(o, k) gives the
// weight of output unit o and input unit k; in_row selects the input slot map.
template <class T, class WF>
__device__ inline void layer_k4(const T (&in)[8], bool in_row, WF w, T (&out)[8]) {
  using V = typename Acc4<T>::type;
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    V acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int s = 0; s < 8; ++s) acc = mfma4(w(16 * t + col, in_row ? kin_row(g, s) : kin_acc<T>(g, s)), in[s], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) out[4 * t + r] = acc[r];
  }
}

// y = W x with 16x16x32 BF16 MFMA and FP32 accumulation; split = BF16x3
// (x = x_hi + x_lo, W = W_hi + W_lo, products hi*hi + hi*lo + lo*hi).
template <class WF>
__device__ inline void layer_bf16(const float (&in)[8], bool in_row, WF w, bool split, float (&out)[8]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  bf16x8 bh, bl;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const __bf16 h = (__bf16)in[s];
    bh[s] = h;
    bl[s] = (__bf16)(in[s] - (float)h);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    bf16x8 ah, al;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float x = w(16 * t + col, in_row ? kin_row(g, s) : kin_acc<float>(g, s));
      const __bf16 h = (__bf16)x;
      ah[s] = h;
      al[s] = (__bf16)(x - (float)h);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
    if (split) {
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) out[4 * t + r] = acc[r];
  }
}

template <int P, class T, class WF>
__device__ inline void layer(const T (&in)[8], bool in_row, WF w, bool first, T (&out)[8]) {
  if constexpr (P == P_BF16) layer_bf16(in, in_row, w, first, out);
  else layer_k4<T>(in, in_row, w, out);
}

// Grid: n_el x wpe workgroups of 4 waves; workgroup (e, b) serves element e,
// its waves striding over that element's 16-atom tiles.  The element's
// padded weights are staged in LDS once per workgroup.
template <int P>
__global__ void __launch_bounds__(256) k_mlp_mfma(MlpArgs<P> a, int wpe) {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  __shared__ T W[NET_STRIDE];
  __shared__ T isc[HID];
  const int e = uniform(blockIdx.x / wpe);
  const int b = blockIdx.x % wpe;
  if (e >= a.n_el) return;
  const T* __restrict__ src = a.nets + (size_t)e * NET_STRIDE;
  for (int i = threadIdx.x; i < NET_STRIDE; i += 256) W[i] = src[i];
  if (threadIdx.x < HID) isc[threadIdx.x] = threadIdx.x < MAX_SF ? (T)a.tab->inv_scale_d[e][threadIdx.x] : T(0);
  __syncthreads();
  const int64_t lo = a.eoff[e], hi = a.eoff[e + 1];
  const int64_t ntiles = (hi - lo + 15) / 16;
  const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
  const int wv = threadIdx.x >> 6;
  T b1[8], b2[8], w3[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int u = kin_acc<T>(g, s);
    b1[s] = W[OFF_B1 + u];
    b2[s] = W[OFF_B2 + u];
    w3[s] = W[OFF_W3 + u];
  }
  const T b3 = W[OFF_B3];
  auto W1 = [&](int o, int k) { return W[OFF_W1 + o * HID + k]; };
  auto W2 = [&](int o, int k) { return W[OFF_W2 + o * HID + k]; };
  auto W2t = [&](int o, int k) { return W[OFF_W2 + k * HID + o]; };
  auto W1t = [&](int o, int k) { return W[OFF_W1 + k * HID + o]; };
  for (int64_t tile = (int64_t)b * 4 + wv; tile < ntiles; tile += (int64_t)wpe * 4) {
    const int64_t atom = lo + tile * 16 + col;
    const bool valid = atom < hi;
    T x[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = valid ? (T)a.G[atom * LD + kin_row(g, s)] : T(0);
    T h1[8], h2[8], d[8], y[8];
    layer<P>(x, true, W1, true, y);
#pragma unroll
    for (int s = 0; s < 8; ++s) h1[s] = tanh_t(y[s] + b1[s]);
    layer<P>(h1, false, W2, false, y);
    T pe = T(0);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      h2[s] = tanh_t(y[s] + b2[s]);
      pe += w3[s] * h2[s];
      d[s] = w3[s] * (T(1) - h2[s] * h2[s]);
    }
    pe += __shfl_xor(pe, 16, 64);
    pe += __shfl_xor(pe, 32, 64);
    if (g == 0 && valid) a.Ei[atom] = (IO)(pe + b3);
    layer<P>(d, false, W2t, false, y);
#pragma unroll
    for (int s = 0; s < 8; ++s) d[s] = y[s] * (T(1) - h1[s] * h1[s]);
    layer<P>(d, false, W1t, true, y);
    if (valid) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int k = kin_acc<T>(g, s);
        a.C[atom * LD + k] = (IO)(y[s] * isc[k]);
      }
    }
  }
}

template <int P>
void launch_mlp(const MlpArgs<P>& a, hipStream_t stream) {
  if (a.n == 0) return;
  int wpe = (int)std::min<int64_t>(512, (a.n + 63) / 64);
  if (wpe < 1) wpe = 1;
  hipLaunchKernelGGL(k_mlp_mfma<P>, dim3((unsigned)(a.n_el * wpe)), dim3(256), 0, stream, a, wpe);
}

// ------------------------------------------------------------ weight gradient
// Per-atom vectors of the forward-over-reverse pass, stored for the
// parameter reduction:  [x, t, h1, dh1, zb1, dzb1, h2, dh2, zb2, dzb2, alpha]
// where t is the tangent (JVP row / scale), dh = tangent of h, zb/dzb the
// adjoints of the pre-activations of the primal and tangent chains.
constexpr int WG_VEC = 11;

// One atom per 32 lanes (two per wave): lane l owns hidden unit l, so every
// layer is one 32-term dot product per lane (a row of W, read four at a time)
// whose inputs come from the atom's other lanes by width-32 shuffles; the
// backward step through W2 has lane l own input l (a column of W2, read
// coalesced across the lanes).  Same expressions and summation order as one
// thread per atom, with 32 times the parallelism.
template <int P>
__global__ void __launch_bounds__(256) k_wgrad_atoms(WGradArgs<P> a) {
  using T = typename Types<P>::T;
  using V4 = typename Vec4<T>::type;
  constexpr int ATOMS = 256 / HID;  // atoms per block
  int e;
  int64_t r0, r1;
  if (!element_tile(blockIdx.x, ATOMS, a.n_el, a.eoff, e, r0, r1)) return;
  e = uniform(e);
  const int l = threadIdx.x & (HID - 1);
  const int64_t r = r0 + (threadIdx.x / HID);
  if (r >= r1) return;  // the atom's 32 lanes leave together
  const T* __restrict__ W = a.nets + (size_t)e * NET_STRIDE;
  T* out = a.vec + r * (WG_VEC * HID);
  const T x = (T)a.G[r * LD + l];
  const T t = (T)a.V[r * LD + l] * (l < MAX_SF ? (T)a.tab->inv_scale_d[e][l] : T(0));
  // layer 1: z = W1 x + b1 and its tangent W1 t (lane = output unit)
  T z = W[OFF_B1 + l], dz = T(0);
#pragma unroll
  for (int kb = 0; kb < HID; kb += 4) {
    const V4 w = *reinterpret_cast<const V4*>(W + OFF_W1 + l * HID + kb);
    const T wk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      z += wk[q] * __shfl(x, kb + q, HID);
      dz += wk[q] * __shfl(t, kb + q, HID);
    }
  }
  const T h1 = tanh_t(z), dz1 = dz;
  const T dh1 = (T(1) - h1 * h1) * dz1;
  out[0 * HID + l] = x;
  out[1 * HID + l] = t;
  out[2 * HID + l] = h1;
  out[3 * HID + l] = dh1;
  const T alpha = a.gE_atom ? (T)a.gE_atom[r] : T(0);
  // layer 2.  Objective J = alpha E - w3 . dh2, dh2 = (1 - h2^2) dz2.
  T z2 = W[OFF_B2 + l], dz2 = T(0);
#pragma unroll
  for (int kb = 0; kb < HID; kb += 4) {
    const V4 w = *reinterpret_cast<const V4*>(W + OFF_W2 + l * HID + kb);
    const T wk[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      z2 += wk[q] * __shfl(h1, kb + q, HID);
      dz2 += wk[q] * __shfl(dh1, kb + q, HID);
    }
  }
  const T h2 = tanh_t(z2);
  const T g2 = T(1) - h2 * h2;
  const T w3 = W[OFF_W3 + l];
  // adjoint of h2: alpha w3 from E, and from -w3 . (1 - h2^2) dz2: +2 w3 h2 dz2
  const T h2bar = alpha * w3 + T(2) * w3 * h2 * dz2;
  const T zb2 = g2 * h2bar, dzb2 = -g2 * w3;
  out[6 * HID + l] = h2;
  out[7 * HID + l] = g2 * dz2;
  out[8 * HID + l] = zb2;
  out[9 * HID + l] = dzb2;
  // back through W2 (lane = input unit of layer 2)
  T hb = T(0), dhb = T(0);
#pragma unroll
  for (int o = 0; o < HID; ++o) {
    const T w = W[OFF_W2 + o * HID + l];
    hb += w * __shfl(zb2, o, HID);
    dhb += w * __shfl(dzb2, o, HID);
  }
  const T g1 = T(1) - h1 * h1;
  // dh1 = (1 - h1^2) dz1 contributes -2 h1 dz1 dhb to the adjoint of h1
  hb += dhb * (T(-2) * h1 * dz1);
  out[4 * HID + l] = g1 * hb;
  out[5 * HID + l] = g1 * dhb;
  if (l == 0) out[10 * HID] = alpha;
}

template <class T> struct PairOf;
template <> struct PairOf<float> { using type = float2; };
template <> struct PairOf<double> { using type = double2; };

// partial[(e * nch + ch) * NET_STRIDE + p]: sum over one chunk of atoms of
// element e of the per-atom gradient of every parameter p (padded layout), in
// FP64.  One 256-thread block per (chunk, element) covers all parameters, so
// each atom's vector is read once per chunk.  The weight gradients are outer
// products (W1: zb1 x^T + dzb1 t^T, W2: zb2 h1^T + dzb2 dh1^T): thread t owns
// the 2 x 2 tile at (o, k) = (2 (t / 16), 2 (t % 16)) of both matrices and
// reads four pairs of each per atom.  Threads 0-31 also own b1, b2 and w3 at
// index t, thread 32 owns b3, and threads 33-63 write the padding (zero).
template <class T>
__global__ void __launch_bounds__(256) k_wgrad_chunks(const int* __restrict__ eoff, int chunk, int nch,
                                                      const T* __restrict__ vec, double* __restrict__ partial) {
  using T2 = typename PairOf<T>::type;
  static_assert(HID == 32 && NET_STRIDE == OFF_B3 + HID, "tile map covers the padded layout exactly");
  const int e = blockIdx.y;
  const int ch = blockIdx.x;
  const int t = threadIdx.x;
  const int o0 = 2 * (t >> 4), k0 = 2 * (t & 15);
  const int64_t lo = eoff[e] + (int64_t)ch * chunk;
  const int64_t hi = min((int64_t)eoff[e + 1], lo + chunk);
  double w1[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, w2[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  double b1 = 0.0, b2 = 0.0, w3 = 0.0, b3 = 0.0;
  for (int64_t r = lo; r < hi; ++r) {
    const T* v = vec + r * (WG_VEC * HID);
    const T2 zb1 = *reinterpret_cast<const T2*>(v + 4 * HID + o0);
    const T2 dzb1 = *reinterpret_cast<const T2*>(v + 5 * HID + o0);
    const T2 x = *reinterpret_cast<const T2*>(v + 0 * HID + k0);
    const T2 tg = *reinterpret_cast<const T2*>(v + 1 * HID + k0);
    const T2 zb2 = *reinterpret_cast<const T2*>(v + 8 * HID + o0);
    const T2 dzb2 = *reinterpret_cast<const T2*>(v + 9 * HID + o0);
    const T2 h1 = *reinterpret_cast<const T2*>(v + 2 * HID + k0);
    const T2 dh1 = *reinterpret_cast<const T2*>(v + 3 * HID + k0);
    const T a_o[2] = {zb1.x, zb1.y}, c_o[2] = {dzb1.x, dzb1.y}, b_k[2] = {x.x, x.y}, d_k[2] = {tg.x, tg.y};
    const T p_o[2] = {zb2.x, zb2.y}, q_o[2] = {dzb2.x, dzb2.y}, u_k[2] = {h1.x, h1.y}, w_k[2] = {dh1.x, dh1.y};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        w1[i][j] += (double)(a_o[i] * b_k[j] + c_o[i] * d_k[j]);
        w2[i][j] += (double)(p_o[i] * u_k[j] + q_o[i] * w_k[j]);
      }
    if (t < HID) {
      b1 += (double)v[4 * HID + t];
      b2 += (double)v[8 * HID + t];
      w3 += (double)(v[10 * HID] * v[6 * HID + t] - v[7 * HID + t]);
    } else if (t == HID) {
      b3 += (double)v[10 * HID];
    }
  }
  double* out = partial + ((size_t)e * nch + ch) * NET_STRIDE;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      out[OFF_W1 + (o0 + i) * HID + k0 + j] = w1[i][j];
      out[OFF_W2 + (o0 + i) * HID + k0 + j] = w2[i][j];
    }
  if (t < HID) {
    out[OFF_B1 + t] = b1;
    out[OFF_B2 + t] = b2;
    out[OFF_W3 + t] = w3;
  } else if (t == HID) {
    out[OFF_B3] = b3;
  } else if (t < 2 * HID) {
    out[OFF_B3 + (t - HID)] = 0.0;
  }
}

// out[e][p] = sum over the chunks of element e (FP64) in a fixed order: eight
// running sums, chunk ch going to sum ch % 8 in chunk order, then the eight
// in order.  A block covers 32 parameters with 8 threads each.
__global__ void __launch_bounds__(256) k_wgrad_final(int nch, const double* __restrict__ partial,
                                                     double* __restrict__ out) {
  __shared__ double red[8][32];
  const int e = blockIdx.y;
  const int pl = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int p = blockIdx.x * 32 + pl;
  double s = 0.0;
  if (p < NET_STRIDE)
    for (int ch = g; ch < nch; ch += 8) s += partial[((size_t)e * nch + ch) * NET_STRIDE + p];
  red[g][pl] = s;
  __syncthreads();
  if (g == 0 && p < NET_STRIDE) {
    double tot = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) tot += red[i][pl];
    out[(size_t)e * NET_STRIDE + p] = tot;
  }
}

// Padded gradient -> caller's flat parameter layout.
__global__ void __launch_bounds__(256) k_unpad(int64_t np, const int* __restrict__ map, const double* __restrict__ padded,
                                               double* __restrict__ flat) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < np) flat[i] = padded[map[i]];
}

template <int P>
void launch_wgrad(const WGradArgs<P>& a, hipStream_t stream) {
  using T = typename Types<P>::T;
  if (a.n > 0) {
    const unsigned g = (unsigned)((a.n + 256 / HID - 1) / (256 / HID) + a.n_el);
    hipLaunchKernelGGL(k_wgrad_atoms<P>, dim3(g), dim3(256), 0, stream, a);
  }
  hipLaunchKernelGGL(k_wgrad_chunks<T>, dim3((unsigned)a.nch, a.n_el), dim3(256), 0, stream, a.eoff, a.chunk, a.nch,
                     (const T*)a.vec, a.partial);
  hipLaunchKernelGGL(k_wgrad_final, dim3((NET_STRIDE + 31) / 32, a.n_el), dim3(256), 0, stream, a.nch, a.partial,
                     a.padded);
  hipLaunchKernelGGL(k_unpad, dim3((unsigned)((a.n_params + 255) / 256)), dim3(256), 0, stream, a.n_params, a.flatmap,
                     a.padded, a.out);
}

template void launch_mlp<P_FP64>(const MlpArgs<P_FP64>&, hipStream_t);
template void launch_mlp<P_FP32>(const MlpArgs<P_FP32>&, hipStream_t);
template void launch_mlp<P_BF16>(const MlpArgs<P_BF16>&, hipStream_t);
template void launch_wgrad<P_FP64>(const WGradArgs<P_FP64>&, hipStream_t);
template void launch_wgrad<P_FP32>(const WGradArgs<P_FP32>&, hipStream_t);

}  // namespace nnp
