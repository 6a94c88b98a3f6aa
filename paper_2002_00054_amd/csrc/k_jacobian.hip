// Stored-Jacobian variant of the differentiation form.
//
// The force step of the method is the chain rule F_m = -sum_i sum_s
// (dE_i/dG_is) dG_is/dr_m (Sec. 3.1, step 3).  The paper recomputes the SF
// derivatives rather than keeping them (Sec. 3.3); this variant keeps them.
// One pass computes the SFs and, for every centre i and neighbour slot t
// (neighbour j), the gradient J_its = dG_is/dr_j of each SF s; forces and the
// force-adjoint product are then contractions of that store:
//   F_j -= sum_s c_is J_its,   F_i += sum_t sum_s c_is J_its,
//   v_is = sum_t (delta_j - delta_i) . J_its,
// where the terms for the centre follow from G_i depending on positions only
// through the differences r_j - r_i.
//
// Gradient of one angular term T = pre (1 + lam cos)^zeta e^{-eta (a^2 + b^2 +
// d^2)} fc(a) fc(b) fc(d), a = |r_ij|, b = |r_ik|, d = |r_k - r_j|, with
// respect to r_j:
//   dT/dcos (r_ik/(a b) - cos r_ij/a^2) + 2 dT/d(a^2) r_ij - 2 dT/d(d^2) (r_k - r_j),
// and of a radial term t = e^{-eta (r - rs)^2} fc(r): dt/dr r_ij/r.  The
// cutoff is the same polynomial in r^2 the other passes use.
//
// k_jac gives each lane of a wave one neighbour j and walks every other
// neighbour k of the centre, so each lane accumulates only its own row of J in
// registers: no atomics and no LDS slot sums, at the price of visiting every
// triplet twice (once from j, once from k).
#include <type_traits>

#include "kernels.h"

namespace nnp {
namespace {

template <int P>
constexpr size_t jac_wave_bytes_of(int lcap) {
  using T = typename Types<P>::T;
  using Acc = typename Types<P>::Acc;
  return (size_t)lcap * 2 * 4 * sizeof(T) + LD * sizeof(Acc);
}

// e^x: FP64 through the device math library; FP32 through the hardware
// base-2 exponential, as in the other passes.
__device__ inline float exp_t(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
__device__ inline double exp_t(double x) { return exp(x); }

// WIDE: the table holds wide angular functions (a separate instantiation, so
// that narrow-only tables keep the register count of the narrow loop).
template <int P, bool WIDE>
__global__ void __launch_bounds__(256) k_jac(JacArgs<P> a) {
  using T = typename Types<P>::T;
  using Acc = typename Types<P>::Acc;
  using IO = typename Types<P>::IO;
  using V4 = typename Vec4<T>::type;

  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = uniform((int)(threadIdx.x >> 6));
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t c = (int64_t)uniform((int)(blk * 4 + wv));
  if (c >= a.n) return;
  const int lcap = a.lcap;
  unsigned char* base = smem + (size_t)wv * jac_wave_bytes_of<P>(lcap);
  V4* rec = reinterpret_cast<V4*>(base);  // (dx, dy, dz, r^2) of each neighbour
  V4* aux = rec + lcap;                   // (r, fc, dfc/d(r^2), 0)
  Acc* gsum = reinterpret_cast<Acc*>(aux + lcap);

  const DevTab<T>* __restrict__ tab = a.tab;
  Cutoff<T> cut;
  cut.load(tab);
  const T rc2 = tab->rc2;
  const double4 pc = a.pos4[c];
  const int ec = uniform(elem_of(pc.w));
  const int n_el = tab->n_el;
  const int ns = uniform(tab->n_sf[ec]);
  const int4 nn = a.nnb[c];
  const int cnt[MAX_EL] = {uniform(nn.x), uniform(nn.y), uniform(nn.z), uniform(nn.w)};
  int off[MAX_EL + 1];
  off[0] = 0;
#pragma unroll
  for (int f = 0; f < MAX_EL; ++f) off[f + 1] = off[f] + (f < n_el ? cnt[f] : 0);
  const int m = off[n_el];
  const V4* __restrict__ row = a.nbr + c * (int64_t)a.cap;
  const int64_t e0 = c * (int64_t)a.cap;
  const int64_t plane = a.plane;

  for (int t = lane; t < m; t += WAVE) {
    const V4 e = row[t];
    V4 r, x;
    r.x = e.x;
    r.y = e.y;
    r.z = e.z;
    r.w = e.x * e.x + e.y * e.y + e.z * e.z;
    T fc, dfc;
    cut.eval(r.w, fc, dfc);
    x.x = sqrt(r.w);
    x.y = fc;
    x.z = dfc;
    x.w = T(0);
    rec[t] = r;
    aux[t] = x;
  }
  if (lane < LD) gsum[lane] = Acc(0);
  __builtin_amdgcn_wave_barrier();

  for (int f = 0; f < n_el; ++f) {
    // SFs of this centre that a neighbour of element f takes part in
    unsigned touched = 0u;
    const int nr = uniform(tab->rad_cnt[ec][f]);
    for (int q = 0; q < nr; ++q) touched |= 1u << tab->rad_out[ec][f][q];
    for (int g = 0; g < n_el; ++g) {
      const int cls = class_index(min(f, g), max(f, g), n_el);
      const int na = uniform(tab->ang_cnt[ec][cls]);
      for (int q = 0; q < na; ++q) touched |= 1u << tab->ang_out[ec][cls][q];
    }
    for (int j0 = off[f]; j0 < off[f + 1]; j0 += WAVE) {
      const int t = j0 + lane;
      const bool jv = t < off[f + 1];
      const V4 ra = rec[jv ? t : j0];
      const V4 xa = aux[jv ? t : j0];
      const T ax = ra.x, ay = ra.y, az = ra.z, a2 = ra.w, ar = xa.x, fca = xa.y, dfca = xa.z;
      const int64_t e = e0 + t;
      for (int s = 0; s < ns; ++s) {
        if (jv && !((touched >> s) & 1u)) {
          a.J[(int64_t)(3 * s + 0) * plane + e] = T(0);
          a.J[(int64_t)(3 * s + 1) * plane + e] = T(0);
          a.J[(int64_t)(3 * s + 2) * plane + e] = T(0);
        }
      }
      // radial terms of the pair (i, j)
      for (int q = 0; q < nr; ++q) {
        const T eta = tab->rad_eta[ec][f][q], rs = tab->rad_rs[ec][f][q];
        const int s = tab->rad_out[ec][f][q];
        const T u = ar - rs;
        const T ex = exp_t(-eta * u * u);
        const T val = jv ? ex * fca : T(0);
        const T dr = ex * (T(-2) * eta * u * fca + dfca * T(2) * ar);  // dt/dr
        const T gs = dr / ar;
        if (jv) {
          a.J[(int64_t)(3 * s + 0) * plane + e] = gs * ax;
          a.J[(int64_t)(3 * s + 1) * plane + e] = gs * ay;
          a.J[(int64_t)(3 * s + 2) * plane + e] = gs * az;
        }
        const Acc tot = wave_sum((Acc)val);
        if (lane == 0) gsum[s] += tot;
      }
      // angular terms (i, j, k) with k in element block g
      const T inv_a2 = T(1) / a2;
      for (int g = 0; g < n_el; ++g) {
        const int cls = class_index(min(f, g), max(f, g), n_el);
        const int na = uniform(tab->ang_cnt[ec][cls]);
        if (na == 0) continue;
        const int ne = uniform(tab->n_eta[ec]);
        T qeta[MAX_ANG], qpre[MAX_ANG], qlam[MAX_ANG], qzeta[MAX_ANG];
        int qzl[MAX_ANG], qni[MAX_ANG];
        bool qwide[MAX_ANG];  // wide function: no r_jk factor or cutoff
        bool any_wide = false;
        T acc[MAX_ANG][3];
        T gacc[MAX_ANG];
#pragma unroll
        for (int q = 0; q < MAX_ANG; ++q) {
          qwide[q] = q < na && tab->ang_wide[ec][cls][q] != 0;
          any_wide |= qwide[q];
          const int bit = q < na ? tab->ang_bit[ec][cls][q] : 0;
          const int qb = bit / MAX_NE;
          qni[q] = bit % MAX_NE;
          qeta[q] = tab->aeta[ec][qni[q]];
          qpre[q] = q < na ? tab->ang_pre[ec][cls][q] : T(0);
          qlam[q] = qb < 6 ? T(1) : T(-1);
          qzl[q] = qb % 6;
          qzeta[q] = T(1 << qzl[q]);
          acc[q][0] = acc[q][1] = acc[q][2] = T(0);
          gacc[q] = T(0);
        }
        T eta_n[MAX_NE];
#pragma unroll
        for (int n = 0; n < MAX_NE; ++n) eta_n[n] = n < ne ? tab->aeta[ec][n] : T(0);
        // the pair loop, compiled without the wide terms for classes that have none
        auto pairs = [&](auto wide_tag) {
          constexpr bool W = decltype(wide_tag)::value;
          if constexpr (W) {
            for (int k = off[g]; k < off[g + 1]; ++k) {
              const V4 rb = rec[k];
              const V4 xb = aux[k];
              const T dx = rb.x - ax, dy = rb.y - ay, dz = rb.z - az;
              const T d2 = dx * dx + dy * dy + dz * dz;
              const bool near = d2 < rc2;
              if (!(jv && k != t && (near || W))) continue;
              T fcd = T(0), dfcd = T(0);
              if (near) cut.eval_in(d2, fcd, dfcd);
              const T b2 = rb.w, fcb = xb.y;
              const T inv_ab = T(1) / (ar * xb.x);
              const T cs = (ax * rb.x + ay * rb.y + az * rb.z) * inv_ab;
              const T ca = cs * inv_a2;
              const T gcx = rb.x * inv_ab - ca * ax, gcy = rb.y * inv_ab - ca * ay, gcz = rb.z * inv_ab - ca * az;
              const T s2 = a2 + b2 + d2, sw = a2 + b2;
              const T f2 = fca * fcb;
              const T f3 = f2 * fcd;
              T exn[MAX_NE], exw[MAX_NE];  // e^{-eta (a^2 + b^2 + d^2)} (narrow), e^{-eta (a^2 + b^2)} (wide)
    #pragma unroll
              for (int n = 0; n < MAX_NE; ++n) {
                exn[n] = n < ne && near ? exp_t(-eta_n[n] * s2) : T(0);
                exw[n] = W && n < ne ? exp_t(-eta_n[n] * sw) : T(0);
              }
    #pragma unroll
              for (int q = 0; q < MAX_ANG; ++q) {
                if (q < na) {
                  const int ni = qni[q];
                  const T en = ni == 0 ? exn[0] : ni == 1 ? exn[1] : ni == 2 ? exn[2] : exn[3];
                  const T ew = ni == 0 ? exw[0] : ni == 1 ? exw[1] : ni == 2 ? exw[2] : exw[3];
                  const bool wq = W && qwide[q];
                  const T ex = qpre[q] * (wq ? ew : en);
                  const T pb = T(1) + qlam[q] * cs;
                  T pz1 = T(1), pw = pb;  // pb^(zeta - 1), pb^zeta
                  for (int i = 0; i < qzl[q]; ++i) {
                    pz1 *= pw;
                    pw *= pw;
                  }
                  // wide: the r_jk factor is 1 (no f_c(r_jk), no d^2 in the exponent)
                  const T fr = wq ? f2 : f3;
                  const T fa = wq ? dfca * fcb : dfca * fcb * fcd;
                  const T fd = wq ? T(0) : fca * fcb * dfcd;
                  const T tq = pw * ex * fr;
                  const T dtdc = qzeta[q] * qlam[q] * pz1 * ex * fr;
                  const T dta = T(2) * (-qeta[q] * tq + pw * ex * fa);
                  const T dtd = wq ? T(0) : T(2) * (-qeta[q] * tq + pw * ex * fd);
                  acc[q][0] += dtdc * gcx + dta * ax - dtd * dx;
                  acc[q][1] += dtdc * gcy + dta * ay - dtd * dy;
                  acc[q][2] += dtdc * gcz + dta * az - dtd * dz;
                  gacc[q] += tq;
                }
              }
            }
          } else {  // narrow functions only
            for (int k = off[g]; k < off[g + 1]; ++k) {
              const V4 rb = rec[k];
              const V4 xb = aux[k];
              const T dx = rb.x - ax, dy = rb.y - ay, dz = rb.z - az;
              const T d2 = dx * dx + dy * dy + dz * dz;
              if (!(jv && k != t && d2 < rc2)) continue;
              T fcd, dfcd;
              cut.eval_in(d2, fcd, dfcd);
              const T b2 = rb.w, fcb = xb.y;
              const T inv_ab = T(1) / (ar * xb.x);
              const T cs = (ax * rb.x + ay * rb.y + az * rb.z) * inv_ab;
              const T ca = cs * inv_a2;
              const T gcx = rb.x * inv_ab - ca * ax, gcy = rb.y * inv_ab - ca * ay, gcz = rb.z * inv_ab - ca * az;
              const T s2 = a2 + b2 + d2;
              const T f3 = fca * fcb * fcd;
              const T fa3 = dfca * fcb * fcd;
              const T fd3 = fca * fcb * dfcd;
              T exn[MAX_NE];
    #pragma unroll
              for (int n = 0; n < MAX_NE; ++n) exn[n] = n < ne ? exp_t(-eta_n[n] * s2) : T(0);
    #pragma unroll
              for (int q = 0; q < MAX_ANG; ++q) {
                if (q < na) {
                  const int ni = qni[q];
                  const T ex = qpre[q] * (ni == 0 ? exn[0] : ni == 1 ? exn[1] : ni == 2 ? exn[2] : exn[3]);
                  const T pb = T(1) + qlam[q] * cs;
                  T pz1 = T(1), pw = pb;  // pb^(zeta - 1), pb^zeta
                  for (int i = 0; i < qzl[q]; ++i) {
                    pz1 *= pw;
                    pw *= pw;
                  }
                  const T tq = pw * ex * f3;
                  const T dtdc = qzeta[q] * qlam[q] * pz1 * ex * f3;
                  const T dta = T(2) * (-qeta[q] * tq + pw * ex * fa3);
                  const T dtd = T(2) * (-qeta[q] * tq + pw * ex * fd3);
                  acc[q][0] += dtdc * gcx + dta * ax - dtd * dx;
                  acc[q][1] += dtdc * gcy + dta * ay - dtd * dy;
                  acc[q][2] += dtdc * gcz + dta * az - dtd * dz;
                  gacc[q] += tq;
                }
              }
            }
          }
        };
        if constexpr (WIDE) {
          if (any_wide) pairs(std::true_type{});
          else pairs(std::false_type{});
        } else {
          pairs(std::false_type{});
        }
#pragma unroll
        for (int q = 0; q < MAX_ANG; ++q) {
          if (q < na) {
            const int s = tab->ang_out[ec][cls][q];
            if (jv) {
              a.J[(int64_t)(3 * s + 0) * plane + e] = acc[q][0];
              a.J[(int64_t)(3 * s + 1) * plane + e] = acc[q][1];
              a.J[(int64_t)(3 * s + 2) * plane + e] = acc[q][2];
            }
            // every unordered pair {j, k} was visited from j and from k
            const Acc tot = wave_sum((Acc)gacc[q]);
            if (lane == 0) gsum[s] += Acc(0.5) * tot;
          }
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < LD) {
    IO v = IO(0);
    if (lane < ns) v = (IO)(((double)gsum[lane] - tab->shift_d[ec][lane]) * tab->inv_scale_d[ec][lane]);
    a.G[c * LD + lane] = v;
  }
}

template <int P>
__global__ void __launch_bounds__(256) k_jac_force(JacArgs<P> a) {
  using T = typename Types<P>::T;
  using FAcc = typename Types<P>::FAcc;
  using IO = typename Types<P>::IO;
  const int lane = threadIdx.x & 63;
  const int wv = uniform((int)(threadIdx.x >> 6));
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t c = (int64_t)uniform((int)(blk * 4 + wv));
  if (c >= a.n) return;
  const DevTab<T>* __restrict__ tab = a.tab;
  const int ec = uniform(elem_of(a.pos4[c].w));
  const int ns = uniform(tab->n_sf[ec]);
  const int4 nn = a.nnb[c];
  const int n_el = tab->n_el;
  const int m = uniform(nn.x + (n_el > 1 ? nn.y : 0) + (n_el > 2 ? nn.z : 0) + (n_el > 3 ? nn.w : 0));
  const IO* __restrict__ crow = a.C + c * LD;
  const int64_t e0 = c * (int64_t)a.cap;
  const int64_t plane = a.plane;
  T fi0 = T(0), fi1 = T(0), fi2 = T(0);
  for (int t = lane; t < m; t += WAVE) {
    const int64_t e = e0 + t;
    T f0 = T(0), f1 = T(0), f2 = T(0);
    for (int s = 0; s < ns; ++s) {
      const T cs = (T)crow[s];
      const T* __restrict__ js = a.J + (int64_t)(3 * s) * plane + e;
      f0 += cs * js[0];
      f1 += cs * js[plane];
      f2 += cs * js[2 * plane];
    }
    const int64_t j = entry_index(a.nbr[e]);
    atomic_add(&a.F[j], (FAcc)(-f0));
    atomic_add(&a.F[a.n + j], (FAcc)(-f1));
    atomic_add(&a.F[2 * a.n + j], (FAcc)(-f2));
    fi0 += f0;
    fi1 += f1;
    fi2 += f2;
  }
  fi0 = wave_sum(fi0);
  fi1 = wave_sum(fi1);
  fi2 = wave_sum(fi2);
  if (lane == 0) {
    atomic_add(&a.F[c], (FAcc)fi0);
    atomic_add(&a.F[a.n + c], (FAcc)fi1);
    atomic_add(&a.F[2 * a.n + c], (FAcc)fi2);
  }
}

template <int P>
__global__ void __launch_bounds__(256) k_jac_jvp(JacArgs<P> a) {
  using T = typename Types<P>::T;
  using Acc = typename Types<P>::Acc;
  using IO = typename Types<P>::IO;
  __shared__ Acc vout[4][LD];
  const int lane = threadIdx.x & 63;
  const int wv = uniform((int)(threadIdx.x >> 6));
  const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t c = (int64_t)uniform((int)(blk * 4 + wv));
  if (c >= a.n) return;
  const DevTab<T>* __restrict__ tab = a.tab;
  const int ec = uniform(elem_of(a.pos4[c].w));
  const int ns = uniform(tab->n_sf[ec]);
  const int4 nn = a.nnb[c];
  const int n_el = tab->n_el;
  const int m = uniform(nn.x + (n_el > 1 ? nn.y : 0) + (n_el > 2 ? nn.z : 0) + (n_el > 3 ? nn.w : 0));
  const int64_t e0 = c * (int64_t)a.cap;
  const int64_t plane = a.plane;
  const T di0 = (T)a.delta[3 * c + 0], di1 = (T)a.delta[3 * c + 1], di2 = (T)a.delta[3 * c + 2];
  Acc acc[MAX_SF];
#pragma unroll
  for (int s = 0; s < MAX_SF; ++s) acc[s] = Acc(0);
  for (int t = lane; t < m; t += WAVE) {
    const int64_t e = e0 + t;
    const int64_t j = entry_index(a.nbr[e]);
    const T d0 = (T)a.delta[3 * j + 0] - di0, d1 = (T)a.delta[3 * j + 1] - di1, d2 = (T)a.delta[3 * j + 2] - di2;
#pragma unroll
    for (int s = 0; s < MAX_SF; ++s) {
      if (s < ns) {
        const T* __restrict__ js = a.J + (int64_t)(3 * s) * plane + e;
        acc[s] += (Acc)(d0 * js[0] + d1 * js[plane] + d2 * js[2 * plane]);
      }
    }
  }
  wave_sum_many<Acc, MAX_SF>(acc, vout[wv], lane);
  __builtin_amdgcn_wave_barrier();
  if (lane < LD) a.V[c * LD + lane] = lane < ns ? (IO)vout[wv][lane] : IO(0);
}

__device__ inline bool same_bits(float x, float y) { return __float_as_int(x) == __float_as_int(y); }
__device__ inline bool same_bits(double x, double y) { return __double_as_longlong(x) == __double_as_longlong(y); }

template <class IO>
__global__ void __launch_bounds__(256) k_same_inputs(int64_t n, const IO* pos, const IO* saved_pos,
                                                     const int32_t* types, const int32_t* saved_types, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool diff = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    diff |= types[i] != saved_types[i];
    diff |= !same_bits(pos[3 * i + 0], saved_pos[3 * i + 0]);
    diff |= !same_bits(pos[3 * i + 1], saved_pos[3 * i + 1]);
    diff |= !same_bits(pos[3 * i + 2], saved_pos[3 * i + 2]);
  }
  if (diff) flag[0] = 1;
}

int64_t wave_blocks(int64_t n) { return (n + 3) / 4; }

}  // namespace

template <int P>
size_t jac_lds_bytes(int lcap) {
  return 4 * jac_wave_bytes_of<P>(lcap);
}

template <int P>
void launch_jac(const JacArgs<P>& a, hipStream_t stream) {
  if (a.n == 0) return;
  const size_t lds = jac_lds_bytes<P>(a.lcap);
  const void* fn = a.wide ? reinterpret_cast<const void*>(&k_jac<P, true>)
                          : reinterpret_cast<const void*>(&k_jac<P, false>);
  if (lds > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (a.wide)
    hipLaunchKernelGGL((k_jac<P, true>), dim3((unsigned)wave_blocks(a.n)), dim3(256), lds, stream, a);
  else
    hipLaunchKernelGGL((k_jac<P, false>), dim3((unsigned)wave_blocks(a.n)), dim3(256), lds, stream, a);
}

template <int P>
void launch_jac_force(const JacArgs<P>& a, hipStream_t stream) {
  if (a.n == 0) return;
  hipLaunchKernelGGL(k_jac_force<P>, dim3((unsigned)wave_blocks(a.n)), dim3(256), 0, stream, a);
}

template <int P>
void launch_jac_jvp(const JacArgs<P>& a, hipStream_t stream) {
  if (a.n == 0) return;
  hipLaunchKernelGGL(k_jac_jvp<P>, dim3((unsigned)wave_blocks(a.n)), dim3(256), 0, stream, a);
}

template <class IO>
void launch_same_inputs(int64_t n, const IO* pos, const IO* saved_pos, const int32_t* types,
                        const int32_t* saved_types, int* flag, hipStream_t stream) {
  if (n == 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_same_inputs<IO>, dim3((unsigned)blocks), dim3(256), 0, stream, n, pos, saved_pos, types,
                     saved_types, flag);
}

template size_t jac_lds_bytes<P_FP64>(int);
template size_t jac_lds_bytes<P_FP32>(int);
template void launch_jac<P_FP64>(const JacArgs<P_FP64>&, hipStream_t);
template void launch_jac<P_FP32>(const JacArgs<P_FP32>&, hipStream_t);
template void launch_jac_force<P_FP64>(const JacArgs<P_FP64>&, hipStream_t);
template void launch_jac_force<P_FP32>(const JacArgs<P_FP32>&, hipStream_t);
template void launch_jac_jvp<P_FP64>(const JacArgs<P_FP64>&, hipStream_t);
template void launch_jac_jvp<P_FP32>(const JacArgs<P_FP32>&, hipStream_t);
template void launch_same_inputs<float>(int64_t, const float*, const float*, const int32_t*, const int32_t*, int*,
                                        hipStream_t);
template void launch_same_inputs<double>(int64_t, const double*, const double*, const int32_t*, const int32_t*,
                                         int*, hipStream_t);

}  // namespace nnp
