// Flat parallelism: one thread per centre atom, the paper's "flat" level
// (threads over atoms only, Sec. 4.3), kept to compare the levels of
// parallelism, and the path of tables with wide angular functions G9 (the
// narrow function without its r_jk factor and cutoff: every pair counts).  Every lane is a centre and walks its own neighbours and
// pairs; a wave per centre (k_triplet) was measured faster on both workloads,
// short neighbour rows included, because here each lane reads its own row
// (64 rows per load instruction) and the pair loop diverges.
//
// SF pass: radial terms over the neighbours, angular terms over the unordered
// pairs (j < k) with r_jk < rc, each SF sum in a thread-private LDS column.
// Force pass: the gradient of sum_s c_s G_s with respect to r_j is built in
// registers by walking, for every neighbour j, every other neighbour k (each
// triplet is visited once from j and once from k, each time for one of its two
// neighbour gradients), then flushed with one atomic per component; the
// centre gets minus the sum over j (G_i depends on positions only through
// r_j - r_i).  The formulas are those of the wave kernels (same cutoff
// polynomial, same angular factorisation):
//   T = pre (1 + lam cos)^zeta e^{-eta (a^2 + b^2 + d^2)} fc(a) fc(b) fc(d),
//   dT/dr_j = dT/dcos (r_ik/(a b) - cos r_ij/a^2) + 2 dT/d(a^2) r_ij - 2 dT/d(d^2) (r_k - r_j).
#include <type_traits>

#include "kernels.h"

namespace nnp {
namespace {

constexpr int FLAT = 64;  // threads (centres) per workgroup: one wave

// Per-class angular parameters of a centre element, in registers.
template <class T>
struct AngClass {
  int na;
  bool any_narrow, any_wide;
  bool wide[MAX_ANG];  // wide function: no r_jk factor or cutoff
  int out[MAX_ANG];
  int ni[MAX_ANG];   // index of the SF's exponent among the centre's distinct ones
  int zl[MAX_ANG];   // log2 zeta
  T pre[MAX_ANG], lam[MAX_ANG], zeta[MAX_ANG], eta[MAX_ANG];
  __device__ inline void load(const DevTab<T>* tab, int ec, int cls) {
    na = tab->ang_cnt[ec][cls];
    any_narrow = any_wide = false;
#pragma unroll
    for (int q = 0; q < MAX_ANG; ++q) {
      wide[q] = q < na && tab->ang_wide[ec][cls][q] != 0;
      any_wide |= wide[q];
      any_narrow |= q < na && !wide[q];
      const int bit = q < na ? tab->ang_bit[ec][cls][q] : 0;
      const int qb = bit / MAX_NE;
      ni[q] = bit % MAX_NE;
      zl[q] = qb % 6;
      lam[q] = qb < 6 ? T(1) : T(-1);
      zeta[q] = T(1 << zl[q]);
      eta[q] = tab->aeta[ec][ni[q]];
      pre[q] = q < na ? tab->ang_pre[ec][cls][q] : T(0);
      out[q] = q < na ? tab->ang_out[ec][cls][q] : 0;
    }
  }
};

template <class T>
__device__ inline T pick(const T (&v)[MAX_NE], int i) {
  return i == 0 ? v[0] : i == 1 ? v[1] : i == 2 ? v[2] : v[3];
}

// (1 + lam c)^zeta and (1 + lam c)^(zeta - 1) for zeta = 2^zl.
template <class T>
__device__ inline void powers(T p, int zl, T& pz, T& pz1) {
  pz1 = T(1);
  pz = p;
  for (int i = 0; i < zl; ++i) {
    pz1 *= pz;
    pz *= pz;
  }
}

// Element blocks of a neighbour row: block f is [lo(f), lo(f + 1)).  Read by
// selection rather than indexing, so that nothing goes to scratch memory.
struct Rows {
  int o1, o2, o3, o4;
  __device__ inline void load(int4 nn, int n_el) {
    o1 = nn.x;
    o2 = o1 + (n_el > 1 ? nn.y : 0);
    o3 = o2 + (n_el > 2 ? nn.z : 0);
    o4 = o3 + (n_el > 3 ? nn.w : 0);
  }
  __device__ inline int lo(int f) const { return f == 0 ? 0 : f == 1 ? o1 : f == 2 ? o2 : f == 3 ? o3 : o4; }
};

template <int P>
__global__ void __launch_bounds__(FLAT) k_flat_sf(TripArgs<P> a) {
  using T = typename Types<P>::T;
  using Acc = typename Types<P>::Acc;
  using IO = typename Types<P>::IO;
  using V4 = typename Vec4<T>::type;
  __shared__ Acc gs[LD][FLAT];
  const int lane = threadIdx.x;
  const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * FLAT + lane;
  if (c >= a.n) return;  // no workgroup barrier below
  const DevTab<T>* __restrict__ tab = a.tab;
  Cutoff<T> cut;
  cut.load(tab);
  const T rc2 = tab->rc2;
  const int n_el = tab->n_el;
  const int ec = elem_of(a.pos4[c].w);
  const int ne = tab->n_eta[ec];
  Rows rw;
  rw.load(a.nnb[c], n_el);
  const V4* __restrict__ row = a.nbr + c * (int64_t)a.cap;
#pragma unroll
  for (int s = 0; s < LD; ++s) gs[s][lane] = Acc(0);
  T eta_n[MAX_NE];
#pragma unroll
  for (int n = 0; n < MAX_NE; ++n) eta_n[n] = n < ne ? tab->aeta[ec][n] : T(0);

  for (int f = 0; f < n_el; ++f) {
    const int nr = tab->rad_cnt[ec][f];
    for (int t = rw.lo(f); t < rw.lo(f + 1); ++t) {
      const V4 e = row[t];
      const T s = e.x * e.x + e.y * e.y + e.z * e.z;
      const T r = sqrt(s);
      T fc, dfc;
      cut.eval(s, fc, dfc);
      for (int q = 0; q < nr; ++q) {
        const T u = r - tab->rad_rs[ec][f][q];
        const T x = -tab->rad_eta[ec][f][q] * u * u;
        gs[tab->rad_out[ec][f][q]][lane] += (Acc)(exp_scaled(x, x * T(1.4426950408889634)) * fc);
      }
    }
  }
  for (int f = 0; f < n_el; ++f) {
    for (int g = f; g < n_el; ++g) {
      AngClass<T> cl;
      cl.load(tab, ec, class_index(f, g, n_el));
      if (cl.na == 0) continue;
      Acc gq[MAX_ANG];
#pragma unroll
      for (int q = 0; q < MAX_ANG; ++q) gq[q] = Acc(0);
      for (int j = rw.lo(f); j < rw.lo(f + 1); ++j) {
        const V4 A = row[j];
        const T a2 = A.x * A.x + A.y * A.y + A.z * A.z;
        const T ia = rsqrt_t(a2);
        const T fca = cut.value(a2);
        // the pair loop, compiled without the wide terms where a class has none
        auto pairs = [&](auto wide_tag) {
          constexpr bool W = decltype(wide_tag)::value;
          for (int k = (f == g ? j + 1 : rw.lo(g)); k < rw.lo(g + 1); ++k) {
            const V4 B = row[k];
            const T dx = B.x - A.x, dy = B.y - A.y, dz = B.z - A.z;
            const T d2 = dx * dx + dy * dy + dz * dz;
            const bool near = d2 < rc2;
            if (!(near || W)) continue;
            const T b2 = B.x * B.x + B.y * B.y + B.z * B.z;
            const T cs = (A.x * B.x + A.y * B.y + A.z * B.z) * ia * rsqrt_t(b2);
            const T f2 = fca * cut.value(b2);
            const T f3 = near ? f2 * cut.value_in(d2) : T(0);
            T ex[MAX_NE], exw[MAX_NE];  // e^{-eta (a^2 + b^2 + d^2)} (narrow), e^{-eta (a^2 + b^2)} (wide)
  #pragma unroll
            for (int n = 0; n < MAX_NE; ++n) {
              const T sn = a2 + b2 + d2, sw = a2 + b2;
              ex[n] = n < ne && near && cl.any_narrow ? exp_scaled(-eta_n[n] * sn, -eta_n[n] * sn * T(1.4426950408889634)) : T(0);
              exw[n] = W && n < ne ? exp_scaled(-eta_n[n] * sw, -eta_n[n] * sw * T(1.4426950408889634)) : T(0);
            }
  #pragma unroll
            for (int q = 0; q < MAX_ANG; ++q) {
              if (q < cl.na) {
                T pz, pz1;
                powers(T(1) + cl.lam[q] * cs, cl.zl[q], pz, pz1);
                gq[q] += (Acc)((W && cl.wide[q]) ? pz * pick(exw, cl.ni[q]) * f2 : pz * pick(ex, cl.ni[q]) * f3);
              }
            }
          }
        };
        if (cl.any_wide) pairs(std::true_type{});
        else pairs(std::false_type{});
      }
#pragma unroll
      for (int q = 0; q < MAX_ANG; ++q)
        if (q < cl.na) gs[cl.out[q]][lane] += (Acc)cl.pre[q] * gq[q];
    }
  }
  const int ns = tab->n_sf[ec];
#pragma unroll
  for (int s = 0; s < LD; ++s) {
    IO v = IO(0);
    if (s < ns) v = (IO)(((double)gs[s][lane] - tab->shift_d[ec][s]) * tab->inv_scale_d[ec][s]);
    a.G[c * LD + s] = v;
  }
}

template <int P>
__global__ void __launch_bounds__(FLAT) k_flat_force(TripArgs<P> a) {
  using T = typename Types<P>::T;
  using FAcc = typename Types<P>::FAcc;
  using V4 = typename Vec4<T>::type;
  __shared__ T cf[LD][FLAT];  // dE/dG of the centre (raw G)
  const int lane = threadIdx.x;
  const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * FLAT + lane;
  if (c >= a.n) return;  // no workgroup barrier below
  const DevTab<T>* __restrict__ tab = a.tab;
  Cutoff<T> cut;
  cut.load(tab);
  const T rc2 = tab->rc2;
  const int n_el = tab->n_el;
  const int ec = elem_of(a.pos4[c].w);
  const int ne = tab->n_eta[ec];
  Rows rw;
  rw.load(a.nnb[c], n_el);
  const V4* __restrict__ row = a.nbr + c * (int64_t)a.cap;
#pragma unroll
  for (int s = 0; s < LD; ++s) cf[s][lane] = (T)a.C[c * LD + s];
  T eta_n[MAX_NE];
#pragma unroll
  for (int n = 0; n < MAX_NE; ++n) eta_n[n] = n < ne ? tab->aeta[ec][n] : T(0);
  T fix = T(0), fiy = T(0), fiz = T(0);

  for (int f = 0; f < n_el; ++f) {
    const int nr = tab->rad_cnt[ec][f];
    for (int j = rw.lo(f); j < rw.lo(f + 1); ++j) {
      const V4 A = row[j];
      const T a2 = A.x * A.x + A.y * A.y + A.z * A.z;
      const T ia = rsqrt_t(a2);
      const T ar = a2 * ia;
      T fca, dfca;
      cut.eval(a2, fca, dfca);  // dfca = dfc/d(a^2)
      // radial: sum_q c_q dt_q/da, t = e^{-eta (a - rs)^2} fc(a)
      T dUa = T(0);
      for (int q = 0; q < nr; ++q) {
        const T eta = tab->rad_eta[ec][f][q];
        const T u = ar - tab->rad_rs[ec][f][q];
        const T x = -eta * u * u;
        const T ex = exp_scaled(x, x * T(1.4426950408889634));
        dUa += cf[tab->rad_out[ec][f][q]][lane] * ex * (T(2) * ar * dfca - T(2) * eta * u * fca);
      }
      T gx = dUa * ia * A.x, gy = dUa * ia * A.y, gz = dUa * ia * A.z;
      const T inv_a2 = ia * ia;
      for (int g = 0; g < n_el; ++g) {
        AngClass<T> cl;
        const int cls = class_index(min(f, g), max(f, g), n_el);
        cl.load(tab, ec, cls);
        if (cl.na == 0) continue;
        T w[MAX_ANG];
#pragma unroll
        for (int q = 0; q < MAX_ANG; ++q) w[q] = q < cl.na ? cf[cl.out[q]][lane] * cl.pre[q] : T(0);
        // the pair loop, compiled without the wide terms where a class has none
        auto pairs = [&](auto wide_tag) {
          constexpr bool W = decltype(wide_tag)::value;
          for (int k = rw.lo(g); k < rw.lo(g + 1); ++k) {
            const V4 B = row[k];
            const T dx = B.x - A.x, dy = B.y - A.y, dz = B.z - A.z;
            const T d2 = dx * dx + dy * dy + dz * dz;
            const bool near = d2 < rc2;
            if (!(k != j && (near || W))) continue;
            const T b2 = B.x * B.x + B.y * B.y + B.z * B.z;
            const T ib = rsqrt_t(b2);
            const T iab = ia * ib;
            const T cs = (A.x * B.x + A.y * B.y + A.z * B.z) * iab;
            const T fcb = cut.value(b2);
            T fcd = T(0), dfcd = T(0);
            if (near) cut.eval_in(d2, fcd, dfcd);
            T ex[MAX_NE], exw[MAX_NE];  // e^{-eta (a^2 + b^2 + d^2)} (narrow), e^{-eta (a^2 + b^2)} (wide)
  #pragma unroll
            for (int n = 0; n < MAX_NE; ++n) {
              const T sn = a2 + b2 + d2, sw = a2 + b2;
              ex[n] = n < ne && near && cl.any_narrow ? exp_scaled(-eta_n[n] * sn, -eta_n[n] * sn * T(1.4426950408889634)) : T(0);
              exw[n] = W && n < ne ? exp_scaled(-eta_n[n] * sw, -eta_n[n] * sw * T(1.4426950408889634)) : T(0);
            }
            // narrow (n) and wide (w) sums: Uc = sum_q w zeta lam pz1 E, Uz = sum_q w pz E, Ue = sum_q w eta pz E
            T Ucn = T(0), Uzn = T(0), Uen = T(0), Ucw = T(0), Uzw = T(0), Uew = T(0);
  #pragma unroll
            for (int q = 0; q < MAX_ANG; ++q) {
              if (q < cl.na) {
                T pz, pz1;
                powers(T(1) + cl.lam[q] * cs, cl.zl[q], pz, pz1);
                const T we = w[q] * ((W && cl.wide[q]) ? pick(exw, cl.ni[q]) : pick(ex, cl.ni[q]));
                const T c1 = we * cl.zeta[q] * cl.lam[q] * pz1, c2 = we * pz, c3 = we * cl.eta[q] * pz;
                if ((W && cl.wide[q])) {
                  Ucw += c1;
                  Uzw += c2;
                  Uew += c3;
                } else {
                  Ucn += c1;
                  Uzn += c2;
                  Uen += c3;
                }
              }
            }
            const T f2 = fca * fcb;
            const T f3 = f2 * fcd;
            const T tc = Ucn * f3 + Ucw * f2;                                                     // dT/dcos
            const T ta = T(2) * (Uzn * dfca * fcb * fcd - Uen * f3 + Uzw * dfca * fcb - Uew * f2);  // 2 dT/d(a^2)
            const T td = T(2) * (Uzn * fca * fcb * dfcd - Uen * f3);                               // 2 dT/d(d^2)
            const T ca = cs * inv_a2;
            gx += tc * (B.x * iab - ca * A.x) + ta * A.x - td * dx;
            gy += tc * (B.y * iab - ca * A.y) + ta * A.y - td * dy;
            gz += tc * (B.z * iab - ca * A.z) + ta * A.z - td * dz;
          }
        };
        if (cl.any_wide) pairs(std::true_type{});
        else pairs(std::false_type{});
      }
      const int64_t jj = entry_index(A);
      atomic_add(&a.F[jj], (FAcc)(-gx));
      atomic_add(&a.F[a.n + jj], (FAcc)(-gy));
      atomic_add(&a.F[2 * a.n + jj], (FAcc)(-gz));
      fix += gx;
      fiy += gy;
      fiz += gz;
    }
  }
  atomic_add(&a.F[c], (FAcc)fix);
  atomic_add(&a.F[a.n + c], (FAcc)fiy);
  atomic_add(&a.F[2 * a.n + c], (FAcc)fiz);
}

// Force-adjoint product of the differentiation form, one thread per centre:
// v_is = sum_m delta_m . dG_is/dr_m = sum_j (delta_j - delta_i) . dG_is/dr_j,
// with the same ordered-pair walk as the force pass (every visit adds the
// r_j gradient of each SF of the pair, projected on delta_j - delta_i).
template <int P>
__global__ void __launch_bounds__(FLAT) k_flat_jvp(TripArgs<P> a) {
  using T = typename Types<P>::T;
  using Acc = typename Types<P>::Acc;
  using IO = typename Types<P>::IO;
  using V4 = typename Vec4<T>::type;
  __shared__ Acc vs[LD][FLAT];
  const int lane = threadIdx.x;
  const int64_t c = xcd_remap(blockIdx.x, gridDim.x) * FLAT + lane;
  if (c >= a.n) return;  // no workgroup barrier below
  const DevTab<T>* __restrict__ tab = a.tab;
  Cutoff<T> cut;
  cut.load(tab);
  const T rc2 = tab->rc2;
  const int n_el = tab->n_el;
  const int ec = elem_of(a.pos4[c].w);
  const int ne = tab->n_eta[ec];
  Rows rw;
  rw.load(a.nnb[c], n_el);
  const V4* __restrict__ row = a.nbr + c * (int64_t)a.cap;
#pragma unroll
  for (int s = 0; s < LD; ++s) vs[s][lane] = Acc(0);
  const T di0 = (T)a.delta[3 * c + 0], di1 = (T)a.delta[3 * c + 1], di2 = (T)a.delta[3 * c + 2];
  T eta_n[MAX_NE];
#pragma unroll
  for (int n = 0; n < MAX_NE; ++n) eta_n[n] = n < ne ? tab->aeta[ec][n] : T(0);

  for (int f = 0; f < n_el; ++f) {
    const int nr = tab->rad_cnt[ec][f];
    for (int j = rw.lo(f); j < rw.lo(f + 1); ++j) {
      const V4 A = row[j];
      const int64_t jj = entry_index(A);
      const T d0 = (T)a.delta[3 * jj + 0] - di0, d1 = (T)a.delta[3 * jj + 1] - di1, d2j = (T)a.delta[3 * jj + 2] - di2;
      const T a2 = A.x * A.x + A.y * A.y + A.z * A.z;
      const T ia = rsqrt_t(a2);
      const T ar = a2 * ia;
      T fca, dfca;
      cut.eval(a2, fca, dfca);
      const T pa = A.x * d0 + A.y * d1 + A.z * d2j;  // r_ij . (delta_j - delta_i)
      for (int q = 0; q < nr; ++q) {
        const T eta = tab->rad_eta[ec][f][q];
        const T u = ar - tab->rad_rs[ec][f][q];
        const T x = -eta * u * u;
        const T ex = exp_scaled(x, x * T(1.4426950408889634));
        const T dt = ex * (T(2) * ar * dfca - T(2) * eta * u * fca);  // dt/da
        vs[tab->rad_out[ec][f][q]][lane] += (Acc)(dt * ia * pa);
      }
      const T inv_a2 = ia * ia;
      for (int g = 0; g < n_el; ++g) {
        AngClass<T> cl;
        cl.load(tab, ec, class_index(min(f, g), max(f, g), n_el));
        if (cl.na == 0) continue;
        Acc vq[MAX_ANG];
#pragma unroll
        for (int q = 0; q < MAX_ANG; ++q) vq[q] = Acc(0);
        // the pair loop, compiled without the wide terms where a class has none
        auto pairs = [&](auto wide_tag) {
          constexpr bool W = decltype(wide_tag)::value;
          for (int k = rw.lo(g); k < rw.lo(g + 1); ++k) {
            const V4 B = row[k];
            const T dx = B.x - A.x, dy = B.y - A.y, dz = B.z - A.z;
            const T d2 = dx * dx + dy * dy + dz * dz;
            const bool near = d2 < rc2;
            if (!(k != j && (near || W))) continue;
            const T b2 = B.x * B.x + B.y * B.y + B.z * B.z;
            const T ib = rsqrt_t(b2);
            const T iab = ia * ib;
            const T cs = (A.x * B.x + A.y * B.y + A.z * B.z) * iab;
            const T fcb = cut.value(b2);
            T fcd = T(0), dfcd = T(0);
            if (near) cut.eval_in(d2, fcd, dfcd);
            T ex[MAX_NE], exw[MAX_NE];
  #pragma unroll
            for (int n = 0; n < MAX_NE; ++n) {
              const T sn = a2 + b2 + d2, sw = a2 + b2;
              ex[n] = n < ne && near && cl.any_narrow ? exp_scaled(-eta_n[n] * sn, -eta_n[n] * sn * T(1.4426950408889634)) : T(0);
              exw[n] = W && n < ne ? exp_scaled(-eta_n[n] * sw, -eta_n[n] * sw * T(1.4426950408889634)) : T(0);
            }
            // projections of dcos/dr_j, r_ij and r_k - r_j on delta_j - delta_i
            const T ca = cs * inv_a2;
            const T pc = (B.x * d0 + B.y * d1 + B.z * d2j) * iab - ca * pa;
            const T pd = dx * d0 + dy * d1 + dz * d2j;
            const T f2 = fca * fcb;
            const T f3 = f2 * fcd;
  #pragma unroll
            for (int q = 0; q < MAX_ANG; ++q) {
              if (q < cl.na) {
                T pz, pz1;
                powers(T(1) + cl.lam[q] * cs, cl.zl[q], pz, pz1);
                T tc, ta, td;
                if ((W && cl.wide[q])) {
                  const T e = pick(exw, cl.ni[q]);
                  tc = e * cl.zeta[q] * cl.lam[q] * pz1 * f2;
                  ta = T(2) * e * pz * (dfca * fcb - cl.eta[q] * f2);
                  td = T(0);
                } else {
                  const T e = pick(ex, cl.ni[q]);
                  tc = e * cl.zeta[q] * cl.lam[q] * pz1 * f3;
                  ta = T(2) * e * pz * (dfca * fcb * fcd - cl.eta[q] * f3);
                  td = T(2) * e * pz * (fca * fcb * dfcd - cl.eta[q] * f3);
                }
                vq[q] += (Acc)(tc * pc + ta * pa - td * pd);
              }
            }
          }
        };
        if (cl.any_wide) pairs(std::true_type{});
        else pairs(std::false_type{});
#pragma unroll
        for (int q = 0; q < MAX_ANG; ++q)
          if (q < cl.na) vs[cl.out[q]][lane] += (Acc)cl.pre[q] * vq[q];
      }
    }
  }
  const int ns = tab->n_sf[ec];
#pragma unroll
  for (int s = 0; s < LD; ++s) a.V[c * LD + s] = s < ns ? (IO)vs[s][lane] : IO(0);
}

}  // namespace

template <int P>
void launch_flat(int mode, const TripArgs<P>& a, hipStream_t stream) {
  if (a.n == 0) return;
  const unsigned nb = (unsigned)((a.n + FLAT - 1) / FLAT);
  if (mode == 0) hipLaunchKernelGGL(k_flat_sf<P>, dim3(nb), dim3(FLAT), 0, stream, a);
  else if (mode == 1) hipLaunchKernelGGL(k_flat_force<P>, dim3(nb), dim3(FLAT), 0, stream, a);
  else hipLaunchKernelGGL(k_flat_jvp<P>, dim3(nb), dim3(FLAT), 0, stream, a);
}

template void launch_flat<P_FP64>(int, const TripArgs<P_FP64>&, hipStream_t);
template void launch_flat<P_FP32>(int, const TripArgs<P_FP32>&, hipStream_t);
template void launch_flat<P_BF16>(int, const TripArgs<P_BF16>&, hipStream_t);

}  // namespace nnp
