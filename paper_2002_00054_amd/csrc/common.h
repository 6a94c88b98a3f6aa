// Shared definitions of the gfx950 kernels and the host layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnp {

// ------------------------------------------------------------------ limits
constexpr int MAX_EL = 4;                            // elements
constexpr int MAX_CLS = MAX_EL * (MAX_EL + 1) / 2;   // unordered neighbour-element pairs
constexpr int MAX_SF = 32;                           // SFs per centre element (network inputs)
constexpr int MAX_RAD = 16;                          // radial SFs per (centre, neighbour element)
constexpr int MAX_ANG = 8;                           // angular SFs per (centre, neighbour pair)
constexpr int MAX_NE = 4;                            // distinct angular eta per centre element
constexpr int HID = 32;                              // padded hidden width and input width
constexpr int LD = 32;                               // row stride of G, dE/dG and JVP rows
constexpr int FC_DEG_MAX = 16;                       // storage bound of the cutoff polynomial
constexpr int WAVE = 64;
constexpr int QCAP = 128;                            // per-wave triplet queue (stack of pairs)

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16 = 2 };

// Arithmetic types of each form.
//  T     symmetry-function and geometry arithmetic
//  Acc   per-atom SF neighbour sums
//  FAcc  force accumulation
//  IO    positions, per-atom energies and forces at the boundary; G~ and dE/dG rows
// Four-vector of the arithmetic type.  Neighbour-list entries use it as
// (dx, dy, dz, j): the minimum-image displacement r_j - r_i rounded once from
// FP64 to T, and the neighbour's sorted index in the bits of w.
template <class T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
__host__ __device__ inline int entry_index(const float4& e) { return __float_as_int(e.w); }
__host__ __device__ inline int entry_index(const double4& e) { return (int)__double_as_longlong(e.w); }
__device__ inline float4 make_entry(double dx, double dy, double dz, int j, float) {
  return make_float4((float)dx, (float)dy, (float)dz, __int_as_float(j));
}
__device__ inline double4 make_entry(double dx, double dy, double dz, int j, double) {
  return make_double4(dx, dy, dz, __longlong_as_double((long long)j));
}
// Entries of type E: displacement + index (float4, double4) or the index alone (int).
__host__ __device__ inline int entry_index(int e) { return e; }
template <class E> __device__ inline E make_entry_as(double dx, double dy, double dz, int j);
template <> __device__ inline float4 make_entry_as<float4>(double dx, double dy, double dz, int j) {
  return make_entry(dx, dy, dz, j, 0.f);
}
template <> __device__ inline double4 make_entry_as<double4>(double dx, double dy, double dz, int j) {
  return make_entry(dx, dy, dz, j, 0.0);
}
template <> __device__ inline int make_entry_as<int>(double, double, double, int j) { return j; }

template <int P> struct Types;
template <> struct Types<P_FP64> { using T = double; using Acc = double; using FAcc = double; using IO = double; };
template <> struct Types<P_FP32> { using T = float;  using Acc = float;  using FAcc = float;  using IO = float; };
template <> struct Types<P_BF16> { using T = float;  using Acc = double; using FAcc = double; using IO = float; };

// -------------------------------------------------------------- SF table
// Device copy of the symmetry-function table, in the arithmetic type T.
// Every field is read with wave-uniform (scalar) loads.
template <class T>
struct DevTab {
  int n_el;
  int n_sf[MAX_EL];
  T rc2;                               // rc^2
  T inv_rc2;                           // 1 / rc^2
  // radial SFs, per (centre e, neighbour element f)
  int rad_cnt[MAX_EL][MAX_EL];
  T rad_eta[MAX_EL][MAX_EL][MAX_RAD];
  T rad_rs[MAX_EL][MAX_EL][MAX_RAD];
  int rad_out[MAX_EL][MAX_EL][MAX_RAD];
  // distinct angular exponents per centre element
  int n_eta[MAX_EL];
  T aeta[MAX_EL][MAX_NE];              // eta
  T aeta2[MAX_EL][MAX_NE];             // eta * log2(e)
  // angular SFs, per (centre e, neighbour-pair class c).  Each SF is the
  // product of a basis function (1 + lambda cos)^zeta, basis index
  // q = 6 [lambda < 0] + log2 zeta, with a radial factor of exponent index n;
  // ang_bit = q * MAX_NE + n.
  int ang_cnt[MAX_EL][MAX_CLS];
  int ang_bit[MAX_EL][MAX_CLS][MAX_ANG];
  T ang_pre[MAX_EL][MAX_CLS][MAX_ANG];     // 2^(1 - zeta)
  int ang_out[MAX_EL][MAX_CLS][MAX_ANG];
  int ang_wide[MAX_EL][MAX_CLS][MAX_ANG];  // 1: wide function (no r_jk factor or cutoff)
  // the same as a map from (q, n) to the one SF of the class using it (-1: none)
  int qn_out[MAX_EL][MAX_CLS][12 * MAX_NE];
  T qn_pre[MAX_EL][MAX_CLS][12 * MAX_NE];
  // centring / scaling of the network inputs (applied in FP64 to the sums)
  double shift_d[MAX_EL][MAX_SF];
  double inv_scale_d[MAX_EL][MAX_SF];
};

// Per-structure geometry of a batch.
struct DevStruct {
  double L[3];
  double invL[3];
  int ncell[3];
  int cellbase;     // first cell id of this structure in the batch-wide cell numbering
  int64_t off;      // first atom (caller order)
  int64_t n;        // atoms
};

// Network parameters of one element, zero-padded to HID x HID (T = math type).
// Layout: W1[HID][HID] (out, in), b1[HID], W2[HID][HID], b2[HID], w3[HID], b3 (+ pad).
constexpr int NET_STRIDE = 2 * HID * HID + 4 * HID;
constexpr int OFF_W1 = 0, OFF_B1 = HID * HID, OFF_W2 = HID * HID + HID, OFF_B2 = 2 * HID * HID + HID,
              OFF_W3 = 2 * HID * HID + 2 * HID, OFF_B3 = 2 * HID * HID + 3 * HID;

// Packed element / structure id stored in the 4th lane of the sorted positions.
__host__ __device__ inline long long pack_ids(int elem, int strct) { return (long long)elem | ((long long)strct << 8); }
__device__ inline int elem_of(double w) { return (int)(__double_as_longlong(w) & 0xff); }
__device__ inline int struct_of(double w) { return (int)(__double_as_longlong(w) >> 8); }

// Neighbour-pair class index of elements e1 <= e2 among n_el elements.
__host__ __device__ inline int class_index(int e1, int e2, int n_el) { return e1 * n_el - e1 * (e1 - 1) / 2 + (e2 - e1); }

// ----------------------------------------------------------- wave helpers
// Sum over the 64 lanes, returned in every lane: an inclusive scan inside
// each 16-lane row with DPP row shifts (1, 2, 4, 8; lanes shifted in from
// outside the row read 0), then the four row totals (lanes 15, 31, 47, 63)
// read out and added in a fixed order.
template <int CTRL>
__device__ inline float dpp_shift(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ inline double dpp_shift(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline float lane_value(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <class T>
__device__ inline T wave_sum(T v) {
  v += dpp_shift<0x111>(v);  // row_shr:1
  v += dpp_shift<0x112>(v);  // row_shr:2
  v += dpp_shift<0x114>(v);  // row_shr:4
  v += dpp_shift<0x118>(v);  // row_shr:8
  return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

__device__ inline int lane_id() { return __lane_id(); }

// Sums K per-lane values over the wave, 8 at a time, and stores total v in
// out[v] (from one lane each).  Three exchange-and-add halvings (lane ^ 32,
// lane ^ 16, lane ^ 8) leave each lane one of the 8 values summed over 8
// lanes; three row shifts finish the sum within each aligned group of 8.
template <class T>
__device__ inline T shfl_xor_t(T v, int m) { return __shfl_xor(v, m); }
// Eight per-lane values summed over the wave: the total of value
// (lane & 32 ? 4 : 0) + (lane & 16 ? 2 : 0) + (lane & 8 ? 1 : 0) is returned
// in the lanes with (lane & 7) == 7.
template <class Acc>
__device__ inline Acc wave_sum8(const Acc (&v)[8], int lane) {
  const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
  Acc a[4], b[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) a[i] = (h32 ? v[i + 4] : v[i]) + shfl_xor_t(h32 ? v[i] : v[i + 4], 32);
#pragma unroll
  for (int i = 0; i < 2; ++i) b[i] = (h16 ? a[i + 2] : a[i]) + shfl_xor_t(h16 ? a[i] : a[i + 2], 16);
  Acc c = (h8 ? b[1] : b[0]) + dpp_shift<0x128>(h8 ? b[0] : b[1]);  // row_ror:8 = lane ^ 8
  c += dpp_shift<0x111>(c);                                          // row_shr:1
  c += dpp_shift<0x112>(c);                                          // row_shr:2
  c += dpp_shift<0x114>(c);                                          // row_shr:4
  return c;
}
__device__ inline int wave_sum8_index(int lane) { return ((lane >> 3) & 4) | ((lane >> 3) & 2) | ((lane >> 3) & 1); }

template <class Acc, int K>
__device__ inline void wave_sum_many(const Acc (&x)[K], Acc* out, int lane) {
  const int vi = wave_sum8_index(lane);
#pragma unroll
  for (int g0 = 0; g0 < K; g0 += 8) {
    Acc v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = g0 + i < K ? x[g0 + i] : Acc(0);
    const Acc c = wave_sum8(v, lane);
    if ((lane & 7) == 7 && g0 + vi < K) out[g0 + vi] = c;
  }
}


__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Workgroup index remapped so that each XCD (workgroups are dealt round-robin
// to the 8 XCDs) works on one contiguous range of centres, i.e. one spatial
// region whose neighbour positions stay in that XCD's L2.
__device__ inline int64_t xcd_remap(int64_t b, int64_t nb) {
  const int64_t per = (nb + 7) / 8;
  const int64_t x = b & 7, r = b >> 3;
  const int64_t full = nb - (per - 1) * 8;  // XCDs that get `per` blocks (others per-1)
  const int64_t start = x < full ? x * per : full * per + (x - full) * (per - 1);
  return start + r;
}

// Number of set bits of mask below this lane.
__device__ inline int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// exp(x) in the arithmetic type: FP64 through the device math library, FP32
// through the hardware base-2 exponential of x log2(e) (the caller passes
// the argument already multiplied by log2(e)).
__device__ inline double exp_scaled(double x_ln, double /*x_log2*/) { return exp(x_ln); }
__device__ inline float exp_scaled(float /*x_ln*/, float x_log2) { return __builtin_amdgcn_exp2f(x_log2); }

// floor(a / b) for 0 <= a < 2^21 and b >= 1, given inv = rcp(b) (v_rcp_f32,
// within 1 ulp): (a + 1/2) / b lies at least 1 / (2b) from an integer, and
// the float error of (a + 1/2) * inv stays below (a + 1/2) 2^-22 / b, so the
// truncation is exact.  A few VALU instructions instead of the integer
// division sequence (about 15).
__device__ inline unsigned small_div(unsigned a, float inv) { return (unsigned)(((float)a + 0.5f) * inv); }
__device__ inline unsigned small_mod(unsigned a, unsigned b, float inv) { return a - b * small_div(a, inv); }

__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline double rsqrt_t(double s) { return 1.0 / sqrt(s); }
__device__ inline float rsqrt_t(float s) { return __builtin_amdgcn_rsqf(s); }

// Cutoff polynomial in t = r^2/rc^2 per arithmetic type: interpolants of
// fc = (1 + cos(pi sqrt(t)))/2 at the Chebyshev points, in the monomial basis
// (gen_cutoff.py).  FP64: degree 10, max error 1.4e-15 (fc) and 1.7e-13
// (dfc/dt).  FP32: degree 6, max error 5.5e-9, below FP32 rounding.  Both are
// several terms shorter than the Taylor series of the same accuracy.
template <class T> struct FcPoly;
template <> struct FcPoly<double> {
  static constexpr int D = 10;
  static constexpr double a(int n) {
    constexpr double c[11] = {0.99999999999999867,    -2.4674011002721739,    2.0293560632041152,
                              -0.66763138438064717,   0.11766531490754019,    -0.012903444753172158,
                              0.00096478511035206918, -5.2316220181516193e-05, 2.1490610761661228e-06,
                              -6.8101185620021584e-08, 1.44427758641541e-09};
    return c[n];
  }
};
template <> struct FcPoly<float> {
  static constexpr int D = 6;
  static constexpr double a(int n) {
    constexpr double c[7] = {0.99999999447228860, -2.4674005583220304, 2.0293473727609408, -0.66757901115278839,
                             0.11751451131309654, -0.012679142877827992, 0.00079683910699860207};
    return c[n];
  }
};

// Cosine cutoff as a polynomial in s = r^2 with compile-time coefficients
// (no square root or cosine per evaluation); exactly 0 for s >= rc^2 unless
// the caller already knows s < rc^2 (the *_in variants).
template <class T>
struct Cutoff {
  static constexpr int D = FcPoly<T>::D;
  T rc2, inv_rc2;
  __device__ inline void load(const DevTab<T>* tab) {
    rc2 = tab->rc2;
    inv_rc2 = tab->inv_rc2;
  }
  // fc and dfc/ds at s = r^2, for s < rc^2.
  __device__ inline void eval_in(T s, T& fc, T& dfc_ds) const {
    const T t = s * inv_rc2;
    T f = T(FcPoly<T>::a(D)), g = T(D * FcPoly<T>::a(D));
#pragma unroll
    for (int n = D - 1; n >= 1; --n) {
      f = f * t + T(FcPoly<T>::a(n));
      g = g * t + T(n * FcPoly<T>::a(n));
    }
    fc = f * t + T(FcPoly<T>::a(0));
    dfc_ds = g * inv_rc2;
  }
  __device__ inline void eval(T s, T& fc, T& dfc_ds) const {
    eval_in(s, fc, dfc_ds);
    const bool in = s < rc2;
    fc = in ? fc : T(0);
    dfc_ds = in ? dfc_ds : T(0);
  }
  __device__ inline T value_in(T s) const {
    const T t = s * inv_rc2;
    T f = T(FcPoly<T>::a(D));
#pragma unroll
    for (int n = D - 1; n >= 0; --n) f = f * t + T(FcPoly<T>::a(n));
    return f;
  }
  __device__ inline T value(T s) const { return s < rc2 ? value_in(s) : T(0); }
};

// ------------------------------------------------------- angular basis
// Basis functions B_q(cos) = (1 + lambda cos)^zeta for lambda = +1 (q = k) and
// lambda = -1 (q = 6 + k), zeta = 2^k, k = 0..5.  A table's use of (q, n)
// pairs (basis function times radial factor of eta index n) is a bit mask;
// kernels are instantiated for a mask, so unused pairs cost nothing.
constexpr int NQ = 12;
__host__ __device__ constexpr int q_lambda(int q) { return q < 6 ? 1 : -1; }
__host__ __device__ constexpr int q_k(int q) { return q % 6; }
__host__ __device__ constexpr int q_zeta(int q) { return 1 << (q % 6); }
__host__ __device__ constexpr uint64_t qn_bit(int q, int n) { return 1ull << (q * MAX_NE + n); }
__host__ __device__ constexpr bool qn_used(uint64_t mask, int q, int n) { return (mask >> (q * MAX_NE + n)) & 1ull; }
__host__ __device__ constexpr int qn_count(uint64_t mask) { return mask ? (int)(mask & 1ull) + qn_count(mask >> 1) : 0; }
__host__ __device__ constexpr bool q_used(uint64_t mask, int q) {
  return ((mask >> (q * MAX_NE)) & ((1ull << MAX_NE) - 1)) != 0;
}
// Largest k used for the basis functions of sign s (0: lambda = +1, 1: -1), -1 if none.
__host__ __device__ constexpr int k_max(uint64_t mask, int s) {
  int m = -1;
  for (int k = 0; k < 6; ++k)
    if (q_used(mask, 6 * s + k)) m = k;
  return m;
}
// The angular structure of the water table: (lambda, zeta, eta index) =
// (+1,1,0), (-1,1,0), (+1,4,0), (-1,4,0), (+1,2,1), (+1,16,1).
constexpr uint64_t QN_WATER = qn_bit(0, 0) | qn_bit(6, 0) | qn_bit(2, 0) | qn_bit(8, 0) | qn_bit(1, 1) | qn_bit(4, 1);
constexpr uint64_t QN_ALL2 = 0x333333333333ull;  // every q with n < 2
constexpr uint64_t QN_ALL4 = 0xffffffffffffull;  // every q with n < 4

// x^n for a wave-uniform integer n >= 0 (binary powering; 0^0 = 1).
template <class T>
__device__ inline T ipow(T x, int n) {
  T r = T(1);
  while (n) {
    if (n & 1) r *= x;
    x *= x;
    n >>= 1;
  }
  return r;
}

// Atomic add without return value (hardware float/double atomics).
__device__ inline void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

}  // namespace nnp
