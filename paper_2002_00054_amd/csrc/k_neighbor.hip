// Wrap + cell binning + counting sort, and the cell-list neighbour build.
//
// The neighbour list is the "random access (neighbor list)" structure the
// paper's kernels loop over (Sec. 4.3); the paper does not say how it is
// built.  Here: atoms are wrapped into the box in FP64, binned into cells of
// edge >= rc, and counting-sorted by (element, structure, cell); each atom's
// full neighbour list (every j != i with |r_ij| < rc under the minimum image)
// is then read from the deduplicated 3x3x3 block of cells around it, grouped
// by neighbour element (all element-0 neighbours first, then element 1, ...).
#include "common.h"
#include "kernels.h"

namespace nnp {

// Structure of atom i (caller order) by binary search of the offsets.
__device__ inline int find_struct(const int64_t* __restrict__ soff, int n_struct, int64_t i) {
  int lo = 0, hi = n_struct - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (soff[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Coordinate wrapped into [0, L); non-finite input maps to 0.
__device__ inline double wrap_coord(double x, double L, double invL) {
  double w = x - L * floor(x * invL);
  if (!(w >= 0.0 && w < L)) w = 0.0;
  return w;
}

__device__ inline int cell_coord(double w, double invL, int n) {
  int k = (int)(w * invL * (double)n);
  return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

template <class TIn>
__global__ void __launch_bounds__(256) k_bin(int64_t n, const TIn* __restrict__ pos, const int32_t* __restrict__ types,
                                             const DevStruct* __restrict__ st, const int64_t* __restrict__ soff,
                                             int n_struct, int n_el, int total_cells, int* __restrict__ key,
                                             int* __restrict__ count, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = find_struct(soff, n_struct, i);
  const DevStruct& S = st[b];
  int e = types[i];
  if (e < 0 || e >= n_el) {
    atomicOr(&flags[0], 1);
    e = 0;  // keep every index in range; the call reports the error
  }
  int c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double w = wrap_coord((double)pos[3 * i + a], S.L[a], S.invL[a]);
    c[a] = cell_coord(w, S.invL[a], S.ncell[a]);
  }
  const int k = e * total_cells + S.cellbase + (c[0] * S.ncell[1] + c[1]) * S.ncell[2] + c[2];
  key[i] = k;
  atomicAdd(&count[k], 1);
}

// Exclusive scan of count[0, n) into start[0, n] (start[n] = total) and
// cursor; one workgroup of 1024 threads, each owning a contiguous chunk.
__global__ void __launch_bounds__(1024) k_scan(int n, const int* __restrict__ count, int* __restrict__ start,
                                               int* __restrict__ cursor) {
  __shared__ int sums[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int b = min(t * chunk, n), e = min(b + chunk, n);
  int s = 0;
  for (int i = b; i < e; ++i) s += count[i];
  sums[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int v = t >= o ? sums[t - o] : 0;
    __syncthreads();
    sums[t] += v;
    __syncthreads();
  }
  int run = t ? sums[t - 1] : 0;
  for (int i = b; i < e; ++i) {
    start[i] = run;
    cursor[i] = run;
    run += count[i];
  }
  if (t == 1023) start[n] = sums[1023];
}

__global__ void __launch_bounds__(256) k_scatter(int64_t n, const int* __restrict__ key, int* __restrict__ cursor,
                                                 int* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = atomicAdd(&cursor[key[i]], 1);
  perm[s] = (int)i;
}

// Within every bin, order atoms by caller index (the scatter's atomics leave
// the order arbitrary; this makes the whole path deterministic up to the
// force atomics).
__global__ void __launch_bounds__(256) k_sort_bins(int nkeys, const int* __restrict__ start, int* __restrict__ perm) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  const int b = start[k], e = start[k + 1];
  for (int i = b + 1; i < e; ++i) {
    const int v = perm[i];
    int j = i - 1;
    while (j >= b && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

// Sorted FP64 positions (wrapped) with the packed element / structure id.
template <class TIn>
__global__ void __launch_bounds__(256) k_fill_sorted(int64_t n, const TIn* __restrict__ pos, const int32_t* __restrict__ types,
                                                     const DevStruct* __restrict__ st, const int64_t* __restrict__ soff,
                                                     int n_struct, int n_el, const int* __restrict__ perm,
                                                     double4* __restrict__ pos4) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t i = perm[s];
  const int b = find_struct(soff, n_struct, i);
  const DevStruct& S = st[b];
  int e = types[i];
  if (e < 0 || e >= n_el) e = 0;
  double4 p;
  p.x = wrap_coord((double)pos[3 * i + 0], S.L[0], S.invL[0]);
  p.y = wrap_coord((double)pos[3 * i + 1], S.L[1], S.invL[1]);
  p.z = wrap_coord((double)pos[3 * i + 2], S.L[2], S.invL[2]);
  p.w = __longlong_as_double(pack_ids(e, b));
  pos4[s] = p;
}

// Element offsets of the sorted order: eoff[f] = first sorted atom of element f.
__global__ void k_element_offsets(int n_el, int total_cells, const int* __restrict__ start, int* __restrict__ eoff) {
  const int f = threadIdx.x;
  if (f <= n_el) eoff[f] = start[f * total_cells];
}

// Neighbours of sorted atom s within rc (see k_neighbors); returns the count.
__device__ int neighbors_of(int64_t s, const double4* __restrict__ pos4, const DevStruct* __restrict__ st,
                            const int* __restrict__ start, int n_el, int total_cells, double rc2, int cap,
                            int* __restrict__ nbr, int4* __restrict__ nnb, int* __restrict__ flags) {
  const double4 p = pos4[s];
  const int b = struct_of(p.w);
  const DevStruct& S = st[b];
  const double L0 = S.L[0], L1 = S.L[1], L2 = S.L[2];
  const double i0 = S.invL[0], i1 = S.invL[1], i2 = S.invL[2];
  const int n0 = S.ncell[0], n1 = S.ncell[1], n2 = S.ncell[2];
  const int c0 = cell_coord(p.x, i0, n0), c1 = cell_coord(p.y, i1, n1), c2 = cell_coord(p.z, i2, n2);
  // Deduplicated stencil: three cells per axis if the axis has >= 3 cells,
  // otherwise every cell of the axis once.
  int cx[3], cy[3], cz[3];
  const int mx = n0 >= 3 ? 3 : n0, my = n1 >= 3 ? 3 : n1, mz = n2 >= 3 ? 3 : n2;
  for (int o = 0; o < 3; ++o) {
    cx[o] = n0 >= 3 ? (c0 - 1 + o + n0) % n0 : o;
    cy[o] = n1 >= 3 ? (c1 - 1 + o + n1) % n1 : o;
    cz[o] = n2 >= 3 ? (c2 - 1 + o + n2) % n2 : o;
  }
  int* row = nbr + s * (int64_t)cap;
  int total = 0;
  int cnt[MAX_EL] = {0, 0, 0, 0};
  for (int f = 0; f < n_el; ++f) {
    const int kb = f * total_cells + S.cellbase;
    for (int ox = 0; ox < mx; ++ox)
      for (int oy = 0; oy < my; ++oy)
        for (int oz = 0; oz < mz; ++oz) {
          const int k = kb + (cx[ox] * n1 + cy[oy]) * n2 + cz[oz];
          const int tb = start[k], te = start[k + 1];
          for (int t = tb; t < te; ++t) {
            if (t == s) continue;
            const double4 q = pos4[t];
            double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
            dx -= L0 * rint(dx * i0);
            dy -= L1 * rint(dy * i1);
            dz -= L2 * rint(dz * i2);
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 < rc2) {
              if (total < cap) {
                row[total] = t;
                ++cnt[f];
              }
              ++total;
            }
          }
        }
  }
  nnb[s] = make_int4(cnt[0], cnt[1], cnt[2], cnt[3]);
  if (total > cap) atomicMax(&flags[1], total);
  return total;
}

// Full neighbour list of every sorted atom, one thread per atom.  Writes at
// most cap entries per row; the number found beyond cap is reported through
// flags[1] (maximum count) so the caller can grow cap and rebuild.  flags[2]
// receives the largest count of any atom (it sizes the pair kernels' LDS).
__global__ void __launch_bounds__(256) k_neighbors(int64_t n, const double4* __restrict__ pos4,
                                                   const DevStruct* __restrict__ st, const int* __restrict__ start,
                                                   int n_el, int total_cells, double rc2, int cap,
                                                   int* __restrict__ nbr, int4* __restrict__ nnb,
                                                   int* __restrict__ flags) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int total = 0;
  if (s < n) total = neighbors_of(s, pos4, st, start, n_el, total_cells, rc2, cap, nbr, nnb, flags);
  // block maximum of the counts, one atomic per block
  __shared__ int bmax[4];
  int w = total;
  for (int o = 32; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o));
  if ((threadIdx.x & 63) == 0) bmax[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int b = max(max(bmax[0], bmax[1]), max(bmax[2], bmax[3]));
    if (b > 0) atomicMax(&flags[2], b);
  }
}

// Work counts of one evaluation, one thread per centre:
//   counts[0] neighbour entries (each unordered pair twice),
//   counts[1] unordered neighbour pairs (j, k) of a centre in element-pair
//             classes that have angular SFs (candidate triplets),
//   counts[2] those with r_jk < rc (triplet terms),
//   counts[3] angular SF-term updates (triplet terms x angular SFs of the class),
//   counts[4] radial SF-term updates (neighbour entries x radial SFs of the
//             centre / neighbour element pair).
__global__ void __launch_bounds__(256) k_count_terms(int64_t n, const double4* __restrict__ pos4,
                                                     const DevStruct* __restrict__ st, const int* __restrict__ nbr,
                                                     const int4* __restrict__ nnb, int cap, int n_el, CountTab ct,
                                                     double rc2, unsigned long long* __restrict__ counts) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double4 p = pos4[s];
  const int e = elem_of(p.w);
  const DevStruct& S = st[struct_of(p.w)];
  const int4 c4 = nnb[s];
  const int cnt[MAX_EL] = {c4.x, c4.y, c4.z, c4.w};
  int off[MAX_EL + 1];
  off[0] = 0;
  for (int f = 0; f < MAX_EL; ++f) off[f + 1] = off[f] + (f < n_el ? cnt[f] : 0);
  const int* row = nbr + s * (int64_t)cap;
  unsigned long long cand = 0, pass = 0, aterms = 0, rterms = 0;
  for (int f = 0; f < n_el; ++f) rterms += (unsigned long long)cnt[f] * ct.rad[e][f];
  for (int e1 = 0; e1 < n_el; ++e1)
    for (int e2 = e1; e2 < n_el; ++e2) {
      const int na = ct.ang[e][class_index(e1, e2, n_el)];
      if (na == 0) continue;
      unsigned long long pc = 0;
      for (int a = off[e1]; a < off[e1] + cnt[e1]; ++a) {
        const double4 qa = pos4[row[a]];
        double ax = qa.x - p.x, ay = qa.y - p.y, az = qa.z - p.z;
        ax -= S.L[0] * rint(ax * S.invL[0]);
        ay -= S.L[1] * rint(ay * S.invL[1]);
        az -= S.L[2] * rint(az * S.invL[2]);
        const int b0 = e1 == e2 ? a + 1 : off[e2];
        for (int b = b0; b < off[e2] + cnt[e2]; ++b) {
          const double4 qb = pos4[row[b]];
          double bx = qb.x - p.x, by = qb.y - p.y, bz = qb.z - p.z;
          bx -= S.L[0] * rint(bx * S.invL[0]);
          by -= S.L[1] * rint(by * S.invL[1]);
          bz -= S.L[2] * rint(bz * S.invL[2]);
          const double wx = bx - ax, wy = by - ay, wz = bz - az;
          ++cand;
          if (wx * wx + wy * wy + wz * wz < rc2) ++pc;
        }
      }
      pass += pc;
      aterms += pc * (unsigned long long)na;
    }
  atomicAdd(&counts[0], (unsigned long long)off[n_el]);
  atomicAdd(&counts[1], cand);
  atomicAdd(&counts[2], pass);
  atomicAdd(&counts[3], aterms);
  atomicAdd(&counts[4], rterms);
}

// ------------------------------------------------------------ launchers
template <class TIn>
void launch_bin_sort(const BinArgs& a, const TIn* pos, hipStream_t stream) {
  const int64_t n = a.n;
  const int nkeys = a.n_el * a.total_cells;
  launch_fill_int(a.count, nkeys + 1, 0, stream);
  if (n > 0) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_bin<TIn>, dim3(g), dim3(256), 0, stream, n, pos, a.types, a.st, a.soff, a.n_struct,
                       a.n_el, a.total_cells, a.key, a.count, a.flags);
  }
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, nkeys, a.count, a.start, a.cursor);
  if (n > 0) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, stream, n, a.key, a.cursor, a.perm);
    hipLaunchKernelGGL(k_sort_bins, dim3((nkeys + 255) / 256), dim3(256), 0, stream, nkeys, a.start, a.perm);
    hipLaunchKernelGGL(k_fill_sorted<TIn>, dim3(g), dim3(256), 0, stream, n, pos, a.types, a.st, a.soff,
                       a.n_struct, a.n_el, a.perm, a.pos4);
  }
  hipLaunchKernelGGL(k_element_offsets, dim3(1), dim3(64), 0, stream, a.n_el, a.total_cells, a.start, a.eoff);
}

template void launch_bin_sort<float>(const BinArgs&, const float*, hipStream_t);
template void launch_bin_sort<double>(const BinArgs&, const double*, hipStream_t);

void launch_neighbors(const BinArgs& a, double rc, int cap, int* nbr, int4* nnb, hipStream_t stream) {
  if (a.n == 0) return;
  const unsigned g = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_neighbors, dim3(g), dim3(256), 0, stream, a.n, a.pos4, a.st, a.start, a.n_el,
                     a.total_cells, rc * rc, cap, nbr, nnb, a.flags);
}

void launch_count_terms(const BinArgs& a, const int* nbr, const int4* nnb, int cap, const CountTab& ct, double rc,
                        unsigned long long* counts, hipStream_t stream) {
  if (a.n == 0) return;
  const unsigned g = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_count_terms, dim3(g), dim3(256), 0, stream, a.n, a.pos4, a.st, nbr, nnb, cap, a.n_el, ct,
                     rc * rc, counts);
}

}  // namespace nnp
