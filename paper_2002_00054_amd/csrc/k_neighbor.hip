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
  bool finite = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double x = (double)pos[3 * i + a];
    finite = finite && isfinite(x);
    const double w = wrap_coord(x, S.L[a], S.invL[a]);
    c[a] = cell_coord(w, S.invL[a], S.ncell[a]);
  }
  if (!finite) atomicOr(&flags[0], 2);  // the call reports NNP_E_ARG
  const int k = e * total_cells + S.cellbase + (c[0] * S.ncell[1] + c[1]) * S.ncell[2] + c[2];
  key[i] = k;
  atomicAdd(&count[k], 1);
}

// Exclusive scan of count[0, n) into start[0, n] (start[n] = total) and
// cursor, in three passes: per-block sums of SCAN_PER keys, one block scanning
// those sums, then each block scanning its keys from its offset.
constexpr int SCAN_PER = 4096;  // keys per block (1024 threads x 4)

// Exclusive scan of v over a 1024-thread block; *total receives the sum.
__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int y = lane < 16 ? sh[lane] : 0;
    for (int o = 1; o < 16; o <<= 1) {
      const int z = __shfl_up(y, o);
      if (lane >= o) y += z;
    }
    if (lane < 16) sh[16 + lane] = y;
  }
  __syncthreads();
  *total = sh[31];
  const int r = (wv ? sh[15 + wv] : 0) + x - v;
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(1024) k_scan_sums(int n, const int* __restrict__ count, int* __restrict__ partial) {
  __shared__ int sh[32];
  const int base = blockIdx.x * SCAN_PER;
  int v = 0;
  for (int i = base + threadIdx.x; i < min(n, base + SCAN_PER); i += 1024) v += count[i];
  int total;
  (void)block_exclusive_scan(v, sh, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// partial[b] <- exclusive prefix of the block sums; start[n] <- total.
__global__ void __launch_bounds__(1024) k_scan_top(int nb, int n, int* __restrict__ partial, int* __restrict__ start) {
  __shared__ int sh[32];
  const int per = (nb + 1023) / 1024;
  const int b0 = min((int)threadIdx.x * per, nb), b1 = min(b0 + per, nb);
  int v = 0;
  for (int b = b0; b < b1; ++b) v += partial[b];
  int total;
  int run = block_exclusive_scan(v, sh, &total);
  for (int b = b0; b < b1; ++b) {
    const int c = partial[b];
    partial[b] = run;
    run += c;
  }
  if (threadIdx.x == 0) start[n] = total;
}

__global__ void __launch_bounds__(1024) k_scan_apply(int n, const int* __restrict__ count,
                                                     const int* __restrict__ partial, int* __restrict__ start,
                                                     int* __restrict__ cursor) {
  __shared__ int sh[32];
  const int i0 = blockIdx.x * SCAN_PER + 4 * threadIdx.x;
  int c[4];
  int v = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = i0 + k < n ? count[i0 + k] : 0;
    v += c[k];
  }
  int total;
  int run = partial[blockIdx.x] + block_exclusive_scan(v, sh, &total);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < n) {
      start[i0 + k] = run;
      cursor[i0 + k] = run;
    }
    run += c[k];
  }
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
// force atomics).  One thread per atom, out of place (raw -> perm): the atom
// the scatter put at slot s of its bin goes to the bin's start plus the
// number of atoms of the bin with a smaller index (indices are distinct), so
// every place lies in the bin and each is written once.
__global__ void __launch_bounds__(256) k_sort_bins(int64_t n, const int* __restrict__ key,
                                                   const int* __restrict__ start, const int* __restrict__ raw,
                                                   int* __restrict__ perm) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int v = raw[s];
  const int k = key[v];
  const int b = start[k], e = start[k + 1];
  int place = b;
  for (int j = b; j < e; ++j) place += raw[j] < v ? 1 : 0;
  perm[place] = v;
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

// Neighbour build, one workgroup per cell.  The candidates of the cell (all
// atoms of the deduplicated 3x3x3 block of cells around it, element by
// element) are staged in LDS in tiles; each wave then takes centres of the
// cell in turn, tests 64 candidates per step in FP64 under the minimum image
// and appends the passing ones to the centre's row with a ballot compaction,
// so rows are written coalesced and grouped by neighbour element.  An entry
// is (r_j - r_i rounded to T, j).  When every axis has >= 3 cells, the
// staged candidates are shifted by the periodic image of their cell so the
// displacement is a plain difference; otherwise the minimum image is taken
// per pair.  At most cap entries are written per row; the largest count
// beyond cap goes to flags[1] (the caller grows cap and rebuilds) and the
// largest count of the cell to cmax[cell].
// Staged candidates per tile: the most that keeps six workgroups on a CU (26.6
// KB of LDS each).  A 2M-atom water box stages about 605 candidates per cell,
// so most cells take one tile: 1.58 -> 1.46 ms against 512-candidate tiles,
// which took two passes per cell at seven workgroups per CU.
constexpr int NB_TILE = 672;
constexpr int NB_MAXC = 64;    // centres per batch (state kept in LDS across tiles)

__device__ inline int centre_of(int ci, const int* cbeg, const int* clen, int n_el) {
  for (int f = 0; f < n_el; ++f) {
    if (ci < clen[f]) return cbeg[f] + ci;
    ci -= clen[f];
  }
  return -1;
}

template <class E>
__global__ void __launch_bounds__(256) k_neighbors(const double4* __restrict__ pos4, const DevStruct* __restrict__ st,
                                                   int n_struct, const int* __restrict__ start, int n_el,
                                                   int total_cells, double rc2, int cap, E* __restrict__ nbr,
                                                   int4* __restrict__ nnb, int* __restrict__ flags,
                                                   int* __restrict__ cmax, const int* __restrict__ roff) {
  __shared__ double4 sp[NB_TILE];
  __shared__ int seg_first[MAX_EL * 27];
  __shared__ int seg_off[MAX_EL * 27 + 1];
  __shared__ double seg_shift[27][3];
  __shared__ double4 cpos[NB_MAXC];
  __shared__ int cidx[NB_MAXC];
  __shared__ int c_tot[NB_MAXC];
  __shared__ int c_bnd[NB_MAXC][MAX_EL];  // passing candidates before element f's block (-1: not reached)
  __shared__ int red[4];
  const int X = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int lo = 0, hi = n_struct - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (st[mid].cellbase <= X) lo = mid; else hi = mid - 1;
  }
  const DevStruct& S = st[lo];
  const int n0 = S.ncell[0], n1 = S.ncell[1], n2 = S.ncell[2];
  const int l = X - S.cellbase;
  const int c0 = l / (n1 * n2), c1 = (l / n2) % n1, c2 = l % n2;
  const bool shifted = n0 >= 3 && n1 >= 3 && n2 >= 3;
  const int mx = n0 >= 3 ? 3 : n0, my = n1 >= 3 ? 3 : n1, mz = n2 >= 3 ? 3 : n2;
  const int nst = mx * my * mz, nseg = n_el * nst;
  const float inv_nst = __builtin_amdgcn_rcpf((float)nst);
  int cbeg[MAX_EL], clen[MAX_EL], nc = 0;
  for (int f = 0; f < MAX_EL; ++f) {
    cbeg[f] = 0;
    clen[f] = 0;
    if (f < n_el) {
      const int k = f * total_cells + X;
      cbeg[f] = start[k];
      clen[f] = start[k + 1] - cbeg[f];
      nc += clen[f];
    }
  }
  if (nc == 0) {
    if (tid == 0) cmax[X] = 0;
    return;
  }
  int len = 0;
  if (tid < nseg) {
    const int f = tid / nst, o = tid - f * nst;
    const int ox = o / (my * mz), oy = (o / mz) % my, oz = o % mz;
    const int cx = n0 >= 3 ? (c0 - 1 + ox + n0) % n0 : ox;
    const int cy = n1 >= 3 ? (c1 - 1 + oy + n1) % n1 : oy;
    const int cz = n2 >= 3 ? (c2 - 1 + oz + n2) % n2 : oz;
    const int k = f * total_cells + S.cellbase + (cx * n1 + cy) * n2 + cz;
    seg_first[tid] = start[k];
    len = start[k + 1] - start[k];
    if (f == 0) {
      const int g[3] = {c0 - 1 + ox, c1 - 1 + oy, c2 - 1 + oz};
      const int nn[3] = {n0, n1, n2};
#pragma unroll
      for (int a = 0; a < 3; ++a) seg_shift[o][a] = !shifted ? 0.0 : (g[a] < 0 ? -S.L[a] : (g[a] >= nn[a] ? S.L[a] : 0.0));
    }
  }
  // inclusive scan of the segment lengths (nseg <= 108: waves 0 and 1)
  for (int o = 1; o < WAVE; o <<= 1) {
    const int y = __shfl_up(len, o);
    if (lane >= o) len += y;
  }
  if (lane == WAVE - 1) red[wv] = len;
  __syncthreads();
  if (wv == 1) len += red[0];
  if (tid < nseg) seg_off[tid + 1] = len;
  if (tid == 0) seg_off[0] = 0;
  __syncthreads();
  const int ntot = seg_off[nseg];
  int ebeg[MAX_EL];  // first candidate index of each element
  for (int f = 0; f < MAX_EL; ++f) ebeg[f] = f < n_el ? seg_off[f * nst] : ntot;
  const double L0 = S.L[0], L1 = S.L[1], L2 = S.L[2];
  const double i0 = S.invL[0], i1 = S.invL[1], i2 = S.invL[2];
  int most = 0;
  for (int cb = 0; cb < nc; cb += NB_MAXC) {
    const int nbc = min(NB_MAXC, nc - cb);
    for (int i = tid; i < nbc; i += 256) {
      const int c = centre_of(cb + i, cbeg, clen, n_el);
      cidx[i] = c;
      cpos[i] = pos4[c];
      c_tot[i] = 0;
      for (int f = 0; f < MAX_EL; ++f) c_bnd[i][f] = f == 0 ? 0 : -1;
    }
    for (int t0 = 0; t0 < ntot; t0 += NB_TILE) {
      const int tl = min(NB_TILE, ntot - t0);
      __syncthreads();
      for (int u = tid; u < tl; u += 256) {
        const int g = t0 + u;
        int a = 0, b = nseg - 1;
        while (a < b) {
          const int m = (a + b + 1) >> 1;
          if (seg_off[m] <= g) a = m; else b = m - 1;
        }
        const int sidx = seg_first[a] + (g - seg_off[a]);
        const int f = (int)small_div((unsigned)a, inv_nst), o = a - f * nst;  // a < 108
        double4 q = pos4[sidx];
        q.x += seg_shift[o][0];
        q.y += seg_shift[o][1];
        q.z += seg_shift[o][2];
        q.w = __longlong_as_double(((long long)f << 32) | (unsigned)sidx);
        sp[u] = q;
      }
      __syncthreads();
      for (int ci = wv; ci < nbc; ci += 4) {
        const int c = uniform(cidx[ci]);  // the wave's centre: its row address is scalar
        const double4 p = cpos[ci];
        int tot = uniform(c_tot[ci]);
        // padded row (stride cap), compact row at roff[c], or none (counting pass: nbr null)
        E* row = nbr ? nbr + (roff ? (int64_t)roff[c] : (int64_t)c * cap) : nullptr;
        // the first element block that starts at or after this tile (blocks
        // start rarely: only steps that reach one look at them)
        int nbnd = ntot;
        for (int e = 1; e < n_el; ++e)
          if (ebeg[e] >= t0 && ebeg[e] < nbnd) nbnd = ebeg[e];
        for (int u0 = 0; u0 < tl; u0 += WAVE) {
          const int u = u0 + lane;
          // every lane reads a staged candidate (the last one past the tile's
          // end); lanes past the end fail the test
          const double4 q = sp[min(u, tl - 1)];
          const int sidx = (int)(__double_as_longlong(q.w) & 0xffffffffll);
          double dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
          if (!shifted) {
            dx -= L0 * rint(dx * i0);
            dy -= L1 * rint(dy * i1);
            dz -= L2 * rint(dz * i2);
          }
          // the three conditions as separate ballots (each is one compare's
          // lane mask), combined in scalar registers
          const unsigned long long msk = __builtin_amdgcn_ballot_w64(u < tl) &
                                         __builtin_amdgcn_ballot_w64(sidx != c) &
                                         __builtin_amdgcn_ballot_w64(dx * dx + dy * dy + dz * dz < rc2);
          const int rank = tot + lanes_below(msk);
          const unsigned long long keep = row ? msk & __builtin_amdgcn_ballot_w64(rank < cap) : 0ull;
          if (__builtin_amdgcn_inverse_ballot_w64(keep))
            *reinterpret_cast<E*>(reinterpret_cast<char*>(row) + (unsigned)rank * (unsigned)sizeof(E)) =
                make_entry_as<E>(dx, dy, dz, sidx);
          // an element block starting inside this step: passing candidates before it
          const int g0 = t0 + u0;
          if (g0 + WAVE > nbnd) {
            int nx = ntot;
            for (int e = 1; e < n_el; ++e) {
              const int b = ebeg[e] - g0;
              if (b >= 0 && b < WAVE && lane == 0)
                c_bnd[ci][e] = tot + __popcll(msk & ((1ull << b) - 1ull));
              if (ebeg[e] >= g0 + WAVE && ebeg[e] < nx) nx = ebeg[e];
            }
            nbnd = nx;
          }
          tot += __popcll(msk);
        }
        if (lane == 0) c_tot[ci] = tot;
      }
    }
    __syncthreads();
    for (int i = tid; i < nbc; i += 256) {
      const int c = cidx[i];
      const int tot = c_tot[i];
      // rows hold the passing candidates in candidate order, clipped at cap
      int kept[MAX_EL + 1];
      for (int f = 0; f < MAX_EL; ++f) kept[f] = min(f < n_el && c_bnd[i][f] >= 0 ? c_bnd[i][f] : tot, cap);
      kept[MAX_EL] = min(tot, cap);
      nnb[c] = make_int4(kept[1] - kept[0], kept[2] - kept[1], kept[3] - kept[2], kept[4] - kept[3]);
      if (tot > cap) atomicMax(&flags[1], tot);
      most = max(most, tot);
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
  if (lane == 0) red[wv] = most;
  __syncthreads();
  if (tid == 0) cmax[X] = max(max(red[0], red[1]), max(red[2], red[3]));
}

// flags[2] = max over cells of cmax: each block takes 4096 cells, then one
// atomic max per block (flags[2] is cleared before the neighbour build).
constexpr int MAXC_PER = 4096;
__global__ void __launch_bounds__(256) k_max_count(int ncells, const int* __restrict__ cmax, int* __restrict__ flags) {
  __shared__ int red[4];
  const int lo = blockIdx.x * MAXC_PER, hi = min(ncells, lo + MAXC_PER);
  int m = 0;
  for (int i = lo + threadIdx.x; i < hi; i += 256) m = max(m, cmax[i]);
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(&flags[2], max(max(red[0], red[1]), max(red[2], red[3])));
}

// Verlet-skin reuse of a neighbour list (molecular dynamics).  The skin
// list holds, for every sorted atom, the indices of the atoms within
// rc + skin at its last build (element-grouped, as above); while no atom has
// moved more than skin/2 since then, every pair within rc is in it, because
// the minimum-image distance obeys the triangle inequality.
//
// k_regather: sorted positions refreshed from the caller's positions in the
// kept sorted order (wrapped in FP64, ids kept), and each atom's
// minimum-image displacement since the build tested against lim2 =
// (skin/2)^2: flags[0] bit 2 if any atom moved farther (the skin list must
// be rebuilt), bit 1 if a coordinate is not finite.
template <class TIn>
__global__ void __launch_bounds__(256) k_regather(int64_t n, const TIn* __restrict__ pos,
                                                  const DevStruct* __restrict__ st, const int* __restrict__ perm,
                                                  double4* __restrict__ pos4, const double4* __restrict__ ref,
                                                  double lim2, int* __restrict__ flags) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool far = false, bad = false;
  if (s < n) {
    const int64_t i = perm[s];
    double4 p = pos4[s];
    const DevStruct& S = st[struct_of(p.w)];
    const double x = (double)pos[3 * i + 0], y = (double)pos[3 * i + 1], z = (double)pos[3 * i + 2];
    bad = !(isfinite(x) && isfinite(y) && isfinite(z));
    p.x = wrap_coord(x, S.L[0], S.invL[0]);
    p.y = wrap_coord(y, S.L[1], S.invL[1]);
    p.z = wrap_coord(z, S.L[2], S.invL[2]);
    const double4 r = ref[s];
    double dx = p.x - r.x, dy = p.y - r.y, dz = p.z - r.z;
    dx -= S.L[0] * rint(dx * S.invL[0]);
    dy -= S.L[1] * rint(dy * S.invL[1]);
    dz -= S.L[2] * rint(dz * S.invL[2]);
    far = dx * dx + dy * dy + dz * dz > lim2;
    pos4[s] = p;
  }
  const unsigned long long fm = __builtin_amdgcn_ballot_w64(far), bm = __builtin_amdgcn_ballot_w64(bad);
  if ((threadIdx.x & 63) == 0) {
    if (fm) atomicOr(&flags[0], 4);
    if (bm) atomicOr(&flags[0], 2);
  }
}

// k_refresh: the rows of (r_j - r_i, j) entries within rc, read from the
// skin list and the current positions (minimum image in FP64), one wave per
// centre, compacted by ballot so that the element grouping is kept.  As in
// the build: at most cap entries per row, flags[1] the largest count beyond
// cap, flags[2] the largest count (one atomic per workgroup).
template <class E>
__global__ void __launch_bounds__(256) k_refresh(int64_t n, int n_el, const double4* __restrict__ pos4,
                                                 const DevStruct* __restrict__ st, const int* __restrict__ snbr,
                                                 const int4* __restrict__ snnb, int scap, double rc2, int cap,
                                                 E* __restrict__ nbr, int4* __restrict__ nnb,
                                                 int* __restrict__ flags) {
  __shared__ int red[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int most = 0;
  for (int64_t c = (int64_t)blockIdx.x * 4 + wv; c < n; c += (int64_t)gridDim.x * 4) {
    const double4 p = pos4[c];
    const DevStruct& S = st[struct_of(p.w)];
    const int4 sc = snnb[c];
    const int scnt[MAX_EL] = {sc.x, sc.y, sc.z, sc.w};
    const int* srow = snbr + c * (int64_t)scap;
    E* row = nbr + c * (int64_t)cap;
    int tot = 0, so = 0;
    int kept[MAX_EL] = {0, 0, 0, 0};
    for (int f = 0; f < n_el; ++f) {
      const int before = tot, end = so + scnt[f];
      for (int t0 = so; t0 < end; t0 += WAVE) {
        const int t = t0 + lane;
        bool pass = false;
        double dx = 0.0, dy = 0.0, dz = 0.0;
        int j = 0;
        if (t < end) {
          j = srow[t];
          const double4 q = pos4[j];
          dx = q.x - p.x;
          dy = q.y - p.y;
          dz = q.z - p.z;
          dx -= S.L[0] * rint(dx * S.invL[0]);
          dy -= S.L[1] * rint(dy * S.invL[1]);
          dz -= S.L[2] * rint(dz * S.invL[2]);
          pass = dx * dx + dy * dy + dz * dz < rc2;
        }
        const unsigned long long msk = __builtin_amdgcn_ballot_w64(pass);
        const int rank = tot + lanes_below(msk);
        if (pass && rank < cap) row[rank] = make_entry_as<E>(dx, dy, dz, j);
        tot += __popcll(msk);
      }
      kept[f] = min(tot, cap) - min(before, cap);
      so = end;
    }
    if (lane == 0) nnb[c] = make_int4(kept[0], kept[1], kept[2], kept[3]);
    most = max(most, tot);
  }
  for (int o = 32; o > 0; o >>= 1) most = max(most, __shfl_xor(most, o));
  if (lane == 0) red[wv] = most;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int m = max(max(red[0], red[1]), max(red[2], red[3]));
    atomicMax(&flags[2], m);
    if (m > cap) atomicMax(&flags[1], m);
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
// One wave per centre (grid-stride): lanes own the j of a class block, the
// k run as a uniform loop (one broadcast read per k).  Partial counts stay in
// registers and are reduced once per wave.
template <class E>
__global__ void __launch_bounds__(256) k_count_terms(int64_t n, const double4* __restrict__ pos4,
                                                     const E* __restrict__ nbr, const int4* __restrict__ nnb, int cap,
                                                     int n_el, CountTab ct, double rc2,
                                                     unsigned long long* __restrict__ counts) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  unsigned long long cand = 0, pass = 0, aterms = 0, entries = 0, rterms = 0;
  for (int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); s < n; s += nwaves) {
    const int e = elem_of(pos4[s].w);
    const int4 c4 = nnb[s];
    const int cnt[MAX_EL] = {c4.x, c4.y, c4.z, c4.w};
    int off[MAX_EL + 1];
    off[0] = 0;
    for (int f = 0; f < MAX_EL; ++f) off[f + 1] = off[f] + (f < n_el ? cnt[f] : 0);
    if (lane == 0) {
      entries += (unsigned long long)off[n_el];
      for (int f = 0; f < n_el; ++f) rterms += (unsigned long long)cnt[f] * ct.rad[e][f];
    }
    const E* row = nbr + s * (int64_t)cap;
    for (int e1 = 0; e1 < n_el; ++e1)
      for (int e2 = e1; e2 < n_el; ++e2) {
        const int na = ct.ang[e][class_index(e1, e2, n_el)];
        if (na == 0) continue;
        const bool same = e1 == e2;
        const int end1 = off[e1] + cnt[e1], end2 = off[e2] + cnt[e2];
        for (int a0 = off[e1]; a0 < end1; a0 += WAVE) {
          const int a = a0 + lane;
          const bool va = a < end1;
          E qa = row[a0];
          if (va) qa = row[a];
          for (int b = same ? a0 + 1 : off[e2]; b < end2; ++b) {
            const E qb = row[b];
            if (va && (!same || b > a)) {
              const double wx = (double)qb.x - (double)qa.x, wy = (double)qb.y - (double)qa.y,
                           wz = (double)qb.z - (double)qa.z;
              ++cand;
              if (wx * wx + wy * wy + wz * wz < rc2) {
                ++pass;
                aterms += (unsigned long long)na;
              }
            }
          }
        }
      }
  }
  unsigned long long v[5] = {entries, cand, pass, aterms, rterms};
  for (int i = 0; i < 5; ++i) {
    for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o);
    if (lane == 0 && v[i]) atomicAdd(&counts[i], v[i]);
  }
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
  const int nb = (nkeys + SCAN_PER - 1) / SCAN_PER;
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, stream, nkeys, a.count, a.scan);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, nb, nkeys, a.scan, a.start);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, stream, nkeys, a.count, a.scan, a.start, a.cursor);
  if (n > 0) {
    const unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, stream, n, a.key, a.cursor, a.perm_raw);
    hipLaunchKernelGGL(k_sort_bins, dim3(g), dim3(256), 0, stream, n, a.key, a.start, a.perm_raw, a.perm);
    hipLaunchKernelGGL(k_fill_sorted<TIn>, dim3(g), dim3(256), 0, stream, n, pos, a.types, a.st, a.soff,
                       a.n_struct, a.n_el, a.perm, a.pos4);
  }
  hipLaunchKernelGGL(k_element_offsets, dim3(1), dim3(64), 0, stream, a.n_el, a.total_cells, a.start, a.eoff);
}

template void launch_bin_sort<float>(const BinArgs&, const float*, hipStream_t);
template void launch_bin_sort<double>(const BinArgs&, const double*, hipStream_t);

template <class E>
void launch_neighbors_as(const BinArgs& a, double rc, int cap, E* nbr, int4* nnb, int* cmax, hipStream_t stream,
                         const int* roff = nullptr) {
  if (a.n == 0) return;
  hipLaunchKernelGGL(k_neighbors<E>, dim3((unsigned)a.total_cells), dim3(256), 0, stream, a.pos4, a.st, a.n_struct,
                     a.start, a.n_el, a.total_cells, rc * rc, cap, nbr, nnb, a.flags, cmax, roff);
  hipLaunchKernelGGL(k_max_count, dim3((unsigned)std::max(1, (a.total_cells + MAXC_PER - 1) / MAXC_PER)), dim3(256), 0,
                     stream, a.total_cells, cmax, a.flags);
}

template <class T>
void launch_neighbors(const BinArgs& a, double rc, int cap, typename Vec4<T>::type* nbr, int4* nnb, int* cmax,
                      hipStream_t stream) {
  launch_neighbors_as<typename Vec4<T>::type>(a, rc, cap, nbr, nnb, cmax, stream);
}
template void launch_neighbors<float>(const BinArgs&, double, int, float4*, int4*, int*, hipStream_t);
template void launch_neighbors<double>(const BinArgs&, double, int, double4*, int4*, int*, hipStream_t);

void launch_neighbor_index(const BinArgs& a, double rc, int cap, int* nbr, int4* nnb, int* cmax, hipStream_t stream) {
  launch_neighbors_as<int>(a, rc, cap, nbr, nnb, cmax, stream);
}

template <class T>
void launch_neighbor_counts(const BinArgs& a, double rc, int4* nnb, int* cmax, hipStream_t stream) {
  launch_neighbors_as<typename Vec4<T>::type>(a, rc, INT32_MAX, nullptr, nnb, cmax, stream);
}
template void launch_neighbor_counts<float>(const BinArgs&, double, int4*, int*, hipStream_t);
template void launch_neighbor_counts<double>(const BinArgs&, double, int4*, int*, hipStream_t);

template <class T>
void launch_neighbors_compact(const BinArgs& a, double rc, const int* roff, typename Vec4<T>::type* nbr, int4* nnb,
                              int* cmax, hipStream_t stream) {
  launch_neighbors_as<typename Vec4<T>::type>(a, rc, INT32_MAX, nbr, nnb, cmax, stream, roff);
}
template void launch_neighbors_compact<float>(const BinArgs&, double, const int*, float4*, int4*, int*, hipStream_t);
template void launch_neighbors_compact<double>(const BinArgs&, double, const int*, double4*, int4*, int*,
                                               hipStream_t);

__global__ void __launch_bounds__(256) k_row_lengths(int64_t n, const int4* __restrict__ nnb, int* __restrict__ len) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int4 v = nnb[c];
  len[c] = v.x + v.y + v.z + v.w;
}

void launch_row_offsets(int64_t n, const int4* nnb, int* len, int* roff, int* tmp, int* partial, hipStream_t stream) {
  if (n == 0) return;
  const int ni = (int)n;
  hipLaunchKernelGGL(k_row_lengths, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n, nnb, len);
  const int nb = (ni + SCAN_PER - 1) / SCAN_PER;
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(1024), 0, stream, ni, len, partial);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, stream, nb, ni, partial, roff);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(1024), 0, stream, ni, len, partial, roff, tmp);
}

template <class TIn>
void launch_regather(const BinArgs& a, const TIn* pos, const double4* ref, double lim, hipStream_t stream) {
  if (a.n == 0) return;
  hipLaunchKernelGGL(k_regather<TIn>, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, stream, a.n, pos, a.st,
                     a.perm, a.pos4, ref, lim * lim, a.flags);
}
template void launch_regather<float>(const BinArgs&, const float*, const double4*, double, hipStream_t);
template void launch_regather<double>(const BinArgs&, const double*, const double4*, double, hipStream_t);

template <class T>
void launch_refresh(const BinArgs& a, const int* snbr, const int4* snnb, int scap, double rc, int cap,
                    typename Vec4<T>::type* nbr, int4* nnb, hipStream_t stream) {
  if (a.n == 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((a.n + 3) / 4, 16384);
  hipLaunchKernelGGL(k_refresh<typename Vec4<T>::type>, dim3(g), dim3(256), 0, stream, a.n, a.n_el, a.pos4, a.st,
                     snbr, snnb, scap, rc * rc, cap, nbr, nnb, a.flags);
}
template void launch_refresh<float>(const BinArgs&, const int*, const int4*, int, double, int, float4*, int4*,
                                    hipStream_t);
template void launch_refresh<double>(const BinArgs&, const int*, const int4*, int, double, int, double4*, int4*,
                                     hipStream_t);

template <class T>
void launch_count_terms(const BinArgs& a, const typename Vec4<T>::type* nbr, const int4* nnb, int cap,
                        const CountTab& ct, double rc, unsigned long long* counts, hipStream_t stream) {
  if (a.n == 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((a.n + 3) / 4, 4096);
  hipLaunchKernelGGL(k_count_terms<typename Vec4<T>::type>, dim3(g), dim3(256), 0, stream, a.n, a.pos4, nbr, nnb,
                     cap, a.n_el, ct, rc * rc, counts);
}
template void launch_count_terms<float>(const BinArgs&, const float4*, const int4*, int, const CountTab&, double,
                                        unsigned long long*, hipStream_t);
template void launch_count_terms<double>(const BinArgs&, const double4*, const int4*, int, const CountTab&, double,
                                         unsigned long long*, hipStream_t);

}  // namespace nnp
