// Launch interfaces of the gfx950 kernels (host side).
#pragma once

#include "common.h"

namespace nnp {

// ---------------------------------------------------------------- K1/K2
struct BinArgs {
  int64_t n;                 // atoms of the batch
  const int32_t* types;      // caller order
  const DevStruct* st;       // [n_struct]
  const int64_t* soff;       // [n_struct + 1] atom offsets (device)
  int n_struct;
  int n_el;
  int total_cells;           // cells of all structures
  int* key;                  // [n]
  int* count;                // [n_el * total_cells + 1]
  int* start;                // [n_el * total_cells + 1]
  int* cursor;               // [n_el * total_cells + 1]
  int* scan;                 // [ceil((n_el * total_cells) / 4096)] block sums of the scan
  int* perm;                 // [n] sorted -> caller index
  int* perm_raw;             // [n] the scatter's order within each bin, before the bin sort
  double4* pos4;             // [n] sorted wrapped positions + ids
  int* eoff;                 // [n_el + 1] element offsets of the sorted order
  int* flags;                // [0] bit 0 bad type, bit 1 non-finite position, bit 2 skin exceeded;
                             // [1] max neighbour count beyond cap, [2] max count, [3] inputs differ
};

void launch_fill_int(int* p, int64_t n, int v, hipStream_t stream);
template <class TIn>
void launch_bin_sort(const BinArgs& a, const TIn* pos, hipStream_t stream);
// Neighbour rows of (dx, dy, dz, j) entries; cmax: [total_cells] scratch.
template <class T>
void launch_neighbors(const BinArgs& a, double rc, int cap, typename Vec4<T>::type* nbr, int4* nnb, int* cmax,
                      hipStream_t stream);
// Rows of neighbour indices alone (the Verlet-skin list of the MD driver and
// the index-entry list layout).
void launch_neighbor_index(const BinArgs& a, double rc, int cap, int* nbr, int4* nnb, int* cmax, hipStream_t stream);
// Compact rows (no padding): a counting pass (nnb receives the exact counts),
// the exclusive scan of the row lengths into roff[0..n] (int; the caller
// checks the total fits), then the write pass into nbr at roff.
template <class T>
void launch_neighbor_counts(const BinArgs& a, double rc, int4* nnb, int* cmax, hipStream_t stream);
void launch_row_offsets(int64_t n, const int4* nnb, int* len, int* roff, int* tmp, int* partial, hipStream_t stream);
template <class T>
void launch_neighbors_compact(const BinArgs& a, double rc, const int* roff, typename Vec4<T>::type* nbr, int4* nnb,
                              int* cmax, hipStream_t stream);
// Sorted positions from the caller's in the kept order; flags[0] bit 2 if any
// atom moved more than lim from ref (its sorted position at the skin build).
template <class TIn>
void launch_regather(const BinArgs& a, const TIn* pos, const double4* ref, double lim, hipStream_t stream);
// Rows of (dx, dy, dz, j) entries within rc from the skin list (scap slots per row).
template <class T>
void launch_refresh(const BinArgs& a, const int* snbr, const int4* snnb, int scap, double rc, int cap,
                    typename Vec4<T>::type* nbr, int4* nnb, hipStream_t stream);
// Angular / radial SF counts per (centre, class) and (centre, neighbour element).
struct CountTab {
  int ang[MAX_EL][MAX_CLS];
  int rad[MAX_EL][MAX_EL];
};
template <class T>
void launch_count_terms(const BinArgs& a, const typename Vec4<T>::type* nbr, const int4* nnb, int cap,
                        const CountTab& ct, double rc, unsigned long long* counts, hipStream_t stream);

// ---------------------------------------------------------------- K3/K5/K7
template <int P>
struct TripArgs {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  using FAcc = typename Types<P>::FAcc;
  int64_t n;                 // sorted atoms
  int cap;                   // neighbour slots per atom (row stride of nbr)
  int lcap;                  // LDS capacity: >= the most neighbours of any atom
  const double4* pos4;
  const typename Vec4<T>::type* nbr;  // [n][cap] (dx, dy, dz, j) entries (null with idx)
  const int* idx;            // or [n][cap] neighbour indices alone (wave-level passes only)
  const int* roff;           // null: row c at c * cap; else compact rows at roff[c] (wave-level passes only)
  int wpc;                   // waves per centre of the wave-level passes (1 or 2)
  const int4* nnb;           // [n] neighbours per element block
  const DevStruct* st;
  const DevTab<T>* tab;
  IO* G;                     // SF: G~ rows [n][LD]
  const IO* C;               // FORCE: dE/dG rows [n][LD]
  FAcc* F;                   // FORCE: force accumulator [3][n] (component planes, sorted order)
  const IO* delta;           // JVP: dL/dF [n][3] (sorted)
  IO* V;                     // JVP: rows [n][LD]
  // Pair-test masks of the one-wave pair walk (wpc 1): the SF pass writes the
  // test of lane l at step s of centre c to bit s % 32 of
  // pm[(c * pm_stride + s / 32) * 64 + l], the force and force-adjoint passes
  // read them instead of repeating the r_jk < rc test.  pm_stride = 0: every
  // pass tests the pairs.  pm_stride >= ceil(pair_step_bound(lcap, n_el) / 32).
  unsigned* pm;
  int pm_stride;
};

// Most steps the one-wave pair walk can take for a centre with m neighbours
// of n_el elements.  A chunk of mJ <= 64 lanes walks a range of D deltas in
// ceil(D / R) steps with R = 1 (mJ > 32) or floor(64 / mJ) (R mJ > 32), so
// at most 2 mJ D / 64 + 1 steps; D = mB across elements and <= mA / 2 within
// one, and summed over the classes the mJ D terms give at most m^2 / 2.  The
// chunks number at most sum over classes of (mA / 64 + 1).
__host__ __device__ constexpr int pair_step_bound(int m, int n_el) {
  return (m * m + n_el * m + 63) / 64 + n_el * (n_el + 1) / 2;
}

template <int P>
void launch_triplet(int mode, int ne, const TripArgs<P>& a, hipStream_t stream);
// One thread per centre (mode 0: SF, 1: force, 2: force-adjoint product).
template <int P>
void launch_flat(int mode, const TripArgs<P>& a, hipStream_t stream);
template <int P>
size_t triplet_lds_bytes(int mode, int ne, int lcap, int wpc);

// ------------------------------------------------- stored-Jacobian form
// J holds, for every centre c and neighbour slot t (entry e = c * cap + t),
// the gradient of each SF s of c with respect to the neighbour's position:
// J[(3 s + x) * plane + e], x = 0..2, plane = n * cap, s < n_sf(element of c).
template <int P>
struct JacArgs {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  using FAcc = typename Types<P>::FAcc;
  int64_t n;                 // sorted atoms
  int cap;                   // neighbour slots per atom
  int lcap;                  // >= the most neighbours of any atom
  int wide;                  // the table holds wide angular functions
  const typename Vec4<T>::type* nbr;  // [n][cap] (dx, dy, dz, j) entries
  const int4* nnb;           // [n] neighbours per element block
  const double4* pos4;       // sorted positions + ids
  const DevTab<T>* tab;
  int64_t plane;             // n * cap
  T* J;                      // [3 * max n_sf][plane]
  IO* G;                     // SF pass: G~ rows [n][LD]
  const IO* C;               // force contraction: dE/dG rows [n][LD]
  FAcc* F;                   // force contraction: accumulator [3][n] (component planes, sorted order)
  const IO* delta;           // JVP contraction: dL/dF [n][3] (sorted)
  IO* V;                     // JVP contraction: rows [n][LD]
};
template <int P>
void launch_jac(const JacArgs<P>& a, hipStream_t stream);          // G~ and J
template <int P>
size_t jac_lds_bytes(int lcap);
template <int P>
void launch_jac_force(const JacArgs<P>& a, hipStream_t stream);    // F from J and dE/dG
template <int P>
void launch_jac_jvp(const JacArgs<P>& a, hipStream_t stream);      // V from J and delta
template <class IO>
void launch_same_inputs(int64_t n, const IO* pos, const IO* saved_pos, const int32_t* types,
                        const int32_t* saved_types, int* flag, hipStream_t stream);

// ------------------------------------------------------ velocity Verlet
struct MdArgs {
  double half_kick[MAX_EL];  // (dt / 2) accel_conv / m_e
  double half_mass[MAX_EL];  // m_e / 2
  double dt;                 // fs
  double L[3], invL[3];      // box edges (A) and inverses
  double ke_conv;            // amu A^2 / fs^2 -> eV
};
int md_blocks(int64_t n);    // blocks of the kinetic-energy partial sums
template <class IO>
void launch_kick_drift(int64_t n, IO* pos, IO* vel, const IO* F, const int32_t* types, const MdArgs& m,
                       hipStream_t stream);
template <class IO>
void launch_kick_ke(int64_t n, IO* vel, const IO* F, const int32_t* types, const MdArgs& m, bool kick,
                    double* partial, double* ke_out, hipStream_t stream);

// ---------------------------------------------------------------- K4/K8
template <int P>
struct MlpArgs {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  int64_t n;                 // sorted atoms
  int n_el;
  const int* eoff;           // [n_el + 1] (device)
  const IO* G;               // [n][LD] scaled inputs
  IO* C;                     // [n][LD] dE/dG (raw G)
  IO* Ei;                    // [n] atomic energies (sorted)
  const T* nets;             // [n_el][NET_STRIDE] padded parameters
  const uint16_t* bf;        // BF16 form: split weights (see k_mlp.hip), else null
  const DevTab<T>* tab;
};
template <int P>
void launch_mlp(const MlpArgs<P>& a, hipStream_t stream);

// Weight gradient of sum_i [a_i E_i - <dE_i/dG~_i, t_i>] with t = V / scale
// (differentiation form), reduced over atoms in FP64 chunks.
template <int P>
struct WGradArgs {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  int64_t n;
  int n_el;
  const int* eoff;
  const IO* G;               // [n][LD] scaled inputs
  const IO* V;               // [n][LD] JVP rows (raw G)
  const double* gE_atom;     // [n] dL/dE of each atom's structure (sorted), or null
  const T* nets;
  const DevTab<T>* tab;
  T* vec;                    // [n][11 * HID] per-atom vectors
  int chunk, nch;            // atoms per partial, partials per element (>= ceil(max N_e / chunk))
  double* partial;           // [n_el][nch][NET_STRIDE]
  double* padded;            // [n_el][NET_STRIDE]
  int64_t n_params;
  const int* flatmap;        // [n_params] flat index -> padded index
  double* out;               // [n_params] caller layout
};
template <int P>
void launch_wgrad(const WGradArgs<P>& a, hipStream_t stream);

// ---------------------------------------------------------------- K6 + misc
template <class T>
void launch_fill(T* p, int64_t n, T v, hipStream_t stream);
template <class IO, class FAcc>
void launch_unpermute(int64_t n, const int* perm, const IO* Ei_s, const FAcc* F_s, double* Ei_o, IO* Ei_out,
                      IO* F_out, hipStream_t stream);
template <class IO>
void launch_permute_rows3(int64_t n, const int* perm, const IO* in, IO* out, hipStream_t stream);
void launch_gather_struct_grad(int64_t n, const int* perm, const int64_t* soff, int n_struct, const double* gE,
                               double* gE_atom, hipStream_t stream);
// Deterministic energy sums: chunk partials then per-structure sums.
void launch_energy(const double* Ei_o, const int64_t* chunk_lo, const int64_t* chunk_hi, int nchunk,
                   const int* struct_chunk, int n_struct, double* partial, double* energies, hipStream_t stream);

}  // namespace nnp
