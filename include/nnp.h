/*
 * nnp.h - C ABI of the MI355X (gfx950) Behler-Parrinello neural-network
 * potential: energy, per-atom energies and forces of periodic orthorhombic
 * structures, and the parameter gradient of an energy+force training loss.
 *
 * Method (Desai, Reeve, Belak, arXiv:2002.00054, Sec. 3.1 and Fig. 1(b)):
 *   step 1  symmetry functions G_i of every atom i from its neighbours within
 *           the cutoff rc: radial G2 (the step-1 formula of Fig. 1(b)) and the
 *           narrow angular G3 of Behler (the paper's ref. [18]; Sec. 3.1 names
 *           the angular loop over neighbours of neighbours without printing
 *           it):
 *             G2 = sum_j exp(-eta (r_ij - rs)^2) fc(r_ij)
 *             G3 = 2^(1-zeta) sum_{j<k} (1 + lambda cos theta_ijk)^zeta
 *                  exp(-eta (r_ij^2 + r_ik^2 + r_jk^2)) fc(r_ij) fc(r_ik) fc(r_jk)
 *           and its wide variant of the same family, without the r_jk factor
 *             G9 = 2^(1-zeta) sum_{j<k} (1 + lambda cos theta_ijk)^zeta
 *                  exp(-eta (r_ij^2 + r_ik^2)) fc(r_ij) fc(r_ik)
 *           with fc(r) = (cos(pi r / rc) + 1) / 2 for r < rc, else 0;
 *   step 2  E_i = NN_{e_i}((G_i - shift) / scale), one feed-forward network per
 *           element (Fig. 1(c)), tanh hidden layers, linear output;
 *           E = sum_i E_i;
 *   step 3  f_m = -dE/dr_m (the sign convention of Fig. 1(a),(b)) by the chain
 *           rule through dE_i/dG_i and dG_i/dr_m.
 *
 * Units: Angstrom and eV.  Neighbours use the minimum image, which needs every
 * box edge > 2 rc.  Positions may lie outside the box; they are wrapped.
 *
 * Threading: a handle may be used by one host thread and one stream at a time.
 * A call that overlaps another call on the same handle (from a second host
 * thread) is refused with NNP_E_STATE before it reads or writes any of the
 * handle's state; nnp_last_error on that thread then names the cause, and the
 * running call is unaffected (nnp_last_timings returns 0 and
 * nnp_workspace_bytes -1 in that case).  Different handles may be used
 * concurrently.  All work of a call is enqueued on the caller's stream; calls
 * that return a host value (the energy) synchronise that stream; the others
 * return with their device outputs ready in the stream's order, and their
 * last kernels may still be running: before using the handle on another
 * stream, synchronise the first one.
 */
#ifndef NNP_H
#define NNP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnp_handle nnp_handle;

typedef enum {
  NNP_OK = 0,
  NNP_E_ARG = -1,   /* invalid argument (null pointer, size, table entry)     */
  NNP_E_BOX = -2,   /* some box edge <= 2 rc (minimum image undefined) or not finite */
  NNP_E_TYPE = -3,  /* an atom type outside [0, n_el); outputs are undefined   */
  NNP_E_HIP = -4,   /* a HIP runtime call failed                              */
  NNP_E_NOMEM = -5, /* device allocation failed                               */
  NNP_E_STATE = -6  /* handle misuse (e.g. backward before any forward)       */
} nnp_status;

/*
 * Arithmetic forms of the whole path.
 *  NNP_FP64        every step in double precision; positions, per-atom
 *                  energies and forces are double.
 *  NNP_FP32        every step in single precision (FP32 MFMA for the network
 *                  layers); positions, per-atom energies and forces are float.
 *  NNP_BF16_MIXED  precision form: symmetry-function terms in FP32 summed per
 *                  atom in FP64; hidden network layer on BF16 MFMA with FP32
 *                  accumulation; first layer (and its transpose in dE/dG) in
 *                  split BF16x3 (x = hi + lo, products hi*hi + hi*lo + lo*hi);
 *                  forces accumulated in FP64 and the energy summed in FP64.
 *                  Positions, per-atom energies and forces are float.
 */
typedef enum { NNP_FP64 = 0, NNP_FP32 = 1, NNP_BF16_MIXED = 2 } nnp_precision;

/* One symmetry function of the table (Sec. 3.1 step 1).
 *  centre    element of the centre atom, in [0, n_el)
 *  kind      2 = radial G2 (neighbour element nbr[0]);
 *            3 = narrow angular G3 (unordered neighbour-element pair nbr[0], nbr[1]);
 *            9 = wide angular G9 (same pair convention).  A table holding any
 *                G9 runs its SF, force and force-adjoint passes one thread per
 *                centre (the stored-Jacobian variant handles G9 directly).
 *  eta       Gaussian exponent, A^-2, >= 0
 *  rs        radial shift, A (G2 only; must be 0 for G3 and G9)
 *  zeta      exponent, one of 1, 2, 4, 8, 16, 32 (G3 and G9 only)
 *  lambda    +1 or -1 (G3 and G9 only)
 *  rc        cutoff radius, A; every entry of one table must use the same rc
 *  shift, scale  centring/scaling: the network sees (G - shift) / scale, scale != 0
 * The order of the entries of one centre element is the order of that
 * element's network inputs. */
typedef struct {
  int centre;
  int kind;
  int nbr[2];
  double eta, rs, zeta, lambda, rc, shift, scale;
} nnp_sf;

/* One element's network (Sec. 3.1 step 2, Fig. 1(c)).
 *  n_layers  number of weight layers, 1..4
 *  sizes     [n_layers + 1] widths: sizes[0] = number of SFs of the element,
 *            sizes[n_layers] = 1, hidden widths <= 32
 *  W[l]      row-major [sizes[l+1]][sizes[l]] (host)
 *  b[l]      [sizes[l+1]] (host)
 *  activation 0 = tanh on hidden layers, linear output (the only one supported) */
typedef struct {
  int n_layers;
  const int* sizes;
  const double* const* W;
  const double* const* b;
  int activation;
} nnp_net;

/*
 * Create a potential.  Deep-copies every host array (the caller may free them
 * afterwards) and uploads the parameters to the current HIP device.
 *  n_el      number of elements, 1..4
 *  elements  [n_el] element names (informational; index = type id), may be NULL
 *  n_sf, sf  the symmetry-function table (see nnp_sf); per element at most 32
 *            entries, per (centre, neighbour element) at most 16 radial, per
 *            (centre, neighbour pair) at most 8 angular, and per centre at most
 *            4 distinct angular eta
 *  nets      [n_el] networks; nets[e].sizes[0] must equal the number of SFs of
 *            centre element e
 *  prec      arithmetic form
 *  out       receives the handle (NULL on failure)
 * Errors: NNP_E_ARG for a malformed table or network, NNP_E_HIP / NNP_E_NOMEM. */
nnp_status nnp_create(int n_el, const char* const* elements, int n_sf, const nnp_sf* sf,
                      const nnp_net* nets, nnp_precision prec, nnp_handle** out);

/*
 * Energy, per-atom energies and forces of one structure (Fig. 1(b) steps 1-3).
 *  n_atoms      number of atoms, >= 0 (0 gives E = 0)
 *  pos          device [n_atoms][3], double (NNP_FP64) or float (other forms)
 *  types        device int32 [n_atoms], element ids in [0, n_el)
 *  box          host double[3], orthorhombic edges; each must exceed 2 rc
 *  energy       host, receives E = sum_i E_i (double); may be NULL
 *  atom_energy  device [n_atoms] E_i in the positions' type; may be NULL
 *  forces       device [n_atoms][3] f = -dE/dr in the positions' type; may be NULL
 *  stream       hipStream_t (NULL = default stream)
 * Outputs are in the caller's atom order.  The neighbour list is rebuilt on
 * every call; if an atom has more neighbours than the current capacity the
 * handle grows it and recomputes (not an error).  Synchronises the stream.
 * Positions may lie outside the box (they are wrapped) but must be finite.
 * Errors: NNP_E_ARG, NNP_E_BOX (checked before any launch), NNP_E_TYPE and
 * NNP_E_ARG for a NaN or infinite coordinate (both detected on the device by
 * the binning pass and reported by the same call, before any SF or force
 * kernel is launched), NNP_E_HIP, NNP_E_NOMEM. */
nnp_status nnp_compute(nnp_handle* h, int64_t n_atoms, const void* pos, const int32_t* types,
                       const double box[3], double* energy, void* atom_energy, void* forces,
                       void* stream);

/*
 * nnp_compute without any allocation, for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments, outputs, errors and
 * synchronisation are those of nnp_compute; the derivatives are always
 * recomputed (the stored-Jacobian mode does not apply) and profiling is off
 * for the call.
 * Every intermediate buffer is carved from one static device array of
 * NNP_NOALLOC_SCRATCH_BYTES bytes that the library holds on each device it
 * runs on until the process ends, shared by every handle on that device; the
 * call makes no hipMalloc, hipFree or other allocating call (the pinned host
 * staging it needs is allocated by nnp_create).  The array keeps the last
 * call's contents; every value a call reads is written or cleared by that
 * call first.  Calls that overlap on one device (two streams, two host
 * threads, two handles) race on the array: serialise them.
 *  n_atoms  at most NNP_NOALLOC_MAX_ATOMS, else NNP_E_ARG before any launch.
 * A structure whose buffers (about 5 KB per atom in FP64 and 2.5 KB in FP32
 * at the water density's 128 neighbour slots) exceed the array returns
 * NNP_E_NOMEM; the handle's device must be the current device (else
 * NNP_E_STATE).  The handle's own workspace is left untouched. */
#define NNP_NOALLOC_MAX_ATOMS 16384
#define NNP_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
nnp_status nnp_compute_noalloc(nnp_handle* h, int64_t n_atoms, const void* pos, const int32_t* types,
                               const double box[3], double* energy, void* atom_energy, void* forces,
                               void* stream);

/*
 * The same for a batch of independent structures stored back to back.
 *  n_struct      number of structures, >= 1
 *  atom_offsets  host int64 [n_struct + 1], offsets[0] = 0, non-decreasing;
 *                structure b holds atoms [offsets[b], offsets[b+1])
 *  pos, types    device, all structures' atoms
 *  boxes         host double [n_struct][3]
 *  energies      device double [n_struct]; may be NULL
 *  atom_energy, forces  as in nnp_compute (batch order); may be NULL
 * Returns once the neighbour list is checked (the stream is synchronised
 * for that) and the remaining kernels are enqueued: the device outputs are
 * ready in the order of `stream` (read them on that stream, or after
 * synchronising it).  With profiling on, the call synchronises at the end. */
nnp_status nnp_compute_batch(nnp_handle* h, int n_struct, const int64_t* atom_offsets, const void* pos,
                             const int32_t* types, const double* boxes, double* energies,
                             void* atom_energy, void* forces, void* stream);

/*
 * Differentiation form: gradient of a scalar loss L(E_b, F) with respect to
 * every network parameter, given dL/dE_b and dL/dF of the batch evaluated by
 * nnp_compute_batch with the same arguments:
 *   dL/dtheta = sum_b dL/dE_b dE_b/dtheta + sum_m dL/dF_m . dF_m/dtheta.
 * By default the descriptor derivatives are recomputed, not stored (see
 * nnp_set_derivative_mode for the stored alternative).  Called with the
 * inputs of the last nnp_compute_batch on this handle (same batch layout and
 * boxes, checked on the host; positions and types bitwise equal, checked on
 * the device, the host waiting for that one flag), it reuses that forward's
 * sorted order, neighbour list and scaled SFs and runs only the
 * force-adjoint product and the weight gradient; with other inputs it
 * rebuilds them first.  Any other call on the handle in between (except
 * nnp_set_params and the query functions) ends the reuse.
 *  dL_dE        device double [n_struct] (may be NULL: no energy term)
 *  dL_dF        device [n_atoms][3] in the positions' type (may be NULL: no force term)
 *  grad_params  device double [nnp_n_params(h)], overwritten; flat layout of
 *               nnp_set_params
 * Like nnp_compute_batch, returns with the gradient ready in the order of
 * `stream`.  Errors as nnp_compute_batch. */
nnp_status nnp_backward(nnp_handle* h, int n_struct, const int64_t* atom_offsets, const void* pos,
                        const int32_t* types, const double* boxes, const double* dL_dE,
                        const void* dL_dF, void* grad_params, void* stream);

/*
 * Molecular dynamics at constant N, V, E around the energy+force path, the
 * setting the method is used in (Sec. 4: an MD proxy application, with energy
 * conservation as its correctness check).  The paper does not name the
 * integrator; this is velocity Verlet:
 *   v += (dt/2) F/m;  x += dt v (then wrapped into [0, L));  F = F(x);  v += (dt/2) F/m.
 * With the default Verlet skin of 0 the neighbour list is rebuilt at every
 * force evaluation; with a skin > 0 (nnp_set_md_skin) a list of the atoms
 * within rc + skin is built with a new sort at the first evaluation and
 * whenever some atom has moved more than skin/2 since the last build, and
 * every evaluation in between takes its pairs within rc from that list.  Both
 * give the same forces up to rounding order (a pair within rc at the current
 * positions is always in the skin list, by the triangle inequality).
 *  n_atoms      atoms of one orthorhombic periodic structure
 *  pos, vel     device [n_atoms][3], positions' type of the handle (FP64 for
 *               NNP_FP64, else FP32), A and A/fs; advanced in place by n_steps
 *  forces       device [n_atoms][3], same type; output: F at the final positions
 *  types        device int32 [n_atoms]
 *  box          host double[3], A
 *  masses       host double[n_el], atomic mass units, finite and > 0
 *  dt_fs        time step in fs, finite and > 0
 *  n_steps      steps (>= 0; 0 evaluates the forces of the initial state only)
 *  epot, ekin   host double [n_steps + 1] or NULL: potential and kinetic energy
 *               (eV) of the initial state and after every step
 * Updates are computed in FP64 and rounded once to the positions' type.  Unit
 * conversions come from the CODATA electron volt and atomic mass constant.
 * Synchronises the stream.  Errors as nnp_compute, checked before any step.
 */
nnp_status nnp_md_run(nnp_handle* h, int64_t n_atoms, void* pos, void* vel, void* forces, const int32_t* types,
                      const double box[3], const double* masses, double dt_fs, int n_steps, double* epot,
                      double* ekin, void* stream);

/*
 * Verlet skin of the MD driver, in A (finite, >= 0; 0, the default, rebuilds
 * the neighbour list at every step).  The paper's MD application reuses
 * neighbour lists between steps in the usual way (Sec. 4, the CabanaMD proxy
 * app); this sets how far beyond rc the reused list reaches.  Takes effect
 * at the next nnp_md_run.  NNP_E_ARG for a negative or non-finite skin.
 */
nnp_status nnp_set_md_skin(nnp_handle* h, double skin);

/* Neighbour-list builds (sorts plus list builds) of the last nnp_md_run on
 * this handle: n_steps + 1 with a skin of 0; -1 while another call holds the
 * handle. */
int64_t nnp_md_list_builds(const nnp_handle* h);

/*
 * Level of parallelism of the SF and force passes (the paper's Sec. 4.3
 * question of threading over atoms only or over atoms and neighbours).
 *  NNP_PAR_WAVE    one 64-lane wavefront per centre atom: lanes over its
 *                  neighbours, then over its neighbour pairs.
 *  NNP_PAR_THREAD  one thread per centre atom, walking its neighbours and
 *                  pairs alone (the paper's flat level); kept for comparison.
 *  NNP_PAR_AUTO    (default) the faster level; on this device that is a
 *                  wave per centre for long and short neighbour rows alike.
 *                  Two waves per centre are taken instead for a batch of at
 *                  most 2,048 atoms (too few centres to fill the device
 *                  otherwise) and for a batch whose densest atom has more
 *                  neighbours than one wave per centre can stage in LDS
 *                  (160 KB per workgroup of four centres: from about 310
 *                  neighbours in the FP64 force-adjoint pass to about 730
 *                  in the FP32 force pass; two waves per centre hold two
 *                  centres per workgroup).  Beyond their LDS too, the batch
 *                  takes the thread level.
 *  NNP_PAR_WAVE2   two wavefronts per centre atom (the paper's third level,
 *                  threads over atoms, neighbours and neighbour pairs): both
 *                  share the centre's neighbour records and force sums in
 *                  LDS; the first stages the neighbours, then the two split
 *                  the walk over neighbour pairs and their SF sums are added.
 * NNP_PAR_WAVE or NNP_PAR_WAVE2 with such a batch is NNP_E_ARG, reported
 * before any SF or force kernel is launched.
 * Both give the same results up to rounding order; the force-adjoint pass of
 * nnp_backward follows the same choice.  An unknown mode is NNP_E_ARG.
 */
typedef enum { NNP_PAR_AUTO = 0, NNP_PAR_WAVE = 1, NNP_PAR_THREAD = 2, NNP_PAR_WAVE2 = 3 } nnp_parallelism;
nnp_status nnp_set_parallelism(nnp_handle* h, int mode);

/*
 * Layout of the neighbour list that the wave-level SF, force and
 * force-adjoint passes read (the data-layout question of Sec. 4.3 and
 * Figs. 6-7, asked here of the one structure the pair passes loop over).
 *  NNP_LIST_PADDED   (default) rows of cap slots per atom; an entry is the
 *                    minimum-image displacement r_j - r_i, formed in FP64 and
 *                    rounded once to the arithmetic type, and the index j
 *                    (16 bytes in FP32 and BF16, 32 in FP64).
 *  NNP_LIST_INDEX    rows of cap slots holding the index j alone (4 bytes);
 *                    the pair passes gather the sorted FP64 positions and
 *                    form the same displacement themselves.
 *  NNP_LIST_COMPACT  displacement entries in rows without padding: the build
 *                    counts first, scans the row lengths into offsets (the
 *                    host waits for the total) and writes each row at its
 *                    offset.
 * Results equal those of the padded layout up to rounding order.  The
 * thread-level passes, the stored-Jacobian form, the Verlet-skin MD path and
 * nnp_count_work always use the padded layout; a call that ends up at the
 * thread level rebuilds its list padded.  An unknown layout is NNP_E_ARG.
 */
typedef enum { NNP_LIST_PADDED = 0, NNP_LIST_INDEX = 1, NNP_LIST_COMPACT = 2 } nnp_list_layout;
nnp_status nnp_set_list_layout(nnp_handle* h, int layout);

/*
 * Pair-test masks (on = 1, the default; 0 = off).  The force pass of
 * Sec. 3.1 step 3 walks the same neighbour pairs (j, k) as the SF pass and,
 * without masks, repeats its test r_jk < rc on each.  With masks the SF pass
 * stores one bit per tested pair and the later passes read them.  (The paper's
 * passes store nothing derived from a pair, Sec. 3.3.)  The workspace is
 * about 8 bytes per 64 pairs: n_atoms * ((m^2 + n_el m) / 64 +
 * n_el (n_el + 1) / 2) * 8 bytes, rounded up to 256-byte blocks per atom, for
 * m the most neighbours of any atom.  Masks are used only when all of these
 * hold:
 *  - the pass runs at the wave level with one wave per centre;
 *  - m is at least 64 (shorter rows gain nothing);
 *  - the workspace is at most 16 GiB.
 * The force-adjoint pass of nnp_backward reads the masks of the SF pass whose
 * neighbour list it uses (the forward's, when the backward reuses it).
 * nnp_compute_noalloc never uses them.  Results equal those without masks up
 * to the rounding of the test itself.
 * on outside {0, 1} is NNP_E_ARG.
 */
nnp_status nnp_set_pair_masks(nnp_handle* h, int on);

/*
 * How the differentiation form obtains the SF derivatives dG_is/dr_m.
 *  NNP_DERIV_RECOMPUTE  (default) the force pass and nnp_backward recompute
 *                       them from the neighbour list, as the paper does
 *                       (Sec. 3.3): nothing per pair or triplet is kept.
 *  NNP_DERIV_STORED     every forward evaluation also stores, for each centre
 *                       i, neighbour slot and SF s, the gradient dG_is/dr_j
 *                       (3 * max n_sf * n_atoms * capacity values of the
 *                       positions' type in the handle's workspace); forces are
 *                       a contraction of that store, and nnp_backward with the
 *                       same inputs as the last forward reuses it instead of
 *                       rebuilding the neighbour list and SFs.  Whether the
 *                       inputs are the same is checked (batch layout on the
 *                       host, positions and types bitwise on the device);
 *                       otherwise nnp_backward recomputes the store first.
 * A batch whose densest atom has more neighbours than the store's kernel can
 * stage in LDS is computed with recomputed derivatives instead.
 * NNP_DERIV_STORED needs an NNP_FP64 or NNP_FP32 handle (NNP_E_STATE
 * otherwise); an unknown mode is NNP_E_ARG.  Takes effect at the next call.
 */
typedef enum { NNP_DERIV_RECOMPUTE = 0, NNP_DERIV_STORED = 1 } nnp_deriv_mode;
nnp_status nnp_set_derivative_mode(nnp_handle* h, int mode);

/* Device memory held by the handle's workspace, in bytes (grow-only buffers
 * kept until nnp_destroy; excludes the parameter and table blocks); -1 while
 * another call holds the handle. */
int64_t nnp_workspace_bytes(const nnp_handle* h);

/* Number of network parameters: sum over elements and layers of out*in + out. */
int64_t nnp_n_params(const nnp_handle* h);

/*
 * Replace every network parameter.  flat_params: double [nnp_n_params(h)],
 * element by element, layer by layer, W row-major [out][in] then b[out];
 * on_device != 0 if it is a device pointer.  The device is synchronised first,
 * so that kernels of earlier calls finish with the old parameters.
 */
nnp_status nnp_set_params(nnp_handle* h, const void* flat_params, int on_device);

/* Copy the current parameters (same layout) into host memory. */
nnp_status nnp_get_params(const nnp_handle* h, double* flat_params_host);

/*
 * Per-kernel timing of the last call on this handle, in milliseconds, from
 * HIP events on the caller's stream, when enabled with nnp_set_profiling.
 *  names: receives up to max_k static kernel-stage names; ms: their times.
 * Returns the number of stages written (0 while another call holds the handle).
 */
nnp_status nnp_set_profiling(nnp_handle* h, int enable);
int nnp_last_timings(const nnp_handle* h, const char** names, double* ms, int max_k);

/*
 * Work counts of one evaluation of a structure (same arguments as
 * nnp_compute, no energies or forces), written to host counts[5]:
 *  [0] neighbour entries of the full lists (each unordered pair within rc twice);
 *  [1] unordered pairs (j, k) of neighbours of a centre in element-pair classes
 *      for which the centre has angular SFs (the candidate triplets);
 *  [2] those with r_jk < rc (the triplet terms of the angular loop, Sec. 3.1);
 *  [3] angular SF-term updates: each triplet term times the number of angular
 *      SFs of its (centre, neighbour-pair) class;
 *  [4] radial SF-term updates: each neighbour entry times the number of radial
 *      SFs of its (centre, neighbour) element pair.
 * Used to state algorithmic work per launch.  Synchronises the stream.
 */
nnp_status nnp_count_work(nnp_handle* h, int64_t n_atoms, const void* pos, const int32_t* types,
                          const double box[3], int64_t counts[5], void* stream);

/* Neighbour capacity (slots per atom) currently allocated. */
int nnp_neighbor_capacity(const nnp_handle* h);

/* Override the neighbour capacity (>= 8): the next call starts from it and
 * regrows on overflow. */
nnp_status nnp_set_neighbor_capacity(nnp_handle* h, int cap);

/* Release the handle and all its device memory.  NULL is allowed. */
void nnp_destroy(nnp_handle* h);

/* Readable message of the last error on this handle ("" if none); with a NULL
 * handle, the last error of nnp_create on this thread.  After a call on this
 * thread was refused because the handle was busy, that refusal's message. */
const char* nnp_last_error(const nnp_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* NNP_H */
