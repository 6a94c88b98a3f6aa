// Host layer of the C ABI in include/nnp.h: argument checks, packing of the
// SF table and networks into device blocks, the growable workspace, and the
// kernel sequence of one call on the caller's stream.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nnp.h"
#include "kernels.h"

// Workspace of nnp_compute_noalloc: a static array, one copy per device,
// kept until the process ends.  Host code never passes this name to a kernel
// or a copy (on the host it stands for the device symbol, not an address):
// the device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[NNP_NOALLOC_SCRATCH_BYTES];

namespace nnp {
namespace {

thread_local std::string g_create_error;

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};  // device address of `scratch`, per device

// Device address of the static workspace on device dev (the current device),
// looked up on the first call for that device.
hipError_t scratch_address(int dev, unsigned char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace
}  // namespace nnp

struct nnp_handle {
  int n_el = 0;
  int prec = NNP_FP32;
  int device = 0;
  std::string err;
  double rc = 0.0;
  int variant = 0;                      // triplet-kernel instantiation (see launch_mode)
  std::vector<int> n_sf;                // per element
  std::vector<std::vector<int>> sizes;  // per element layer widths
  std::vector<double> params;           // flat caller layout
  std::vector<int> flatmap;             // flat index -> padded index
  nnp::DevTab<double> tab_d;            // host copy (double)
  // device parameter blocks
  void* d_tab = nullptr;                // DevTab<T>
  void* d_nets = nullptr;               // [n_el][NET_STRIDE] T
  int* d_flatmap = nullptr;
  // workspace
  std::map<std::string, nnp::DevBuf> ws;
  int cap = 0;                          // neighbour slots per atom
  int lcap = 0;                         // most neighbours of any atom in the last build, rounded up
  int cap_override = 0;
  // pinned staging for small uploads / readbacks
  void* h_stage = nullptr;
  size_t h_stage_bytes = 0;
  int* h_flags = nullptr;               // pinned [4]
  double* h_energy = nullptr;           // pinned [1]
  // profiling
  bool prof = false;
  std::vector<const char*> t_names;
  std::vector<double> t_ms;
  std::vector<hipEvent_t> events;
  bool has_forward = false;
  int parallelism = NNP_PAR_AUTO;        // SF and force passes: wave or thread per centre
  bool has_wide = false;                 // the table holds wide angular SFs (thread-per-centre passes only)
  int deriv_mode = NNP_DERIV_RECOMPUTE;
  // The last batch forward's inputs, for nnp_backward: while fwd_valid, the
  // workspace holds that forward's sorted order, neighbour list and G~ (and
  // its J store in the stored-Jacobian mode).
  bool fwd_valid = false;
  int fwd_cap = 0;
  std::vector<int64_t> fwd_offs;
  std::vector<double> fwd_boxes;
  std::atomic<int> busy{0};              // an ABI call is running on this handle
  // MD driver: Verlet skin (A; 0 = rebuild the list at every step), the skin
  // list's state and capacity, and the neighbour-list builds of the last run
  int list_layout = NNP_LIST_PADDED;     // of the wave-level passes with recomputed derivatives
  int pair_masks = 1;                    // SF pass records its pair tests for the force pass
  unsigned* fwd_pm = nullptr;            // the masks the last SF pass wrote, and their stride
  int fwd_pm_stride = 0;                 // (0: none; valid with the forward's list, fwd_valid)
  size_t compact_entries = 0;            // entries of the last compact list
  int fwd_layout = NNP_LIST_PADDED;      // layout of the list the last batch forward left
  double md_skin = 0.0;
  bool skin_ok = false;
  int scap = 0;
  int64_t md_builds = 0;
  // nnp_compute_noalloc: while arena_on, named buffers are carved from the
  // device's static workspace (bump order, reset at every such call) instead
  // of the handle's own allocations, and nothing is allocated.
  unsigned char* scratch = nullptr;      // this device's copy of the static workspace
  bool arena_on = false;
  size_t arena_used = 0;
  std::map<std::string, nnp::DevBuf> arena_bufs;
};

namespace nnp {
namespace {

nnp_status fail(nnp_handle* h, nnp_status st, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return st;
}

// A call refused because its handle was busy reports through these (per host
// thread): the running call owns the handle's own message.
thread_local const nnp_handle* t_busy_handle = nullptr;
thread_local std::string t_busy_error;

// Holds the handle for the duration of one ABI call.  A call that overlaps
// another on the same handle (from a second host thread) is refused with
// NNP_E_STATE before it reads or writes any of the handle's state.
struct Claim {
  nnp_handle* h;
  bool ok;
  explicit Claim(nnp_handle* h_) : h(h_) {
    int idle = 0;
    ok = h->busy.compare_exchange_strong(idle, 1, std::memory_order_acquire);
    if (ok) {
      t_busy_handle = nullptr;
      h->err.clear();
    } else {
      t_busy_handle = h;
      t_busy_error = "the handle is in use by another call (one host thread and one stream at a time)";
    }
  }
  ~Claim() {
    if (ok) h->busy.store(0, std::memory_order_release);
  }
  Claim(const Claim&) = delete;
  Claim& operator=(const Claim&) = delete;
};

#define NNP_HIP(h, call)                                                                             \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess)                                                                             \
      return fail(h, e_ == hipErrorOutOfMemory ? NNP_E_NOMEM : NNP_E_HIP,                             \
                  std::string(#call) + ": " + hipGetErrorString(e_));                                 \
  } while (0)

// Error of the last launches on this thread, if any.
nnp_status check_launch(nnp_handle* h, const char* stage) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, NNP_E_HIP, std::string(stage) + ": " + hipGetErrorString(e));
  return NNP_OK;
}

// Largest dynamic LDS a workgroup may use on the current device.
size_t lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
  return (size_t)v;
}

// Named buffer of the static workspace (no allocation): reused while large
// enough, grown in place if it is the last one carved, else carved anew.
nnp_status ensure_arena(nnp_handle* h, const char* name, size_t bytes, void** out) {
  DevBuf& b = h->arena_bufs[name];
  if (b.bytes < bytes) {
    const size_t nb = (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
    const bool last = b.p && static_cast<unsigned char*>(b.p) + b.bytes == h->scratch + h->arena_used;
    const size_t start = last ? (size_t)(static_cast<unsigned char*>(b.p) - h->scratch) : h->arena_used;
    if (start + nb > (size_t)NNP_NOALLOC_SCRATCH_BYTES)
      return fail(h, NNP_E_NOMEM, std::string("the call needs more than the ") +
                                      std::to_string((long long)NNP_NOALLOC_SCRATCH_BYTES) +
                                      " bytes of the static workspace (buffer " + name + ")");
    b.p = h->scratch + start;
    b.bytes = nb;
    h->arena_used = start + nb;
  }
  *out = b.p;
  return NNP_OK;
}

// Grow-only named device buffer.
nnp_status ensure(nnp_handle* h, const char* name, size_t bytes, void** out) {
  if (h->arena_on) return ensure_arena(h, name, bytes, out);
  DevBuf& b = h->ws[name];
  if (b.bytes < bytes) {
    if (b.p) {
      // an earlier call may have returned with kernels still using the buffer
      hipError_t e = hipDeviceSynchronize();
      if (e == hipSuccess) e = hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
      if (e != hipSuccess) return fail(h, NNP_E_HIP, std::string("hipFree: ") + hipGetErrorString(e));
    }
    size_t nb = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, nb);
    if (e != hipSuccess) {
      b.p = nullptr;
      return fail(h, NNP_E_NOMEM, std::string("hipMalloc(") + name + ", " + std::to_string(nb) + "): " +
                                      hipGetErrorString(e));
    }
    b.bytes = nb;
  }
  *out = b.p;
  return NNP_OK;
}

template <class X>
nnp_status ensure_t(nnp_handle* h, const char* name, size_t count, X** out) {
  void* p = nullptr;
  nnp_status st = ensure(h, name, count * sizeof(X), &p);
  *out = reinterpret_cast<X*>(p);
  return st;
}

nnp_status stage(nnp_handle* h, size_t bytes) {
  if (h->h_stage_bytes >= bytes) return NNP_OK;
  if (h->arena_on) return fail(h, NNP_E_NOMEM, "the batch description exceeds the pinned staging block");
  if (h->h_stage) (void)hipHostFree(h->h_stage);
  h->h_stage = nullptr;
  h->h_stage_bytes = 0;
  NNP_HIP(h, hipHostMalloc(&h->h_stage, std::max<size_t>(bytes, 4096), hipHostMallocDefault));
  h->h_stage_bytes = std::max<size_t>(bytes, 4096);
  return NNP_OK;
}

template <class T>
DevTab<T> convert_tab(const DevTab<double>& s) {
  DevTab<T> t;
  std::memset(&t, 0, sizeof(t));
  t.n_el = s.n_el;
  for (int e = 0; e < MAX_EL; ++e) t.n_sf[e] = s.n_sf[e];
  t.rc2 = (T)s.rc2;
  t.inv_rc2 = (T)s.inv_rc2;
  for (int e = 0; e < MAX_EL; ++e) {
    for (int f = 0; f < MAX_EL; ++f) {
      t.rad_cnt[e][f] = s.rad_cnt[e][f];
      for (int k = 0; k < MAX_RAD; ++k) {
        t.rad_eta[e][f][k] = (T)s.rad_eta[e][f][k];
        t.rad_rs[e][f][k] = (T)s.rad_rs[e][f][k];
        t.rad_out[e][f][k] = s.rad_out[e][f][k];
      }
    }
    t.n_eta[e] = s.n_eta[e];
    for (int n = 0; n < MAX_NE; ++n) {
      t.aeta[e][n] = (T)s.aeta[e][n];
      t.aeta2[e][n] = (T)s.aeta2[e][n];
    }
    for (int c = 0; c < MAX_CLS; ++c) {
      t.ang_cnt[e][c] = s.ang_cnt[e][c];
      for (int k = 0; k < MAX_ANG; ++k) {
        t.ang_bit[e][c][k] = s.ang_bit[e][c][k];
        t.ang_pre[e][c][k] = (T)s.ang_pre[e][c][k];
        t.ang_out[e][c][k] = s.ang_out[e][c][k];
        t.ang_wide[e][c][k] = s.ang_wide[e][c][k];
      }
    }
    for (int c = 0; c < MAX_CLS; ++c)
      for (int b = 0; b < 12 * MAX_NE; ++b) {
        t.qn_out[e][c][b] = s.qn_out[e][c][b];
        t.qn_pre[e][c][b] = (T)s.qn_pre[e][c][b];
      }
    for (int k = 0; k < MAX_SF; ++k) {
      t.shift_d[e][k] = s.shift_d[e][k];
      t.inv_scale_d[e][k] = s.inv_scale_d[e][k];
    }
  }
  return t;
}

// Upload the padded networks (type T) from the flat caller layout.
template <class T>
nnp_status upload_nets(nnp_handle* h) {
  std::vector<T> pad((size_t)h->n_el * NET_STRIDE, T(0));
  for (size_t i = 0; i < h->params.size(); ++i) pad[h->flatmap[i]] = (T)h->params[i];
  if (!h->d_nets) NNP_HIP(h, hipMalloc(&h->d_nets, pad.size() * sizeof(T)));
  NNP_HIP(h, hipMemcpy(h->d_nets, pad.data(), pad.size() * sizeof(T), hipMemcpyHostToDevice));
  return NNP_OK;
}

nnp_status upload_params(nnp_handle* h) {
  if (h->prec == NNP_FP64) return upload_nets<double>(h);
  return upload_nets<float>(h);
}

// ------------------------------------------------------------------ batch
struct Batch {
  int n_struct = 0;
  int64_t n = 0;
  std::vector<DevStruct> st;
  std::vector<int64_t> soff;
  int total_cells = 0;
  std::vector<int64_t> chunk_lo, chunk_hi;
  std::vector<int> struct_chunk;
};

// Batch description; cells have edge >= rcell (default: the cutoff).
nnp_status make_batch(nnp_handle* h, int n_struct, const int64_t* offs, const double* boxes, Batch& B,
                      double rcell = 0.0) {
  if (rcell <= 0.0) rcell = h->rc;
  if (n_struct < 1) return fail(h, NNP_E_ARG, "n_struct must be >= 1");
  if (!offs || !boxes) return fail(h, NNP_E_ARG, "atom_offsets and boxes must not be NULL");
  if (offs[0] != 0) return fail(h, NNP_E_ARG, "atom_offsets[0] must be 0");
  B.n_struct = n_struct;
  B.soff.assign(offs, offs + n_struct + 1);
  B.n = offs[n_struct];
  if (B.n > (int64_t)INT32_MAX / 2) return fail(h, NNP_E_ARG, "too many atoms");
  int64_t cells = 0;
  const int64_t chunk = 4096;
  for (int b = 0; b < n_struct; ++b) {
    if (offs[b + 1] < offs[b]) return fail(h, NNP_E_ARG, "atom_offsets must be non-decreasing");
    DevStruct s;
    std::memset(&s, 0, sizeof(s));
    const int64_t nb = offs[b + 1] - offs[b];
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
      const double L = boxes[3 * b + a];
      if (!std::isfinite(L) || !(L > 2.0 * h->rc))
        return fail(h, NNP_E_BOX, "box edge " + std::to_string(L) + " of structure " + std::to_string(b) +
                                      " must be finite and exceed 2 rc = " + std::to_string(2.0 * h->rc));
      s.L[a] = L;
      s.invL[a] = 1.0 / L;
      s.ncell[a] = std::max(1, (int)std::floor(L / rcell));
      ncell *= s.ncell[a];
    }
    // Bound the cell count of sparse boxes: coarser cells stay >= rc.
    const int64_t limit = std::max<int64_t>(64, 8 * nb);
    while (ncell > limit) {
      ncell = 1;
      for (int a = 0; a < 3; ++a) {
        s.ncell[a] = std::max(1, s.ncell[a] / 2);
        ncell *= s.ncell[a];
      }
    }
    s.cellbase = (int)cells;
    s.off = offs[b];
    s.n = nb;
    cells += ncell;
    if (cells * h->n_el > (int64_t)1 << 28) return fail(h, NNP_E_ARG, "too many cells");
    B.st.push_back(s);
    B.struct_chunk.push_back((int)B.chunk_lo.size());
    for (int64_t c0 = offs[b]; c0 < offs[b + 1]; c0 += chunk) {
      B.chunk_lo.push_back(c0);
      B.chunk_hi.push_back(std::min(offs[b + 1], c0 + chunk));
    }
  }
  B.struct_chunk.push_back((int)B.chunk_lo.size());
  B.total_cells = (int)cells;
  return NNP_OK;
}

// Profiling marks on the caller's stream.
struct Marks {
  nnp_handle* h;
  hipStream_t s;
  int k = 0;
  Marks(nnp_handle* h_, hipStream_t s_) : h(h_), s(s_) {
    h->t_names.clear();
    h->t_ms.clear();
    if (h->prof) mark(nullptr);
  }
  void mark(const char* name) {
    if (!h->prof) return;
    if ((int)h->events.size() <= k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      h->events.push_back(e);
    }
    (void)hipEventRecord(h->events[k], s);
    if (name) h->t_names.push_back(name);
    ++k;
  }
  void finish() {
    if (!h->prof) return;
    for (int i = 0; i + 1 < k && i < (int)h->t_names.size(); ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, h->events[i], h->events[i + 1]);
      h->t_ms.push_back(ms);
    }
  }
};

// Neighbour capacity from the densest structure: mean count * 1.2 + 16,
// rounded up to a multiple of 16 (a denser spot triggers a regrow).
int initial_cap(nnp_handle* h, const Batch& B) {
  if (h->cap_override) return h->cap_override;
  double rho = 0.0;
  for (const auto& s : B.st) rho = std::max(rho, (double)s.n / (s.L[0] * s.L[1] * s.L[2]));
  const double mean = rho * 4.0 / 3.0 * M_PI * h->rc * h->rc * h->rc;
  int cap = (int)std::ceil(mean * 1.2 + 16.0);
  cap = (cap + 15) / 16 * 16;
  return std::max(cap, std::max(h->cap, 32));
}

struct Common {
  Batch B;
  int64_t* d_soff = nullptr;
  DevStruct* d_st = nullptr;
  int64_t* d_clo = nullptr;
  int64_t* d_chi = nullptr;
  int* d_sc = nullptr;
  BinArgs bin;
  int layout = NNP_LIST_PADDED;
  void* nbr = nullptr;   // [n][cap] Vec4<T> entries of the form's arithmetic type (compact: at roff)
  int* idx = nullptr;    // index layout: [n][cap] neighbour indices
  int* roff = nullptr;   // compact layout: [n + 1] row offsets
  int4* nnb = nullptr;
};

// Uploads the batch description and runs wrap + bin + counting sort.
// With sort = false the buffers are only bound (their contents are those of
// the last sorted batch) and nothing is launched.
template <class IO>
nnp_status prepare(nnp_handle* h, Common& cm, const IO* pos, const int32_t* types, hipStream_t stream,
                   bool sort = true) {
  Batch& B = cm.B;
  const int64_t n = B.n;
  const int nkeys = h->n_el * B.total_cells;
  nnp_status st;
  const size_t nst = B.st.size(), nso = B.soff.size(), nch = B.chunk_lo.size(), nsc = B.struct_chunk.size();
  // The batch description goes up in one copy: its five arrays are packed,
  // 16-byte aligned, into one pinned staging block and one device block.
  auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
  const size_t o_st = 0, o_soff = o_st + al(nst * sizeof(DevStruct)), o_clo = o_soff + al(nso * sizeof(int64_t)),
               o_chi = o_clo + al(std::max<size_t>(nch, 1) * sizeof(int64_t)),
               o_sc = o_chi + al(std::max<size_t>(nch, 1) * sizeof(int64_t)), bytes = o_sc + al(nsc * sizeof(int));
  unsigned char* d_desc = nullptr;
  if ((st = ensure_t(h, "batch_desc", bytes, &d_desc))) return st;
  if ((st = stage(h, bytes))) return st;
  unsigned char* hs = (unsigned char*)h->h_stage;
  std::memcpy(hs + o_st, B.st.data(), nst * sizeof(DevStruct));
  std::memcpy(hs + o_soff, B.soff.data(), nso * sizeof(int64_t));
  if (nch) {
    std::memcpy(hs + o_clo, B.chunk_lo.data(), nch * sizeof(int64_t));
    std::memcpy(hs + o_chi, B.chunk_hi.data(), nch * sizeof(int64_t));
  }
  std::memcpy(hs + o_sc, B.struct_chunk.data(), nsc * sizeof(int));
  NNP_HIP(h, hipMemcpyAsync(d_desc, hs, bytes, hipMemcpyHostToDevice, stream));
  cm.d_st = reinterpret_cast<DevStruct*>(d_desc + o_st);
  cm.d_soff = reinterpret_cast<int64_t*>(d_desc + o_soff);
  cm.d_clo = reinterpret_cast<int64_t*>(d_desc + o_clo);
  cm.d_chi = reinterpret_cast<int64_t*>(d_desc + o_chi);
  cm.d_sc = reinterpret_cast<int*>(d_desc + o_sc);

  BinArgs& a = cm.bin;
  a.n = n;
  a.types = types;
  a.st = cm.d_st;
  a.soff = cm.d_soff;
  a.n_struct = B.n_struct;
  a.n_el = h->n_el;
  a.total_cells = B.total_cells;
  if ((st = ensure_t(h, "key", std::max<int64_t>(n, 1), &a.key))) return st;
  if ((st = ensure_t(h, "count", nkeys + 1, &a.count))) return st;
  if ((st = ensure_t(h, "start", nkeys + 1, &a.start))) return st;
  if ((st = ensure_t(h, "cursor", nkeys + 1, &a.cursor))) return st;
  if ((st = ensure_t(h, "scan", nkeys / 4096 + 1, &a.scan))) return st;
  if ((st = ensure_t(h, "perm", std::max<int64_t>(n, 1), &a.perm))) return st;
  if ((st = ensure_t(h, "perm_raw", std::max<int64_t>(n, 1), &a.perm_raw))) return st;
  if ((st = ensure_t(h, "pos4", std::max<int64_t>(n, 1), &a.pos4))) return st;
  if ((st = ensure_t(h, "eoff", MAX_EL + 1, &a.eoff))) return st;
  if ((st = ensure_t(h, "flags", 4, &a.flags))) return st;
  if (!sort) return NNP_OK;
  h->fwd_valid = false;  // the sorted order, neighbour list, G~ and J store are about to change
  h->fwd_pm = nullptr;   // and so are the pair-test masks
  h->fwd_pm_stride = 0;
  h->skin_ok = false;    // and the Verlet-skin list with them
  launch_fill_int(a.flags, 4, 0, stream);
  launch_bin_sort<IO>(a, pos, stream);
  return NNP_OK;
}

// Binds the neighbour list of the given layout that the workspace holds
// (padded entries, index entries, or compact entries with their offsets).
template <class T>
nnp_status bind_neighbors(nnp_handle* h, Common& cm, int layout = NNP_LIST_PADDED) {
  using E = typename Vec4<T>::type;
  nnp_status st;
  const int64_t n = std::max<int64_t>(cm.B.n, 1);
  cm.layout = layout;
  cm.nbr = nullptr;
  cm.idx = nullptr;
  cm.roff = nullptr;
  if ((st = ensure_t(h, "nnb", n, &cm.nnb))) return st;
  if (layout == NNP_LIST_INDEX) return ensure_t(h, "nbr_idx", (size_t)n * h->cap, &cm.idx);
  E* nbr = nullptr;
  if (layout == NNP_LIST_COMPACT) {
    if ((st = ensure_t(h, "roff", (size_t)n + 1, &cm.roff))) return st;
    if ((st = ensure_t(h, "nbr", std::max<size_t>(h->compact_entries, 1), &nbr))) return st;
  } else if ((st = ensure_t(h, "nbr", (size_t)n * h->cap, &nbr))) {
    return st;
  }
  cm.nbr = nbr;
  return NNP_OK;
}

// The neighbour build in the given layout.  The compact layout counts first,
// scans the row lengths and reads the total back (a host wait) to size the
// list, then writes it; its rows never overflow.
template <class T>
nnp_status build_neighbors(nnp_handle* h, Common& cm, hipStream_t stream, int layout = NNP_LIST_PADDED) {
  using E = typename Vec4<T>::type;
  nnp_status st;
  const int64_t n = std::max<int64_t>(cm.B.n, 1);
  int* cmax = nullptr;
  if ((st = ensure_t(h, "cmax", std::max(cm.B.total_cells, 1), &cmax))) return st;
  launch_fill_int(cm.bin.flags + 1, 2, 0, stream);
  if (layout == NNP_LIST_COMPACT) {
    int *len, *tmp, *part, *roff;
    int4* nnb;
    if ((st = ensure_t(h, "nnb", n, &nnb))) return st;
    if ((st = ensure_t(h, "roff", (size_t)n + 1, &roff))) return st;
    if ((st = ensure_t(h, "row_len", n, &len))) return st;
    if ((st = ensure_t(h, "row_tmp", n, &tmp))) return st;
    if ((st = ensure_t(h, "row_part", n / 4096 + 1, &part))) return st;
    if (cm.B.n > 0) {
      launch_neighbor_counts<T>(cm.bin, h->rc, nnb, cmax, stream);
      launch_row_offsets(cm.B.n, nnb, len, roff, tmp, part, stream);
      int total = 0;
      NNP_HIP(h, hipMemcpyAsync(h->h_flags, roff + cm.B.n, sizeof(int), hipMemcpyDeviceToHost, stream));
      NNP_HIP(h, hipStreamSynchronize(stream));
      total = h->h_flags[0];
      if (total < 0) return fail(h, NNP_E_ARG, "too many neighbour entries for the compact layout");
      h->compact_entries = (size_t)total;
    } else {
      h->compact_entries = 0;
    }
    if ((st = bind_neighbors<T>(h, cm, layout))) return st;
    launch_neighbors_compact<T>(cm.bin, h->rc, cm.roff, reinterpret_cast<E*>(cm.nbr), cm.nnb, cmax, stream);
    return NNP_OK;
  }
  if ((st = bind_neighbors<T>(h, cm, layout))) return st;
  if (layout == NNP_LIST_INDEX) launch_neighbor_index(cm.bin, h->rc, h->cap, cm.idx, cm.nnb, cmax, stream);
  else launch_neighbors<T>(cm.bin, h->rc, h->cap, reinterpret_cast<E*>(cm.nbr), cm.nnb, cmax, stream);
  return NNP_OK;
}

template <int P>
TripArgs<P> trip_args(nnp_handle* h, Common& cm) {
  TripArgs<P> t;
  std::memset(&t, 0, sizeof(t));
  t.n = cm.B.n;
  t.cap = h->cap;
  t.lcap = h->lcap;
  t.pos4 = cm.bin.pos4;
  t.nbr = reinterpret_cast<const typename Vec4<typename Types<P>::T>::type*>(cm.nbr);
  t.idx = cm.idx;
  t.roff = cm.roff;
  t.wpc = 1;  // set with the level (use_flat)
  t.nnb = cm.nnb;
  t.st = cm.d_st;
  t.tab = reinterpret_cast<const DevTab<typename Types<P>::T>*>(h->d_tab);
  return t;
}

// Reads back the flags after a neighbour build; returns 1 if the neighbour
// capacity overflowed (cap has been grown: rebuild), 0 if all is well (lcap
// then bounds every atom's count), <0 on error.
int check_flags(nnp_handle* h, hipStream_t stream, Common& cm, nnp_status* st) {
  hipError_t e = hipMemcpyAsync(h->h_flags, cm.bin.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    *st = fail(h, NNP_E_HIP, std::string("readback: ") + hipGetErrorString(e));
    return -1;
  }
  if (h->h_flags[0] & 1) {
    *st = fail(h, NNP_E_TYPE, "atom type outside [0, n_el)");
    return -1;
  }
  if (h->h_flags[0] & 2) {
    *st = fail(h, NNP_E_ARG, "non-finite atom position (NaN or infinity)");
    return -1;
  }
  if (h->h_flags[1] > h->cap) {
    int nc = (int)std::ceil(h->h_flags[1] * 1.15) + 8;
    h->cap = (nc + 15) / 16 * 16;
    return 1;
  }
  const int most = std::max(h->h_flags[2], 1);
  h->lcap = std::min(h->cap, (most + 7) / 8 * 8);
  return 0;
}

// Level of the pair passes of modes mode_a and mode_b (0 SF, 1 force, 2
// force-adjoint product): *flat for a thread per centre, else *wpc waves per
// centre.  A thread per centre when asked for or when the table holds wide
// angular SFs; the wave levels when asked for, refused before any launch if
// an atom has more neighbours than they can stage in LDS.  NNP_PAR_AUTO
// takes one wave per centre (measured the fastest on both workloads, short
// rows included); for an atom beyond its LDS, two waves per centre (a
// workgroup then holds two centres, not four), and beyond that the thread
// level, which reads the rows from HBM.  Small batches take two waves per
// centre under NNP_PAR_AUTO (AUTO_WAVE2_ATOMS).
// Batches of at most this many atoms take two waves per centre under
// NNP_PAR_AUTO: with fewer than 8 centres per CU the second wave of each
// centre fills the machine (measured on water: 192 and 1,536 atoms 5-20 %
// faster SF and force passes, 12,288 atoms 12 % slower).
constexpr int64_t AUTO_WAVE2_ATOMS = 2048;
// Largest pair-mask buffer (n atoms x pair_step_bound(lcap) steps, 8 bytes each);
// beyond it the force pass tests the pairs itself.
constexpr size_t PAIR_MASK_MAX_BYTES = (size_t)16 << 30;
// Masks pay when rows are long: measured at 2M water atoms (112 neighbours
// at most) the step is 7 % faster with them, on the 1.5M-atom fcc metal (24)
// 1.4 % slower.  They are used from this many neighbours on.
constexpr int PAIR_MASK_MIN_NEIGHBORS = 64;

template <int P>
nnp_status use_flat(nnp_handle* h, int mode_a, int mode_b, bool* flat, int* wpc = nullptr, int64_t n_atoms = -1) {
  int w = h->parallelism == NNP_PAR_WAVE2 ||
                  (h->parallelism == NNP_PAR_AUTO && n_atoms >= 0 && n_atoms <= AUTO_WAVE2_ATOMS)
              ? 2
              : 1;
  if (wpc) *wpc = w;
  *flat = h->parallelism == NNP_PAR_THREAD || h->has_wide;
  if (*flat) return NNP_OK;
  auto lds_of = [&](int k) {
    return std::max(triplet_lds_bytes<P>(mode_a, h->variant, h->lcap, k),
                    triplet_lds_bytes<P>(mode_b, h->variant, h->lcap, k));
  };
  const size_t lds = lds_of(w);
  if (lds <= lds_limit()) return NNP_OK;
  if (h->parallelism == NNP_PAR_WAVE || h->parallelism == NNP_PAR_WAVE2)
    return fail(h, NNP_E_ARG, "an atom with " + std::to_string(h->lcap) + " neighbours needs " + std::to_string(lds) +
                                  " bytes of LDS per workgroup at the wave level, more than the device allows");
  if (lds_of(2) <= lds_limit()) {
    if (wpc) *wpc = 2;
    return NNP_OK;
  }
  *flat = true;
  return NNP_OK;
}

// The stored-Jacobian form applies to the FP64 and FP32 handles, and to
// batches whose densest atom its kernel can stage in LDS; otherwise the
// call recomputes the derivatives.
template <int P>
bool use_store(const nnp_handle* h) {
  if constexpr (P == P_BF16) {
    return false;
  } else {
    return h->deriv_mode == NNP_DERIV_STORED && !h->arena_on && jac_lds_bytes<P>(h->lcap) <= lds_limit();
  }
}

// Layout of the neighbour list for the next build: the handle's choice where
// only wave-level passes with recomputed derivatives will read it, otherwise
// the padded entries every pass reads.
template <int P>
int list_layout(const nnp_handle* h) {
  if (h->list_layout == NNP_LIST_PADDED || h->parallelism == NNP_PAR_THREAD || h->has_wide) return NNP_LIST_PADDED;
  if (h->deriv_mode == NNP_DERIV_STORED && P != P_BF16) return NNP_LIST_PADDED;
  return h->list_layout;
}

template <int P>
nnp_status jac_setup(nnp_handle* h, Common& cm, JacArgs<P>& j) {
  using T = typename Types<P>::T;
  std::memset(&j, 0, sizeof(j));
  int ns_max = 1;
  for (int e = 0; e < h->n_el; ++e) ns_max = std::max(ns_max, h->n_sf[e]);
  const int64_t n1 = std::max<int64_t>(cm.B.n, 1);
  j.n = cm.B.n;
  j.cap = h->cap;
  j.lcap = h->lcap;
  j.wide = h->has_wide ? 1 : 0;
  j.nbr = reinterpret_cast<const typename Vec4<T>::type*>(cm.nbr);
  j.nnb = cm.nnb;
  j.pos4 = cm.bin.pos4;
  j.tab = reinterpret_cast<const DevTab<T>*>(h->d_tab);
  j.plane = n1 * h->cap;
  return ensure_t(h, "J", (size_t)3 * ns_max * j.plane, &j.J);
}

// Keeps a copy of the inputs whose sorted order, neighbour list and G~ (and
// J store) are now in the workspace.
template <class IO>
nnp_status fwd_remember(nnp_handle* h, const Common& cm, const IO* pos, const int32_t* types, hipStream_t stream) {
  const int64_t n = cm.B.n;
  IO* sp;
  int32_t* stp;
  nnp_status st;
  if ((st = ensure_t(h, "jpos", (size_t)std::max<int64_t>(n, 1) * 3, &sp))) return st;
  if ((st = ensure_t(h, "jtypes", (size_t)std::max<int64_t>(n, 1), &stp))) return st;
  if (n > 0) {
    NNP_HIP(h, hipMemcpyAsync(sp, pos, (size_t)n * 3 * sizeof(IO), hipMemcpyDeviceToDevice, stream));
    NNP_HIP(h, hipMemcpyAsync(stp, types, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
  }
  h->fwd_offs.assign(cm.B.soff.begin(), cm.B.soff.end());
  h->fwd_boxes.clear();
  for (const auto& d : cm.B.st) h->fwd_boxes.insert(h->fwd_boxes.end(), d.L, d.L + 3);
  h->fwd_cap = h->cap;
  h->fwd_layout = cm.layout;
  return NNP_OK;
}

// True if the workspace still holds the forward results of exactly these
// inputs (same batch layout, same capacity, bitwise equal positions and
// types, compared on the device; the host waits for that one flag).  Binds
// the sorted-order buffers of cm either way.
template <class IO>
bool fwd_reusable(nnp_handle* h, Common& cm, const IO* pos, const int32_t* types, hipStream_t stream,
                  nnp_status* st) {
  *st = NNP_OK;
  if (!h->fwd_valid || h->fwd_cap != h->cap) return false;
  if (h->fwd_offs.size() != cm.B.soff.size() ||
      !std::equal(h->fwd_offs.begin(), h->fwd_offs.end(), cm.B.soff.begin()))
    return false;
  std::vector<double> boxes;
  for (const auto& d : cm.B.st) boxes.insert(boxes.end(), d.L, d.L + 3);
  if (boxes != h->fwd_boxes) return false;
  IO* sp;
  int32_t* stp;
  if ((*st = ensure_t(h, "jpos", (size_t)std::max<int64_t>(cm.B.n, 1) * 3, &sp))) return false;
  if ((*st = ensure_t(h, "jtypes", (size_t)std::max<int64_t>(cm.B.n, 1), &stp))) return false;
  if ((*st = prepare<IO>(h, cm, pos, types, stream, false))) return false;
  launch_fill_int(cm.bin.flags + 3, 1, 0, stream);
  launch_same_inputs<IO>(cm.B.n, pos, sp, types, stp, cm.bin.flags + 3, stream);
  hipError_t e = hipMemcpyAsync(h->h_flags + 3, cm.bin.flags + 3, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    *st = fail(h, NNP_E_HIP, std::string("readback: ") + hipGetErrorString(e));
    return false;
  }
  return h->h_flags[3] == 0;
}

// Buffers of one forward evaluation (sorted order unless stated).
// Pair-test masks for an SF pass at the wave level (ta.wpc set), when they are
// switched on and pay (rows of PAIR_MASK_MIN_NEIGHBORS or more) and fit:
// sets ta.pm and ta.pm_stride, and remembers them for the passes that read
// them (the force pass, and the backward's force-adjoint pass while the
// forward's list is reused).
template <int P>
nnp_status pair_mask_buffer(nnp_handle* h, int64_t n, TripArgs<P>& ta) {
  h->fwd_pm = nullptr;
  h->fwd_pm_stride = 0;
  if (ta.wpc != 1 || !h->pair_masks || h->arena_on || h->lcap < PAIR_MASK_MIN_NEIGHBORS) return NNP_OK;
  const int blocks = (pair_step_bound(h->lcap, h->n_el) + 31) / 32;
  const size_t words = (size_t)n * blocks * WAVE;
  if (words * sizeof(unsigned) > PAIR_MASK_MAX_BYTES) return NNP_OK;
  nnp_status st;
  if ((st = ensure_t(h, "pair_masks", words, &ta.pm))) return st;
  ta.pm_stride = blocks;
  h->fwd_pm = ta.pm;
  h->fwd_pm_stride = blocks;
  return NNP_OK;
}

template <int P>
struct FwdBufs {
  using IO = typename Types<P>::IO;
  using FAcc = typename Types<P>::FAcc;
  IO *G = nullptr, *C = nullptr, *Ei_s = nullptr;
  FAcc* F_s = nullptr;
  double *Ei_o = nullptr, *partial = nullptr, *energies = nullptr;  // Ei_o in caller order
};

template <int P>
nnp_status fwd_buffers(nnp_handle* h, const Common& cm, int n_struct, FwdBufs<P>& b) {
  nnp_status st;
  const int64_t n1 = std::max<int64_t>(cm.B.n, 1);
  if ((st = ensure_t(h, "G", (size_t)n1 * LD, &b.G))) return st;
  if ((st = ensure_t(h, "C", (size_t)n1 * LD, &b.C))) return st;
  if ((st = ensure_t(h, "Ei_s", n1, &b.Ei_s))) return st;
  if ((st = ensure_t(h, "F_s", (size_t)n1 * 3, &b.F_s))) return st;
  if ((st = ensure_t(h, "Ei_o", n1, &b.Ei_o))) return st;
  if ((st = ensure_t(h, "partial", std::max<size_t>(cm.B.chunk_lo.size(), 1), &b.partial))) return st;
  if ((st = ensure_t(h, "energies", n_struct, &b.energies))) return st;
  return NNP_OK;
}

// Everything after the neighbour list (held in cm, with h->lcap set): SF,
// networks and dE/dG, forces, outputs in the caller's order and the energies.
template <int P>
nnp_status evaluate(nnp_handle* h, Common& cm, Marks& mk, const FwdBufs<P>& b, int n_struct,
                    const typename Types<P>::IO* pos, const int32_t* types, double* energies_dev, double* energy_host,
                    void* ei_v, void* f_v, hipStream_t stream, bool remember) {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  using FAcc = typename Types<P>::FAcc;
  nnp_status st;
  const int64_t n = cm.B.n;
  TripArgs<P> ta = trip_args<P>(h, cm);
  MlpArgs<P> ma;
  std::memset(&ma, 0, sizeof(ma));
  ma.n = n;
  ma.n_el = h->n_el;
  ma.eoff = cm.bin.eoff;
  ma.G = b.G;
  ma.C = b.C;
  ma.Ei = b.Ei_s;
  ma.nets = reinterpret_cast<const T*>(h->d_nets);
  ma.tab = ta.tab;
  const bool store = use_store<P>(h);
  if constexpr (P != P_BF16) {
    if (store) {
      JacArgs<P> ja;
      if ((st = jac_setup<P>(h, cm, ja))) return st;
      ja.G = b.G;
      launch_jac<P>(ja, stream);
      mk.mark("sf");
      launch_fill<FAcc>(b.F_s, n * 3, FAcc(0), stream);
      launch_mlp<P>(ma, stream);
      mk.mark("mlp");
      ja.C = b.C;
      ja.F = b.F_s;
      launch_jac_force<P>(ja, stream);
      mk.mark("force");
    }
  }
  if (!store) {
    bool flat = false;
    if ((st = use_flat<P>(h, 0, 1, &flat, &ta.wpc, n))) return st;
    if (!flat && (st = pair_mask_buffer<P>(h, n, ta))) return st;
    ta.G = b.G;
    if (flat) launch_flat<P>(0, ta, stream);
    else launch_triplet<P>(0, h->variant, ta, stream);
    mk.mark("sf");
    launch_fill<FAcc>(b.F_s, n * 3, FAcc(0), stream);
    launch_mlp<P>(ma, stream);
    mk.mark("mlp");
    ta.C = b.C;
    ta.F = b.F_s;
    if (flat) launch_flat<P>(1, ta, stream);
    else launch_triplet<P>(1, h->variant, ta, stream);
    mk.mark("force");
  }
  const bool keep = remember || store;
  if (keep && (st = fwd_remember<IO>(h, cm, pos, types, stream))) return st;
  launch_unpermute<IO, FAcc>(n, cm.bin.perm, b.Ei_s, b.F_s, b.Ei_o, reinterpret_cast<IO*>(ei_v),
                             reinterpret_cast<IO*>(f_v), stream);
  launch_energy(b.Ei_o, cm.d_clo, cm.d_chi, (int)cm.B.chunk_lo.size(), cm.d_sc, n_struct, b.partial, b.energies,
                stream);
  if (energies_dev)
    NNP_HIP(h, hipMemcpyAsync(energies_dev, b.energies, n_struct * sizeof(double), hipMemcpyDeviceToDevice, stream));
  if (energy_host)
    NNP_HIP(h, hipMemcpyAsync(h->h_energy, b.energies, sizeof(double), hipMemcpyDeviceToHost, stream));
  mk.mark("finish");
  if ((st = check_launch(h, "forward"))) return st;
  // Device outputs are ready in stream order; the host waits only for a
  // host energy or for the profiling events.
  if (energy_host || h->prof) NNP_HIP(h, hipStreamSynchronize(stream));
  if (energy_host) *energy_host = *h->h_energy;
  mk.finish();
  h->has_forward = true;
  h->fwd_valid = keep;
  return NNP_OK;
}

template <int P>
nnp_status forward(nnp_handle* h, int n_struct, const int64_t* offs, const void* pos_v, const int32_t* types,
                   const double* boxes, double* energies_dev, double* energy_host, void* ei_v, void* f_v,
                   hipStream_t stream, bool remember = false) {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  Common cm;
  nnp_status st;
  if ((st = make_batch(h, n_struct, offs, boxes, cm.B))) return st;
  const int64_t n = cm.B.n;
  if (n > 0 && (!pos_v || !types)) return fail(h, NNP_E_ARG, "pos and types must not be NULL");
  const IO* pos = reinterpret_cast<const IO*>(pos_v);
  h->cap = initial_cap(h, cm.B);
  Marks mk(h, stream);
  (void)hipGetLastError();
  if ((st = prepare<IO>(h, cm, pos, types, stream))) return st;
  mk.mark("bin_sort");
  FwdBufs<P> bufs;
  if ((st = fwd_buffers<P>(h, cm, n_struct, bufs))) return st;
  int layout = list_layout<P>(h);
  for (int attempt = 0; attempt < 8; ++attempt) {
    if ((st = build_neighbors<T>(h, cm, stream, layout))) return st;
    const int r = check_flags(h, stream, cm, &st);
    if (r < 0) return st;
    if (r > 0) continue;  // capacity grew: rebuild the neighbour list
    if (layout != NNP_LIST_PADDED) {
      bool flat = false;
      if ((st = use_flat<P>(h, 0, 1, &flat))) return st;
      if (flat) {  // the thread level reads padded entries only
        layout = NNP_LIST_PADDED;
        continue;
      }
    }
    mk.mark("neighbors");
    return evaluate<P>(h, cm, mk, bufs, n_struct, pos, types, energies_dev, energy_host, ei_v, f_v, stream, remember);
  }
  return fail(h, NNP_E_STATE, "neighbour capacity did not converge");
}

// Forward evaluation of one structure with a Verlet-skin neighbour list (the
// MD driver): the list of atoms within rc + skin is built with the sorted
// order and reused while no atom has moved more than skin/2 since; each call
// re-gathers the sorted positions and extracts the rows within rc from it.
// The skin list is rebuilt (with a new sort) when the displacement test
// fails or h->skin_ok is false.
template <int P>
nnp_status forward_skin(nnp_handle* h, int64_t n, const void* pos_v, const int32_t* types, const double box[3],
                        double* energies_dev, void* f_v, hipStream_t stream) {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  Common cm;
  nnp_status st;
  const int64_t offs[2] = {0, n};
  const double rs = h->rc + h->md_skin;
  if ((st = make_batch(h, 1, offs, box, cm.B, rs))) return st;
  const IO* pos = reinterpret_cast<const IO*>(pos_v);
  h->cap = initial_cap(h, cm.B);
  {
    const double rho = (double)n / (box[0] * box[1] * box[2]);
    int sc = (int)std::ceil(rho * 4.0 / 3.0 * M_PI * rs * rs * rs * 1.2 + 16.0);
    sc = (sc + 15) / 16 * 16;
    h->scap = std::max(h->scap, std::max(sc, 32));
  }
  Marks mk(h, stream);
  (void)hipGetLastError();
  FwdBufs<P> bufs;
  if ((st = fwd_buffers<P>(h, cm, 1, bufs))) return st;
  const int64_t n1 = std::max<int64_t>(n, 1);
  double4* ref = nullptr;
  if ((st = ensure_t(h, "skin_ref", n1, &ref))) return st;
  for (int attempt = 0; attempt < 16; ++attempt) {
    int* snbr = nullptr;
    int4* snnb = nullptr;
    if ((st = ensure_t(h, "skin_nbr", (size_t)n1 * h->scap, &snbr))) return st;
    if ((st = ensure_t(h, "skin_nnb", n1, &snnb))) return st;
    if (!h->skin_ok) {
      if ((st = prepare<IO>(h, cm, pos, types, stream))) return st;  // clears the flags
      int* cmax = nullptr;
      if ((st = ensure_t(h, "cmax", std::max(cm.B.total_cells, 1), &cmax))) return st;
      launch_neighbor_index(cm.bin, rs, h->scap, snbr, snnb, cmax, stream);
      NNP_HIP(h, hipMemcpyAsync(h->h_flags, cm.bin.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, stream));
      NNP_HIP(h, hipStreamSynchronize(stream));
      if (h->h_flags[0] & 1) return fail(h, NNP_E_TYPE, "atom type outside [0, n_el)");
      if (h->h_flags[0] & 2) return fail(h, NNP_E_ARG, "non-finite atom position (NaN or infinity)");
      if (h->h_flags[1] > h->scap) {  // skin capacity too small: grow it and build again
        h->scap = ((int)std::ceil(h->h_flags[1] * 1.15) + 8 + 15) / 16 * 16;
        continue;
      }
      if (n > 0) NNP_HIP(h, hipMemcpyAsync(ref, cm.bin.pos4, (size_t)n * sizeof(double4), hipMemcpyDeviceToDevice, stream));
      h->skin_ok = true;
      ++h->md_builds;
      mk.mark("skin_build");
      launch_fill_int(cm.bin.flags, 4, 0, stream);
    } else {
      if ((st = prepare<IO>(h, cm, pos, types, stream, false))) return st;  // binds the kept sorted order
      launch_fill_int(cm.bin.flags, 4, 0, stream);
      launch_regather<IO>(cm.bin, pos, ref, 0.5 * h->md_skin, stream);
      mk.mark("regather");
    }
    if ((st = bind_neighbors<T>(h, cm))) return st;
    launch_refresh<T>(cm.bin, snbr, snnb, h->scap, h->rc, h->cap, reinterpret_cast<typename Vec4<T>::type*>(cm.nbr),
                      cm.nnb, stream);
    NNP_HIP(h, hipMemcpyAsync(h->h_flags, cm.bin.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, stream));
    NNP_HIP(h, hipStreamSynchronize(stream));
    if (h->h_flags[0] & 2) return fail(h, NNP_E_ARG, "non-finite atom position (NaN or infinity)");
    if (h->h_flags[0] & 4) {  // an atom moved more than skin/2: new sort and skin list
      h->skin_ok = false;
      continue;
    }
    if (h->h_flags[1] > h->cap) {
      const int nc = (int)std::ceil(h->h_flags[1] * 1.15) + 8;
      h->cap = (nc + 15) / 16 * 16;
      continue;  // the next round re-gathers (unchanged) and refreshes into the larger rows
    }
    h->lcap = std::min(h->cap, (std::max(h->h_flags[2], 1) + 7) / 8 * 8);
    mk.mark("neighbors");
    return evaluate<P>(h, cm, mk, bufs, 1, pos, types, energies_dev, nullptr, nullptr, f_v, stream, false);
  }
  return fail(h, NNP_E_STATE, "neighbour capacity did not converge");
}

template <int P>
nnp_status backward(nnp_handle* h, int n_struct, const int64_t* offs, const void* pos_v, const int32_t* types,
                    const double* boxes, const double* dL_dE, const void* dL_dF_v, double* grad, hipStream_t stream) {
  using T = typename Types<P>::T;
  using IO = typename Types<P>::IO;
  Common cm;
  nnp_status st;
  if ((st = make_batch(h, n_struct, offs, boxes, cm.B))) return st;
  const int64_t n = cm.B.n;
  if (n > 0 && (!pos_v || !types)) return fail(h, NNP_E_ARG, "pos and types must not be NULL");
  if (!grad) return fail(h, NNP_E_ARG, "grad_params must not be NULL");
  const IO* pos = reinterpret_cast<const IO*>(pos_v);
  const IO* dLdF = reinterpret_cast<const IO*>(dL_dF_v);
  h->cap = initial_cap(h, cm.B);
  Marks mk(h, stream);
  (void)hipGetLastError();
  IO *G, *V, *delta;
  double *gE_atom, *part, *padded;
  T* vec;
  const int64_t n1 = std::max<int64_t>(n, 1);
  // atoms per chunk of the weight-gradient reduction: 64, or more once there
  // would be over 4096 chunks (bounds the FP64 partial sums)
  const int chunk = (int)std::max<int64_t>(64, (n1 + 4095) / 4096);
  const int nch = (int)((n1 + chunk - 1) / chunk);
  if ((st = ensure_t(h, "G", (size_t)n1 * LD, &G))) return st;
  if ((st = ensure_t(h, "V", (size_t)n1 * LD, &V))) return st;
  if ((st = ensure_t(h, "delta", (size_t)n1 * 3, &delta))) return st;
  if ((st = ensure_t(h, "gE_atom", n1, &gE_atom))) return st;
  if ((st = ensure_t(h, "wvec", (size_t)n1 * 11 * HID, &vec))) return st;
  if ((st = ensure_t(h, "wpart", (size_t)h->n_el * nch * NET_STRIDE, &part))) return st;
  if ((st = ensure_t(h, "wpad", (size_t)h->n_el * NET_STRIDE, &padded))) return st;
  // With the inputs of the last batch forward, its sorted order, neighbour
  // list and G~ (and J store) are reused: only the force-adjoint product and
  // the weight gradient run.  Otherwise they are rebuilt first.
  bool ready = fwd_reusable<IO>(h, cm, pos, types, stream, &st);
  if (st) return st;
  if (ready && h->fwd_layout != NNP_LIST_PADDED) {  // a thread-level product needs padded entries
    bool flat = false;
    if ((st = use_flat<P>(h, 2, 2, &flat))) return st;
    ready = !flat;
  }
  if (ready) {
    if ((st = bind_neighbors<T>(h, cm, h->fwd_layout))) return st;
    mk.mark("reuse");
  } else {
    if ((st = prepare<IO>(h, cm, pos, types, stream))) return st;
    mk.mark("bin_sort");
  }
  int layout = list_layout<P>(h);
  for (int attempt = 0; attempt < 8 && !ready; ++attempt) {
    if ((st = build_neighbors<T>(h, cm, stream, layout))) return st;
    const int r = check_flags(h, stream, cm, &st);
    if (r < 0) return st;
    if (r > 0) continue;  // capacity grew: rebuild the neighbour list
    if (layout != NNP_LIST_PADDED) {
      bool f_sf = false, f_jvp = false;
      if ((st = use_flat<P>(h, 0, 0, &f_sf))) return st;
      if ((st = use_flat<P>(h, 2, 2, &f_jvp))) return st;
      if (f_sf || f_jvp) {  // the thread level reads padded entries only
        layout = NNP_LIST_PADDED;
        continue;
      }
    }
    mk.mark("neighbors");
    const bool store = use_store<P>(h);
    if constexpr (P != P_BF16) {
      if (store) {
        JacArgs<P> ja;
        if ((st = jac_setup<P>(h, cm, ja))) return st;
        ja.G = G;
        launch_jac<P>(ja, stream);
        mk.mark("sf");
      }
    }
    if (!store) {
      TripArgs<P> ta = trip_args<P>(h, cm);
      bool flat = false;
      if ((st = use_flat<P>(h, 0, 0, &flat, &ta.wpc, n))) return st;
      if (!flat && (st = pair_mask_buffer<P>(h, n, ta))) return st;
      ta.G = G;
      if (flat) launch_flat<P>(0, ta, stream);
      else launch_triplet<P>(0, h->variant, ta, stream);
      mk.mark("sf");
    }
    if ((st = fwd_remember<IO>(h, cm, pos, types, stream))) return st;
    h->fwd_valid = true;
    ready = true;
  }
  if (!ready) return fail(h, NNP_E_STATE, "neighbour capacity did not converge");
  if (dLdF) launch_permute_rows3<IO>(n, cm.bin.perm, dLdF, delta, stream);
  else launch_fill<IO>(delta, n * 3, IO(0), stream);
  const bool store = use_store<P>(h);
  if constexpr (P != P_BF16) {
    if (store) {
      JacArgs<P> ja;
      if ((st = jac_setup<P>(h, cm, ja))) return st;
      ja.delta = delta;
      ja.V = V;
      launch_jac_jvp<P>(ja, stream);
    }
  }
  if (!store) {
    TripArgs<P> ta = trip_args<P>(h, cm);
    bool flat = false;
    if ((st = use_flat<P>(h, 2, 2, &flat, &ta.wpc, n))) return st;
    if (!flat && ta.wpc == 1 && h->fwd_pm_stride > 0) {  // the SF pass's tests of this list
      ta.pm = h->fwd_pm;
      ta.pm_stride = h->fwd_pm_stride;
    }
    ta.delta = delta;
    ta.V = V;
    if (flat) launch_flat<P>(2, ta, stream);
    else launch_triplet<P>(2, h->variant, ta, stream);
  }
  mk.mark("jvp");
  launch_gather_struct_grad(n, cm.bin.perm, cm.d_soff, n_struct, dL_dE, gE_atom, stream);
  WGradArgs<P> wa;
  std::memset(&wa, 0, sizeof(wa));
  wa.n = n;
  wa.n_el = h->n_el;
  wa.eoff = cm.bin.eoff;
  wa.G = G;
  wa.V = V;
  wa.gE_atom = gE_atom;
  wa.nets = reinterpret_cast<const T*>(h->d_nets);
  wa.tab = reinterpret_cast<const DevTab<T>*>(h->d_tab);
  wa.vec = vec;
  wa.chunk = chunk;
  wa.nch = nch;
  wa.partial = part;
  wa.padded = padded;
  wa.n_params = (int64_t)h->params.size();
  wa.flatmap = h->d_flatmap;
  wa.out = grad;
  launch_wgrad<P>(wa, stream);
  mk.mark("wgrad");
  if ((st = check_launch(h, "backward"))) return st;
  // the gradient is ready in stream order; the host waits only for profiling
  if (h->prof) NNP_HIP(h, hipStreamSynchronize(stream));
  mk.finish();
  return NNP_OK;
}

// Unit conversions of the MD driver from the CODATA values of the electron
// volt (J), the atomic mass constant (kg) and the angstrom and femtosecond.
constexpr double EV_J = 1.602176634e-19, AMU_KG = 1.66053906660e-27;
constexpr double ACCEL_CONV = EV_J / 1e-10 / AMU_KG * 1e-30 / 1e-10;  // eV/(A amu) -> A/fs^2
constexpr double KE_CONV = AMU_KG * 1e10 / EV_J;                       // amu A^2/fs^2 -> eV

template <int P>
nnp_status md_run(nnp_handle* h, int64_t n, void* pos_v, void* vel_v, void* f_v, const int32_t* types,
                  const double box[3], const double* masses, double dt, int n_steps, double* epot, double* ekin,
                  hipStream_t stream) {
  using IO = typename Types<P>::IO;
  IO* pos = reinterpret_cast<IO*>(pos_v);
  IO* vel = reinterpret_cast<IO*>(vel_v);
  IO* F = reinterpret_cast<IO*>(f_v);
  MdArgs m;
  std::memset(&m, 0, sizeof(m));
  for (int e = 0; e < h->n_el; ++e) {
    m.half_kick[e] = 0.5 * dt * ACCEL_CONV / masses[e];
    m.half_mass[e] = 0.5 * masses[e];
  }
  m.dt = dt;
  for (int x = 0; x < 3; ++x) {
    m.L[x] = box[x];
    m.invL[x] = 1.0 / box[x];
  }
  m.ke_conv = KE_CONV;
  double *e_dev, *k_dev, *part;
  nnp_status st;
  if ((st = ensure_t(h, "md_epot", (size_t)n_steps + 1, &e_dev))) return st;
  if ((st = ensure_t(h, "md_ekin", (size_t)n_steps + 1, &k_dev))) return st;
  if ((st = ensure_t(h, "md_part", (size_t)md_blocks(n), &part))) return st;
  const int64_t offs[2] = {0, n};
  h->skin_ok = false;  // the first evaluation builds the skin list
  h->md_builds = 0;
  auto force_at = [&](double* e_out) -> nnp_status {
    if (h->md_skin > 0.0) return forward_skin<P>(h, n, pos, types, box, e_out, F, stream);
    ++h->md_builds;
    return forward<P>(h, 1, offs, pos, types, box, e_out, nullptr, nullptr, F, stream);
  };
  if ((st = force_at(e_dev))) return st;
  launch_kick_ke<IO>(n, vel, F, types, m, false, part, k_dev, stream);
  for (int s = 1; s <= n_steps; ++s) {
    launch_kick_drift<IO>(n, pos, vel, F, types, m, stream);
    if ((st = force_at(e_dev + s))) return st;
    launch_kick_ke<IO>(n, vel, F, types, m, true, part, k_dev + s, stream);
  }
  if ((st = check_launch(h, "md"))) return st;
  if (epot) NNP_HIP(h, hipMemcpyAsync(epot, e_dev, ((size_t)n_steps + 1) * sizeof(double), hipMemcpyDeviceToHost, stream));
  if (ekin) NNP_HIP(h, hipMemcpyAsync(ekin, k_dev, ((size_t)n_steps + 1) * sizeof(double), hipMemcpyDeviceToHost, stream));
  NNP_HIP(h, hipStreamSynchronize(stream));
  return NNP_OK;
}

// --------------------------------------------------------------- create
nnp_status build_table(nnp_handle* h, int n_el, int n_sf, const nnp_sf* sf, const nnp_net* nets) {
  DevTab<double>& t = h->tab_d;
  std::memset(&t, 0, sizeof(t));
  t.n_el = n_el;
  for (int e = 0; e < MAX_EL; ++e)
    for (int c = 0; c < MAX_CLS; ++c)
      for (int b = 0; b < 12 * MAX_NE; ++b) t.qn_out[e][c][b] = -1;
  h->rc = 0.0;
  std::vector<std::vector<double>> etas(n_el);
  std::vector<int> count(n_el, 0);
  uint64_t qn_mask = 0;
  for (int s = 0; s < n_sf; ++s) {
    const nnp_sf& d = sf[s];
    const std::string at = "sf[" + std::to_string(s) + "]: ";
    if (d.centre < 0 || d.centre >= n_el) return fail(nullptr, NNP_E_ARG, at + "centre out of range");
    if (d.kind != 2 && d.kind != 3 && d.kind != 9) return fail(nullptr, NNP_E_ARG, at + "kind must be 2, 3 or 9");
    if (d.nbr[0] < 0 || d.nbr[0] >= n_el) return fail(nullptr, NNP_E_ARG, at + "nbr[0] out of range");
    if (d.kind != 2 && (d.nbr[1] < 0 || d.nbr[1] >= n_el)) return fail(nullptr, NNP_E_ARG, at + "nbr[1] out of range");
    if (!std::isfinite(d.eta) || d.eta < 0) return fail(nullptr, NNP_E_ARG, at + "eta must be finite and >= 0");
    if (!std::isfinite(d.rc) || d.rc <= 0) return fail(nullptr, NNP_E_ARG, at + "rc must be > 0");
    if (h->rc == 0.0) h->rc = d.rc;
    if (d.rc != h->rc) return fail(nullptr, NNP_E_ARG, at + "all SFs must share one rc");
    if (!std::isfinite(d.scale) || d.scale == 0.0 || !std::isfinite(d.shift))
      return fail(nullptr, NNP_E_ARG, at + "shift must be finite and scale finite and non-zero");
    const int e = d.centre;
    const int k = count[e]++;
    if (k >= MAX_SF) return fail(nullptr, NNP_E_ARG, at + "more than 32 SFs for one element");
    t.shift_d[e][k] = d.shift;
    t.inv_scale_d[e][k] = 1.0 / d.scale;
    if (d.kind == 2) {
      if (!std::isfinite(d.rs)) return fail(nullptr, NNP_E_ARG, at + "rs must be finite");
      const int f = d.nbr[0];
      const int q = t.rad_cnt[e][f]++;
      if (q >= MAX_RAD) return fail(nullptr, NNP_E_ARG, at + "more than 16 radial SFs for one element pair");
      t.rad_eta[e][f][q] = d.eta;
      t.rad_rs[e][f][q] = d.rs;
      t.rad_out[e][f][q] = k;
    } else {
      if (d.rs != 0.0) return fail(nullptr, NNP_E_ARG, at + "rs must be 0 for angular SFs");
      int kz = -1;
      for (int k = 0; k < 6; ++k)
        if (d.zeta == (double)(1 << k)) kz = k;
      if (kz < 0) return fail(nullptr, NNP_E_ARG, at + "zeta must be one of 1, 2, 4, 8, 16, 32");
      if (d.lambda != 1.0 && d.lambda != -1.0) return fail(nullptr, NNP_E_ARG, at + "lambda must be +1 or -1");
      const int e1 = std::min(d.nbr[0], d.nbr[1]), e2 = std::max(d.nbr[0], d.nbr[1]);
      const int cls = class_index(e1, e2, n_el);
      const int q = t.ang_cnt[e][cls]++;
      if (q >= MAX_ANG) return fail(nullptr, NNP_E_ARG, at + "more than 8 angular SFs for one neighbour pair");
      int ei = -1;
      for (size_t x = 0; x < etas[e].size(); ++x)
        if (etas[e][x] == d.eta) ei = (int)x;
      if (ei < 0) {
        if ((int)etas[e].size() >= MAX_NE)
          return fail(nullptr, NNP_E_ARG, at + "more than 4 distinct angular eta for one element");
        ei = (int)etas[e].size();
        etas[e].push_back(d.eta);
      }
      const int qb = (d.lambda > 0 ? 0 : 6) + kz;
      if (d.kind == 3) {  // the (q, n) slot map of the wave kernels covers the narrow functions
        if (t.qn_out[e][cls][qb * MAX_NE + ei] >= 0)
          return fail(nullptr, NNP_E_ARG, at + "duplicate angular SF (same class, eta, zeta and lambda)");
        t.qn_out[e][cls][qb * MAX_NE + ei] = k;
        t.qn_pre[e][cls][qb * MAX_NE + ei] = std::pow(2.0, 1.0 - d.zeta);
        qn_mask |= qn_bit(qb, ei);
      } else {
        t.ang_wide[e][cls][q] = 1;
        h->has_wide = true;
      }
      t.ang_bit[e][cls][q] = qb * MAX_NE + ei;
      t.ang_pre[e][cls][q] = std::pow(2.0, 1.0 - d.zeta);
      t.ang_out[e][cls][q] = k;
    }
  }
  int ne_max = 1;
  for (int e = 0; e < n_el; ++e) {
    t.n_sf[e] = count[e];
    t.n_eta[e] = (int)etas[e].size();
    for (size_t x = 0; x < etas[e].size(); ++x) {
      t.aeta[e][x] = etas[e][x];
      t.aeta2[e][x] = etas[e][x] * 1.4426950408889634074;
    }
    ne_max = std::max(ne_max, t.n_eta[e]);
  }
  if (ne_max > 2) h->variant = 2;
  else if ((qn_mask & ~QN_WATER) == 0) h->variant = 0;
  else h->variant = 1;
  t.rc2 = h->rc * h->rc;
  t.inv_rc2 = 1.0 / t.rc2;
  h->n_sf = count;
  // networks
  h->sizes.clear();
  h->params.clear();
  h->flatmap.clear();
  for (int e = 0; e < n_el; ++e) {
    const nnp_net& nt = nets[e];
    const std::string at = "nets[" + std::to_string(e) + "]: ";
    if (nt.n_layers != 3) return fail(nullptr, NNP_E_ARG, at + "exactly two hidden layers (n_layers = 3) are supported");
    if (!nt.sizes || !nt.W || !nt.b) return fail(nullptr, NNP_E_ARG, at + "NULL sizes/W/b");
    if (nt.activation != 0) return fail(nullptr, NNP_E_ARG, at + "only activation 0 (tanh) is supported");
    std::vector<int> sz(nt.sizes, nt.sizes + 4);
    if (sz[0] != count[e]) return fail(nullptr, NNP_E_ARG, at + "sizes[0] must equal the element's SF count");
    if (sz[3] != 1) return fail(nullptr, NNP_E_ARG, at + "output width must be 1");
    if (sz[1] < 1 || sz[1] > HID || sz[2] < 1 || sz[2] > HID)
      return fail(nullptr, NNP_E_ARG, at + "hidden widths must be in [1, 32]");
    const int offW[3] = {OFF_W1, OFF_W2, OFF_W3}, offB[3] = {OFF_B1, OFF_B2, OFF_B3};
    for (int l = 0; l < 3; ++l) {
      if (!nt.W[l] || !nt.b[l]) return fail(nullptr, NNP_E_ARG, at + "NULL layer array");
      for (int o = 0; o < sz[l + 1]; ++o)
        for (int i = 0; i < sz[l]; ++i) {
          const double w = nt.W[l][(size_t)o * sz[l] + i];
          if (!std::isfinite(w)) return fail(nullptr, NNP_E_ARG, at + "non-finite weight");
          h->params.push_back(w);
          h->flatmap.push_back(e * NET_STRIDE + (l < 2 ? offW[l] + o * HID + i : offW[l] + i));
        }
      for (int o = 0; o < sz[l + 1]; ++o) {
        const double bv = nt.b[l][o];
        if (!std::isfinite(bv)) return fail(nullptr, NNP_E_ARG, at + "non-finite bias");
        h->params.push_back(bv);
        h->flatmap.push_back(e * NET_STRIDE + offB[l] + o);
      }
    }
    h->sizes.push_back(sz);
  }
  return NNP_OK;
}

}  // namespace
}  // namespace nnp

using namespace nnp;

extern "C" {

nnp_status nnp_create(int n_el, const char* const* elements, int n_sf, const nnp_sf* sf, const nnp_net* nets,
                      nnp_precision prec, nnp_handle** out) {
  (void)elements;
  g_create_error.clear();
  if (!out) return fail(nullptr, NNP_E_ARG, "out must not be NULL");
  *out = nullptr;
  if (n_el < 1 || n_el > MAX_EL) return fail(nullptr, NNP_E_ARG, "n_el must be in [1, 4]");
  if (n_sf < 1 || !sf || !nets) return fail(nullptr, NNP_E_ARG, "empty SF table or NULL nets");
  if (prec != NNP_FP64 && prec != NNP_FP32 && prec != NNP_BF16_MIXED) return fail(nullptr, NNP_E_ARG, "bad precision");
  nnp_handle* h = new nnp_handle();
  h->n_el = n_el;
  h->prec = prec;
  nnp_status st = build_table(h, n_el, n_sf, sf, nets);
  if (st) {
    delete h;
    return st;
  }
  auto bail = [&](nnp_status s) {
    g_create_error = h->err;
    nnp_destroy(h);
    return s;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(fail(h, NNP_E_HIP, "hipGetDevice failed"));
  {
    const hipError_t e = scratch_address(h->device, &h->scratch);
    if (e != hipSuccess) return bail(fail(h, NNP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)));
  }
  if (prec == NNP_FP64) {
    if (hipMalloc(&h->d_tab, sizeof(DevTab<double>)) != hipSuccess) return bail(fail(h, NNP_E_NOMEM, "table alloc"));
    if (hipMemcpy(h->d_tab, &h->tab_d, sizeof(DevTab<double>), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(h, NNP_E_HIP, "table upload failed"));
  } else {
    DevTab<float> tf = convert_tab<float>(h->tab_d);
    if (hipMalloc(&h->d_tab, sizeof(DevTab<float>)) != hipSuccess) return bail(fail(h, NNP_E_NOMEM, "table alloc"));
    if (hipMemcpy(h->d_tab, &tf, sizeof(DevTab<float>), hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(h, NNP_E_HIP, "table upload failed"));
  }
  if (hipMalloc(&h->d_flatmap, h->flatmap.size() * sizeof(int)) != hipSuccess)
    return bail(fail(h, NNP_E_NOMEM, "flatmap alloc"));
  if (hipMemcpy(h->d_flatmap, h->flatmap.data(), h->flatmap.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(h, NNP_E_HIP, "flatmap upload"));
  if ((st = upload_params(h))) return bail(st);
  if (hipHostMalloc((void**)&h->h_flags, 4 * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return bail(fail(h, NNP_E_NOMEM, "pinned flags"));
  if (hipHostMalloc((void**)&h->h_energy, sizeof(double), hipHostMallocDefault) != hipSuccess)
    return bail(fail(h, NNP_E_NOMEM, "pinned energy"));
  if ((st = stage(h, 4096))) return bail(st);  // staging of one structure's batch description
  *out = h;
  return NNP_OK;
}

nnp_status nnp_count_work(nnp_handle* h, int64_t n_atoms, const void* pos, const int32_t* types, const double box[3],
                          int64_t counts[5], void* stream) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (!counts || !box || n_atoms < 0) return fail(h, NNP_E_ARG, "bad arguments");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int64_t offs[2] = {0, n_atoms};
  Common cm;
  nnp_status st;
  if ((st = make_batch(h, 1, offs, box, cm.B))) return st;
  if (n_atoms > 0 && (!pos || !types)) return fail(h, NNP_E_ARG, "pos and types must not be NULL");
  h->cap = initial_cap(h, cm.B);
  (void)hipGetLastError();
  if (h->prec == NNP_FP64) st = prepare<double>(h, cm, (const double*)pos, types, s);
  else st = prepare<float>(h, cm, (const float*)pos, types, s);
  if (st) return st;
  CountTab ct;
  std::memset(&ct, 0, sizeof(ct));
  for (int e = 0; e < MAX_EL; ++e) {
    for (int c = 0; c < MAX_CLS; ++c) ct.ang[e][c] = h->tab_d.ang_cnt[e][c];
    for (int f = 0; f < MAX_EL; ++f) ct.rad[e][f] = h->tab_d.rad_cnt[e][f];
  }
  unsigned long long* d_cnt;
  if ((st = ensure_t(h, "counts", 8, &d_cnt))) return st;
  bool built = false;
  for (int attempt = 0; attempt < 8 && !built; ++attempt) {
    st = h->prec == NNP_FP64 ? build_neighbors<double>(h, cm, s) : build_neighbors<float>(h, cm, s);
    if (st) return st;
    const int r = check_flags(h, s, cm, &st);
    if (r < 0) return st;
    built = r == 0;
  }
  if (!built) return fail(h, NNP_E_STATE, "neighbour capacity did not converge");
  launch_fill_int(reinterpret_cast<int*>(d_cnt), 16, 0, s);
  if (h->prec == NNP_FP64)
    launch_count_terms<double>(cm.bin, reinterpret_cast<const double4*>(cm.nbr), cm.nnb, h->cap, ct, h->rc, d_cnt, s);
  else
    launch_count_terms<float>(cm.bin, reinterpret_cast<const float4*>(cm.nbr), cm.nnb, h->cap, ct, h->rc, d_cnt, s);
  if ((st = check_launch(h, "count"))) return st;
  unsigned long long c[8];
  NNP_HIP(h, hipMemcpy(c, d_cnt, sizeof(c), hipMemcpyDeviceToHost));
  for (int i = 0; i < 5; ++i) counts[i] = (int64_t)c[i];
  return NNP_OK;
}

nnp_status nnp_compute_batch(nnp_handle* h, int n_struct, const int64_t* atom_offsets, const void* pos,
                             const int32_t* types, const double* boxes, double* energies, void* atom_energy,
                             void* forces, void* stream) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  switch (h->prec) {
    case NNP_FP64: return forward<P_FP64>(h, n_struct, atom_offsets, pos, types, boxes, energies, nullptr, atom_energy, forces, s, true);
    case NNP_FP32: return forward<P_FP32>(h, n_struct, atom_offsets, pos, types, boxes, energies, nullptr, atom_energy, forces, s, true);
    default: return forward<P_BF16>(h, n_struct, atom_offsets, pos, types, boxes, energies, nullptr, atom_energy, forces, s, true);
  }
}

nnp_status nnp_compute(nnp_handle* h, int64_t n_atoms, const void* pos, const int32_t* types, const double box[3],
                       double* energy, void* atom_energy, void* forces, void* stream) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (n_atoms < 0) return fail(h, NNP_E_ARG, "n_atoms must be >= 0");
  if (!box) return fail(h, NNP_E_ARG, "box must not be NULL");
  const int64_t offs[2] = {0, n_atoms};
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double e = 0.0;
  nnp_status st;
  switch (h->prec) {
    case NNP_FP64: st = forward<P_FP64>(h, 1, offs, pos, types, box, nullptr, &e, atom_energy, forces, s); break;
    case NNP_FP32: st = forward<P_FP32>(h, 1, offs, pos, types, box, nullptr, &e, atom_energy, forces, s); break;
    default: st = forward<P_BF16>(h, 1, offs, pos, types, box, nullptr, &e, atom_energy, forces, s); break;
  }
  if (st == NNP_OK && energy) *energy = e;
  return st;
}

nnp_status nnp_compute_noalloc(nnp_handle* h, int64_t n_atoms, const void* pos, const int32_t* types,
                               const double box[3], double* energy, void* atom_energy, void* forces, void* stream) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (n_atoms < 0 || n_atoms > NNP_NOALLOC_MAX_ATOMS)
    return fail(h, NNP_E_ARG, "n_atoms must be in [0, " + std::to_string(NNP_NOALLOC_MAX_ATOMS) + "]");
  if (!box) return fail(h, NNP_E_ARG, "box must not be NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
    return fail(h, NNP_E_STATE, "the handle's device must be the current device");
  const int64_t offs[2] = {0, n_atoms};
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // Every named buffer of the call is carved from this device's static
  // workspace; profiling (which creates events) is off for the call.
  h->arena_on = true;
  h->arena_used = 0;
  h->arena_bufs.clear();
  const bool prof = h->prof;
  h->prof = false;
  double e = 0.0;
  nnp_status st;
  switch (h->prec) {
    case NNP_FP64: st = forward<P_FP64>(h, 1, offs, pos, types, box, nullptr, &e, atom_energy, forces, s); break;
    case NNP_FP32: st = forward<P_FP32>(h, 1, offs, pos, types, box, nullptr, &e, atom_energy, forces, s); break;
    default: st = forward<P_BF16>(h, 1, offs, pos, types, box, nullptr, &e, atom_energy, forces, s); break;
  }
  h->prof = prof;
  h->arena_on = false;
  h->arena_bufs.clear();
  if (st == NNP_OK && energy) *energy = e;
  return st;
}

nnp_status nnp_backward(nnp_handle* h, int n_struct, const int64_t* atom_offsets, const void* pos,
                        const int32_t* types, const double* boxes, const double* dL_dE, const void* dL_dF,
                        void* grad_params, void* stream) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  switch (h->prec) {
    case NNP_FP64: return backward<P_FP64>(h, n_struct, atom_offsets, pos, types, boxes, dL_dE, dL_dF, (double*)grad_params, s);
    case NNP_FP32: return backward<P_FP32>(h, n_struct, atom_offsets, pos, types, boxes, dL_dE, dL_dF, (double*)grad_params, s);
    default: return fail(h, NNP_E_STATE, "nnp_backward needs an NNP_FP64 or NNP_FP32 handle");
  }
}

int64_t nnp_n_params(const nnp_handle* h) { return h ? (int64_t)h->params.size() : 0; }

nnp_status nnp_set_params(nnp_handle* h, const void* flat, int on_device) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (!flat) return fail(h, NNP_E_ARG, "flat_params must not be NULL");
  std::vector<double> p(h->params.size());
  // calls may return with kernels still reading the networks: let them finish
  NNP_HIP(h, hipDeviceSynchronize());
  if (on_device) {
    NNP_HIP(h, hipMemcpy(p.data(), flat, p.size() * sizeof(double), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(p.data(), flat, p.size() * sizeof(double));
  }
  for (double v : p)
    if (!std::isfinite(v)) return fail(h, NNP_E_ARG, "non-finite parameter");
  h->params = p;
  return upload_params(h);
}

nnp_status nnp_get_params(const nnp_handle* h, double* out) {
  if (!h || !out) return NNP_E_ARG;
  Claim claim(const_cast<nnp_handle*>(h));
  if (!claim.ok) return NNP_E_STATE;
  std::memcpy(out, h->params.data(), h->params.size() * sizeof(double));
  return NNP_OK;
}

nnp_status nnp_set_profiling(nnp_handle* h, int enable) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  h->prof = enable != 0;
  return NNP_OK;
}

int nnp_last_timings(const nnp_handle* h, const char** names, double* ms, int max_k) {
  if (!h) return 0;
  Claim claim(const_cast<nnp_handle*>(h));
  if (!claim.ok) return 0;
  const int k = std::min<int>(max_k, (int)h->t_ms.size());
  for (int i = 0; i < k; ++i) {
    if (names) names[i] = h->t_names[i];
    if (ms) ms[i] = h->t_ms[i];
  }
  return k;
}

nnp_status nnp_md_run(nnp_handle* h, int64_t n_atoms, void* pos, void* vel, void* forces, const int32_t* types,
                      const double box[3], const double* masses, double dt_fs, int n_steps, double* epot,
                      double* ekin, void* stream) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (n_atoms < 0 || n_steps < 0) return fail(h, NNP_E_ARG, "n_atoms and n_steps must be >= 0");
  if (n_atoms > 0 && (!pos || !vel || !forces || !types))
    return fail(h, NNP_E_ARG, "pos, vel, forces and types must not be NULL");
  if (!box || !masses) return fail(h, NNP_E_ARG, "box and masses must not be NULL");
  if (!(std::isfinite(dt_fs) && dt_fs > 0.0)) return fail(h, NNP_E_ARG, "dt must be finite and > 0");
  for (int e = 0; e < h->n_el; ++e)
    if (!(std::isfinite(masses[e]) && masses[e] > 0.0)) return fail(h, NNP_E_ARG, "masses must be finite and > 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  switch (h->prec) {
    case NNP_FP64: return md_run<P_FP64>(h, n_atoms, pos, vel, forces, types, box, masses, dt_fs, n_steps, epot, ekin, s);
    case NNP_FP32: return md_run<P_FP32>(h, n_atoms, pos, vel, forces, types, box, masses, dt_fs, n_steps, epot, ekin, s);
    default: return md_run<P_BF16>(h, n_atoms, pos, vel, forces, types, box, masses, dt_fs, n_steps, epot, ekin, s);
  }
}

nnp_status nnp_set_list_layout(nnp_handle* h, int layout) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (layout != NNP_LIST_PADDED && layout != NNP_LIST_INDEX && layout != NNP_LIST_COMPACT)
    return fail(h, NNP_E_ARG, "layout must be NNP_LIST_PADDED, NNP_LIST_INDEX or NNP_LIST_COMPACT");
  h->list_layout = layout;
  return NNP_OK;
}

nnp_status nnp_set_pair_masks(nnp_handle* h, int on) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (on != 0 && on != 1) return fail(h, NNP_E_ARG, "on must be 0 or 1");
  h->pair_masks = on;
  return NNP_OK;
}

nnp_status nnp_set_md_skin(nnp_handle* h, double skin) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (!(std::isfinite(skin) && skin >= 0.0)) return fail(h, NNP_E_ARG, "skin must be finite and >= 0");
  h->md_skin = skin;
  h->skin_ok = false;
  return NNP_OK;
}

int64_t nnp_md_list_builds(const nnp_handle* h) {
  if (!h) return -1;
  Claim claim(const_cast<nnp_handle*>(h));
  if (!claim.ok) return -1;
  return h->md_builds;
}

nnp_status nnp_set_parallelism(nnp_handle* h, int mode) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (mode != NNP_PAR_AUTO && mode != NNP_PAR_WAVE && mode != NNP_PAR_THREAD && mode != NNP_PAR_WAVE2)
    return fail(h, NNP_E_ARG, "parallelism must be NNP_PAR_AUTO, NNP_PAR_WAVE, NNP_PAR_THREAD or NNP_PAR_WAVE2");
  h->parallelism = mode;
  return NNP_OK;
}

nnp_status nnp_set_derivative_mode(nnp_handle* h, int mode) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (mode != NNP_DERIV_RECOMPUTE && mode != NNP_DERIV_STORED)
    return fail(h, NNP_E_ARG, "derivative mode must be NNP_DERIV_RECOMPUTE or NNP_DERIV_STORED");
  if (mode == NNP_DERIV_STORED && h->prec == NNP_BF16_MIXED)
    return fail(h, NNP_E_STATE, "the stored-Jacobian mode needs an NNP_FP64 or NNP_FP32 handle");
  if (mode != h->deriv_mode) h->fwd_valid = false;
  h->deriv_mode = mode;
  return NNP_OK;
}

int64_t nnp_workspace_bytes(const nnp_handle* h) {
  if (!h) return 0;
  Claim claim(const_cast<nnp_handle*>(h));
  if (!claim.ok) return -1;
  int64_t b = 0;
  for (const auto& kv : h->ws) b += (int64_t)kv.second.bytes;
  return b;
}

int nnp_neighbor_capacity(const nnp_handle* h) { return h ? h->cap : 0; }

nnp_status nnp_set_neighbor_capacity(nnp_handle* h, int cap) {
  if (!h) return NNP_E_ARG;
  Claim claim(h);
  if (!claim.ok) return NNP_E_STATE;
  if (cap < 8) return fail(h, NNP_E_ARG, "capacity must be >= 8");
  h->cap_override = cap;
  h->cap = cap;
  h->fwd_valid = false;
  return NNP_OK;
}

void nnp_destroy(nnp_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();  // calls may return with kernels still using the workspace
  for (auto& kv : h->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (h->d_tab) (void)hipFree(h->d_tab);
  if (h->d_nets) (void)hipFree(h->d_nets);
  if (h->d_flatmap) (void)hipFree(h->d_flatmap);
  if (h->h_stage) (void)hipHostFree(h->h_stage);
  if (h->h_flags) (void)hipHostFree(h->h_flags);
  if (h->h_energy) (void)hipHostFree(h->h_energy);
  for (auto e : h->events) (void)hipEventDestroy(e);
  delete h;
}

const char* nnp_last_error(const nnp_handle* h) {
  if (!h) return nnp::g_create_error.c_str();
  if (h == nnp::t_busy_handle) return nnp::t_busy_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
