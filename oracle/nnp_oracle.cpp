// Plain FP64 CPU oracle of the Behler-Parrinello energy+force evaluation.
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// definition that the HIP path is checked against.  Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// library under paper_2002_00054_amd/ never does, and the two share no code.
//
// What is computed (Desai, Reeve, Belak, "Implementing a neural network
// interatomic model with performance portability ...", Sec. 3.1, Fig. 1(b)):
//   step 1  symmetry functions G_i of every atom from its neighbours inside
//           the cutoff: radial G2 (the printed formula of step 1) and the
//           angular G3 over pairs of neighbours (the "extra loop over
//           neighbors of neighbors"; the paper does not print it, so the
//           narrow angular function of Behler, the paper's ref. [18], is
//           used); also its wide variant G9 (no r_jk factor: every pair of
//           neighbours within the cutoff of i counts), the other angular
//           function of that family;
//   step 2  E_i = NN_{e_i}(G_i), one network per element (Fig. 1(c));
//           E = sum_i E_i;
//   step 3  forces f = -dE/dr (sign convention of Fig. 1(a)/(b)), by the
//           chain rule through dE_i/dG_i and dG_i/dr.
// Readings where the paper is silent are the ones listed with the design
// notes: full neighbour list with minimum image (box edges > 2 rc), unordered
// neighbour pairs j<k in G3, r_jk taken as |r_ik - r_ij|, integer zeta by
// repeated multiplication with 0^0 = 1, frozen shift/scale
// G~ = (G - shift)/scale, tanh hidden layers and a linear output.
//
// Everything is double precision, no fast-math, brute-force loops; OpenMP
// only splits the outer loop over centre atoms.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// Potential description, flat arrays (one entry per SF of the table).
typedef struct {
  int n_el;
  int n_sf;                 // table entries over all centre elements
  const int* centre;        // [n_sf] centre element
  const int* kind;          // [n_sf] 2 = radial G2, 3 = narrow angular G3, 9 = wide angular G9
  const int* nbr0;          // [n_sf] neighbour element (G2) / first of pair (G3)
  const int* nbr1;          // [n_sf] second of pair (G3), ignored for G2
  const double* eta;        // [n_sf] A^-2
  const double* rs;         // [n_sf] A (G2 only)
  const double* zeta;       // [n_sf] integer-valued (G3 only)
  const double* lam;        // [n_sf] +-1 (G3 only)
  const double* rc;         // [n_sf] cutoff radius, A
  const double* shift;      // [n_sf]
  const double* scale;      // [n_sf]
  int n_layers;             // weight layers per net (3 for n_sf->25->25->1)
  const int* sizes;         // [n_el][n_layers+1]
  const double* params;     // per element, per layer: W[out][in] then b[out]
} opot;

}  // extern "C"

namespace {

const double kPi = 3.14159265358979323846;

struct SFDef {
  int kind, n0, n1;
  double eta, rs, zeta, lam, rc, shift, scale;
};

struct Net {
  std::vector<int> sizes;
  std::vector<std::vector<double>> W, b;  // W[l][out*in + in_idx]
};

struct Pot {
  int n_el = 0;
  std::vector<std::vector<SFDef>> sf;  // per centre element, table order
  std::vector<Net> net;
  double rc_max = 0.0;
};

Pot parse(const opot* p) {
  Pot P;
  P.n_el = p->n_el;
  P.sf.resize(P.n_el);
  for (int s = 0; s < p->n_sf; ++s) {
    SFDef d;
    d.kind = p->kind[s];
    d.n0 = p->nbr0[s];
    d.n1 = p->nbr1[s];
    d.eta = p->eta[s];
    d.rs = p->rs[s];
    d.zeta = p->zeta[s];
    d.lam = p->lam[s];
    d.rc = p->rc[s];
    d.shift = p->shift[s];
    d.scale = p->scale[s];
    P.sf[p->centre[s]].push_back(d);
    P.rc_max = std::max(P.rc_max, d.rc);
  }
  P.net.resize(P.n_el);
  const double* q = p->params;
  for (int e = 0; e < P.n_el; ++e) {
    Net& n = P.net[e];
    n.sizes.assign(p->sizes + e * (p->n_layers + 1), p->sizes + (e + 1) * (p->n_layers + 1));
    for (int l = 0; l < p->n_layers; ++l) {
      int fi = n.sizes[l], fo = n.sizes[l + 1];
      n.W.emplace_back(q, q + (size_t)fo * fi);
      q += (size_t)fo * fi;
      n.b.emplace_back(q, q + fo);
      q += fo;
    }
  }
  return P;
}

// ---------------------------------------------------------------- geometry
// Minimum-image displacement r_j - r_i along one axis of edge L.
double min_image(double d, double L) { return d - L * std::nearbyint(d / L); }

void displacement(const double* pos, int64_t i, int64_t j, const double* box, double out[3]) {
  for (int a = 0; a < 3; ++a) out[a] = min_image(pos[3 * j + a] - pos[3 * i + a], box[a]);
}

double norm3(const double v[3]) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }
double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Cosine cutoff f_c(r) = (cos(pi r / rc) + 1) / 2 inside rc, 0 outside; and its derivative.
double fcut(double r, double rc) { return r < rc ? 0.5 * (std::cos(kPi * r / rc) + 1.0) : 0.0; }
double dfcut(double r, double rc) { return r < rc ? -0.5 * (kPi / rc) * std::sin(kPi * r / rc) : 0.0; }

// x^n for integer n >= 0 by repeated multiplication (0^0 = 1).
double ipow(double x, int n) {
  double r = 1.0;
  for (int k = 0; k < n; ++k) r *= x;
  return r;
}

// ---------------------------------------------------------- neighbour lists
// Brute force: every j != i with |min-image r_ij| < rc, ascending j.
void neighbours_brute(int64_t N, const double* pos, const double* box, double rc,
                      std::vector<std::vector<int64_t>>& nb) {
  nb.assign(N, {});
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < N; ++i) {
    for (int64_t j = 0; j < N; ++j) {
      if (j == i) continue;
      double d[3];
      displacement(pos, i, j, box, d);
      if (norm3(d) < rc) nb[i].push_back(j);
    }
  }
}

// Cell list: cells of edge >= rc per axis, atoms of the (deduplicated) 3x3x3
// block of cells around the centre's cell, minimum-image distance test; the
// result is sorted ascending so it equals the brute-force list.
struct Cells {
  int n[3];
  std::vector<std::vector<int64_t>> members;
  int cell_of(const double* x, const double* box) const {
    int c[3];
    for (int a = 0; a < 3; ++a) {
      double w = x[a] - box[a] * std::floor(x[a] / box[a]);
      int k = (int)std::floor(w / box[a] * n[a]);
      c[a] = std::min(std::max(k, 0), n[a] - 1);
    }
    return (c[0] * n[1] + c[1]) * n[2] + c[2];
  }
};

Cells build_cells(int64_t N, const double* pos, const double* box, double rc) {
  Cells C;
  for (int a = 0; a < 3; ++a) C.n[a] = std::max(1, (int)std::floor(box[a] / rc));
  C.members.assign((size_t)C.n[0] * C.n[1] * C.n[2], {});
  for (int64_t i = 0; i < N; ++i) C.members[C.cell_of(pos + 3 * i, box)].push_back(i);
  return C;
}

void neighbours_of(const Cells& C, int64_t i, const double* pos, const double* box, double rc,
                   std::vector<int64_t>& out) {
  out.clear();
  int cid = C.cell_of(pos + 3 * i, box);
  int ci[3] = {cid / (C.n[1] * C.n[2]), (cid / C.n[2]) % C.n[1], cid % C.n[2]};
  std::vector<int> offs[3];
  for (int a = 0; a < 3; ++a) {
    for (int o = -1; o <= 1; ++o) {
      int k = ((ci[a] + o) % C.n[a] + C.n[a]) % C.n[a];
      if (std::find(offs[a].begin(), offs[a].end(), k) == offs[a].end()) offs[a].push_back(k);
    }
  }
  for (int x : offs[0])
    for (int y : offs[1])
      for (int z : offs[2])
        for (int64_t j : C.members[(x * C.n[1] + y) * C.n[2] + z]) {
          if (j == i) continue;
          double d[3];
          displacement(pos, i, j, box, d);
          if (norm3(d) < rc) out.push_back(j);
        }
  std::sort(out.begin(), out.end());
}

void neighbours_cells(int64_t N, const double* pos, const double* box, double rc,
                      std::vector<std::vector<int64_t>>& nb) {
  Cells C = build_cells(N, pos, box, rc);
  nb.assign(N, {});
#pragma omp parallel
  {
    std::vector<int64_t> tmp;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
      neighbours_of(C, i, pos, box, rc, tmp);
      nb[i] = tmp;
    }
  }
}

// ------------------------------------------------------ symmetry functions
// Raw (unscaled) G of centre i, Sec. 3.1 step 1.
void descriptors(const Pot& P, int64_t i, const std::vector<int64_t>& nb, const double* pos,
                 const int* types, const double* box, double* G) {
  const std::vector<SFDef>& S = P.sf[types[i]];
  const int ns = (int)S.size();
  for (int s = 0; s < ns; ++s) G[s] = 0.0;
  const size_t m = nb.size();
  std::vector<double> rv(3 * m), rl(m);
  for (size_t a = 0; a < m; ++a) {
    displacement(pos, i, nb[a], box, &rv[3 * a]);
    rl[a] = norm3(&rv[3 * a]);
  }
  // Radial: G2 = sum_j exp(-eta (r_ij - rs)^2) f_c(r_ij) over neighbours of element nbr0.
  for (size_t a = 0; a < m; ++a) {
    const int ej = types[nb[a]];
    const double r = rl[a];
    for (int s = 0; s < ns; ++s) {
      const SFDef& d = S[s];
      if (d.kind != 2 || d.n0 != ej || r >= d.rc) continue;
      G[s] += std::exp(-d.eta * (r - d.rs) * (r - d.rs)) * fcut(r, d.rc);
    }
  }
  // Angular: G3 = 2^(1-zeta) sum_{j<k} (1 + lam cos theta_ijk)^zeta
  //              exp(-eta (r_ij^2 + r_ik^2 + r_jk^2)) f_c(r_ij) f_c(r_ik) f_c(r_jk)
  // over unordered neighbour pairs whose elements match {nbr0, nbr1}.
  for (size_t a = 0; a < m; ++a) {
    for (size_t b = a + 1; b < m; ++b) {
      const int ej = types[nb[a]], ek = types[nb[b]];
      const double* u = &rv[3 * a];
      const double* v = &rv[3 * b];
      const double w[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
      const double ra = rl[a], rb = rl[b], rd = norm3(w);
      const double cth = dot3(u, v) / (ra * rb);
      for (int s = 0; s < ns; ++s) {
        const SFDef& d = S[s];
        if (d.kind != 3 && d.kind != 9) continue;
        const bool match = (d.n0 == ej && d.n1 == ek) || (d.n0 == ek && d.n1 == ej);
        if (!match || ra >= d.rc || rb >= d.rc) continue;
        const int z = (int)d.zeta;
        const double ang = std::pow(2.0, 1.0 - d.zeta) * ipow(1.0 + d.lam * cth, z);
        if (d.kind == 3) {
          if (rd >= d.rc) continue;
          G[s] += ang * std::exp(-d.eta * (ra * ra + rb * rb + rd * rd)) * fcut(ra, d.rc) * fcut(rb, d.rc) *
                  fcut(rd, d.rc);
        } else {
          // G9 = 2^(1-zeta) sum_{j<k} (1 + lam cos)^zeta exp(-eta (r_ij^2 + r_ik^2)) f_c(r_ij) f_c(r_ik)
          G[s] += ang * std::exp(-d.eta * (ra * ra + rb * rb)) * fcut(ra, d.rc) * fcut(rb, d.rc);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ networks
// E_i = NN(G~) with tanh hidden layers and a linear output (Sec. 3.1 step 2),
// and dE_i/dG (raw G: includes the 1/scale of the centring/scaling).
double network(const Pot& P, int e, const double* G, double* dEdG) {
  const Net& n = P.net[e];
  const std::vector<SFDef>& S = P.sf[e];
  const int L = (int)n.W.size();
  std::vector<std::vector<double>> act(L + 1);
  act[0].resize(n.sizes[0]);
  for (int s = 0; s < n.sizes[0]; ++s) act[0][s] = (G[s] - S[s].shift) / S[s].scale;
  for (int l = 0; l < L; ++l) {
    const int fi = n.sizes[l], fo = n.sizes[l + 1];
    act[l + 1].assign(fo, 0.0);
    for (int o = 0; o < fo; ++o) {
      double z = n.b[l][o];
      for (int k = 0; k < fi; ++k) z += n.W[l][(size_t)o * fi + k] * act[l][k];
      act[l + 1][o] = (l < L - 1) ? std::tanh(z) : z;
    }
  }
  const double E = act[L][0];
  if (dEdG) {
    // Backpropagation of the scalar output to the inputs.
    std::vector<double> g(1, 1.0);  // dE/d(output pre-activation)
    for (int l = L - 1; l >= 0; --l) {
      const int fi = n.sizes[l], fo = n.sizes[l + 1];
      std::vector<double> gin(fi, 0.0);
      for (int k = 0; k < fi; ++k)
        for (int o = 0; o < fo; ++o) gin[k] += n.W[l][(size_t)o * fi + k] * g[o];
      if (l > 0)
        for (int k = 0; k < fi; ++k) gin[k] *= 1.0 - act[l][k] * act[l][k];
      g.swap(gin);
    }
    for (int s = 0; s < n.sizes[0]; ++s) dEdG[s] = g[s] / S[s].scale;
  }
  return E;
}

// --------------------------------------------------------------- gradients
// For centre i, call sink(m, grad[3], s) with grad = dG_is / dr_m for every
// term of every SF s.  Pair term t(r) = exp(-eta (r-rs)^2) f_c(r); triplet
// term T(a, b, d, cos) with a = r_ij, b = r_ik, d = r_jk as in `descriptors`.
template <class Sink>
void descriptor_gradients(const Pot& P, int64_t i, const std::vector<int64_t>& nb, const double* pos,
                          const int* types, const double* box, Sink&& sink) {
  const std::vector<SFDef>& S = P.sf[types[i]];
  const int ns = (int)S.size();
  const size_t m = nb.size();
  std::vector<double> rv(3 * m), rl(m);
  for (size_t a = 0; a < m; ++a) {
    displacement(pos, i, nb[a], box, &rv[3 * a]);
    rl[a] = norm3(&rv[3 * a]);
  }
  for (size_t a = 0; a < m; ++a) {
    const int ej = types[nb[a]];
    const double r = rl[a];
    const double* u = &rv[3 * a];
    for (int s = 0; s < ns; ++s) {
      const SFDef& d = S[s];
      if (d.kind != 2 || d.n0 != ej || r >= d.rc) continue;
      const double ex = std::exp(-d.eta * (r - d.rs) * (r - d.rs));
      const double dt = ex * (-2.0 * d.eta * (r - d.rs) * fcut(r, d.rc) + dfcut(r, d.rc));
      // dr/dr_j = u/r, dr/dr_i = -u/r.
      double gj[3], gi[3];
      for (int c = 0; c < 3; ++c) {
        gj[c] = dt * u[c] / r;
        gi[c] = -dt * u[c] / r;
      }
      sink(nb[a], gj, s);
      sink(i, gi, s);
    }
  }
  for (size_t a = 0; a < m; ++a) {
    for (size_t b = a + 1; b < m; ++b) {
      const int ej = types[nb[a]], ek = types[nb[b]];
      const double* u = &rv[3 * a];
      const double* v = &rv[3 * b];
      const double w[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
      const double ra = rl[a], rb = rl[b], rd = norm3(w);
      const double cth = dot3(u, v) / (ra * rb);
      // d cos / d u and d cos / d v (u = r_j - r_i, v = r_k - r_i).
      double dcu[3], dcv[3];
      for (int c = 0; c < 3; ++c) {
        dcu[c] = v[c] / (ra * rb) - cth * u[c] / (ra * ra);
        dcv[c] = u[c] / (ra * rb) - cth * v[c] / (rb * rb);
      }
      for (int s = 0; s < ns; ++s) {
        const SFDef& d = S[s];
        if (d.kind != 3 && d.kind != 9) continue;
        const bool match = (d.n0 == ej && d.n1 == ek) || (d.n0 == ek && d.n1 == ej);
        if (!match || ra >= d.rc || rb >= d.rc) continue;
        const bool wide = d.kind == 9;  // G9: no r_jk factor, no r_jk cutoff
        if (!wide && rd >= d.rc) continue;
        const int z = (int)d.zeta;
        const double pre = std::pow(2.0, 1.0 - d.zeta);
        const double Pb = 1.0 + d.lam * cth;
        const double X = std::exp(-d.eta * (ra * ra + rb * rb + (wide ? 0.0 : rd * rd)));
        const double fa = fcut(ra, d.rc), fb = fcut(rb, d.rc), fd = wide ? 1.0 : fcut(rd, d.rc);
        const double dfa = dfcut(ra, d.rc), dfb = dfcut(rb, d.rc);
        // wide: T does not depend on r_jk, so dT/dd = 0 (fd = 1, dfd = 0, no eta d^2 term)
        const double dfd = wide ? 0.0 : dfcut(rd, d.rc) - 2.0 * d.eta * rd * fd;
        const double Pz = ipow(Pb, z);
        const double dT_dc = pre * z * d.lam * ipow(Pb, z - 1) * X * fa * fb * fd;
        const double dT_da = pre * Pz * X * (-2.0 * d.eta * ra * fa + dfa) * fb * fd;
        const double dT_db = pre * Pz * X * fa * (-2.0 * d.eta * rb * fb + dfb) * fd;
        const double dT_dd = pre * Pz * X * fa * fb * dfd;
        double gi[3], gj[3], gk[3];
        for (int c = 0; c < 3; ++c) {
          // a depends on r_i, r_j; b on r_i, r_k; d on r_j, r_k; cos on all three.
          gj[c] = dT_da * u[c] / ra - dT_dd * w[c] / rd + dT_dc * dcu[c];
          gk[c] = dT_db * v[c] / rb + dT_dd * w[c] / rd + dT_dc * dcv[c];
          gi[c] = -dT_da * u[c] / ra - dT_db * v[c] / rb - dT_dc * (dcu[c] + dcv[c]);
        }
        sink(nb[a], gj, s);
        sink(nb[b], gk, s);
        sink(i, gi, s);
      }
    }
  }
}

int max_sf(const Pot& P) {
  int m = 0;
  for (const auto& v : P.sf) m = std::max(m, (int)v.size());
  return m;
}

void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

void neighbour_lists(const Pot& P, int64_t N, const double* pos, const double* box, int use_cells,
                     std::vector<std::vector<int64_t>>& nb) {
  if (use_cells)
    neighbours_cells(N, pos, box, P.rc_max, nb);
  else
    neighbours_brute(N, pos, box, P.rc_max, nb);
}

}  // namespace

extern "C" {

int oracle_max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Neighbour lists (ascending indices) by brute force (use_cells = 0) or by
// the cell list (use_cells = 1).  counts[N]; list[N][cap].  Returns 1 if some
// atom has more than cap neighbours (its count is still exact), else 0.
int oracle_neighbors(int64_t N, const double* pos, const double* box, double rc, int use_cells,
                     int64_t cap, int32_t* counts, int32_t* list) {
  std::vector<std::vector<int64_t>> nb;
  if (use_cells)
    neighbours_cells(N, pos, box, rc, nb);
  else
    neighbours_brute(N, pos, box, rc, nb);
  int over = 0;
  for (int64_t i = 0; i < N; ++i) {
    counts[i] = (int32_t)nb[i].size();
    if ((int64_t)nb[i].size() > cap) over = 1;
    for (size_t a = 0; a < nb[i].size() && (int64_t)a < cap; ++a) list[i * cap + a] = (int32_t)nb[i][a];
  }
  return over;
}

// Raw descriptors G[N][ld] (row i holds the SFs of element types[i] in table order).
int oracle_descriptors(const opot* p, int64_t N, const double* pos, const int* types, const double* box,
                       double* G, int ld, int use_cells, int nthreads) {
  set_threads(nthreads);
  Pot P = parse(p);
  if (ld < max_sf(P)) return -1;
  std::vector<std::vector<int64_t>> nb;
  neighbour_lists(P, N, pos, box, use_cells, nb);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < N; ++i) descriptors(P, i, nb[i], pos, types, box, G + i * ld);
  return 0;
}

// Energy, per-atom energies and forces.  Optional G and dEdG [N][ld].
int oracle_compute(const opot* p, int64_t N, const double* pos, const int* types, const double* box,
                   double* E, double* Ei, double* F, double* Gout, double* dEdGout, int ld, int use_cells,
                   int nthreads) {
  set_threads(nthreads);
  Pot P = parse(p);
  const int ms = max_sf(P);
  if (ld < ms) return -1;
  std::vector<std::vector<int64_t>> nb;
  neighbour_lists(P, N, pos, box, use_cells, nb);
  std::vector<double> G((size_t)N * ms, 0.0), C((size_t)N * ms, 0.0), ei(N);
  // Pass 1: descriptors, atomic energies and dE_i/dG_i.
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < N; ++i) {
    descriptors(P, i, nb[i], pos, types, box, &G[i * ms]);
    ei[i] = network(P, types[i], &G[i * ms], &C[i * ms]);
  }
  // Pass 2: forces f_m = -sum_i sum_s dE_i/dG_is dG_is/dr_m, per-thread buffers.
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> Fb(nt, std::vector<double>((size_t)3 * N, 0.0));
#pragma omp parallel
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    std::vector<double>& fb = Fb[t];
#pragma omp for schedule(dynamic, 8)
    for (int64_t i = 0; i < N; ++i) {
      const double* c = &C[i * ms];
      descriptor_gradients(P, i, nb[i], pos, types, box, [&](int64_t m, const double g[3], int s) {
        for (int a = 0; a < 3; ++a) fb[3 * m + a] -= c[s] * g[a];
      });
    }
  }
  for (int64_t k = 0; k < 3 * N; ++k) {
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += Fb[t][k];
    if (F) F[k] = s;
  }
  double Et = 0.0;
  for (int64_t i = 0; i < N; ++i) Et += ei[i];
  if (E) *E = Et;
  if (Ei)
    for (int64_t i = 0; i < N; ++i) Ei[i] = ei[i];
  for (int64_t i = 0; i < N; ++i)
    for (int s = 0; s < ms; ++s) {
      if (Gout) Gout[i * ld + s] = G[i * ms + s];
      if (dEdGout) dEdGout[i * ld + s] = C[i * ms + s];
    }
  return 0;
}

// The same evaluation restricted to the centres [lo, hi): their atomic
// energies go to Ei[0 .. hi-lo), and the force terms they contribute,
// -dE_i/dG_is dG_is/dr_m for every atom m, are ADDED to F (3 N values, set
// by the caller).  Summed over centre ranges that cover every atom, this is
// oracle_compute (forces are a sum over centres, Fig. 1(b) step 3); it lets a
// large box be evaluated in parts that each finish.  Neighbours come from the
// cell list of the whole box.
int oracle_compute_centres(const opot* p, int64_t N, const double* pos, const int* types, const double* box,
                           int64_t lo, int64_t hi, double* Ei, double* F, int nthreads) {
  if (lo < 0 || hi > N || lo > hi) return -1;
  set_threads(nthreads);
  Pot P = parse(p);
  const int ms = max_sf(P);
  Cells C = build_cells(N, pos, box, P.rc_max);
  const int64_t n = hi - lo;
  std::vector<std::vector<int64_t>> nb(n);
  std::vector<double> G((size_t)n * ms, 0.0), Cc((size_t)n * ms, 0.0);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t q = 0; q < n; ++q) {
    neighbours_of(C, lo + q, pos, box, P.rc_max, nb[q]);
    descriptors(P, lo + q, nb[q], pos, types, box, &G[q * ms]);
    Ei[q] = network(P, types[lo + q], &G[q * ms], &Cc[q * ms]);
  }
  int nt = 1;
#ifdef _OPENMP
  nt = omp_get_max_threads();
#endif
  std::vector<std::vector<double>> Fb(nt, std::vector<double>((size_t)3 * N, 0.0));
#pragma omp parallel
  {
    int t = 0;
#ifdef _OPENMP
    t = omp_get_thread_num();
#endif
    std::vector<double>& fb = Fb[t];
#pragma omp for schedule(dynamic, 8)
    for (int64_t q = 0; q < n; ++q) {
      const double* c = &Cc[q * ms];
      descriptor_gradients(P, lo + q, nb[q], pos, types, box, [&](int64_t m, const double g[3], int s) {
        for (int a = 0; a < 3; ++a) fb[3 * m + a] -= c[s] * g[a];
      });
    }
  }
  for (int64_t k = 0; k < 3 * N; ++k) {
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += Fb[t][k];
    F[k] += s;
  }
  return 0;
}

// Descriptor-Jacobian-vector product v[i][s] = sum_m delta_m . dG_is/dr_m
// (raw G), for the force term of the training-loss gradient.
int oracle_sf_jvp(const opot* p, int64_t N, const double* pos, const int* types, const double* box,
                  const double* delta, double* v, int ld, int use_cells, int nthreads) {
  set_threads(nthreads);
  Pot P = parse(p);
  if (ld < max_sf(P)) return -1;
  std::vector<std::vector<int64_t>> nb;
  neighbour_lists(P, N, pos, box, use_cells, nb);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < N; ++i) {
    double* vi = v + i * ld;
    for (int s = 0; s < ld; ++s) vi[s] = 0.0;
    descriptor_gradients(P, i, nb[i], pos, types, box, [&](int64_t m, const double g[3], int s) {
      vi[s] += delta[3 * m] * g[0] + delta[3 * m + 1] * g[1] + delta[3 * m + 2] * g[2];
    });
  }
  return 0;
}

// Per-atom energies and forces of selected atoms only, for boxes too large for
// oracle_compute: uses the cell list, computes G and dE/dG of every centre
// within the cutoff of a selected atom and sums their gradient terms on it.
int oracle_sampled(const opot* p, int64_t N, const double* pos, const int* types, const double* box,
                   int64_t n_samp, const int64_t* idx, double* Ei, double* F, int nthreads) {
  set_threads(nthreads);
  Pot P = parse(p);
  const int ms = max_sf(P);
  Cells C = build_cells(N, pos, box, P.rc_max);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t q = 0; q < n_samp; ++q) {
    const int64_t a = idx[q];
    std::vector<int64_t> nba, nbi;
    std::vector<double> G(ms), c(ms);
    neighbours_of(C, a, pos, box, P.rc_max, nba);
    descriptors(P, a, nba, pos, types, box, G.data());
    Ei[q] = network(P, types[a], G.data(), nullptr);
    double f[3] = {0.0, 0.0, 0.0};
    // Centres whose energy depends on r_a: a itself and its neighbours.
    std::vector<int64_t> centres(1, a);
    centres.insert(centres.end(), nba.begin(), nba.end());
    for (int64_t i : centres) {
      neighbours_of(C, i, pos, box, P.rc_max, nbi);
      descriptors(P, i, nbi, pos, types, box, G.data());
      network(P, types[i], G.data(), c.data());
      descriptor_gradients(P, i, nbi, pos, types, box, [&](int64_t m, const double g[3], int s) {
        if (m != a) return;
        for (int k = 0; k < 3; ++k) f[k] -= c[s] * g[k];
      });
    }
    for (int k = 0; k < 3; ++k) F[3 * q + k] = f[k];
  }
  return 0;
}

}  // extern "C"
