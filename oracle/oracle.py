"""ctypes front end of the FP64 CPU oracle (``nnp_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark; never by the library.  It takes the
potential as plain objects (an SF table of records with ``centre, kind, nbr,
eta, rs, zeta, lam, rc, shift, scale`` and networks with ``W``/``b`` lists) and
numpy arrays, and imports nothing from the HIP package.

Also holds the training-loss gradient of the differentiation form (loss of
energies and forces, gradient with respect to every network parameter),
written with plain float64 PyTorch autograd on the CPU over the per-atom
networks, with the descriptor-Jacobian-vector products taken from the C++
oracle; and a velocity Verlet integrator over the oracle's forces.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nnp_oracle.cpp")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "libnnp_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ -O2 -fopenmp (no fast-math)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, SRC]
        )
        os.replace(tmp, LIB)
    return LIB


class _OPot(C.Structure):
    _fields_ = [
        ("n_el", C.c_int),
        ("n_sf", C.c_int),
        ("centre", C.POINTER(C.c_int)),
        ("kind", C.POINTER(C.c_int)),
        ("nbr0", C.POINTER(C.c_int)),
        ("nbr1", C.POINTER(C.c_int)),
        ("eta", C.POINTER(C.c_double)),
        ("rs", C.POINTER(C.c_double)),
        ("zeta", C.POINTER(C.c_double)),
        ("lam", C.POINTER(C.c_double)),
        ("rc", C.POINTER(C.c_double)),
        ("shift", C.POINTER(C.c_double)),
        ("scale", C.POINTER(C.c_double)),
        ("n_layers", C.c_int),
        ("sizes", C.POINTER(C.c_int)),
        ("params", C.POINTER(C.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        L.oracle_neighbors.argtypes = [C.c_int64, dp, dp, C.c_double, C.c_int, C.c_int64,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.oracle_descriptors.argtypes = [C.POINTER(_OPot), C.c_int64, dp, ip, dp, dp, C.c_int, C.c_int, C.c_int]
        L.oracle_compute.argtypes = [C.POINTER(_OPot), C.c_int64, dp, ip, dp, dp, dp, dp, dp, dp,
                                     C.c_int, C.c_int, C.c_int]
        L.oracle_sf_jvp.argtypes = [C.POINTER(_OPot), C.c_int64, dp, ip, dp, dp, dp, C.c_int, C.c_int, C.c_int]
        L.oracle_sampled.argtypes = [C.POINTER(_OPot), C.c_int64, dp, ip, dp, C.c_int64,
                                     C.POINTER(C.c_int64), dp, dp, C.c_int]
        L.oracle_compute_centres.argtypes = [C.POINTER(_OPot), C.c_int64, dp, ip, dp, C.c_int64, C.c_int64, dp, dp,
                                             C.c_int]
        L.oracle_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class Potential:
    """Oracle-side copy of a potential: SF table + per-element networks."""

    def __init__(self, table, nets, n_el=None):
        self.table = list(table)
        self.nets = list(nets)
        self.n_el = n_el if n_el is not None else len(nets)
        t = self.table
        self._a = dict(
            centre=np.array([s.centre for s in t], dtype=np.int32),
            kind=np.array([s.kind for s in t], dtype=np.int32),
            nbr0=np.array([s.nbr[0] for s in t], dtype=np.int32),
            nbr1=np.array([s.nbr[-1] for s in t], dtype=np.int32),
            eta=np.array([s.eta for s in t], dtype=np.float64),
            rs=np.array([s.rs for s in t], dtype=np.float64),
            zeta=np.array([s.zeta for s in t], dtype=np.float64),
            lam=np.array([s.lam for s in t], dtype=np.float64),
            rc=np.array([s.rc for s in t], dtype=np.float64),
            shift=np.array([s.shift for s in t], dtype=np.float64),
            scale=np.array([s.scale for s in t], dtype=np.float64),
        )
        n_layers = len(nets[0].W)
        sizes = []
        for n in nets:
            if len(n.W) != n_layers:
                raise ValueError("all networks must have the same depth")
            sizes += [n.W[0].shape[1]] + [w.shape[0] for w in n.W]
        self._sizes = np.array(sizes, dtype=np.int32)
        self._params = np.concatenate(
            [np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in zip(n.W, n.b)]) for n in nets]
        ).astype(np.float64)
        a = self._a
        self._s = _OPot(self.n_el, len(t), _ip(a["centre"]), _ip(a["kind"]), _ip(a["nbr0"]), _ip(a["nbr1"]),
                        _dp(a["eta"]), _dp(a["rs"]), _dp(a["zeta"]), _dp(a["lam"]), _dp(a["rc"]),
                        _dp(a["shift"]), _dp(a["scale"]), n_layers, _ip(self._sizes), _dp(self._params))
        self.n_sf = [int(np.sum(a["centre"] == e)) for e in range(self.n_el)]
        self.max_sf = max(self.n_sf)
        self.rc = float(np.max(a["rc"]))

    # -- helpers ---------------------------------------------------------
    @staticmethod
    def _inputs(pos, types, box):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        types = np.ascontiguousarray(types, dtype=np.int32)
        box = np.ascontiguousarray(box, dtype=np.float64)
        return pos, types, box

    def descriptors(self, pos, types, box, use_cells=False, nthreads=0):
        pos, types, box = self._inputs(pos, types, box)
        n = pos.shape[0]
        G = np.zeros((n, self.max_sf))
        rc = lib().oracle_descriptors(C.byref(self._s), n, _dp(pos), _ip(types), _dp(box), _dp(G),
                                      self.max_sf, int(use_cells), nthreads)
        assert rc == 0
        return G

    def compute(self, pos, types, box, use_cells=False, nthreads=0, want_g=False):
        """Returns dict(E, Ei, F[, G, dEdG])."""
        pos, types, box = self._inputs(pos, types, box)
        n = pos.shape[0]
        E = np.zeros(1)
        Ei = np.zeros(n)
        F = np.zeros((n, 3))
        G = np.zeros((n, self.max_sf)) if want_g else None
        D = np.zeros((n, self.max_sf)) if want_g else None
        null = C.POINTER(C.c_double)()
        rc = lib().oracle_compute(C.byref(self._s), n, _dp(pos), _ip(types), _dp(box), _dp(E), _dp(Ei), _dp(F),
                                  _dp(G) if want_g else null, _dp(D) if want_g else null, self.max_sf,
                                  int(use_cells), nthreads)
        assert rc == 0
        out = dict(E=float(E[0]), Ei=Ei, F=F)
        if want_g:
            out["G"] = G
            out["dEdG"] = D
        return out

    def sf_jvp(self, pos, types, box, delta, use_cells=False, nthreads=0):
        pos, types, box = self._inputs(pos, types, box)
        delta = np.ascontiguousarray(delta, dtype=np.float64)
        n = pos.shape[0]
        v = np.zeros((n, self.max_sf))
        rc = lib().oracle_sf_jvp(C.byref(self._s), n, _dp(pos), _ip(types), _dp(box), _dp(delta), _dp(v),
                                 self.max_sf, int(use_cells), nthreads)
        assert rc == 0
        return v

    def compute_centres(self, pos, types, box, lo, hi, F, nthreads=0):
        """E_i of the centres [lo, hi) (returned) and their force terms added
        into F (n x 3, float64, set by the caller); cell list, any box size."""
        pos, types, box = self._inputs(pos, types, box)
        assert F.dtype == np.float64 and F.flags.c_contiguous and F.shape == (pos.shape[0], 3)
        Ei = np.zeros(hi - lo)
        rc = lib().oracle_compute_centres(C.byref(self._s), pos.shape[0], _dp(pos), _ip(types), _dp(box),
                                          int(lo), int(hi), _dp(Ei), _dp(F), nthreads)
        assert rc == 0
        return Ei

    def sampled(self, pos, types, box, idx, nthreads=0):
        """E_i and F_i of the atoms ``idx`` only (cell list; any box size)."""
        pos, types, box = self._inputs(pos, types, box)
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        Ei = np.zeros(len(idx))
        F = np.zeros((len(idx), 3))
        rc = lib().oracle_sampled(C.byref(self._s), pos.shape[0], _dp(pos), _ip(types), _dp(box), len(idx),
                                  idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(Ei), _dp(F), nthreads)
        assert rc == 0
        return Ei, F


def neighbors(pos, box, rc, use_cells=False, cap=256):
    """(counts[N], list[N][cap]) of the oracle's neighbour search."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    n = pos.shape[0]
    counts = np.zeros(n, dtype=np.int32)
    lst = np.full((n, cap), -1, dtype=np.int32)
    over = lib().oracle_neighbors(n, _dp(pos), _dp(box), rc, int(use_cells), cap,
                                  counts.ctypes.data_as(C.POINTER(C.c_int32)),
                                  lst.ctypes.data_as(C.POINTER(C.c_int32)))
    if over:
        raise ValueError("neighbour capacity exceeded")
    return counts, lst


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ---------------------------------------------------------------------------
# Differentiation form: energy+force loss and its parameter gradient
# ---------------------------------------------------------------------------
def loss_terms(E, Ehat, N, F, Fhat, wF=0.1):
    """L = (1/B) sum_b ((E_b - Ehat_b)/N_b)^2 + wF/(3 sum_b N_b) sum (F - Fhat)^2.

    Returns (L, dL/dE [B], dL/dF [sum N, 3]).
    """
    E = np.asarray(E, dtype=np.float64)
    Ehat = np.asarray(Ehat, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    B = len(E)
    rE = (E - Ehat) / N
    nF = 3.0 * np.sum(N)
    dF = F - Fhat
    L = np.mean(rE ** 2) + wF * np.sum(dF ** 2) / nF
    gE = 2.0 * rE / N / B
    gF = 2.0 * wF * dF / nF
    return float(L), gE, gF


def batch_energy_forces(pot: Potential, boxes, nthreads=0):
    Es, Fs = [], []
    for b in boxes:
        out = pot.compute(b.pos, b.types, b.box, nthreads=nthreads)
        Es.append(out["E"])
        Fs.append(out["F"])
    return np.array(Es), np.concatenate(Fs, axis=0)


def loss(pot: Potential, boxes, Ehat, Fhat, wF=0.1, nthreads=0):
    E, F = batch_energy_forces(pot, boxes, nthreads)
    N = [b.n_atoms for b in boxes]
    return loss_terms(E, Ehat, N, F, Fhat, wF)[0]


def loss_and_grad(pot: Potential, boxes, Ehat, Fhat, wF=0.1, nthreads=0):
    """Loss and its gradient w.r.t. the flat parameter vector (element by
    element, layer by layer, W row-major then b).

    With delta = dL/dF and g_b = dL/dE_b, and F_m = -sum_i sum_s
    dE_i/dG_is dG_is/dr_m, the gradient is
        sum_b g_b dE_b/dtheta - sum_i d/dtheta <dE_i/dG_i (theta), v_i>,
    where v_i[s] = sum_m delta_m . dG_is/dr_m does not depend on theta.
    The first and second derivatives of each atom's network are taken with
    float64 torch autograd on the CPU; v comes from ``Potential.sf_jvp``.
    """
    import torch

    E, F = batch_energy_forces(pot, boxes, nthreads)
    N = [b.n_atoms for b in boxes]
    L, gE, gF = loss_terms(E, Ehat, N, F, Fhat, wF)
    Gs, Vs, Ts, Bs = [], [], [], []
    o = 0
    for bi, b in enumerate(boxes):
        n = b.n_atoms
        Gs.append(pot.descriptors(b.pos, b.types, b.box, nthreads=nthreads))
        Vs.append(pot.sf_jvp(b.pos, b.types, b.box, gF[o:o + n], nthreads=nthreads))
        Ts.append(b.types)
        Bs.append(np.full(n, bi))
        o += n
    G = np.concatenate(Gs)
    V = np.concatenate(Vs)
    T = np.concatenate(Ts)
    Bidx = np.concatenate(Bs)
    shift = pot._a["shift"]
    scale = pot._a["scale"]
    centre = pot._a["centre"]
    params = []
    total = torch.zeros((), dtype=torch.float64)
    for e, net in enumerate(pot.nets):
        sel = np.nonzero(T == e)[0]
        ns = pot.n_sf[e]
        sh = torch.tensor(shift[centre == e])
        sc = torch.tensor(scale[centre == e])
        Ws = [torch.tensor(w, requires_grad=True) for w in net.W]
        bs = [torch.tensor(bb, requires_grad=True) for bb in net.b]
        for w, bb in zip(Ws, bs):
            params += [w, bb]
        g_raw = torch.tensor(G[sel, :ns], requires_grad=True)
        h = (g_raw - sh) / sc
        for l, (w, bb) in enumerate(zip(Ws, bs)):
            z = h @ w.T + bb
            h = torch.tanh(z) if l < len(Ws) - 1 else z
        Ei = h[:, 0]
        (c,) = torch.autograd.grad(Ei.sum(), g_raw, create_graph=True)  # dE_i/dG_i, raw G
        gE_atom = torch.tensor(gE[Bidx[sel]])
        total = total + torch.sum(gE_atom * Ei) - torch.sum(c * torch.tensor(V[sel, :ns]))
    grads = torch.autograd.grad(total, params)
    flat = np.concatenate([g.detach().numpy().ravel() for g in grads])
    return L, flat


# ---------------------------------------------------------------------------
# Molecular dynamics at constant N, V, E (the setting of the method, Sec. 4)
# ---------------------------------------------------------------------------
# Unit conversions from the CODATA electron volt (J) and atomic mass constant
# (kg), with 1 A = 1e-10 m and 1 fs = 1e-15 s.
EV_J = 1.602176634e-19
AMU_KG = 1.66053906660e-27
ACCEL_CONV = (EV_J / 1e-10) / AMU_KG / (1e-10 / 1e-15 ** 2)  # eV/(A amu) -> A/fs^2
KE_CONV = AMU_KG * (1e-10 / 1e-15) ** 2 / EV_J                # amu (A/fs)^2 -> eV


def kinetic_energy(vel, m_atom):
    """sum_i m_i |v_i|^2 / 2 in eV (vel in A/fs, masses in amu)."""
    return 0.5 * KE_CONV * float(np.sum(m_atom[:, None] * vel * vel))


def velocity_verlet(pot: Potential, pos, vel, types, box, masses, dt, n_steps, nthreads=0):
    """Velocity Verlet, the textbook NVE integrator (the paper does not name
    its integrator): half kick with F(t), drift by dt, forces at the new
    positions, half kick with F(t + dt).  Positions are wrapped into [0, L)
    after each drift.  Returns (pos, vel, F, epot[n+1], ekin[n+1]) in FP64."""
    types = np.asarray(types)
    box = np.asarray(box, dtype=np.float64)
    m_atom = np.asarray(masses, dtype=np.float64)[types]
    x = np.array(pos, dtype=np.float64)
    v = np.array(vel, dtype=np.float64)
    out = pot.compute(x, types, box, use_cells=True, nthreads=nthreads)
    F = out["F"]
    epot, ekin = [out["E"]], [kinetic_energy(v, m_atom)]
    for _ in range(n_steps):
        v = v + 0.5 * dt * ACCEL_CONV * F / m_atom[:, None]
        x = x + dt * v
        x = x - box * np.floor(x / box)
        out = pot.compute(x, types, box, use_cells=True, nthreads=nthreads)
        F = out["F"]
        v = v + 0.5 * dt * ACCEL_CONV * F / m_atom[:, None]
        epot.append(out["E"])
        ekin.append(kinetic_energy(v, m_atom))
    return x, v, F, np.array(epot), np.array(ekin)
