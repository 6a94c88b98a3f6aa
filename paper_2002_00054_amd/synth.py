"""Seeded synthetic inputs for the Behler-Parrinello water potential.

This module is shared by the HIP path and by the CPU oracle used in tests.  It
holds no arithmetic of the method itself (no cutoff, no symmetry function, no
network evaluation): only

* water-like periodic boxes (positions and element types),
* the symmetry-function parameter table (which SFs exist, with which eta,
  zeta, lambda), and
* Xavier-initialised network weights,

all drawn from ``numpy.random.default_rng`` with fixed seeds so that every
consumer sees bit-identical inputs.

Element ids: H = 0, O = 1 (the index into ``ELEMENTS``).

The paper's own water model (n2p2 H2O, 6.4 A cutoff; Sec. 3.3 and Sec. 4.1)
and its training data are not available, so these boxes and this table stand
in for it with the shapes of the paper's water workload: liquid-density water,
~86 neighbours per atom inside a 6 A cosine cutoff, two elements, per-element
networks of two hidden layers of ~30 units (Sec. 3.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ELEMENTS = ("H", "O")
H, O = 0, 1

#: Lattice spacing of one water molecule per site at ~1 g/cm^3 (A).
WATER_SPACING = 3.105
#: O-H bond length (A) and H-O-H angle (degrees) of the rigid monomer.
OH_BOND = 0.96
HOH_ANGLE_DEG = 104.5
#: Half-width of the uniform per-coordinate jitter of the O site (A).
JITTER = 0.3
#: Cosine cutoff radius of every symmetry function (A).
RCUT = 6.0


# --------------------------------------------------------------------------
# Boxes
# --------------------------------------------------------------------------
@dataclass
class Box:
    """One periodic orthorhombic structure: positions (A), types, box edges."""

    pos: np.ndarray  # float64 [N, 3], wrapped into [0, L)
    types: np.ndarray  # int32 [N]
    box: np.ndarray  # float64 [3]
    seed: int = 0
    n_side: int = 0

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])


def _quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [M,3,3] from unit quaternions [M,4] (w, x, y, z)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = np.empty((q.shape[0], 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def water_box(n: int, seed: int, spacing: float = WATER_SPACING) -> Box:
    """n^3 water molecules on a jittered cubic lattice, one per site.

    * box edge L = spacing * n (3.105 A gives ~1 g/cm^3);
    * O at spacing*(ix, iy, iz) + U(-0.3, 0.3)^3, sites in C order of
      ``meshgrid(indexing='ij')``;
    * each molecule rotated by a uniform random rotation (normalised
      N(0,1)^4 quaternion); H1 = O + R (0.96, 0, 0),
      H2 = O + R (0.96 cos 104.5deg, 0.96 sin 104.5deg, 0);
    * atoms interleaved O, H, H per molecule, wrapped into [0, L).

    The jitter is drawn before the quaternions, both from
    ``default_rng(seed)``.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    m = n * n * n
    L = spacing * n
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    sites = spacing * np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    jitter = rng.uniform(-JITTER, JITTER, size=(m, 3))
    q = rng.standard_normal(size=(m, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rot = _quat_to_matrix(q)
    th = math.radians(HOH_ANGLE_DEG)
    h1_body = np.array([OH_BOND, 0.0, 0.0])
    h2_body = np.array([OH_BOND * math.cos(th), OH_BOND * math.sin(th), 0.0])
    o = sites + jitter
    h1 = o + rot @ h1_body
    h2 = o + rot @ h2_body
    pos = np.empty((3 * m, 3))
    pos[0::3] = o
    pos[1::3] = h1
    pos[2::3] = h2
    pos = np.mod(pos, L)
    pos[pos >= L] = 0.0  # np.mod can round up to L for tiny negatives
    types = np.empty(3 * m, dtype=np.int32)
    types[0::3] = O
    types[1::3] = H
    types[2::3] = H
    return Box(pos=pos, types=types, box=np.array([L, L, L]), seed=seed, n_side=n)


def tile_box(b: Box, k: int) -> Box:
    """Periodic k x k x k replica of ``b`` (no re-jitter).

    Atom order: replica-major, replica index r = (a*k + b)*k + c for the
    shift (a, b, c) * L, each replica holding ``b``'s atoms in order.
    """
    n = b.n_atoms
    shifts = np.array([(a, bb, c) for a in range(k) for bb in range(k) for c in range(k)], dtype=np.float64)
    pos = (b.pos[None, :, :] + shifts[:, None, :] * b.box[None, None, :]).reshape(-1, 3)
    types = np.tile(b.types, k ** 3)
    return Box(pos=pos, types=types.astype(np.int32), box=b.box * k, seed=b.seed, n_side=b.n_side * k)


# Workload recipes ----------------------------------------------------------
#: (n, seeds) for the named workloads; atoms = 3 n^3, L = 3.105 n.
CONFIG0 = dict(n=4, scaling_seed=0, parity_seeds=(1, 2, 3, 4))  # 192 atoms, 12.42 A
CONFIG1 = dict(n=16, seeds=(11, 12, 13))  # 12,288 atoms, 49.68 A
CONFIG2 = dict(n=88, seed=22)  # 2,044,416 atoms, 273.24 A
SWEEP_N = (16, 24, 32, 44, 56, 70, 88)  # weak-scaling sweep, seed 100 + n

# Standard atomic weights of H and O (amu), the masses of the MD runs.
WATER_MASSES = (1.00794, 15.9994)


def thermal_velocities(types: np.ndarray, masses=WATER_MASSES, temperature: float = 300.0,
                       seed: int = 0) -> np.ndarray:
    """Seeded initial velocities (A/fs): each component N(0, kB T / m) with
    kB = 8.617333262e-5 eV/K and 1 amu (A/fs)^2 = 103.6427 eV, the centre of
    mass at rest."""
    m = np.asarray(masses, dtype=np.float64)[np.asarray(types)]
    sigma = np.sqrt(8.617333262e-5 * temperature / (m * 103.64269652680505))
    v = np.random.default_rng(seed).normal(size=(len(m), 3)) * sigma[:, None]
    return v - np.sum(m[:, None] * v, axis=0) / np.sum(m)


def training_batch_sizes(n_struct: int = 32, seed: int = 4) -> np.ndarray:
    """Lattice sides n in {4..8} of the uneven training batch (192-1536 atoms)."""
    return np.random.default_rng(seed).integers(4, 9, size=n_struct)


def training_batch(n_struct: int = 32, first_seed: int = 40) -> list[Box]:
    """32 boxes of uneven size, box b with side n_b and seed first_seed + b."""
    sides = training_batch_sizes(n_struct)
    return [water_box(int(s), first_seed + i) for i, s in enumerate(sides)]


# --------------------------------------------------------------------------
# Symmetry-function table
# --------------------------------------------------------------------------
@dataclass
class SF:
    """One symmetry function of one centre element.

    kind 2: radial, neighbour element ``nbr[0]``;
    kind 3: narrow angular, unordered neighbour-element pair ``nbr``;
    kind 9: wide angular (no r_jk factor), unordered pair ``nbr``.
    ``shift``/``scale`` are the frozen centring/scaling constants
    (G_scaled = (G - shift) / scale); 0/1 until set.
    """

    centre: int
    kind: int
    nbr: tuple
    eta: float
    rs: float = 0.0
    zeta: float = 1.0
    lam: float = 1.0
    rc: float = RCUT
    shift: float = 0.0
    scale: float = 1.0


#: Radial exponents (A^-2): 0.001 * 500^(k/5), k = 0..5, log-spaced in [0.001, 0.5].
RADIAL_ETAS = tuple(0.001 * 500.0 ** (k / 5.0) for k in range(6))
#: Angular base list: (eta [A^-2], zeta, lambda).
ANGULAR_BASE = (
    (0.001, 1, -1.0),
    (0.001, 1, +1.0),
    (0.001, 4, -1.0),
    (0.001, 4, +1.0),
    (0.03, 2, +1.0),
    (0.03, 16, +1.0),
)
#: Neighbour-pair classes in table order.
PAIR_CLASSES = ((H, H), (H, O), (O, O))


def water_sf_table() -> list[SF]:
    """The water SF table: 27 SFs for an H centre, 30 for an O centre.

    Order per centre: radial with neighbour H (6 eta ascending), radial with
    neighbour O (6 eta), then angular blocks HH, HO, OO, each holding the
    first 5 (H centre) or all 6 (O centre) entries of ``ANGULAR_BASE``.
    """
    table: list[SF] = []
    for centre in (H, O):
        for nb in (H, O):
            for eta in RADIAL_ETAS:
                table.append(SF(centre, 2, (nb,), eta))
        n_ang = 5 if centre == H else 6
        for cls in PAIR_CLASSES:
            for eta, zeta, lam in ANGULAR_BASE[:n_ang]:
                table.append(SF(centre, 3, cls, eta, 0.0, float(zeta), lam))
    return table


def sf_counts(table: list[SF], n_el: int = 2) -> list[int]:
    return [sum(1 for s in table if s.centre == e) for e in range(n_el)]


# --------------------------------------------------------------------------
# Network weights
# --------------------------------------------------------------------------
@dataclass
class Net:
    """Feed-forward net: tanh hidden layers, linear output.

    ``W[l]`` has shape [out, in] (row-major), ``b[l]`` shape [out].
    """

    W: list = field(default_factory=list)
    b: list = field(default_factory=list)

    @property
    def sizes(self) -> list[int]:
        return [self.W[0].shape[1]] + [w.shape[0] for w in self.W]

    def flat(self) -> np.ndarray:
        """Parameters flattened layer by layer as W (row-major) then b."""
        parts = []
        for w, bb in zip(self.W, self.b):
            parts.append(w.ravel())
            parts.append(bb.ravel())
        return np.concatenate(parts)

    @staticmethod
    def from_flat(flat: np.ndarray, sizes: list[int]) -> "Net":
        net = Net()
        o = 0
        for l in range(len(sizes) - 1):
            fi, fo = sizes[l], sizes[l + 1]
            net.W.append(np.array(flat[o:o + fo * fi]).reshape(fo, fi))
            o += fo * fi
            net.b.append(np.array(flat[o:o + fo]))
            o += fo
        return net


HIDDEN = (25, 25)


def xavier_nets(n_sf: list[int], seed: int = 1000, hidden=HIDDEN, bias_halfwidth: float = 0.0) -> list[Net]:
    """Glorot-uniform weights, W ~ U(+-sqrt(6/(fan_in+fan_out))).

    Drawn from ``default_rng(seed)`` element by element, all weight matrices
    of an element first (W1, W2, W3), then, if ``bias_halfwidth`` > 0, its
    biases b1, b2, b3 ~ U(+-bias_halfwidth); otherwise biases are zero.
    """
    rng = np.random.default_rng(seed)
    nets = []
    for ns in n_sf:
        sizes = [ns, *hidden, 1]
        net = Net()
        for l in range(len(sizes) - 1):
            fi, fo = sizes[l], sizes[l + 1]
            lim = math.sqrt(6.0 / (fi + fo))
            net.W.append(rng.uniform(-lim, lim, size=(fo, fi)))
        for l in range(len(sizes) - 1):
            fo = sizes[l + 1]
            if bias_halfwidth > 0:
                net.b.append(rng.uniform(-bias_halfwidth, bias_halfwidth, size=fo))
            else:
                net.b.append(np.zeros(fo))
        nets.append(net)
    return nets


def water_nets(seed: int = 1000) -> list[Net]:
    """The main (student) potential's networks."""
    return xavier_nets(sf_counts(water_sf_table()), seed)


def teacher_nets(seed: int = 7) -> list[Net]:
    """The fixed teacher that labels the training batch (biases U(+-0.1))."""
    return xavier_nets(sf_counts(water_sf_table()), seed, bias_halfwidth=0.1)


def flat_params(nets: list[Net]) -> np.ndarray:
    """All parameters, element by element, in ``Net.flat`` order."""
    return np.concatenate([n.flat() for n in nets])


# --------------------------------------------------------------------------
# Frozen scaling constants
# --------------------------------------------------------------------------
def load_scaling(path: str | None = None) -> dict:
    """Frozen per-(element, SF) shift/scale of the water table (JSON)."""
    import json
    import os

    if path is None:
        path = os.path.join(os.path.dirname(__file__), "data", "water_scaling.json")
    with open(path) as f:
        return json.load(f)


def water_table_scaled(path: str | None = None) -> list[SF]:
    """``water_sf_table`` with the stored shift/scale filled in."""
    sc = load_scaling(path)
    table = water_sf_table()
    counters = {e: 0 for e in range(len(ELEMENTS))}
    for s in table:
        e = s.centre
        k = counters[e]
        s.shift = float(sc["shift"][ELEMENTS[e]][k])
        s.scale = float(sc["scale"][ELEMENTS[e]][k])
        counters[e] += 1
    return table


# --------------------------------------------------------------------------
# Second workload: a single-element fcc metal with a short cutoff (Ni-like)
# --------------------------------------------------------------------------
#: fcc lattice constant (A), cutoff of the paper's Ni model (A), displacement
#: half-width (A) of each coordinate, and the atomic weight (amu).
NI_LATTICE = 3.52
NI_RCUT = 3.9
NI_JITTER = 0.1
NI_MASS = 58.6934
#: fcc basis in units of the lattice constant.
FCC_BASIS = ((0.0, 0.0, 0.0), (0.5, 0.5, 0.0), (0.5, 0.0, 0.5), (0.0, 0.5, 0.5))


def fcc_box(n: int, seed: int, a: float = NI_LATTICE, jitter: float = NI_JITTER) -> Box:
    """n^3 cubic cells of 4 atoms (L = n a), every coordinate displaced by
    U(+-jitter) drawn from ``default_rng(seed)``, all atoms of type 0, sites in
    C order of the cells then the basis, wrapped into [0, L)."""
    ijk = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), axis=-1).reshape(-1, 3)
    pos = ((ijk[:, None, :] + np.asarray(FCC_BASIS)[None, :, :]) * a).reshape(-1, 3)
    if jitter > 0:
        pos = pos + np.random.default_rng(seed).uniform(-jitter, jitter, size=pos.shape)
    L = n * a
    box = np.array([L, L, L])
    pos = np.mod(pos, box)
    pos[pos >= L] = 0.0
    return Box(pos=pos, types=np.zeros(len(pos), dtype=np.int32), box=box, seed=seed, n_side=n)


#: Radial exponents of the Ni table (A^-2): 0.003 * 500^(k/7), k = 0..7.
NI_RADIAL_ETAS = tuple(0.003 * 500.0 ** (k / 7.0) for k in range(8))
#: Angular list of the Ni table: (eta [A^-2], zeta, lambda); the same (zeta,
#: lambda, eta-index) structure as the water table's base list.
NI_ANGULAR = (
    (0.003, 1, -1.0),
    (0.003, 1, +1.0),
    (0.003, 4, -1.0),
    (0.003, 4, +1.0),
    (0.05, 2, +1.0),
    (0.05, 16, +1.0),
)


def ni_sf_table() -> list[SF]:
    """14 SFs of the single element: 8 radial (eta ascending), then 6 narrow angular."""
    table = [SF(0, 2, (0,), eta, rc=NI_RCUT) for eta in NI_RADIAL_ETAS]
    table += [SF(0, 3, (0, 0), eta, 0.0, float(zeta), lam, rc=NI_RCUT) for eta, zeta, lam in NI_ANGULAR]
    return table


def ni_g9_sf_table() -> list[SF]:
    """The wide variant of the Ni table: the same 8 radial SFs, then the 6
    angular ones as wide functions G9 (kind 9: no r_jk factor or cutoff)."""
    table = [SF(0, 2, (0,), eta, rc=NI_RCUT) for eta in NI_RADIAL_ETAS]
    table += [SF(0, 9, (0, 0), eta, 0.0, float(zeta), lam, rc=NI_RCUT) for eta, zeta, lam in NI_ANGULAR]
    return table


def ni_nets(seed: int = 2000) -> list[Net]:
    return xavier_nets(sf_counts(ni_sf_table(), n_el=1), seed)


def ni_table_scaled(path: str | None = None, wide: bool = False) -> list[SF]:
    """``ni_sf_table`` (or, with ``wide``, ``ni_g9_sf_table``) with the stored
    shift/scale filled in."""
    import os

    if path is None:
        path = os.path.join(os.path.dirname(__file__), "data", "ni_g9_scaling.json" if wide else "ni_scaling.json")
    sc = load_scaling(path)
    table = ni_g9_sf_table() if wide else ni_sf_table()
    for k, s in enumerate(table):
        s.shift = float(sc["shift"]["Ni"][k])
        s.scale = float(sc["scale"]["Ni"][k])
    return table
