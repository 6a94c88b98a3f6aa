"""Pins of the oracle on the second workload: a single-element fcc metal with
the 3.9 A cutoff of the paper's Ni model (CPU).

- the perfect lattice has 12 neighbours at a/sqrt(2) and 6 more at a within
  the cutoff (neighbour search and minimum image on a cubic box);
- every SF of the perfect lattice equals the lattice sum written from exact
  integer neighbour vectors (units of a/2), with no neighbour search: 12 + 6
  radial terms, and the angular terms of every unordered neighbour pair closer
  than the cutoff, with the cosine and r_jk from the integer vectors;
- the perfect lattice has identical atomic energies and zero forces
  (inversion symmetry);
- a 2 x 2 x 2 tiling of a jittered box repeats every E_i and F_i.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2002_00054_amd import synth


def _fc(r, rc):
    return 0.5 * (math.cos(math.pi * r / rc) + 1.0) if r < rc else 0.0


def _shell_vectors():
    """Integer neighbour vectors (units of a/2) of the first two fcc shells."""
    v = []
    for p in itertools.product((-2, -1, 0, 1, 2), repeat=3):
        n2 = p[0] ** 2 + p[1] ** 2 + p[2] ** 2
        if (n2 == 2 and sum(abs(x) for x in p) == 2) or (n2 == 4 and sorted(map(abs, p)) == [0, 0, 2]):
            v.append(np.array(p))
    return v


def test_perfect_lattice_shells():
    b = synth.fcc_box(4, 0, jitter=0.0)
    for rc, want in ((2.6, 12), (3.5, 12), (3.9, 18)):
        counts, _ = oracle.neighbors(b.pos, b.box, rc, use_cells=True)
        assert np.all(counts == want), (rc, np.unique(counts))
    assert len(_shell_vectors()) == 18


def test_perfect_lattice_sfs_match_lattice_sums():
    a, rc = synth.NI_LATTICE, synth.NI_RCUT
    table = synth.ni_sf_table()
    pot = oracle.Potential(table, synth.ni_nets(), n_el=1)
    b = synth.fcc_box(3, 0, jitter=0.0)
    G = pot.descriptors(b.pos, b.types, b.box)[:, : len(table)]
    vec = _shell_vectors()
    h = a / 2.0
    want = []
    for s in table:
        if s.kind == 2:
            want.append(sum(math.exp(-s.eta * (h * h * (v @ v))) * _fc(h * math.sqrt(v @ v), rc) for v in vec))
            continue
        tot = 0.0
        for vj, vk in itertools.combinations(vec, 2):
            d = vk - vj
            rij, rik, rjk = (h * math.sqrt(x @ x) for x in (vj, vk, d))
            if rjk >= rc:
                continue
            cos = (vj @ vk) / math.sqrt((vj @ vj) * (vk @ vk))
            tot += ((1.0 + s.lam * cos) ** s.zeta * math.exp(-s.eta * (rij ** 2 + rik ** 2 + rjk ** 2))
                    * _fc(rij, rc) * _fc(rik, rc) * _fc(rjk, rc))
        want.append(2.0 ** (1.0 - s.zeta) * tot)
    want = np.array(want)
    np.testing.assert_allclose(G, np.broadcast_to(want, G.shape), rtol=1e-12, atol=1e-14)


def test_perfect_lattice_zero_force_equal_energies():
    pot = oracle.Potential(synth.ni_table_scaled(), synth.ni_nets(), n_el=1)
    b = synth.fcc_box(4, 0, jitter=0.0)
    out = pot.compute(b.pos, b.types, b.box, use_cells=True)
    assert np.max(np.abs(out["F"])) < 1e-12
    assert np.ptp(out["Ei"]) < 1e-12 * max(1.0, abs(out["Ei"][0]))


def test_tiling_repeats_atoms():
    pot = oracle.Potential(synth.ni_table_scaled(), synth.ni_nets(), n_el=1)
    b = synth.fcc_box(3, 7)
    t = synth.tile_box(b, 2)
    o1 = pot.compute(b.pos, b.types, b.box)
    o8 = pot.compute(t.pos, t.types, t.box, use_cells=True)
    n = b.n_atoms
    for c in range(8):
        np.testing.assert_allclose(o8["Ei"][c * n:(c + 1) * n], o1["Ei"], rtol=0, atol=1e-12)
        np.testing.assert_allclose(o8["F"][c * n:(c + 1) * n], o1["F"], rtol=0, atol=1e-11)
    assert o8["E"] == pytest.approx(8 * o1["E"], rel=1e-12)
