"""Pins of the oracle's wide angular function G9 (CPU):

  G9_i = 2^(1-zeta) sum_{j<k} (1 + lam cos theta_ijk)^zeta e^{-eta (r_ij^2 + r_ik^2)} f_c(r_ij) f_c(r_ik)

- an isolated trimer with both neighbours at r from the centre, at several
  angles, including the straight one where r_jk = 2r is beyond the cutoff:
  there the narrow G3 of the same parameters is 0 and G9 is not;
- the perfect fcc lattice: every G9 equals the sum over all 153 unordered
  pairs of the 18 neighbour vectors, from exact integer vectors;
- forces of a mixed narrow + wide table against central differences of E;
- rotation invariance of a cluster;
- the sampled evaluator (used at full size) against the full one.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from common import random_rotation
from paper_2002_00054_amd import synth

RC = synth.NI_RCUT


def _fc(r):
    return 0.5 * (math.cos(math.pi * r / RC) + 1.0) if r < RC else 0.0


def _table(kind):
    return [synth.SF(0, kind, (0, 0), eta, 0.0, float(zeta), lam, rc=RC) for eta, zeta, lam in synth.NI_ANGULAR]


def _pot(table):
    return oracle.Potential(table, synth.xavier_nets(synth.sf_counts(table, n_el=1), 3), n_el=1)


@pytest.mark.parametrize("theta_deg", [60.0, 90.0, 131.0, 180.0])
def test_trimer_closed_form(theta_deg):
    r, L = 2.5, 40.0
    th = math.radians(theta_deg)
    pos = np.array([[20.0, 20.0, 20.0], [20.0 + r, 20.0, 20.0],
                    [20.0 + r * math.cos(th), 20.0 + r * math.sin(th), 20.0]])
    types = np.zeros(3, dtype=np.int32)
    box = np.array([L, L, L])
    G9 = _pot(_table(9)).descriptors(pos, types, box)[0, :6]
    G3 = _pot(_table(3)).descriptors(pos, types, box)[0, :6]
    rjk = 2.0 * r * math.sin(th / 2.0)
    for s, (eta, zeta, lam) in enumerate(synth.NI_ANGULAR):
        ang = 2.0 ** (1.0 - zeta) * (1.0 + lam * math.cos(th)) ** zeta
        want9 = ang * math.exp(-eta * 2 * r * r) * _fc(r) ** 2
        want3 = ang * math.exp(-eta * (2 * r * r + rjk * rjk)) * _fc(r) ** 2 * _fc(rjk)
        assert G9[s] == pytest.approx(want9, rel=1e-13, abs=1e-300)
        assert G3[s] == pytest.approx(want3, rel=1e-13, abs=1e-300)
    if theta_deg == 180.0:
        assert np.all(G3 == 0.0) and np.any(G9 > 0.0)


def test_perfect_lattice_sum():
    a = synth.NI_LATTICE
    table = _table(9)
    b = synth.fcc_box(3, 0, jitter=0.0)
    G = _pot(table).descriptors(b.pos, b.types, b.box)[:, :6]
    vec = [np.array(p) for p in itertools.product((-2, -1, 0, 1, 2), repeat=3)
           if (p[0] ** 2 + p[1] ** 2 + p[2] ** 2 == 2 and sum(map(abs, p)) == 2)
           or (p[0] ** 2 + p[1] ** 2 + p[2] ** 2 == 4 and sorted(map(abs, p)) == [0, 0, 2])]
    assert len(vec) == 18
    h = a / 2.0
    for s, (eta, zeta, lam) in enumerate(synth.NI_ANGULAR):
        tot = 0.0
        for vj, vk in itertools.combinations(vec, 2):
            rij, rik = h * math.sqrt(vj @ vj), h * math.sqrt(vk @ vk)
            cos = (vj @ vk) / math.sqrt((vj @ vj) * (vk @ vk))
            tot += (1.0 + lam * cos) ** zeta * math.exp(-eta * (rij ** 2 + rik ** 2)) * _fc(rij) * _fc(rik)
        np.testing.assert_allclose(G[:, s], 2.0 ** (1.0 - zeta) * tot, rtol=1e-12)


def test_forces_central_differences_mixed_table():
    table = [synth.SF(0, 2, (0,), eta, rc=RC) for eta in synth.NI_RADIAL_ETAS[:4]] + _table(3) + _table(9)
    pot = _pot(table)
    b = synth.fcc_box(3, 4)
    F = pot.compute(b.pos, b.types, b.box)["F"]
    h = 1e-5
    rng = np.random.default_rng(9)
    for i, c in zip(rng.choice(b.n_atoms, 8, replace=False), rng.integers(0, 3, 8)):
        p = b.pos.copy()
        p[i, c] += h
        ep = pot.compute(p, b.types, b.box)["E"]
        p[i, c] -= 2 * h
        em = pot.compute(p, b.types, b.box)["E"]
        assert abs(-(ep - em) / (2 * h) - F[i, c]) < 1e-6
    assert np.max(np.abs(F.sum(axis=0))) < 1e-10


def test_rotation_invariance():
    rng = np.random.default_rng(2)
    pts = rng.uniform(-2.5, 2.5, size=(9, 3))
    pts = pts[np.linalg.norm(pts, axis=1) > 0.5]
    L = 40.0
    box = np.array([L, L, L])
    types = np.zeros(len(pts), dtype=np.int32)
    pot = _pot(_table(9))
    e0 = pot.compute(pts + 20.0, types, box)["Ei"]
    R = random_rotation(rng)
    e1 = pot.compute(pts @ R.T + 20.0, types, box)["Ei"]
    np.testing.assert_allclose(e1, e0, rtol=1e-12, atol=1e-12)


def test_sampled_matches_full_with_wide_functions():
    """The sampled evaluator (used at full size) equals the full one on a mixed table."""
    table = [synth.SF(0, 2, (0,), eta, rc=RC) for eta in synth.NI_RADIAL_ETAS[:4]] + _table(3) + _table(9)
    pot = _pot(table)
    b = synth.fcc_box(4, 8)
    full = pot.compute(b.pos, b.types, b.box, use_cells=True)
    idx = np.array([0, 5, 77, 130, 255], dtype=np.int64)
    Ei, F = pot.sampled(b.pos, b.types, b.box, idx)
    np.testing.assert_allclose(Ei, full["Ei"][idx], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(F, full["F"][idx], rtol=1e-11, atol=1e-12)
