"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: exact closed-form values of
small geometries (tests/golden), central finite differences of the energy,
the invariances the descriptors must carry (translation, rotation,
permutation; Sec. 2), extensivity of replicated boxes, the brute-force
neighbour set, the network against torch's layers, and special parameter
choices that collapse the network.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from common import LN2, cluster, nets_for, oracle_water, random_rotation, tiny_table, water_potential
from paper_2002_00054_amd import synth

H, O = synth.H, synth.O
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_form_sf.json")))


def _box(L=30.0):
    return np.array([L, L, L])


# ---------------------------------------------------------------- P1 dimer
def test_dimer_exact_values():
    """Radial SF of an isolated O-H pair equals the single term (golden)."""
    cases = GOLD["dimer"]["cases"]
    radial = []
    for c in cases:
        eta = c.get("eta", None)
        if eta is None:
            eta = c["eta_times_r2_over_ln2"] * LN2 / c["r"] ** 2
        radial.append((H, eta))
    radial.append((O, 0.0))  # no O neighbour of the O centre: stays 0
    table = tiny_table(radial=radial, angular=[((H, H), 0.0, 1, 1.0)])
    pot = oracle.Potential(table, nets_for(table))
    for k, c in enumerate(cases):
        # O near the box corner, H across the periodic boundary: minimum image.
        pos = np.array([[0.5, 7.0, 7.0], [0.5 - c["r"] + 30.0, 7.0, 7.0]])
        G = pot.descriptors(pos, np.array([O, H]), _box())
        n = len(radial) + 1
        assert G[0, k] == pytest.approx(c["value"], rel=1e-14, abs=1e-300), c["derivation"]
        # the other slots of the O centre: other etas may be non-zero, O-neighbour and angular are 0
        assert G[0, len(cases)] == 0.0 and G[0, n - 1] == 0.0


def test_dimer_water_table_closed_form():
    """Water table, O-H dimer at 0.96 and 5.9 A: G2_O[H, eta] = exp(-eta r^2) f_c(r),
    G2_O[O, .] = 0 and every angular SF 0."""
    pot = oracle_water()
    table = synth.water_sf_table()
    o_rows = [s for s in table if s.centre == O]
    for r in (0.96, 5.9):
        pos = np.array([[5.0, 5.0, 5.0], [5.0 + r * 0.6, 5.0 + r * 0.8, 5.0]])
        G = pot.descriptors(pos, np.array([O, H]), _box())
        fc = 0.5 * (math.cos(math.pi * r / 6.0) + 1.0)
        for k, s in enumerate(o_rows):
            if s.kind == 2 and s.nbr[0] == H:
                assert G[0, k] == pytest.approx(math.exp(-s.eta * r * r) * fc, rel=1e-14)
            else:
                assert G[0, k] == 0.0


# -------------------------------------------------------------- P2 trimer
def _trimer_check(section, pos, types, centre_row, cls):
    cases = GOLD[section]["cases"]
    ang = []
    for c in cases:
        eta = c.get("eta", None)
        if eta is None:
            eta = c["eta_times_12_over_ln2"] * LN2 / 12.0
        ang.append((cls, eta, c["zeta"], c["lambda"]))
    table = tiny_table(radial=[(H, 0.0)], angular=ang)
    pot = oracle.Potential(table, nets_for(table))
    G = pot.descriptors(pos, types, _box())
    for k, c in enumerate(cases):
        assert G[centre_row, 1 + k] == pytest.approx(c["value"], rel=1e-14, abs=1e-15), c["derivation"]
    return G


def test_equilateral_trimer_exact_values():
    s3 = math.sqrt(3.0)
    pos = np.array([[10.0, 10.0, 10.0], [12.0, 10.0, 10.0], [11.0, 10.0 + s3, 10.0]])
    types = np.array([O, H, H])
    _trimer_check("equilateral", pos, types, 0, (H, H))
    # the same triangle seen from an H centre is in the mixed class {H, O}
    # (either order of the class names), with identical values
    _trimer_check("equilateral", pos, types, 1, (O, H))
    _trimer_check("equilateral", pos, types, 2, (H, O))


def test_collinear_trimer_exact_values():
    pos = np.array([[10.0, 10.0, 10.0], [8.0, 10.0, 10.0], [12.0, 10.0, 10.0]])
    _trimer_check("collinear", pos, np.array([O, H, H]), 0, (H, H))


def test_water_monomer_angular_closed_form():
    """O-centre angular SFs of one rigid water molecule: a single (j, k) pair,
    with the angle 104.5 deg, sides 0.96 and r_HH from the law of cosines."""
    th = math.radians(104.5)
    pos = np.array([[5.0, 5.0, 5.0], [5.96, 5.0, 5.0], [5.0 + 0.96 * math.cos(th), 5.0 + 0.96 * math.sin(th), 5.0]])
    pot = oracle_water()
    G = pot.descriptors(pos, np.array([O, H, H]), _box())
    rhh = math.sqrt(2 * 0.96 ** 2 * (1 - math.cos(th)))
    fc = lambda r: 0.5 * (math.cos(math.pi * r / 6.0) + 1.0)
    o_rows = [s for s in synth.water_sf_table() if s.centre == O]
    for k, s in enumerate(o_rows):
        if s.kind == 3 and s.nbr == (H, H):
            want = (2.0 ** (1 - s.zeta) * (1 + s.lam * math.cos(th)) ** s.zeta
                    * math.exp(-s.eta * (2 * 0.96 ** 2 + rhh ** 2)) * fc(0.96) ** 2 * fc(rhh))
            assert G[0, k] == pytest.approx(want, rel=1e-13)
    assert rhh == pytest.approx(1.518123981588179, rel=1e-14)


# ------------------------------------------------------------ P11 special
def test_zero_first_layer_gives_constant_energy_zero_force():
    """W1 = 0, b1 = 0: h1 = 0, so E_i = w3 . tanh(b2) + b3 for every atom and F = 0."""
    table, nets = water_potential()
    nets = [synth.Net([w.copy() for w in n.W], [b.copy() for b in n.b]) for n in nets]
    rng = np.random.default_rng(3)
    for n in nets:
        n.W[0][:] = 0.0
        n.b[1] = rng.uniform(-1, 1, size=n.b[1].shape)
        n.b[2] = rng.uniform(-1, 1, size=n.b[2].shape)
    pot = oracle.Potential(table, nets)
    b = synth.water_box(4, 1)
    out = pot.compute(b.pos, b.types, b.box)
    for e in (H, O):
        want = float(nets[e].W[2][0] @ np.tanh(nets[e].b[1]) + nets[e].b[2][0])
        np.testing.assert_allclose(out["Ei"][b.types == e], want, rtol=1e-14)
    assert np.all(out["F"] == 0.0)


def test_network_matches_torch_layers():
    """E_i of the oracle equals torch's Linear/Tanh stack on the scaled G."""
    import torch

    table, nets = water_potential()
    pot = oracle.Potential(table, nets)
    b = synth.water_box(4, 2)
    out = pot.compute(b.pos, b.types, b.box, want_g=True)
    for e in (H, O):
        rows = [s for s in table if s.centre == e]
        sh = np.array([s.shift for s in rows])
        sc = np.array([s.scale for s in rows])
        g = out["G"][b.types == e, :len(rows)]
        x = torch.tensor((g - sh) / sc)
        layers = []
        for l, (w, bb) in enumerate(zip(nets[e].W, nets[e].b)):
            lin = torch.nn.Linear(w.shape[1], w.shape[0]).double()
            with torch.no_grad():
                lin.weight.copy_(torch.tensor(w))
                lin.bias.copy_(torch.tensor(bb))
            layers.append(lin)
            if l < len(nets[e].W) - 1:
                layers.append(torch.nn.Tanh())
        y = torch.nn.Sequential(*layers)(x)[:, 0].detach().numpy()
        np.testing.assert_allclose(out["Ei"][b.types == e], y, rtol=1e-13, atol=1e-13)
        # dE/dG (raw) against torch autograd
        xg = torch.tensor(g, requires_grad=True)
        yy = torch.nn.Sequential(*layers)((xg - torch.tensor(sh)) / torch.tensor(sc))[:, 0].sum()
        (dg,) = torch.autograd.grad(yy, xg)
        np.testing.assert_allclose(out["dEdG"][b.types == e, :len(rows)], dg.numpy(), rtol=1e-12, atol=1e-13)


def test_scaling_is_divide_by_scale_after_subtracting_shift():
    """(G - shift)/scale: multiplying scale by k and W1 by k, or moving shift by
    D while moving b1 by W1 D/scale, leaves every energy unchanged."""
    table, nets = water_potential()
    b = synth.water_box(4, 3)
    ref = oracle.Potential(table, nets).compute(b.pos, b.types, b.box)["Ei"]
    t2 = [synth.SF(**{**s.__dict__}) for s in table]
    n2 = [synth.Net([w.copy() for w in n.W], [x.copy() for x in n.b]) for n in nets]
    rng = np.random.default_rng(9)
    for e in (H, O):
        rows = [i for i, s in enumerate(t2) if s.centre == e]
        k = rng.uniform(0.5, 2.0, size=len(rows))
        D = rng.uniform(-1, 1, size=len(rows))
        sc = np.array([t2[i].scale for i in rows])
        n2[e].b[0] = n2[e].b[0] + n2[e].W[0] @ (D / sc)
        for j, i in enumerate(rows):
            t2[i].shift += D[j]
            t2[i].scale *= k[j]
        n2[e].W[0] = n2[e].W[0] * k[None, :]
    got = oracle.Potential(t2, n2).compute(b.pos, b.types, b.box)["Ei"]
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-12)


# --------------------------------------------------------- P3 / P4 forces
def _fd_check(pot, pos, types, box, pairs, h=1e-5, tol=1e-6):
    F = pot.compute(pos, types, box)["F"]
    for i, a in pairs:
        p = pos.copy()
        p[i, a] += h
        Ep = pot.compute(p, types, box)["E"]
        p[i, a] -= 2 * h
        Em = pot.compute(p, types, box)["E"]
        fd = -(Ep - Em) / (2 * h)
        assert abs(fd - F[i, a]) <= tol, (i, a, fd, F[i, a])


def test_forces_match_central_differences_periodic():
    pot = oracle_water()
    b = synth.water_box(4, 1)
    rng = np.random.default_rng(11)
    pairs = list(zip(rng.integers(0, b.n_atoms, 30), rng.integers(0, 3, 30)))
    _fd_check(pot, b.pos, b.types, b.box, pairs)


def test_forces_match_central_differences_cluster():
    pot = oracle_water()
    c = cluster()
    pairs = [(i, a) for i in range(c.n_atoms) for a in range(3)]
    _fd_check(pot, c.pos, c.types, c.box, pairs)


def test_forces_match_central_differences_special_geometries():
    """Collinear and equilateral trimers with zeta = 1 (0^0 in dT/dcos) and zeta = 16."""
    table = tiny_table(radial=[(H, 0.01), (O, 0.2)],
                       angular=[((H, H), 0.001, 1, 1.0), ((H, H), 0.03, 16, -1.0), ((H, O), 0.01, 1, -1.0),
                                ((H, O), 0.0, 2, 1.0), ((O, O), 0.01, 4, 1.0)])
    pot = oracle.Potential(table, nets_for(table, bias=0.3))
    s3 = math.sqrt(3.0)
    for pos in (np.array([[10.0, 10.0, 10.0], [8.0, 10.0, 10.0], [12.0, 10.0, 10.0]]),
                np.array([[10.0, 10.0, 10.0], [12.0, 10.0, 10.0], [11.0, 10.0 + s3, 10.0]])):
        pairs = [(i, a) for i in range(3) for a in range(3)]
        _fd_check(pot, pos, np.array([O, H, H]), _box(), pairs, h=1e-6, tol=1e-7)


def test_net_force_vanishes():
    pot = oracle_water()
    for seed in (1, 2):
        b = synth.water_box(4, seed)
        F = pot.compute(b.pos, b.types, b.box)["F"]
        rms = np.sqrt(np.mean(F ** 2))
        assert np.all(np.abs(F.sum(axis=0)) <= 1e-10 * b.n_atoms * rms)


# ---------------------------------------------------- P5-P7 invariances
def test_translation_invariance():
    pot = oracle_water()
    b = synth.water_box(4, 2)
    ref = pot.compute(b.pos, b.types, b.box)
    rng = np.random.default_rng(1)
    for _ in range(3):
        p = np.mod(b.pos + rng.uniform(-50, 50, size=3), b.box)
        out = pot.compute(p, b.types, b.box)
        np.testing.assert_allclose(out["Ei"], ref["Ei"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out["F"], ref["F"], rtol=1e-10, atol=1e-11)


def test_cubic_point_group_invariance_periodic():
    """All 48 axis permutations x sign flips map the cubic box onto itself."""
    pot = oracle_water()
    b = synth.water_box(4, 3)
    ref = pot.compute(b.pos, b.types, b.box)
    L = b.box[0]
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            R = np.zeros((3, 3))
            for r, (c, s) in enumerate(zip(perm, signs)):
                R[r, c] = s
            p = np.mod(b.pos @ R.T, L)
            out = pot.compute(p, b.types, b.box)
            np.testing.assert_allclose(out["Ei"], ref["Ei"], rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(out["F"], ref["F"] @ R.T, rtol=1e-10, atol=1e-11)


def test_rotation_invariance_cluster():
    pot = oracle_water()
    c = cluster()
    ref = pot.compute(c.pos, c.types, c.box)
    rng = np.random.default_rng(4)
    ctr = c.box / 2
    for _ in range(4):
        R = random_rotation(rng)
        p = (c.pos - ctr) @ R.T + ctr
        out = pot.compute(p, c.types, c.box)
        np.testing.assert_allclose(out["Ei"], ref["Ei"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out["F"], ref["F"] @ R.T, rtol=1e-10, atol=1e-11)


def test_permutation_invariance():
    pot = oracle_water()
    b = synth.water_box(4, 4)
    ref = pot.compute(b.pos, b.types, b.box)
    perm = np.random.default_rng(2).permutation(b.n_atoms)
    out = pot.compute(b.pos[perm], b.types[perm], b.box)
    assert out["E"] == pytest.approx(ref["E"], rel=1e-12)
    np.testing.assert_allclose(out["Ei"], ref["Ei"][perm], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["F"], ref["F"][perm], rtol=1e-10, atol=1e-11)
    # swapping the positions of two same-element atoms
    hs = np.nonzero(b.types == H)[0][:2]
    p = b.pos.copy()
    p[[hs[0], hs[1]]] = p[[hs[1], hs[0]]]
    out = pot.compute(p, b.types, b.box)
    assert out["Ei"][hs[0]] == pytest.approx(ref["Ei"][hs[1]], rel=1e-12)
    np.testing.assert_allclose(out["F"][hs[1]], ref["F"][hs[0]], rtol=1e-10, atol=1e-11)


# ------------------------------------------------------- P8 extensivity
def test_extensivity_of_replicated_box():
    pot = oracle_water()
    b = synth.water_box(4, 0)
    ref = pot.compute(b.pos, b.types, b.box)
    t = synth.tile_box(b, 2)
    out = pot.compute(t.pos, t.types, t.box, use_cells=True)
    n = b.n_atoms
    for r in range(8):
        np.testing.assert_allclose(out["Ei"][r * n:(r + 1) * n], ref["Ei"], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out["F"][r * n:(r + 1) * n], ref["F"], rtol=1e-10, atol=1e-11)
    assert out["E"] == pytest.approx(8 * ref["E"], rel=1e-12)


# ------------------------------------------------------ P9 neighbour sets
@pytest.mark.parametrize("n,seed", [(4, 1), (6, 2)])
def test_cell_list_equals_brute_force(n, seed):
    b = synth.water_box(n, seed)
    c1, l1 = oracle.neighbors(b.pos, b.box, 6.0, use_cells=False)
    c2, l2 = oracle.neighbors(b.pos, b.box, 6.0, use_cells=True)
    assert np.array_equal(c1, c2) and np.array_equal(l1, l2)
    # neighbour relation is symmetric
    pairs = {(i, int(j)) for i in range(b.n_atoms) for j in l1[i, :c1[i]]}
    assert all((j, i) in pairs for i, j in pairs)
    assert 80 <= c1.mean() <= 92  # ~86 neighbours per atom at 1 g/cm^3 inside 6 A


def test_triangle_count_identity():
    """Sum over centres of neighbour pairs within the cutoff of each other = 3 x triangles."""
    b = synth.water_box(4, 1)
    c, l = oracle.neighbors(b.pos, b.box, 6.0)
    nbs = [set(l[i, :c[i]].tolist()) for i in range(b.n_atoms)]
    per_centre = 0
    for i in range(b.n_atoms):
        nb = sorted(nbs[i])
        per_centre += sum(1 for x in range(len(nb)) for y in range(x + 1, len(nb)) if nb[y] in nbs[nb[x]])
    tri = sum(1 for i in range(b.n_atoms) for j in nbs[i] if j > i for k in nbs[i] & nbs[j] if k > j)
    assert per_centre == 3 * tri


def test_sampled_matches_full():
    """The sampled evaluator (for boxes too big for the full one) equals the full one."""
    pot = oracle_water()
    b = synth.water_box(6, 5)
    full = pot.compute(b.pos, b.types, b.box)
    idx = np.array([0, 1, 2, 100, 377, b.n_atoms - 1])
    Ei, F = pot.sampled(b.pos, b.types, b.box, idx)
    np.testing.assert_allclose(Ei, full["Ei"][idx], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(F, full["F"][idx], rtol=1e-10, atol=1e-11)


def test_centre_ranges_sum_to_full():
    """The centre-range evaluator (for timing a box too big for one silent
    run) over uneven ranges covering every atom equals the full one: the
    energies per centre, and the forces as the sum of the ranges' terms.  An
    empty range adds nothing, and the summed forces still cancel."""
    pot = oracle_water()
    b = synth.water_box(6, 5)
    full = pot.compute(b.pos, b.types, b.box)
    F = np.zeros((b.n_atoms, 3))
    cuts = [0, 1, 200, 200, 513, b.n_atoms]
    Ei = np.concatenate([pot.compute_centres(b.pos, b.types, b.box, lo, hi, F) for lo, hi in zip(cuts, cuts[1:])])
    np.testing.assert_allclose(Ei, full["Ei"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(F, full["F"], rtol=1e-10, atol=1e-11)
    assert np.max(np.abs(F.sum(axis=0))) < 1e-9


# -------------------------------------------------- P10 loss gradient
@pytest.mark.slow
def test_loss_gradient_matches_finite_differences():
    table, nets = water_potential()
    teacher = oracle.Potential(table, synth.teacher_nets())
    boxes = [synth.water_box(4, 40), synth.water_box(4, 41)]
    Ehat, Fhat = oracle.batch_energy_forces(teacher, boxes)
    flat = synth.flat_params(nets)
    sizes = [n.sizes for n in nets]
    counts = [len(n.flat()) for n in nets]

    def pot_of(theta):
        ns, o = [], 0
        for s, c in zip(sizes, counts):
            ns.append(synth.Net.from_flat(theta[o:o + c], s))
            o += c
        return oracle.Potential(table, ns)

    L0, g = oracle.loss_and_grad(pot_of(flat), boxes, Ehat, Fhat)
    rng = np.random.default_rng(10)
    idx = rng.choice(len(flat), size=24, replace=False)
    h = 1e-5
    for k in idx:
        tp = flat.copy()
        tp[k] += h
        tm = flat.copy()
        tm[k] -= h
        fd = (oracle.loss(pot_of(tp), boxes, Ehat, Fhat) - oracle.loss(pot_of(tm), boxes, Ehat, Fhat)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])
