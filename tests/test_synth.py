"""The seeded generators: shapes, determinism, geometry of the molecules."""
import math

import numpy as np

from paper_2002_00054_amd import synth


def test_water_box_shape_and_density():
    b = synth.water_box(4, 0)
    assert b.pos.shape == (192, 3) and b.types.shape == (192,)
    assert np.allclose(b.box, 12.42)
    assert np.all((b.pos >= 0) & (b.pos < b.box))
    assert (b.types == synth.O).sum() == 64 and (b.types == synth.H).sum() == 128
    # 18.015 g/mol per molecule, A^3 -> cm^3: ~1 g/cm^3
    rho = 64 * 18.015 / 6.02214076e23 / (12.42e-8) ** 3
    assert abs(rho - 1.0) < 0.01


def test_water_box_is_deterministic_and_seeded():
    a = synth.water_box(4, 1)
    b = synth.water_box(4, 1)
    c = synth.water_box(4, 2)
    assert np.array_equal(a.pos, b.pos)
    assert not np.allclose(a.pos, c.pos)


def test_monomer_geometry():
    b = synth.water_box(5, 3)
    o, h1, h2 = b.pos[0::3], b.pos[1::3], b.pos[2::3]

    def mi(d):
        return d - b.box * np.round(d / b.box)

    d1, d2 = mi(h1 - o), mi(h2 - o)
    assert np.allclose(np.linalg.norm(d1, axis=1), 0.96)
    assert np.allclose(np.linalg.norm(d2, axis=1), 0.96)
    cosang = np.sum(d1 * d2, axis=1) / 0.96 ** 2
    assert np.allclose(cosang, math.cos(math.radians(104.5)))


def test_sf_table_counts_and_ranges():
    t = synth.water_sf_table()
    assert synth.sf_counts(t) == [27, 30]
    etas2 = sorted({s.eta for s in t if s.kind == 2})
    assert math.isclose(etas2[0], 0.001) and math.isclose(etas2[-1], 0.5)
    assert {s.zeta for s in t if s.kind == 3} == {1.0, 2.0, 4.0, 16.0}
    assert {s.lam for s in t if s.kind == 3} == {1.0, -1.0}


def test_xavier_nets():
    nets = synth.water_nets()
    assert [n.sizes for n in nets] == [[27, 25, 25, 1], [30, 25, 25, 1]]
    for n in nets:
        for w in n.W:
            lim = math.sqrt(6.0 / (w.shape[0] + w.shape[1]))
            assert np.all(np.abs(w) <= lim)
        assert all(np.all(b == 0) for b in n.b)
    flat = synth.flat_params(nets)
    assert flat.size == 1376 + 1451


def test_tile_box():
    b = synth.water_box(4, 0)
    t = synth.tile_box(b, 2)
    assert t.n_atoms == 8 * 192 and np.allclose(t.box, 2 * b.box)
    assert np.array_equal(t.pos[:192], b.pos)


def test_training_batch_sizes():
    s = synth.training_batch_sizes()
    assert len(s) == 32 and s.min() >= 4 and s.max() <= 8
