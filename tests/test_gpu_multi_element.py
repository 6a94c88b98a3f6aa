"""Potentials of three and four elements on the GPU against the FP64 oracle.

The inputs are the generator's water boxes, with every atom's type drawn
uniformly from n_el elements (seeded). The tables fill every element-pair
class:
- n_el = 3 with two angular eta per centre, which takes the kernels'
  two-eta, all-(q, n) instantiation;
- n_el = 4 with four angular eta, which takes the four-eta instantiation.

Both use zeta in {1, 2, 4, 16} with either sign of lambda. The SF shift and
scale are the mean and spread of the oracle's raw values on the box, so the
networks see inputs of order one.

Energies and forces are held to the water bars (FP64 1e-9 relative, FP32
1e-5 eV / 1e-4 eV/A) at the three levels of parallelism. The weight
gradient of a three-box batch is checked per parameter tensor in FP64.
"""
import numpy as np
import pytest

import oracle
from gpu_common import check_fp32, check_fp64, gpu_loss_and_grad, oracle_input, per_tensor_rel, run, say
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu

NAMES = ("A", "B", "C", "D")


def _raw_table(n_el):
    t = []
    if n_el == 3:
        # two angular eta: 6 radial + 6 classes x 4 angular = 30 SFs per centre
        ang = ((0.002, 1.0, -1.0), (0.002, 4.0, 1.0), (0.03, 2.0, 1.0), (0.03, 16.0, -1.0))
        for c in range(n_el):
            for nb in range(n_el):
                for eta in (0.004, 0.05):
                    t.append(synth.SF(c, 2, (nb,), eta))
            for e1 in range(n_el):
                for e2 in range(e1, n_el):
                    for eta, zeta, lam in ang:
                        t.append(synth.SF(c, 3, (e1, e2), eta, 0.0, zeta, lam))
    else:
        # four angular eta, one per class in turn: 4 radial + 10 classes x 2
        etas = (0.001, 0.004, 0.02, 0.05)
        for c in range(n_el):
            for nb in range(n_el):
                t.append(synth.SF(c, 2, (nb,), 0.01))
            k = 0
            for e1 in range(n_el):
                for e2 in range(e1, n_el):
                    zl = ((1.0, -1.0), (4.0, 1.0)) if k % 2 == 0 else ((2.0, 1.0), (16.0, -1.0))
                    for zeta, lam in zl:
                        t.append(synth.SF(c, 3, (e1, e2), etas[k % 4], 0.0, zeta, lam))
                    k += 1
    return t


def _typed_box(side, seed, n_el):
    b = synth.water_box(side, seed)
    types = np.random.default_rng(1000 + seed).integers(0, n_el, b.n_atoms).astype(np.int32)
    return synth.Box(pos=b.pos, types=types, box=b.box)


def _scaled_table(n_el, box):
    """The raw table with shift/scale set from the oracle's values on box."""
    t = _raw_table(n_el)
    counts = synth.sf_counts(t, n_el)
    nets = synth.xavier_nets(counts, 3)
    G = oracle.Potential(t, nets, n_el=n_el).descriptors(box.pos, box.types, box.box, use_cells=True)
    col = {e: 0 for e in range(n_el)}
    for s in t:
        g = G[box.types == s.centre, col[s.centre]]
        col[s.centre] += 1
        s.shift = float(np.mean(g))
        s.scale = float(max(np.std(g), 1e-3))
    return t


def _setup(n_el):
    scale_box = _typed_box(6, 90 + n_el, n_el)
    table = _scaled_table(n_el, scale_box)
    nets = synth.xavier_nets(synth.sf_counts(table, n_el), 11 + n_el, hidden=(12, 8), bias_halfwidth=0.1)
    return table, nets


def _potential(table, nets, n_el, form):
    from paper_2002_00054_amd.nnp import Potential

    return Potential(table, nets, precision=form, elements=NAMES[:n_el])


@pytest.fixture(scope="module", params=[3, 4])
def system(request):
    n_el = request.param
    table, nets = _setup(n_el)
    return n_el, table, nets


@pytest.mark.parametrize("level", ["auto", "wave", "thread"])
@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("side,seed", [(5, 1), (8, 2)])
def test_energies_forces_match_oracle(system, level, form, side, seed):
    n_el, table, nets = system
    b = _typed_box(side, seed, n_el)
    say("elements", n_el, "atoms", b.n_atoms, form, level)
    ref = oracle.Potential(table, nets, n_el=n_el).compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    # the forces are not trivially small: the networks are not saturated
    assert np.sqrt(np.mean(ref["F"] ** 2)) > 1e-3
    pot = _potential(table, nets, n_el, form)
    if level != "auto":
        pot.set_parallelism(level)
    e, ei, f = run(pot, b)
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
        assert e == pytest.approx(ref["E"], rel=1e-10)
    else:
        check_fp32(ei, f, ref["Ei"], ref["F"])
    pot.close()


def test_weight_gradient_matches_oracle(system):
    """Forward and backward on three boxes (192, 375 and 192 atoms): the
    force-adjoint pass over every class, per parameter tensor."""
    n_el, table, nets = system
    boxes = [_typed_box(s, 60 + i, n_el) for i, s in enumerate((4, 5, 4))]
    teacher = oracle.Potential(table, synth.xavier_nets(synth.sf_counts(table, n_el), 77, hidden=(12, 8),
                                                        bias_halfwidth=0.1), n_el=n_el)
    Ehat, Fhat = oracle.batch_energy_forces(teacher, boxes)
    L_ref, g_ref = oracle.loss_and_grad(oracle.Potential(table, nets, n_el=n_el), boxes, Ehat, Fhat)
    pot = _potential(table, nets, n_el, "fp64")
    L, g = gpu_loss_and_grad(pot, boxes, Ehat, Fhat, synth.flat_params(nets))
    rel = per_tensor_rel(g, g_ref, nets)
    say("elements", n_el, "fp64 weight-gradient rel-L2 per tensor, max", rel.max())
    assert L == pytest.approx(L_ref, rel=1e-10)
    assert rel.max() < 1e-8
    pot.close()
