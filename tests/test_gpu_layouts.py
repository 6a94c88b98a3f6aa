"""The neighbour-list layouts of the wave-level passes (nnp_set_list_layout):
padded displacement entries (the default), index entries with the
positions gathered by the pair passes, and compact rows without padding.

Every layout is held to the same bars against the FP64 oracle as the
default one (FP64 1e-9 relative, FP32 1e-5 eV / 1e-4 eV/A), on both
workloads: water (two elements, 6 A) from the 192-atom box (two cells per
axis: the deduplicated stencil and minimum images) to 12,288 atoms, and the
fcc metal (3.9 A).  The weight gradient (force-adjoint pass on the same
list) matches the oracle per parameter tensor, and a batch too dense for
one wave per centre runs the index layout with two.
"""
import numpy as np
import pytest

import oracle
from common import oracle_water, water_potential
from gpu_common import (check_fp32, check_fp64, gpu_loss_and_grad, make_potential, oracle_input, per_tensor_rel,
                        run, say)
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu

LAYOUTS = ["index", "compact"]


def _check(form, ei, f, ref):
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    else:
        check_fp32(ei, f, ref["Ei"], ref["F"])


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("side,seed", [(4, 1), (7, 5), (16, 12)])
def test_water_layout_matches_oracle(layout, form, side, seed):
    b = synth.water_box(side, seed)
    say("water", layout, form, b.n_atoms, "atoms")
    pot = make_potential(form)
    pot.set_list_layout(layout)
    e, ei, f = run(pot, b)
    ref = oracle_water().compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    _check(form, ei, f, ref)
    assert abs(e - ref["E"]) <= (1e-9 if form == "fp64" else 1e-5) * b.n_atoms
    pot.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_water_layout_bf16_equals_padded(layout):
    """The precision form reads the same list: its results equal the padded
    layout's up to rounding order."""
    b = synth.water_box(16, 13)
    pot = make_potential("bf16")
    _, ei0, f0 = run(pot, b)
    pot.set_list_layout(layout)
    _, ei1, f1 = run(pot, b)
    assert np.max(np.abs(ei1 - ei0)) < 1e-5 and np.max(np.abs(f1 - f0)) < 1e-4
    pot.close()


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_fcc_layout_matches_oracle(layout, form):
    table, nets = synth.ni_table_scaled(), synth.ni_nets()
    b = synth.fcc_box(8, 2)
    say("fcc", layout, form, b.n_atoms, "atoms")
    pot = make_potential(form, table, nets)
    pot.set_list_layout(layout)
    e, ei, f = run(pot, b)
    ref = oracle.Potential(table, nets, n_el=1).compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    _check(form, ei, f, ref)
    pot.close()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_layout_weight_gradient_matches_oracle(layout):
    """Forward and backward on the 3-box training batch: the backward reuses
    the forward's list in the chosen layout for its force-adjoint pass."""
    table, nets = water_potential()
    teacher = oracle.Potential(table, synth.teacher_nets())
    boxes = [synth.water_box(s, 40 + i) for i, s in enumerate((4, 5, 4))]
    Ehat, Fhat = oracle.batch_energy_forces(teacher, boxes)
    L_ref, g_ref = oracle.loss_and_grad(oracle.Potential(table, nets), boxes, Ehat, Fhat)
    pot = make_potential("fp64")
    pot.set_list_layout(layout)
    L, g = gpu_loss_and_grad(pot, boxes, Ehat, Fhat, synth.flat_params(nets))
    rel = per_tensor_rel(g, g_ref, nets)
    say(layout, "fp64 weight-gradient rel-L2 per tensor, max", rel.max())
    assert L == pytest.approx(L_ref, rel=1e-10)
    assert rel.max() < 1e-8
    pot.close()


def test_index_layout_dense_batch_falls_back():
    """A ball of ~580 atoms all within rc of each other is beyond one wave
    per centre; under the default parallelism it takes two, which read the
    index layout as well, and matches the oracle.  Named explicitly, the
    thread level rebuilds padded rows and matches too."""
    rng = np.random.default_rng(17)
    g = np.arange(-2.9, 2.9001, 0.56)
    pts = np.array([(x, y, z) for x in g for y in g for z in g])
    pts = pts[np.einsum("ij,ij->i", pts, pts) <= 2.9 ** 2]
    pts = pts + rng.uniform(-0.04, 0.04, pts.shape)
    types = np.where(np.arange(len(pts)) % 3 == 0, synth.O, synth.H).astype(np.int32)
    b = synth.Box(pos=pts + 7.0, types=types, box=np.array([14.0, 14.0, 14.0]))
    ref = oracle_water().compute(b.pos, b.types, b.box, use_cells=True)
    pot = make_potential("fp64")
    pot.set_list_layout("index")
    e, ei, f = run(pot, b)
    check_fp64(ei, f, ref["Ei"], ref["F"])
    pot.set_parallelism("thread")
    e, ei, f = run(pot, b)
    check_fp64(ei, f, ref["Ei"], ref["F"])
    pot.close()


def test_layout_argument_errors():
    pot = make_potential("fp32")
    assert pot._L.nnp_set_list_layout(pot._h, 7) == -1  # NNP_E_ARG through the C ABI
    assert "layout" in pot._L.nnp_last_error(pot._h).decode()
    pot.close()
