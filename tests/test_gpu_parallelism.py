"""The levels of parallelism of the SF and force passes (nnp_set_parallelism)
against the FP64 oracle, on both workloads: one thread per centre on the
water boxes (86 neighbours) and on the fcc boxes (18 neighbours), one wave
per centre (also the default) named explicitly on the fcc boxes, two waves
per centre on both, at the usual bars, and the levels against each other."""
import numpy as np
import pytest

import oracle
from common import oracle_water, water_potential
from gpu_common import (check_fp32, check_fp64, gpu_loss_and_grad, make_potential, oracle_input,
                        per_tensor_rel, run, say)
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("side,seed", [(4, 1), (16, 11)])
def test_water_thread_per_centre(form, side, seed):
    b = synth.water_box(side, seed)
    say("water thread", form, b.n_atoms)
    pot = make_potential(form)
    pot.set_parallelism("thread")
    e, ei, f = run(pot, b)
    ref = oracle_water().compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    elif form == "fp32":
        check_fp32(ei, f, ref["Ei"], ref["F"])
    else:
        assert float(np.sqrt(np.mean((f - ref["F"]) ** 2))) <= 5e-3
    pot.close()


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("side,seed", [(4, 1), (7, 3), (16, 11)])
def test_water_two_waves_per_centre(form, side, seed):
    b = synth.water_box(side, seed)
    say("water wave2", form, b.n_atoms)
    pot = make_potential(form)
    pot.set_parallelism("wave2")
    e, ei, f = run(pot, b)
    ref = oracle_water().compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    elif form == "fp32":
        check_fp32(ei, f, ref["Ei"], ref["F"])
    else:
        assert float(np.sqrt(np.mean((f - ref["F"]) ** 2))) <= 5e-3
    pot.close()


def test_two_waves_weight_gradient_matches_oracle():
    """The force-adjoint pass with two waves per centre (3-box training
    batch, FP64, per tensor)."""
    table, nets = water_potential()
    teacher = oracle.Potential(table, synth.teacher_nets())
    boxes = [synth.water_box(s, 40 + i) for i, s in enumerate((4, 5, 4))]
    Ehat, Fhat = oracle.batch_energy_forces(teacher, boxes)
    L_ref, g_ref = oracle.loss_and_grad(oracle.Potential(table, nets), boxes, Ehat, Fhat)
    pot = make_potential("fp64")
    pot.set_parallelism("wave2")
    L, g = gpu_loss_and_grad(pot, boxes, Ehat, Fhat, synth.flat_params(nets))
    rel = per_tensor_rel(g, g_ref, nets)
    say("wave2 fp64 weight-gradient rel-L2 per tensor, max", rel.max())
    assert L == pytest.approx(L_ref, rel=1e-10)
    assert rel.max() < 1e-8
    pot.close()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("mode", ["wave", "wave2", "thread"])
def test_fcc_levels(form, mode):
    table, nets = synth.ni_table_scaled(), synth.ni_nets()
    b = synth.fcc_box(8, 2)
    pot = make_potential(form, table, nets)
    pot.set_parallelism(mode)
    e, ei, f = run(pot, b)
    ref = oracle.Potential(table, nets, n_el=1).compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    else:
        check_fp32(ei, f, ref["Ei"], ref["F"])
    pot.close()


def test_levels_agree_fp64():
    table, nets = synth.ni_table_scaled(), synth.ni_nets()
    b = synth.fcc_box(20, 3)
    out = {}
    for mode in ("wave", "thread", "wave2"):
        pot = make_potential("fp64", table, nets)
        pot.set_parallelism(mode)
        out[mode] = run(pot, b)
        pot.close()
    e1, ei1, f1 = out["wave"]
    for other in ("thread", "wave2"):
        e2, ei2, f2 = out[other]
        assert e2 == pytest.approx(e1, rel=1e-13)
        assert np.max(np.abs(ei2 - ei1)) < 1e-12 * np.max(np.abs(ei1))
        assert np.max(np.abs(f2 - f1)) < 1e-12 * np.max(np.abs(f1))


def test_bad_mode():
    from paper_2002_00054_amd.nnp import NNPError

    pot = make_potential("fp32")
    with pytest.raises(NNPError, match="NNP_E_ARG"):
        pot._check(pot._L.nnp_set_parallelism(pot._h, 9))
    pot.close()


def _dense_ball():
    """A jittered cubic lattice (spacing 0.56 A) inside a ball of radius 2.9 A,
    H and O mixed: ~580 atoms, every pair closer than rc = 6 A."""
    rng = np.random.default_rng(17)
    g = np.arange(-2.9, 2.9001, 0.56)
    pts = np.array([(x, y, z) for x in g for y in g for z in g])
    pts = pts[np.einsum("ij,ij->i", pts, pts) <= 2.9 ** 2]
    pts = pts + rng.uniform(-0.04, 0.04, pts.shape)
    types = np.where(np.arange(len(pts)) % 3 == 0, synth.O, synth.H).astype(np.int32)
    return synth.Box(pos=pts + 7.0, types=types, box=np.array([14.0, 14.0, 14.0]))


def test_dense_cluster_beyond_wave_lds():
    """Atoms with more neighbours than one wave per centre can stage in LDS
    (about 580 per atom: over 190 KB per workgroup of four centres in FP64,
    above the 160 KB a workgroup can have).  Under the default level the
    handle takes two waves per centre (two centres per workgroup, about half
    the LDS) and matches the oracle (FP64), forward and weight gradient
    alike; an explicit request for one wave per centre is refused with
    NNP_E_ARG before any launch, and two waves per centre named explicitly
    match the oracle too."""
    from paper_2002_00054_amd.nnp import NNPError

    b = _dense_ball()
    assert b.n_atoms > 560
    d2 = np.sum((b.pos[:, None, :] - b.pos[None, :, :]) ** 2, axis=-1)
    assert np.max(d2) < synth.RCUT ** 2
    say("dense ball", b.n_atoms)
    ref = oracle_water().compute(b.pos, b.types, b.box, use_cells=True)
    pot = make_potential("fp64")
    e, ei, f = run(pot, b)
    check_fp64(ei, f, ref["Ei"], ref["F"])
    assert e == pytest.approx(float(np.sum(ref["Ei"])), rel=1e-10)
    pot.set_parallelism("wave")
    with pytest.raises(NNPError, match="NNP_E_ARG.*LDS"):
        run(pot, b)
    # two waves per centre put two centres, not four, in a workgroup: the
    # ball fits its LDS
    pot.set_parallelism("wave2")
    e, ei, f = run(pot, b)
    check_fp64(ei, f, ref["Ei"], ref["F"])
    pot.close()


def test_dense_cluster_gradient_default_level():
    """The weight gradient of the dense ball under the default level (its
    force-adjoint pass also takes two waves per centre) against the oracle,
    FP64, 1e-8 per parameter tensor."""
    b = _dense_ball()
    table, nets = water_potential()
    teacher = synth.teacher_nets()
    Ehat, Fhat = oracle.batch_energy_forces(oracle.Potential(table, teacher), [b])
    L_ref, g_ref = oracle.loss_and_grad(oracle.Potential(table, nets), [b], Ehat, Fhat)
    pot = make_potential("fp64")
    L, g = gpu_loss_and_grad(pot, [b], Ehat, Fhat, synth.flat_params(nets))
    per = per_tensor_rel(g, g_ref, nets)
    say("dense ball gradient per-tensor rel-L2 max", float(per.max()))
    assert L == pytest.approx(L_ref, rel=1e-10)
    assert per.max() < 1e-8, per
    pot.close()
