"""Pair-test masks (nnp_set_pair_masks): the SF pass stores its r_jk < rc
decisions, one bit per tested pair in blocks of 32 steps of the pair walk,
and the force pass reads them instead of testing again.

Masks are on by default for rows of at least 64 neighbours, so every water
test at one wave per centre already runs through them (the fcc metal, 18
neighbours, does not).  These tests add what the default workloads do not
reach: many mask blocks per centre (a compressed water box, about 170
neighbours and eight blocks per atom, and a dense ball where every pair is
within rc: over 80 blocks), masks on against masks off on the same input,
and the argument check."""
import numpy as np
import pytest

from common import oracle_water
from gpu_common import check_fp32, check_fp64, make_potential, oracle_input, run, say
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


def _compressed_water(side, seed, scale=0.8):
    b = synth.water_box(side, seed)
    return synth.Box(pos=b.pos * scale, types=b.types, box=b.box * scale)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_compressed_water_matches_oracle(form):
    b = _compressed_water(5, 7)
    ref = oracle_water().compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    say("compressed water", form, b.n_atoms, "atoms")
    pot = make_potential(form)
    pot.set_parallelism("wave")
    e, ei, f = run(pot, b)
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    else:
        check_fp32(ei, f, ref["Ei"], ref["F"], tol_e=1e-5, tol_f=2e-4)
    pot.close()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_masks_on_and_off_agree(form):
    """Same pairs, same order: the two differ by the order of the global
    force sums alone (FP64), plus the rounding of the pair test (FP32)."""
    b = synth.water_box(16, 14)
    out = []
    for on in (True, False):
        pot = make_potential(form)
        pot.set_pair_masks(on)
        out.append(run(pot, b))
        pot.close()
    (e1, ei1, f1), (e0, ei0, f0) = out
    rms_f = np.sqrt(np.mean(f0 ** 2))
    if form == "fp64":
        assert np.max(np.abs(ei1 - ei0)) <= 1e-13 * np.max(np.abs(ei0))
        assert np.max(np.abs(f1 - f0)) <= 1e-12 * rms_f
    else:
        ref = oracle_water().compute(oracle_input(b, form), b.types, b.box, use_cells=True)
        check_fp32(ei1, f1, ref["Ei"], ref["F"])
        check_fp32(ei0, f0, ref["Ei"], ref["F"])


def _dense_ball():
    """A jittered cubic lattice (spacing 0.56 A) in a ball of radius 2.9 A:
    ~580 atoms, every pair within rc = 6 A (no pair near the cutoff)."""
    rng = np.random.default_rng(23)
    g = np.arange(-2.9, 2.9001, 0.56)
    pts = np.array([(x, y, z) for x in g for y in g for z in g])
    pts = pts[np.einsum("ij,ij->i", pts, pts) <= 2.9 ** 2]
    pts = pts + rng.uniform(-0.04, 0.04, pts.shape)
    types = np.where(np.arange(len(pts)) % 3 == 0, synth.O, synth.H).astype(np.int32)
    return synth.Box(pos=pts + 7.0, types=types, box=np.array([14.0, 14.0, 14.0]))


def test_dense_ball_one_wave_fp32():
    """FP32 stages the ball's ~580 neighbours per centre with one wave per
    centre (its records are half the FP64 size), so the masks span over 80
    blocks per atom.  Every pair is inside rc, so masks on and off test the
    same pairs and agree to the order of the force sums.  Against the FP64
    oracle the bars are FP32's on this input: each force is a sum of about
    1.7e5 triplet terms with |F| up to 30 eV/A (measured 4e-5 rms E_i and
    5e-3 rms F, the same with masks off)."""
    b = _dense_ball()
    ref = oracle_water().compute(oracle_input(b, "fp32"), b.types, b.box, use_cells=True)
    res = []
    for on in (True, False):
        pot = make_potential("fp32")
        pot.set_parallelism("wave")
        pot.set_pair_masks(on)
        res.append(run(pot, b))
        pot.close()
    rms_e, rms_f = np.sqrt(np.mean(ref["Ei"] ** 2)), np.sqrt(np.mean(ref["F"] ** 2))
    for e, ei, f in res:
        say("dense ball fp32 max dEi/rms", np.max(np.abs(ei - ref["Ei"])) / rms_e,
            "max dF/rms", np.max(np.abs(f - ref["F"])) / rms_f)
        assert np.max(np.abs(ei - ref["Ei"])) <= 1e-4 * rms_e
        assert np.max(np.abs(f - ref["F"])) <= 1e-2 * rms_f
    assert np.max(np.abs(res[0][1] - res[1][1])) <= 1e-6 * rms_e
    assert np.max(np.abs(res[0][2] - res[1][2])) <= 1e-5 * rms_f


def test_pair_masks_argument_errors():
    pot = make_potential("fp32")
    assert pot._L.nnp_set_pair_masks(pot._h, 2) == -1  # NNP_E_ARG through the C ABI
    assert "on must be" in pot._L.nnp_last_error(pot._h).decode()
    pot.close()


@pytest.mark.parametrize("form", ["fp64", "fp32"])
def test_backward_reads_the_masks(form):
    """The force-adjoint pass of nnp_backward reads the pair-test masks: of
    the forward whose list it reuses (a compute_batch on the same inputs just
    before), or of its own SF pass (a backward alone).  Both, with masks on,
    equal masks off to the order of the sums.  (One wave per centre named
    explicitly: a batch this small would otherwise take two, without masks.)"""
    import torch

    boxes = [synth.water_box(s, 60 + i) for i, s in enumerate((4, 5, 4, 6))]
    pos = np.concatenate([b.pos for b in boxes])
    types = np.concatenate([b.types for b in boxes]).astype(np.int32)
    offs = np.cumsum([0] + [b.n_atoms for b in boxes])
    bx = np.stack([b.box for b in boxes])
    rng = np.random.default_rng(3)
    gE = rng.normal(size=len(boxes))
    gF = rng.normal(size=pos.shape)
    grads = {}
    for on in (True, False):
        for reuse in (True, False):
            pot = make_potential(form)
            pot.set_parallelism("wave")
            pot.set_pair_masks(on)
            x = torch.tensor(pos, dtype=pot.dtype, device="cuda")
            t = torch.tensor(types, device="cuda")
            if reuse:
                pot.compute_batch(x, t, offs, bx)
            g = pot.backward(x, t, offs, bx, torch.tensor(gE, device="cuda"),
                             torch.tensor(gF, dtype=pot.dtype, device="cuda"))
            grads[(on, reuse)] = g.cpu().numpy()
            pot.close()
    ref = grads[(False, False)]
    scale = np.max(np.abs(ref))
    for key, g in grads.items():
        d = np.max(np.abs(g - ref)) / scale
        say("backward", form, "masks", key[0], "reuse", key[1], "max rel diff", d)
        assert d <= (1e-12 if form == "fp64" else 1e-4), (key, d)


def test_mask_workspace_and_row_threshold():
    """Masks take a whole number of 256-byte blocks per atom on water (86
    neighbours), within the step bound of rows of at most 2 * 86; on the fcc
    metal (18 neighbours, below the 64 from which they pay) they are not
    allocated at all."""
    def workspace(table_nets, b, on):
        pot = make_potential("fp32", *table_nets) if table_nets else make_potential("fp32")
        pot.set_pair_masks(on)
        run(pot, b)
        ws = pot.workspace_bytes
        pot.close()
        return ws

    b = synth.water_box(16, 12)
    extra = workspace(None, b, True) - workspace(None, b, False)
    per_atom = extra / b.n_atoms
    say("mask workspace per atom (B)", per_atom)
    assert extra > 0 and extra % (256 * b.n_atoms) == 0
    m = 2 * 86
    assert per_atom <= 256 * (((m * m + 2 * m + 63) // 64 + 3 + 31) // 32)
    f = synth.fcc_box(8, 2)
    tn = (synth.ni_table_scaled(), synth.ni_nets())
    assert workspace(tn, f, True) == workspace(tn, f, False)
