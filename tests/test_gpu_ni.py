"""Second workload on the GPU through the C ABI: the single-element fcc metal
with the 3.9 A cutoff of the paper's Ni model (14 SFs, SF-25-25-1).

Parity against the FP64 oracle at the same bars as water (FP64 1e-9
relative, FP32 1e-5 eV / 1e-4 eV/A, BF16 force RMSE 5e-3 eV/A), from a box
with two cells per axis (the deduplicated cell stencil) up to the
1,492,992-atom box of the paper's Ni runs (sampled atoms there), and the
perfect lattice's zero forces.
"""
import numpy as np
import pytest

import oracle
from gpu_common import check_fp32, check_fp64, make_potential, oracle_input, run, say
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


def _pots(form):
    table, nets = synth.ni_table_scaled(), synth.ni_nets()
    return make_potential(form, table, nets), oracle.Potential(table, nets, n_el=1)


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("n,seed", [(3, 1), (8, 2), (20, 3)])
def test_ni_matches_oracle(form, n, seed):
    b = synth.fcc_box(n, seed)
    say("ni", form, b.n_atoms, "atoms")
    pot, ref_pot = _pots(form)
    e, ei, f = run(pot, b)
    ref = ref_pot.compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    else:
        check_fp32(ei, f, ref["Ei"], ref["F"])
    pot.close()


def test_ni_bf16_force_rmse():
    b = synth.fcc_box(20, 3)
    pot, ref_pot = _pots("bf16")
    e, ei, f = run(pot, b)
    ref = ref_pot.compute(oracle_input(b, "bf16"), b.types, b.box, use_cells=True)
    rmse = float(np.sqrt(np.mean((f - ref["F"]) ** 2)))
    say("ni bf16 force RMSE", rmse)
    assert rmse <= 5e-3
    pot.close()


def test_ni_perfect_lattice_zero_force():
    b = synth.fcc_box(8, 0, jitter=0.0)
    pot, _ = _pots("fp64")
    e, ei, f = run(pot, b)
    assert np.max(np.abs(f)) < 1e-10
    assert np.ptp(ei) < 1e-11
    pot.close()


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_ni_fullsize_sampled(form):
    """1,492,992 atoms (72 cells per axis), as the report times it."""
    b = synth.fcc_box(72, 72)
    rng = np.random.default_rng(72)
    idx = list(rng.choice(b.n_atoms, size=120, replace=False))
    for a in range(3):
        idx += [int(np.argmin(b.pos[:, a])), int(np.argmax(b.pos[:, a]))]
    idx = np.array(sorted(set(idx)), dtype=np.int64)
    say("ni fullsize", form, b.n_atoms, "atoms, sampled", len(idx))
    pot, ref_pot = _pots(form)
    e, ei, f = run(pot, b)
    Ei, F = ref_pot.sampled(oracle_input(b, form), b.types, b.box, idx)
    if form == "fp64":
        check_fp64(ei[idx], f[idx], Ei, F)
        assert np.max(np.abs(np.sum(f, axis=0))) < 1e-8
    else:
        check_fp32(ei[idx], f[idx], Ei, F)
        assert np.max(np.abs(np.sum(f, axis=0))) < 0.05
    assert abs(e - float(np.sum(ei))) <= 1e-12 * abs(e) + 1e-9
    pot.close()


def test_ni_weight_gradient_matches_oracle():
    """Differentiation form on the second workload (10,976 + 108 atoms: the
    triplet kernels' multi-centre waves in the SF, force and JVP passes)."""
    import torch

    from paper_2002_00054_amd.nnp import energy_forces

    table, nets = synth.ni_table_scaled(), synth.ni_nets()
    teacher = synth.xavier_nets(synth.sf_counts(table, n_el=1), 7, bias_halfwidth=0.1)
    boxes = [synth.fcc_box(14, 5), synth.fcc_box(3, 6)]
    Ehat, Fhat = oracle.batch_energy_forces(oracle.Potential(table, teacher, n_el=1), boxes)
    L_ref, g_ref = oracle.loss_and_grad(oracle.Potential(table, nets, n_el=1), boxes, Ehat, Fhat)
    pot = make_potential("fp64", table, nets)
    pos = torch.tensor(np.concatenate([b.pos for b in boxes]), dtype=torch.float64, device="cuda")
    types = torch.tensor(np.concatenate([b.types for b in boxes]), dtype=torch.int32, device="cuda")
    offs = np.cumsum([0] + [b.n_atoms for b in boxes])
    th = torch.tensor(synth.flat_params(nets), dtype=torch.float64, device="cuda", requires_grad=True)
    E, F = energy_forces(th, pos, pot, types, offs, np.stack([b.box for b in boxes]))
    N = torch.tensor([b.n_atoms for b in boxes], dtype=torch.float64, device="cuda")
    L = torch.mean(((E - torch.tensor(Ehat, device="cuda")) / N) ** 2) + \
        0.1 * torch.sum((F - torch.tensor(Fhat, device="cuda")) ** 2) / (3 * N.sum())
    (g,) = torch.autograd.grad(L, th)
    rel = float(np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref))
    say("ni fp64 weight-gradient rel-L2", rel)
    assert rel < 1e-8
    assert L.item() == pytest.approx(L_ref, rel=1e-10)
    pot.close()
