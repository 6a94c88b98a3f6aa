"""The two AI-systems forms beside the plain path, on the GPU through the C ABI.

Precision form (NNP_BF16_MIXED): errors against the FP64 oracle on a fresh
12,288-atom box; the force RMSE must stay within 5e-3 eV/A.

Differentiation form: forces are the adjoint of the energy (gradcheck in
FP64), and the parameter gradient of the energy+force loss from
nnp_backward matches the FP64 oracle's gradient (FP64 to 1e-8, FP32 to 1e-4
relative L2 per layer) and central differences of the GPU loss.
"""
import json

import numpy as np
import pytest

import oracle
from common import oracle_water, water_potential
from gpu_common import (check_fp32, check_fp64, gpu_loss_and_grad, make_potential, oracle_input,
                        per_tensor_rel, run, say)
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


def test_bf16_form_errors_vs_oracle():
    b = synth.water_box(16, 12)
    pot = make_potential("bf16")
    e, ei, f = run(pot, b)
    ref = oracle_water().compute(oracle_input(b, "bf16"), b.types, b.box, use_cells=True)
    de = ei - ref["Ei"]
    df = f - ref["F"]
    rmse_f = float(np.sqrt(np.mean(df ** 2)))
    say(f"bf16 form: E/atom err {abs(e - ref['E']) / b.n_atoms:.3e} eV, Ei rmse {np.sqrt(np.mean(de ** 2)):.3e} "
        f"max {np.max(np.abs(de)):.3e} eV, F rmse {rmse_f:.3e} max {np.max(np.abs(df)):.3e} eV/A "
        f"(mean |F| {np.mean(np.abs(ref['F'])):.3e})")
    assert rmse_f <= 5e-3
    assert np.max(np.abs(de)) <= 5e-2


@pytest.mark.parametrize("form", ["fp64", "fp32", "bf16"])
def test_accuracy_table_12288(form):
    """Each form against the FP64 oracle on a 12,288-atom box (lattice side 16,
    seed 12), printed as one JSON line: the accuracy column of the measured
    results table.  Bars: FP64 1e-9 relative, FP32 1e-5 eV / 1e-4 eV/A,
    BF16 force RMSE 5e-3 eV/A."""
    b = synth.water_box(16, 12)
    pot = make_potential(form)
    e, ei, f = run(pot, b)
    ref = oracle_water().compute(oracle_input(b, form), b.types, b.box, use_cells=True)
    de, df = ei - ref["Ei"], f - ref["F"]
    rmse_f = float(np.sqrt(np.mean(df ** 2)))
    say(json.dumps({"report": "accuracy", "form": form, "atoms": b.n_atoms,
                    "E_per_atom_abs_err": abs(e - ref["E"]) / b.n_atoms,
                    "Ei_max_abs_err": float(np.max(np.abs(de))),
                    "Ei_max_rel_err": float(np.max(np.abs(de) / np.maximum(np.abs(ref["Ei"]), 1e-300))),
                    "F_max_abs_err": float(np.max(np.abs(df))), "F_rmse": rmse_f}))
    if form == "fp64":
        check_fp64(ei, f, ref["Ei"], ref["F"])
    elif form == "fp32":
        check_fp32(ei, f, ref["Ei"], ref["F"])
    else:
        assert rmse_f <= 5e-3
    pot.close()


def test_fp32_mfma_network_matches_oracle_tightly():
    """The FP32 network on MFMA (not only the SF terms) is within FP32 error."""
    b = synth.water_box(6, 9)
    pot = make_potential("fp32")
    e, ei, f = run(pot, b)
    ref = oracle_water().compute(oracle_input(b, "fp32"), b.types, b.box)
    assert np.max(np.abs(ei - ref["Ei"])) < 2e-6
    assert np.max(np.abs(f - ref["F"])) < 2e-5


# ----------------------------------------------------------- differentiation
def test_energy_gradient_is_minus_force_gradcheck():
    import torch

    from paper_2002_00054_amd.nnp import energy

    c = synth.water_box(4, 6)
    pot = make_potential("fp64")
    pos = torch.tensor(c.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    types = torch.tensor(c.types, dtype=torch.int32, device="cuda")
    E = energy(pos, pot, types, c.box)
    (g,) = torch.autograd.grad(E, pos)
    _, _, f = pot.compute(pos.detach(), types, c.box)
    # two evaluations differ only by the order of the force atomics
    assert torch.allclose(g, -f, rtol=0, atol=1e-12 * f.abs().max().item())
    # central differences of E through the GPU path on a few coordinates
    idx = [(0, 0), (5, 2), (77, 1), (191, 0)]
    for i, a in idx:
        p = pos.detach().clone()
        p[i, a] += 1e-5
        ep = pot.compute(p, types, c.box)[0]
        p[i, a] -= 2e-5
        em = pot.compute(p, types, c.box)[0]
        assert abs((ep - em) / 2e-5 - g[i, a].item()) < 1e-6


def _batch(n_boxes=3):
    sides = [4, 5, 4][:n_boxes]
    boxes = [synth.water_box(s, 40 + i) for i, s in enumerate(sides)]
    return boxes


@pytest.fixture(scope="module")
def train_setup():
    table, nets = water_potential()
    teacher = oracle.Potential(table, synth.teacher_nets())
    boxes = _batch()
    Ehat, Fhat = oracle.batch_energy_forces(teacher, boxes)
    student = oracle.Potential(table, nets)
    L, g = oracle.loss_and_grad(student, boxes, Ehat, Fhat)
    return dict(table=table, nets=nets, boxes=boxes, Ehat=Ehat, Fhat=Fhat, L=L, g=g,
                params=synth.flat_params(nets))


def test_weight_gradient_fp64_matches_oracle(train_setup):
    s = train_setup
    pot = make_potential("fp64")
    L, g = gpu_loss_and_grad(pot, s["boxes"], s["Ehat"], s["Fhat"], s["params"])
    assert L == pytest.approx(s["L"], rel=1e-10)
    rel = per_tensor_rel(g, s["g"], s["nets"])
    say("fp64 weight-gradient rel-L2 per tensor, max", rel.max())
    assert rel.max() < 1e-8


def test_weight_gradient_fp32_matches_oracle(train_setup):
    s = train_setup
    pot = make_potential("fp32")
    L, g = gpu_loss_and_grad(pot, s["boxes"], s["Ehat"], s["Fhat"], s["params"])
    rel = per_tensor_rel(g, s["g"], s["nets"])
    say("fp32 weight-gradient rel-L2 per tensor, max", rel.max())
    assert L == pytest.approx(s["L"], rel=1e-4)
    assert rel.max() < 1e-4


def test_weight_gradient_finite_differences_gpu(train_setup):
    s = train_setup
    pot = make_potential("fp64")
    p0 = s["params"].copy()
    L, g = gpu_loss_and_grad(pot, s["boxes"], s["Ehat"], s["Fhat"], p0)
    rng = np.random.default_rng(3)
    h = 1e-5
    for k in rng.choice(len(p0), size=12, replace=False):
        pp = p0.copy()
        pp[k] += h
        pm = p0.copy()
        pm[k] -= h
        Lp, _ = gpu_loss_and_grad(pot, s["boxes"], s["Ehat"], s["Fhat"], pp)
        Lm, _ = gpu_loss_and_grad(pot, s["boxes"], s["Ehat"], s["Fhat"], pm)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_position_gradient_of_forces_raises(train_setup):
    import torch

    from paper_2002_00054_amd.nnp import energy_forces

    s = train_setup
    pot = make_potential("fp64")
    b = s["boxes"][0]
    pos = torch.tensor(b.pos, dtype=torch.float64, device="cuda", requires_grad=True)
    types = torch.tensor(b.types, dtype=torch.int32, device="cuda")
    th = torch.tensor(s["params"], dtype=torch.float64, device="cuda", requires_grad=True)
    E, F = energy_forces(th, pos, pot, types, [0, b.n_atoms], b.box[None])
    with pytest.raises(NotImplementedError):
        torch.autograd.grad(F.sum(), pos)


@pytest.fixture(scope="module")
def full_batch():
    """The 32-box training batch (192-1536 atoms per box, 30,108 atoms),
    labelled by the teacher, with the oracle's loss gradient."""
    table, nets = water_potential()
    boxes = synth.training_batch()
    Ehat, Fhat = oracle.batch_energy_forces(oracle.Potential(table, synth.teacher_nets()), boxes)
    L, g = oracle.loss_and_grad(oracle.Potential(table, nets), boxes, Ehat, Fhat)
    return dict(boxes=boxes, Ehat=Ehat, Fhat=Fhat, L=L, g=g, params=synth.flat_params(nets), nets=nets)


@pytest.mark.parametrize("form,tol", [("fp64", 1e-8), ("fp32", 1e-4)])
def test_weight_gradient_full_training_batch(full_batch, form, tol):
    s = full_batch
    pot = make_potential(form)
    L, g = gpu_loss_and_grad(pot, s["boxes"], s["Ehat"], s["Fhat"], s["params"])
    rel = float(np.linalg.norm(g - s["g"]) / np.linalg.norm(s["g"]))
    per = per_tensor_rel(g, s["g"], s["nets"])
    say(json.dumps({"report": "training_gradient", "form": form, "boxes": len(s["boxes"]),
                    "atoms": int(sum(b.n_atoms for b in s["boxes"])), "loss_rel_err": abs(L - s["L"]) / s["L"],
                    "grad_rel_l2_vs_oracle": rel, "grad_rel_l2_max_per_tensor": float(per.max())}))
    assert per.max() < tol, per
    assert L == pytest.approx(s["L"], rel=tol)
    pot.close()
