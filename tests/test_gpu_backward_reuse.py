"""nnp_backward after nnp_compute_batch with the same inputs reuses that
forward's sorted order, neighbour list and scaled SFs (the paper's
recompute principle, Sec. 3.3, concerns the per-pair derivatives, which
the force-adjoint pass still recomputes), and with other inputs rebuilds
them.  Both derivative modes; the gradients are compared bitwise with the
rebuilding path (every pass of the weight gradient is deterministic) and
per tensor with the FP64 oracle."""
import numpy as np
import pytest

import oracle
from common import water_potential
from gpu_common import make_potential, per_tensor_rel, say
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


def _batch():
    return [synth.water_box(4, 40), synth.water_box(5, 41), synth.water_box(4, 42)]


def _dev(boxes, dtype):
    import torch

    pos = torch.tensor(np.concatenate([b.pos for b in boxes]), dtype=dtype, device="cuda")
    types = torch.tensor(np.concatenate([b.types for b in boxes]), dtype=torch.int32, device="cuda")
    offs = np.cumsum([0] + [b.n_atoms for b in boxes])
    bx = np.stack([b.box for b in boxes])
    return pos, types, offs, bx


def _grads(pot, pos, types, offs, bx, seed=3):
    import torch

    rng = np.random.default_rng(seed)
    gE = torch.tensor(rng.standard_normal(len(offs) - 1), dtype=torch.float64, device="cuda")
    gF = torch.tensor(rng.standard_normal((pos.shape[0], 3)) * 1e-2, dtype=pot.dtype, device="cuda")
    return gE, gF


@pytest.mark.parametrize("mode", ["recompute", "stored"])
def test_backward_reuses_forward(mode):
    import torch

    boxes = _batch()
    pot = make_potential("fp64")
    pot.set_derivative_mode(mode)
    pos, types, offs, bx = _dev(boxes, torch.float64)
    gE, gF = _grads(pot, pos, types, offs, bx)
    pot.set_profiling(True)
    pot.compute_batch(pos, types, offs, bx)
    g_reuse = pot.backward(pos, types, offs, bx, gE, gF).cpu().numpy()
    names = pot.timings()
    say(mode, "backward stages after a forward of the same inputs:", sorted(names))
    assert "reuse" in names and "neighbors" not in names and "sf" not in names
    # a second backward of the same inputs still reuses them
    g_again = pot.backward(pos, types, offs, bx, gE, gF).cpu().numpy()
    assert "reuse" in pot.timings()
    # an intervening call on other inputs ends the reuse: the backward rebuilds
    other = synth.water_box(4, 7)
    p2 = torch.tensor(other.pos, dtype=torch.float64, device="cuda")
    t2 = torch.tensor(other.types, dtype=torch.int32, device="cuda")
    pot.compute(p2, t2, other.box)
    g_rebuilt = pot.backward(pos, types, offs, bx, gE, gF).cpu().numpy()
    names = pot.timings()
    assert "neighbors" in names and "sf" in names and "reuse" not in names
    assert np.array_equal(g_reuse, g_again)
    assert np.array_equal(g_reuse, g_rebuilt)
    pot.close()


@pytest.mark.parametrize("form,tol", [("fp64", 1e-8), ("fp32", 1e-4)])
def test_backward_with_moved_atom_rebuilds(form, tol):
    """Positions that differ from the forward's (one coordinate moved by
    0.05 A) are detected on the device: the backward rebuilds and its
    gradient is the oracle's for the moved positions."""
    import torch

    boxes = _batch()
    table, nets = water_potential()
    pot = make_potential(form)
    pos, types, offs, bx = _dev(boxes, pot.dtype)
    moved = [synth.Box(pos=b.pos.copy(), types=b.types, box=b.box) for b in boxes]
    moved[1].pos[10, 2] += 0.05
    if form == "fp32":
        moved = [synth.Box(pos=b.pos.astype(np.float32).astype(np.float64), types=b.types, box=b.box)
                 for b in moved]
    pos_m, _, _, _ = _dev(moved, pot.dtype)
    teacher = oracle.Potential(table, synth.teacher_nets())
    Ehat, Fhat = oracle.batch_energy_forces(teacher, moved)
    student = oracle.Potential(table, nets)
    E, F = oracle.batch_energy_forces(student, moved)
    N = [b.n_atoms for b in moved]
    _, gE, gF = oracle.loss_terms(E, Ehat, N, F, Fhat)
    _, g_ref = oracle.loss_and_grad(student, moved, Ehat, Fhat)
    pot.set_profiling(True)
    pot.compute_batch(pos, types, offs, bx)  # forward of the original positions
    g = pot.backward(pos_m, types, offs, bx, torch.tensor(gE, device="cuda"),
                     torch.tensor(gF, dtype=pot.dtype, device="cuda")).cpu().numpy()
    assert "neighbors" in pot.timings()
    per = per_tensor_rel(g, g_ref, nets)
    say(form, "moved-atom backward per-tensor rel-L2 max", float(per.max()))
    assert per.max() < tol, per
    pot.close()
