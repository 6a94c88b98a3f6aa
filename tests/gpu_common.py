"""Helpers of the GPU tests: potentials on the device, tolerance checks."""
import sys

import numpy as np

from common import water_potential


def dev():
    import torch

    return torch.device("cuda:0")


def make_potential(precision, table=None, nets=None):
    from paper_2002_00054_amd.nnp import Potential

    if table is None:
        table, nets = water_potential()
    return Potential(table, nets, precision=precision)


def to_dev(box_obj, dtype):
    import torch

    pos = torch.tensor(box_obj.pos, dtype=dtype, device=dev())
    types = torch.tensor(box_obj.types, dtype=torch.int32, device=dev())
    return pos, types


def run(pot, box_obj):
    """(E, Ei, F) as numpy float64 of one structure."""
    pos, types = to_dev(box_obj, pot.dtype)
    e, ei, f = pot.compute(pos, types, box_obj.box)
    return e, ei.double().cpu().numpy(), f.double().cpu().numpy()


def oracle_input(box_obj, precision):
    """Positions as the GPU sees them: rounded to float32 for FP32 forms."""
    if precision == "fp64":
        return box_obj.pos
    return box_obj.pos.astype(np.float32).astype(np.float64)


def check_fp64(ei, f, ref_ei, ref_f, rel=1e-9):
    """|dE_i| <= rel max(|E_i|, rms E) and |dF| <= rel rms(F)."""
    rms_e = np.sqrt(np.mean(ref_ei ** 2))
    rms_f = np.sqrt(np.mean(ref_f ** 2))
    tol_e = rel * np.maximum(np.abs(ref_ei), rms_e)
    assert np.all(np.abs(ei - ref_ei) <= tol_e), np.max(np.abs(ei - ref_ei) / tol_e)
    assert np.all(np.abs(f - ref_f) <= rel * rms_f), np.max(np.abs(f - ref_f)) / (rel * rms_f)


def check_fp32(ei, f, ref_ei, ref_f, tol_e=1e-5, tol_f=1e-4):
    de = np.max(np.abs(ei - ref_ei))
    df = np.max(np.abs(f - ref_f))
    assert de <= tol_e and df <= tol_f, (de, df)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_loss_and_grad(pot, boxes, Ehat, Fhat, params):
    """Energy+force loss of a batch (per-atom energy MSE + 0.1 force MSE)
    and its parameter gradient, through the autograd function over
    nnp_compute_batch / nnp_backward."""
    import torch

    from paper_2002_00054_amd.nnp import energy_forces

    dt = pot.dtype
    pos = torch.tensor(np.concatenate([b.pos for b in boxes]), dtype=dt, device="cuda")
    types = torch.tensor(np.concatenate([b.types for b in boxes]), dtype=torch.int32, device="cuda")
    offs = np.cumsum([0] + [b.n_atoms for b in boxes])
    bx = np.stack([b.box for b in boxes])
    th = torch.tensor(params, dtype=torch.float64, device="cuda", requires_grad=True)
    E, F = energy_forces(th, pos, pot, types, offs, bx)
    N = torch.tensor([b.n_atoms for b in boxes], dtype=torch.float64, device="cuda")
    Eh = torch.tensor(Ehat, dtype=torch.float64, device="cuda")
    Fh = torch.tensor(Fhat, dtype=dt, device="cuda")
    L = torch.mean(((E - Eh) / N) ** 2) + 0.1 * torch.sum((F - Fh).double() ** 2) / (3 * N.sum())
    (g,) = torch.autograd.grad(L, th)
    return L.item(), g.cpu().numpy()


def per_tensor_rel(g, ref, nets):
    """Relative L2 error of each parameter tensor (W1, b1, W2, b2, w3, b3 per
    element, in the flat parameter order)."""
    out = []
    o = 0
    for n in nets:
        for w, b in zip(n.W, n.b):
            for sz in (w.size, b.size):
                a, r = g[o:o + sz], ref[o:o + sz]
                out.append(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300))
                o += sz
    return np.array(out)
