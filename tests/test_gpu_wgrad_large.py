"""Weight gradient (nnp_backward, FP64) of a 292,008-atom box against central
differences of the forward.  At this size the reduction over atoms takes
chunks of more than 64 atoms (at most 4096 chunks), a path the 30,108-atom
training batch does not reach.  Loss: L = g_E E + sum_i delta_i . F_i with a
seeded random delta; the forward gives L directly, so the differences need no
oracle, and both the energy and the force-adjoint terms are exercised."""
import numpy as np
import pytest

from gpu_common import make_potential, say, to_dev
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


def test_weight_gradient_large_box_central_differences():
    import torch

    b = synth.water_box(46, 5)
    assert b.n_atoms > 4096 * 64
    pot = make_potential("fp64")
    pos, types = to_dev(b, torch.float64)
    rng = np.random.default_rng(3)
    delta = torch.tensor(rng.normal(0.0, 1.0, (b.n_atoms, 3)), dtype=torch.float64, device="cuda")
    gE = 0.7
    say("wgrad large", b.n_atoms)
    g = pot.backward(pos, types, [0, b.n_atoms], [b.box], dL_dE=torch.tensor([gE], device="cuda"),
                     dL_dF=delta).cpu().numpy()
    theta = synth.flat_params(synth.water_nets())
    nH = 27 * 25 + 25 + 25 * 25 + 25 + 25 + 1
    # W1, b1, W2, b2, w3, b3 of H, then W1, W2, w3, b3 of O
    idx = [0, 300, 680, 1000, 1330, 1355, nH - 1, nH + 100, nH + 900, nH + 1430, len(theta) - 1]
    assert len(theta) == pot.n_params and nH == 1376

    def loss(th):
        pot.set_params(th)
        e, _, f = pot.compute(pos, types, b.box)
        return gE * e + float(torch.sum(delta * f).item())

    h = 1e-5
    fd = []
    for p in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fd.append((loss(tp) - loss(tm)) / (2 * h))
    pot.set_params(theta)
    fd = np.array(fd)
    scale = np.max(np.abs(fd))
    err = np.max(np.abs(g[idx] - fd)) / scale
    say("wgrad large: max |analytic - central difference| / max |gradient|", err)
    assert err < 1e-6
    pot.close()
