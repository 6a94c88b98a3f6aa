"""The GPU path at the full benchmark size, in the configuration bench.py times.

The 2,044,416-atom water box (lattice side 88, seed 22) is too large for the
full oracle, so each form is compared with the oracle's sampled evaluator
(E_i and F_i of chosen atoms, computed one by one from their neighbourhoods):
a seeded random sample plus the atoms closest to every box face, where the
minimum image and the periodic cell shifts matter.  Tolerances are those of
the small-box parity tests.  Properties that hold at any size are checked on
all atoms: E = sum_i E_i and a vanishing net force.
"""
import numpy as np
import pytest

from common import oracle_water
from gpu_common import check_fp32, check_fp64, make_potential, oracle_input, run, say
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    return synth.water_box(88, 22)


@pytest.fixture(scope="module")
def sample(big):
    rng = np.random.default_rng(88)
    idx = list(rng.choice(big.n_atoms, size=160, replace=False))
    w = np.mod(big.pos, big.box)
    for a in range(3):
        idx += [int(np.argmin(w[:, a])), int(np.argmax(w[:, a]))]
    return np.array(sorted(set(idx)), dtype=np.int64)


def _sampled(big, idx, precision):
    return oracle_water().sampled(oracle_input(big, precision), big.types, big.box, idx)


def _properties(e, ei, f, tol_net):
    assert abs(e - float(np.sum(ei))) <= 1e-12 * abs(e) + 1e-9
    net = np.abs(np.sum(f, axis=0))
    assert np.all(net <= tol_net), net


def test_fullsize_fp32(big, sample):
    say("fp32", big.n_atoms, "atoms, sampled", len(sample))
    e, ei, f = run(make_potential("fp32"), big)
    Ei, F = _sampled(big, sample, "fp32")
    check_fp32(ei[sample], f[sample], Ei, F)
    # FP32 force atomics: per-atom errors of ~1e-6 eV/A summed over 2M atoms
    _properties(e, ei, f, tol_net=0.05)


def test_fullsize_fp64(big, sample):
    say("fp64", big.n_atoms, "atoms, sampled", len(sample))
    e, ei, f = run(make_potential("fp64"), big)
    Ei, F = _sampled(big, sample, "fp64")
    check_fp64(ei[sample], f[sample], Ei, F)
    _properties(e, ei, f, tol_net=1e-8)


def test_fullsize_bf16_force_rmse(big, sample):
    say("bf16", big.n_atoms, "atoms, sampled", len(sample))
    e, ei, f = run(make_potential("bf16"), big)
    Ei, F = _sampled(big, sample, "bf16")
    rmse = float(np.sqrt(np.mean((f[sample] - F) ** 2)))
    say("bf16 sampled force RMSE", rmse, "max |dE_i|", float(np.max(np.abs(ei[sample] - Ei))))
    assert rmse <= 5e-3
    assert np.max(np.abs(ei[sample] - Ei)) <= 5e-2
