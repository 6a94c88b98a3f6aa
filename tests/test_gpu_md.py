"""The MD driver (nnp_md_run, velocity Verlet on the device) through the C ABI.

Parity: trajectories, forces and energies against the oracle's integrator
over the oracle's forces, from the same seeded start (FP64 to 1e-8 A and
A/fs, FP32 to 1e-4).  Properties that hold at any size: constant-energy
drift bounds, the scheme's second order and its time reversibility.
"""
import numpy as np
import pytest

import oracle
from common import oracle_water
from gpu_common import make_potential, say
from paper_2002_00054_amd import synth

pytestmark = pytest.mark.gpu

MASSES = synth.WATER_MASSES


def _gpu_run(pot, b, v0, dt, steps, pos=None, skin=0.0):
    import torch

    pot.set_md_skin(skin)
    x = torch.tensor(b.pos if pos is None else pos, dtype=pot.dtype, device="cuda")
    v = torch.tensor(v0, dtype=pot.dtype, device="cuda")
    t = torch.tensor(b.types, dtype=torch.int32, device="cuda")
    f, ep, ek = pot.md_run(x, v, t, b.box, MASSES, dt, steps)
    return x.double().cpu().numpy(), v.double().cpu().numpy(), f.double().cpu().numpy(), ep, ek


def _mod_diff(a, b, box):
    return (a - b + 0.5 * box) % box - 0.5 * box


@pytest.mark.parametrize("skin", [0.0, 1.0, 0.3])
@pytest.mark.parametrize("side,seed,steps", [(4, 3, 20), (16, 11, 4)])
def test_md_fp64_matches_oracle(side, seed, steps, skin):
    """Per-step rebuild (skin 0) and skin lists of 1 A and 0.3 A (rebuilt
    every few steps) follow the oracle's trajectory."""
    b = synth.water_box(side, seed)
    v0 = synth.thermal_velocities(b.types, seed=seed)
    say("md fp64", b.n_atoms, "atoms", steps, "steps, skin", skin)
    pot = make_potential("fp64")
    x, v, f, ep, ek = _gpu_run(pot, b, v0, 0.5, steps, skin=skin)
    say("  neighbour-list builds", pot.md_list_builds)
    if skin == 0.0:
        assert pot.md_list_builds == steps + 1
    else:  # atoms here move up to about 1 A in 10 fs: rebuilds every few steps
        assert 1 <= pot.md_list_builds <= steps + 1
    rx, rv, rf, rep, rek = oracle.velocity_verlet(oracle_water(), b.pos, v0, b.types, b.box, MASSES, 0.5, steps)
    assert np.max(np.abs(_mod_diff(x, rx, b.box))) < 1e-8
    assert np.max(np.abs(v - rv)) < 1e-8
    assert np.max(np.abs(f - rf)) < 1e-7
    np.testing.assert_allclose(ep, rep, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(ek, rek, rtol=1e-9)


@pytest.mark.parametrize("skin", [0.0, 1.0])
def test_md_fp32_matches_oracle(skin):
    b = synth.water_box(4, 3)
    v0 = synth.thermal_velocities(b.types, seed=3)
    x0 = b.pos.astype(np.float32).astype(np.float64)
    v0 = v0.astype(np.float32).astype(np.float64)
    x, v, f, ep, ek = _gpu_run(make_potential("fp32"), b, v0, 0.5, 10, pos=x0, skin=skin)
    rx, rv, rf, rep, rek = oracle.velocity_verlet(oracle_water(), x0, v0, b.types, b.box, MASSES, 0.5, 10)
    say("md fp32 max dx", np.max(np.abs(_mod_diff(x, rx, b.box))), "dv", np.max(np.abs(v - rv)))
    assert np.max(np.abs(_mod_diff(x, rx, b.box))) < 1e-4
    assert np.max(np.abs(v - rv)) < 1e-4
    assert np.max(np.abs(ep - rep)) / b.n_atoms < 1e-5
    assert np.max(np.abs(ek - rek)) / b.n_atoms < 1e-5


def test_md_zero_steps_is_one_force_evaluation():
    import torch

    b = synth.water_box(4, 2)
    pot = make_potential("fp64")
    x, v, f, ep, ek = _gpu_run(pot, b, synth.thermal_velocities(b.types, seed=2), 0.5, 0)
    e, _, f_ref = pot.compute(torch.tensor(b.pos, dtype=torch.float64, device="cuda"),
                              torch.tensor(b.types, dtype=torch.int32, device="cuda"), b.box)
    assert ep.shape == (1,) and ep[0] == pytest.approx(e, rel=1e-13)
    assert np.max(np.abs(f - f_ref.cpu().numpy())) < 1e-12
    m = np.asarray(MASSES)[b.types]
    assert ek[0] == pytest.approx(oracle.kinetic_energy(synth.thermal_velocities(b.types, seed=2), m), rel=1e-12)


@pytest.mark.parametrize("skin", [0.0, 1.0])
@pytest.mark.parametrize("form,bound", [("fp64", 2e-4), ("fp32", 5e-4)])
def test_md_energy_conservation(form, bound, skin):
    """12,288 atoms, 200 steps of 0.25 fs: the total energy stays within the
    integrator's bound, and over 8 fs its deviation falls about fourfold when
    dt halves (FP64)."""
    b = synth.water_box(16, 12)
    v0 = synth.thermal_velocities(b.types, seed=12)
    pot = make_potential(form)
    _, _, _, ep, ek = _gpu_run(pot, b, v0, 0.25, 200, skin=skin)
    et = ep + ek
    drift = np.max(np.abs(et - et[0])) / b.n_atoms
    say("md", form, "skin", skin, "max |dE_total| per atom over 50 fs", drift, "ekin", ek[0], ek[-1],
        "builds", pot.md_list_builds)
    assert drift < bound
    if form == "fp64":
        dev = []
        for dt in (0.5, 0.25):
            _, _, _, ep, ek = _gpu_run(pot, b, v0, dt, int(round(8.0 / dt)), skin=skin)
            dev.append(np.max(np.abs(ep + ek - ep[0] - ek[0])))
        assert 3.0 < dev[0] / dev[1] < 5.0, dev


def test_md_time_reversibility_fp64():
    b = synth.water_box(6, 4)
    v0 = synth.thermal_velocities(b.types, seed=4)
    pot = make_potential("fp64")
    x1, v1, _, _, _ = _gpu_run(pot, b, v0, 0.5, 20)
    x2, v2, _, _, _ = _gpu_run(pot, b, -v1, 0.5, 20, pos=x1)
    assert np.max(np.abs(_mod_diff(x2, b.pos, b.box))) < 1e-8
    assert np.max(np.abs(v2 + v0)) < 1e-8


def test_md_argument_errors():
    import torch

    from paper_2002_00054_amd.nnp import NNPError

    b = synth.water_box(4, 1)
    pot = make_potential("fp64")
    x = torch.tensor(b.pos, dtype=torch.float64, device="cuda")
    v = torch.zeros_like(x)
    t = torch.tensor(b.types, dtype=torch.int32, device="cuda")
    for masses, dt in (((1.0, 0.0), 0.5), ((1.0, 16.0), 0.0), ((1.0, 16.0), float("nan"))):
        with pytest.raises(NNPError, match="NNP_E_ARG"):
            pot.md_run(x, v, t, b.box, masses, dt, 3)
    np.testing.assert_array_equal(x.cpu().numpy(), b.pos)  # nothing ran


def test_md_skin_list_equals_rebuild_fp64():
    """The same 40-step run with the list rebuilt every step and with skins of
    1 A and 0.1 A: equal trajectories up to rounding order, and the skin
    saves builds (the more, the wider it is)."""
    b = synth.water_box(16, 13)
    v0 = synth.thermal_velocities(b.types, seed=13)
    pot = make_potential("fp64")
    ref = _gpu_run(pot, b, v0, 0.5, 40)
    assert pot.md_list_builds == 41
    counts = []
    for skin in (1.0, 0.1):
        out = _gpu_run(pot, b, v0, 0.5, 40, skin=skin)
        builds = pot.md_list_builds
        counts.append(builds)
        say("skin", skin, "builds", builds)
        assert 1 <= builds < 41
        assert np.max(np.abs(_mod_diff(out[0], ref[0], b.box))) < 1e-10
        assert np.max(np.abs(out[1] - ref[1])) < 1e-10
        assert np.max(np.abs(out[2] - ref[2])) < 1e-9
        np.testing.assert_allclose(out[3], ref[3], rtol=1e-12)
    assert counts[0] < counts[1]


def test_md_skin_argument_errors():
    from paper_2002_00054_amd.nnp import NNPError

    pot = make_potential("fp64")
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(NNPError, match="NNP_E_ARG"):
            pot.set_md_skin(bad)
