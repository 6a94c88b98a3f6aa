"""Pins of the oracle's velocity Verlet integrator (CPU).

- the unit conversions against an independent published value (the
  mass-velocity-squared to energy factor of the metal unit system,
  1.0364269e-4 eV per amu (A/ps)^2) and against each other;
- free flight: with zero forces (first layer and its bias zero) positions move
  by dt v per step exactly and the velocities and kinetic energy stay fixed;
- time reversibility of the scheme: n steps, velocity reversal, n steps
  return to the start;
- the scheme's second order: the largest total-energy deviation over a fixed
  time falls about fourfold when dt halves, and stays small.
A dropped or doubled half-kick, a sign error or a wrong unit factor fails
one of these.
"""
import numpy as np
import pytest

import oracle
from common import oracle_water, water_potential
from paper_2002_00054_amd import synth


def test_unit_conversions():
    assert oracle.KE_CONV == pytest.approx(1.0364269e-4 * 1e6, rel=1e-7)
    assert oracle.ACCEL_CONV * oracle.KE_CONV == pytest.approx(1.0, rel=1e-14)


def test_free_flight_with_zero_forces():
    table, nets = water_potential()
    nets = [synth.Net([w.copy() for w in n.W], [b.copy() for b in n.b]) for n in nets]
    for n in nets:
        n.W[0][:] = 0.0
        n.b[0][:] = 0.0
    pot = oracle.Potential(table, nets)
    b = synth.water_box(4, 1)
    v0 = synth.thermal_velocities(b.types, seed=1)
    dt, steps = 0.5, 7
    x, v, F, ep, ek = oracle.velocity_verlet(pot, b.pos, v0, b.types, b.box, synth.WATER_MASSES, dt, steps)
    assert np.all(F == 0.0)
    np.testing.assert_array_equal(v, v0)
    want = np.mod(np.mod(b.pos, b.box) + steps * dt * v0, b.box)
    d = (x - want + 0.5 * b.box) % b.box - 0.5 * b.box  # compare modulo the box
    assert np.max(np.abs(d)) < 1e-12
    assert np.ptp(ek) < 1e-12 * ek[0]
    assert np.ptp(ep) <= 1e-12 * abs(ep[0])


def test_time_reversibility():
    pot = oracle_water()
    b = synth.water_box(4, 3)
    v0 = synth.thermal_velocities(b.types, seed=3)
    x1, v1, _, _, _ = oracle.velocity_verlet(pot, b.pos, v0, b.types, b.box, synth.WATER_MASSES, 0.5, 12)
    assert np.max(np.abs(v1 - v0)) > 1e-3  # the forces did act
    x2, v2, _, _, _ = oracle.velocity_verlet(pot, x1, -v1, b.types, b.box, synth.WATER_MASSES, 0.5, 12)
    d = (x2 - b.pos + 0.5 * b.box) % b.box - 0.5 * b.box
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v2 + v0)) < 1e-9


def test_second_order_energy_error():
    pot = oracle_water()
    b = synth.water_box(4, 3)
    v0 = synth.thermal_velocities(b.types, seed=0)
    dev = []
    for dt in (0.5, 0.25):
        _, _, _, ep, ek = oracle.velocity_verlet(pot, b.pos, v0, b.types, b.box, synth.WATER_MASSES, dt,
                                                 int(round(8.0 / dt)))
        et = ep + ek
        dev.append(np.max(np.abs(et - et[0])))
    assert 3.0 < dev[0] / dev[1] < 5.0, dev
    assert dev[1] / b.n_atoms < 2e-4  # eV per atom at dt = 0.25 fs
