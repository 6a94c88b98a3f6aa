"""Shared fixtures of the test suite: the water potential and small tables."""
import math

import numpy as np

from paper_2002_00054_amd import synth


def water_potential():
    """(SF table with frozen shift/scale, per-element nets) of the water potential."""
    return synth.water_table_scaled(), synth.water_nets()


def oracle_water():
    import oracle

    t, n = water_potential()
    return oracle.Potential(t, n)


def tiny_table(radial=(), angular=(), rc=synth.RCUT):
    """Table where both centre elements get the same SFs.

    radial: list of (nbr element, eta); angular: list of ((e1, e2), eta, zeta, lam).
    """
    t = []
    for c in (synth.H, synth.O):
        for nb, eta in radial:
            t.append(synth.SF(c, 2, (nb,), eta, rc=rc))
        for cls, eta, zeta, lam in angular:
            t.append(synth.SF(c, 3, tuple(cls), eta, 0.0, float(zeta), float(lam), rc=rc))
    return t


def nets_for(table, seed=5, hidden=(4, 3), bias=0.0):
    counts = synth.sf_counts(table)
    return synth.xavier_nets(counts, seed, hidden=hidden, bias_halfwidth=bias)


def cluster(n_mol=5, seed=5, L=40.0):
    """Isolated cluster of the n_mol molecules nearest to molecule 0 of a
    192-atom box, unwrapped and centred in an L-edge box."""
    b = synth.water_box(4, seed)
    o = b.pos[0::3]
    d = o - o[0]
    d -= b.box * np.round(d / b.box)
    order = np.argsort(np.linalg.norm(d, axis=1))[:n_mol]
    pos, types = [], []
    for m in order:
        for a in range(3):
            x = b.pos[3 * m + a] - o[0]
            x -= b.box * np.round(x / b.box)
            pos.append(x)
            types.append(b.types[3 * m + a])
    pos = np.array(pos)
    pos = pos - pos.mean(axis=0) + L / 2
    return synth.Box(pos=pos, types=np.array(types, dtype=np.int32), box=np.array([L, L, L]))


def random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    return synth._quat_to_matrix(q[None, :])[0]


LN2 = math.log(2.0)
