"""Write the frozen centring/scaling constants of the Ni SF tables (narrow
and wide angular).

As for water: for every SF the shift is the mean and the scale the range
(max - min) of the raw SF over the 256 atoms of the reference fcc box
(4 cells per axis, seed 0), computed with the FP64 oracle; a range below
1e-12 gives scale 1.

Run from the repository root:  python oracle/make_ni_scaling.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "oracle"))

from paper_2002_00054_amd import synth  # noqa: E402  (seeded inputs only)
import oracle  # noqa: E402

DATA = os.path.join(ROOT, "paper_2002_00054_amd", "data")


def write(table, name, what):
    pot = oracle.Potential(table, synth.ni_nets(), n_el=1)
    b = synth.fcc_box(4, 0)
    G = pot.descriptors(b.pos, b.types, b.box)[:, :pot.n_sf[0]]
    rng = G.max(axis=0) - G.min(axis=0)
    doc = {
        "what": f"frozen shift (mean) and scale (max-min) of raw SFs, {what}, "
                "256-atom fcc box 4 cells per axis seed 0, FP64 oracle",
        "shift": {"Ni": [float(x) for x in G.mean(axis=0)]},
        "scale": {"Ni": [float(x) for x in np.where(rng < 1e-12, 1.0, rng)]},
    }
    out = os.path.join(DATA, name)
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", out)


def main():
    # shift 0, scale 1 in the tables: raw G
    write(synth.ni_sf_table(), "ni_scaling.json", "Ni table")
    write(synth.ni_g9_sf_table(), "ni_g9_scaling.json", "Ni table with wide angular SFs")


if __name__ == "__main__":
    main()
