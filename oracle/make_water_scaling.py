"""Write the frozen centring/scaling constants of the water SF table.

For every (centre element, SF) the shift is the mean and the scale the range
(max - min) of the raw SF over the atoms of that element in the 192-atom
reference box (lattice side 4, seed 0), computed with the FP64 oracle; a range
below 1e-12 gives scale 1.  The constants are frozen: every other box reuses
them, so that E stays a sum of per-atom terms.

Run from the repository root:  python oracle/make_water_scaling.py
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

OUT = os.path.join(ROOT, "paper_2002_00054_amd", "data", "water_scaling.json")


def main():
    table = synth.water_sf_table()  # shift 0, scale 1: raw G
    nets = synth.water_nets()
    pot = oracle.Potential(table, nets)
    b = synth.water_box(synth.CONFIG0["n"], synth.CONFIG0["scaling_seed"])
    G = pot.descriptors(b.pos, b.types, b.box)
    shift, scale = {}, {}
    for e, name in enumerate(synth.ELEMENTS):
        ns = pot.n_sf[e]
        g = G[b.types == e, :ns]
        mean = g.mean(axis=0)
        rng = g.max(axis=0) - g.min(axis=0)
        rng = np.where(rng < 1e-12, 1.0, rng)
        shift[name] = [float(x) for x in mean]
        scale[name] = [float(x) for x in rng]
    doc = {
        "what": "frozen shift (mean) and scale (max-min) of raw SFs, water table, "
                "192-atom box side 4 seed 0, FP64 oracle",
        "shift": shift,
        "scale": scale,
    }
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
