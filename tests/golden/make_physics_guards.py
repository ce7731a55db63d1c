"""Writes physics_guards.json: the oracle's lead-field error against the
closed-form multilayer-sphere potential, on the first oracle run.

The paper prints no accuracy figures for its lead fields, so these guards are
measured, not quoted: mean RDM and mean |MAG-1| over 6 fixed dipoles x 3
orientations at 32 Fibonacci electrodes, for a homogeneous sphere and for the
four-layer sphere, at 8 mm, 4 mm and 2 mm.  Calls only the oracle and the seeded
input generator.

    python tests/golden/make_physics_guards.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fem, leadfield as lf, solve, source, sphere  # noqa: E402
from paper_1811_07717_amd import headmodel as hm  # noqa: E402

RADII = [r * 1e-3 for r in hm.RADII_MM]
FIXED_DIPOLES = np.array([[0.0, 0, 0], [0.03, 0.01, -0.02], [-0.05, 0.02, 0.01],
                          [0.01, -0.06, 0.03], [0.0, 0.0, 0.065], [0.04, 0.04, -0.03]])


def physics_errors(h_mm, sigmas):
    H = hm.make_head(h_mm, L=32, m=1, seed=5, sigmas=sigmas)
    cen = H.nodes[H.tets].mean(1)
    dip = np.array([np.argmin(((cen - f) ** 2).sum(1)) for f in FIXED_DIPOLES],
                   dtype=np.int32)
    S = fem.assemble(H.nodes, H.tets, H.sigma, H.tris, H.tri_electrode, H.Z)
    T = solve.transfer_reference(S["A"], S["B"], tol=1e-10)
    G = source.point_dipole_matrix(H.nodes, H.tets, dip)
    LF = lf.leadfield(T, S["B"], S["C"], G)
    pos = cen[dip]
    R = lf.average_reference(32)
    ana = np.zeros_like(LF)
    for d in range(len(dip)):
        for k in range(3):
            ana[:, 3 * d + k] = R @ sphere.potential(H.centres, pos[d], np.eye(3)[k],
                                                     RADII, sigmas)
    return float(lf.rdm(LF, ana).mean()), float(np.abs(lf.mag(LF, ana) - 1).mean())


def main():
    out = {"_source": "tests/golden/make_physics_guards.py (oracle only)"}
    for case, sig in (("homogeneous", (0.33,) * 4), ("four_layer", hm.SIGMAS)):
        out[case] = {}
        for h in (8.0, 4.0, 2.0):
            r, m = physics_errors(h, sig)
            out[case]["%d" % h] = {"rdm": r, "mag": m}
            print(case, h, r, m, flush=True)
    with open(os.path.join(HERE, "physics_guards.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
