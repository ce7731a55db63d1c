"""The HIP lead field against the closed-form multilayer-sphere potential at
2 mm (homogeneous and four-layer sphere, 32 electrodes, 6 fixed dipoles x 3
orientations): the mean RDM and |MAG-1| must equal the oracle's stored 2 mm
values (tests/golden/physics_guards.json, make_physics_guards.py) to within
the solver tolerance's effect, and stay below the 4 mm values."""
import importlib.util
import json
import os

import numpy as np
import pytest

from oracle import leadfield as lf, sphere
from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _guards_module():
    spec = importlib.util.spec_from_file_location(
        "make_physics_guards", os.path.join(GOLDEN, "make_physics_guards.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("case", ["homogeneous", "four_layer"])
def test_gpu_leadfield_against_sphere_series_2mm(case):
    from paper_1811_07717_amd import zi
    mod = _guards_module()
    sig = (0.33,) * 4 if case == "homogeneous" else hm.SIGMAS
    with open(os.path.join(GOLDEN, "physics_guards.json")) as f:
        guards = json.load(f)[case]
    H = hm.make_head(2.0, L=32, m=1, seed=5, sigmas=sig)
    cen = H.nodes[H.tets].mean(1)
    dip = np.array([np.argmin(((cen - f) ** 2).sum(1)) for f in mod.FIXED_DIPOLES],
                   dtype=np.int32)
    print(f"[case] physics {case} 2 mm: n={H.n} L={H.L}", flush=True)
    g = zi.System.from_head(H)
    T, _ = g.transfer_solve(tol=1e-10)
    G = g.point_dipoles(torch.from_numpy(dip).cuda())
    LF = g.leadfield(T, G).cpu().numpy()
    g.close()
    R = lf.average_reference(H.L)
    pos = cen[dip]
    ana = np.zeros_like(LF)
    for d in range(len(dip)):
        for k in range(3):
            ana[:, 3 * d + k] = R @ sphere.potential(H.centres, pos[d], np.eye(3)[k],
                                                     mod.RADII, sig)
    rdm = float(lf.rdm(LF, ana).mean())
    mag = float(np.abs(lf.mag(LF, ana) - 1).mean())
    print(f"[2mm] {case}: GPU mean RDM {rdm:.5f} |MAG-1| {mag:.5f}; oracle "
          f"{guards['2']['rdm']:.5f} {guards['2']['mag']:.5f}", flush=True)
    assert rdm == pytest.approx(guards["2"]["rdm"], rel=1e-3, abs=1e-6)
    assert mag == pytest.approx(guards["2"]["mag"], rel=1e-3, abs=1e-6)
    assert rdm < guards["4"]["rdm"] and mag < guards["4"]["mag"]
