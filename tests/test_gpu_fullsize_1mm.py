"""1 mm sphere, 256 electrodes, 100 000 dipoles: properties at full size.

The oracle cannot assemble and solve this size in a test's time, so the
checks are ones that hold at any size: the mesh-graph sizes equal the counts
taken independently of this code from the same seeded fixture mesh (n, e and
nnz of the 1 mm configuration), sampled electrode columns reach the FP64 true
residual, and every lead-field column sums to zero (average reference)."""
import numpy as np
import pytest

from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def test_sizes_residual_and_reference():
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere1mm_L256")
    say(f"[case] sphere1mm_L256: n={H.n} e={H.e} L={H.L} m={H.m}")
    assert (H.n, H.e) == (3339581, 19572768)
    g = zi.System.from_head(H)
    assert g.nnz == 49471669
    cols = [0, 101, 255]
    say("[gpu] zi_transfer_solve 1 mm, 3 columns")
    T, st = g.transfer_solve(tol=1e-8, columns=cols)
    say(f"[1mm] iterations {st['iters'].tolist()}, true residual {st['relres_true'].max():.2e}")
    assert st["relres_true"].max() <= 1.5e-8
    assert np.all(st["iters"] > 0)
    say("[gpu] full transfer solve + lead field for 300 dipole columns")
    Tall, st_all = g.transfer_solve(tol=1e-8)
    assert st_all["relres_true"].max() <= 1.5e-8
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets[:100]).cuda())
    LF = g.leadfield(Tall, G)
    s = LF.sum(dim=0).abs().max().item()
    say(f"[1mm] LF {tuple(LF.shape)}, max |column sum| {s:.2e}, max |LF| {LF.abs().max().item():.2e}")
    assert s <= 1e-9 * LF.abs().max().item()
    g.close()
