"""The library's device block cache: a system built on blocks that another
system of the same sizes left behind must give exactly the results of one
built on fresh memory (no state may leak through reused blocks)."""
import dataclasses

import numpy as np
import pytest

from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def build_solve(H):
    from paper_1811_07717_amd import zi
    g = zi.System.from_head(H)
    T, st = g.transfer_solve(tol=1e-8)
    G = g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda())
    LF = g.leadfield(T, G)
    v = g.view()
    vals = v["val"].clone()
    g.close()
    return T, st, LF, vals


def test_cached_blocks_do_not_leak_state():
    from paper_1811_07717_amd import zi
    H = hm.workload("sphere8mm_L37")
    zi.release_cached_memory()
    print("[gpu] fresh build 8 mm L37", flush=True)
    T1, s1, LF1, v1 = build_solve(H)
    # same sizes, other values: its blocks go back to the cache dirty
    H2 = dataclasses.replace(H, sigma=H.sigma * 3.7, Z=H.Z * 0.3)
    print("[gpu] build with other values, same sizes", flush=True)
    build_solve(H2)
    print("[gpu] build on cached blocks", flush=True)
    T2, s2, LF2, v2 = build_solve(H)
    assert torch.equal(v1, v2)
    assert torch.equal(T1, T2)
    np.testing.assert_array_equal(s1["iters"], s2["iters"])
    assert torch.equal(LF1, LF2)
    zi.release_cached_memory()
    T3, s3, LF3, _ = build_solve(H)
    assert torch.equal(T1, T3)
    zi.release_cached_memory()
