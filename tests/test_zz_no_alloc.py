"""zi_leadfield_noalloc (the lead field with its workspace in a fixed device
array) against zi_leadfield on the same inputs: bit for bit, on two calls
in a row, the second with a smaller source matrix, and on a source matrix
longer than one workspace chunk."""
import numpy as np
import pytest

from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def solved():
    from paper_1811_07717_amd import zi
    H = hm.make_head(8.0, L=32, m=22000, seed=1812)
    say(f"[case] noalloc: 8 mm, L={H.L}, m={H.m}")
    g = zi.System.from_head(H)
    T, _ = g.transfer_solve(tol=1e-8)
    yield H, g, T
    g.close()


def test_noalloc_matches_leadfield(solved):
    from paper_1811_07717_amd import zi
    H, g, T = solved
    chunk = int(zi.lib().zi_leadfield_noalloc_max_cols(H.L))
    assert chunk > 0
    assert int(zi.lib().zi_leadfield_noalloc_max_cols(257)) == 0
    dip = torch.from_numpy(H.dipole_tets).cuda()
    G_big = g.point_dipoles(dip)
    G_small = g.point_dipoles(dip[:100])
    ncols = 3 * H.m
    assert ncols > chunk, "the first call must span more than one workspace chunk"
    for G, what in ((G_big, f"{ncols} columns ({chunk} per chunk)"), (G_small, "300 columns")):
        for prec in (0, 1):
            say(f"[gpu] zi_leadfield / zi_leadfield_noalloc, {what}, precision {prec}")
            ref = g.leadfield(T, G, precision=prec)
            out = torch.full_like(ref, np.nan)
            got = g.leadfield(T, G, precision=prec, out=out, noalloc=True)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (what, prec, (got - ref).abs().max().item())


def test_noalloc_rejects_bad_source(solved):
    from paper_1811_07717_amd import zi
    H, g, T = solved
    cp = torch.tensor([0, 1], dtype=torch.int32, device="cuda")
    ri = torch.tensor([H.n], dtype=torch.int32, device="cuda")   # row out of range
    gv = torch.ones(1, dtype=torch.float64, device="cuda")
    with pytest.raises(zi.ZiError) as e:
        g.leadfield(T, (cp, ri, gv), noalloc=True)
    assert e.value.status == zi.ZI_EINVAL
