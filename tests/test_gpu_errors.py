"""Error paths of the C-ABI on the device.  Every invalid input here is one
the library's own validation kernels reject before any indexed access."""
import numpy as np
import pytest

from paper_1811_07717_amd import headmodel as hm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def head():
    return hm.make_head(8.0, L=8, m=5, seed=11)


def build(H, **over):
    from paper_1811_07717_amd import zi
    d = dict(nodes=H.nodes.copy(), tets=H.tets.copy(), sigma=H.sigma.copy(), tris=H.tris.copy(),
             te=H.tri_electrode.copy(), Z=H.Z.copy(), ground=-1)
    d.update(over)
    c = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return zi.System(c(d["nodes"]), c(d["tets"]), c(d["sigma"]), c(d["tris"]), c(d["te"]),
                     d["Z"], ground=d["ground"])


def status_of(H, **over):
    from paper_1811_07717_amd import zi
    try:
        build(H, **over).close()
        return zi.ZI_OK
    except zi.ZiError as e:
        return e.status


def test_valid_input_assembles(head):
    from paper_1811_07717_amd import zi
    assert status_of(head) == zi.ZI_OK


def test_index_out_of_range(head):
    from paper_1811_07717_amd import zi
    t = head.tets.copy()
    t[17, 2] = head.n
    assert status_of(head, tets=t) == zi.ZI_EMESH
    t = head.tets.copy()
    t[5, 1] = -1
    assert status_of(head, tets=t) == zi.ZI_EMESH


def test_repeated_vertex(head):
    from paper_1811_07717_amd import zi
    t = head.tets.copy()
    t[3, 3] = t[3, 0]
    assert status_of(head, tets=t) == zi.ZI_EMESH


def test_degenerate_tet(head):
    from paper_1811_07717_amd import zi
    x = head.nodes.copy()
    t = head.tets[100]
    x[t[3]] = (x[t[0]] + x[t[1]]) / 2       # flatten onto an edge
    assert status_of(head, nodes=x) == zi.ZI_EMESH


def test_bad_conductivity(head):
    from paper_1811_07717_amd import zi
    s = head.sigma.copy()
    s[7] = 0.0
    assert status_of(head, sigma=s) == zi.ZI_EMESH
    s[7] = -0.3
    assert status_of(head, sigma=s) == zi.ZI_EMESH
    s[7] = np.nan
    assert status_of(head, sigma=s) == zi.ZI_EMESH


def test_nonfinite_coordinate(head):
    from paper_1811_07717_amd import zi
    x = head.nodes.copy()
    x[3, 1] = np.inf
    assert status_of(head, nodes=x) == zi.ZI_EMESH


def test_electrode_triangle_not_boundary(head):
    from paper_1811_07717_amd import zi
    tr = head.tris.copy()
    # an interior face: three vertices of an interior tetrahedron
    inner = np.argmin((head.nodes[head.tets].mean(1) ** 2).sum(1))
    tr[0] = head.tets[inner][:3]
    assert status_of(head, tris=tr) == zi.ZI_EMESH
    tr = head.tris.copy()
    tr[0] = [0, head.n - 1, head.n // 2]        # not even a mesh face
    assert status_of(head, tris=tr) == zi.ZI_EMESH


def test_electrode_index_and_empty_electrode(head):
    from paper_1811_07717_amd import zi
    te = head.tri_electrode.copy()
    te[0] = head.L
    assert status_of(head, te=te) == zi.ZI_EMESH
    te = head.tri_electrode.copy()
    te[te == 3] = 2                              # electrode 3 loses its triangles
    assert status_of(head, te=te) == zi.ZI_EMESH


def test_contact_impedance(head):
    from paper_1811_07717_amd import zi
    Z = head.Z.copy()
    Z[1] = 0.0
    assert status_of(head, Z=Z) == zi.ZI_EMESH


def test_inadmissible_ground(head):
    from paper_1811_07717_amd import zi
    inner = int(np.argmin((head.nodes ** 2).sum(1)))
    assert status_of(head, ground=inner) == zi.ZI_EINVAL      # not on the boundary
    assert status_of(head, ground=int(head.tris[0, 0])) == zi.ZI_EINVAL   # on an electrode


def test_explicit_ground_accepted(head):
    g = build(head)
    gnd = g.ground
    g.close()
    g2 = build(head, ground=gnd)
    assert g2.ground == gnd
    g2.close()


def test_bad_dipole_and_source_matrix(head):
    from paper_1811_07717_amd import zi
    g = build(head)
    with pytest.raises(zi.ZiError) as e:
        g.point_dipoles(torch.tensor([0, head.e], dtype=torch.int32, device="cuda"))
    assert e.value.status == zi.ZI_EINVAL
    T, _ = g.transfer_solve(tol=1e-8)
    cp = torch.tensor([0, 2], dtype=torch.int32, device="cuda")
    ri = torch.tensor([0, head.n], dtype=torch.int32, device="cuda")
    gv = torch.ones(2, dtype=torch.float64, device="cuda")
    with pytest.raises(zi.ZiError) as e:
        g.leadfield(T, (cp, ri, gv))
    assert e.value.status == zi.ZI_EINVAL
    g.close()


def test_single_electrode_leadfield_is_zero():
    from paper_1811_07717_amd import zi
    H = hm.make_head(8.0, L=1, m=4, seed=2)
    g = zi.System.from_head(H)
    T, _ = g.transfer_solve(tol=1e-8)
    LF = g.leadfield(T, g.point_dipoles(torch.from_numpy(H.dipole_tets).cuda()))
    assert torch.all(LF == 0)
    g.close()


def test_pcg_form_options(head):
    from paper_1811_07717_amd import zi
    g = build(head)
    _, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir", form="single",
                             raise_on_error=False)
    assert st["status"] == zi.ZI_EINVAL
    zi.PCG_FORM["bogus"] = 7
    try:
        _, st = g.transfer_solve(tol=1e-8, form="bogus", raise_on_error=False)
        assert st["status"] == zi.ZI_EINVAL
    finally:
        del zi.PCG_FORM["bogus"]
    _, st = g.transfer_solve(tol=1e-8, precision="fp32_spmm_ir", form="classic")
    assert st["status"] == zi.ZI_OK
    g.close()


def test_empty_source_matrix_and_no_dipoles(head):
    # Degenerate sizes: a source matrix with no columns gives an L x 0 lead
    # field, and zero dipoles give the column pointer [0].
    g = build(head)
    T, _ = g.transfer_solve(tol=1e-8)
    cp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ri = torch.empty(0, dtype=torch.int32, device="cuda")
    gv = torch.empty(0, dtype=torch.float64, device="cuda")
    LF = g.leadfield(T, (cp, ri, gv))
    assert tuple(LF.shape) == (head.L, 0)
    cp0, ri0, gv0 = g.point_dipoles(torch.empty(0, dtype=torch.int32, device="cuda"))
    assert cp0.tolist() == [0] and ri0.numel() == 0 and gv0.numel() == 0
    g.close()
