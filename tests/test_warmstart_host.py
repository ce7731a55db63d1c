"""Host logic of the learned warm start (no GPU): the padded node-to-tet
incidence table and the per-node mean it serves."""
import numpy as np
import pytest

from paper_1811_07717_amd import headmodel as hm
from paper_1811_07717_amd.warmstart import _incidence, _node_mean

torch = pytest.importorskip("torch")


def test_incidence_lists_every_tet_of_every_node_in_order():
    H = hm.make_head(8.0, L=8, m=1, seed=3)
    inc, cnt = _incidence(H)
    assert inc.shape == (H.n, cnt.max())
    for v in (0, H.n // 2, H.n - 1):
        want = np.nonzero((H.tets == v).any(axis=1))[0]
        np.testing.assert_array_equal(inc[v, :cnt[v]], want)
        assert (inc[v, cnt[v]:] == -1).all()
    assert np.array_equal(np.sort(inc[inc >= 0]), np.repeat(np.arange(H.e), 4))


def test_padded_mean_matches_bincount_mean():
    H = hm.make_head(8.0, L=8, m=1, seed=3)
    vals = hm.perturbed_sigma(H, seed=5)
    inc, cnt = _incidence(H)
    d = torch.from_numpy(np.log(vals) - np.log(H.sigma))
    it = torch.from_numpy(inc)
    g = torch.where(it >= 0, d[it.clamp(min=0)], torch.zeros((), dtype=d.dtype))
    got = (g.sum(dim=1) / torch.from_numpy(cnt.astype(np.float64))).numpy()
    ref = _node_mean(H, np.log(vals) - np.log(H.sigma))
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()
