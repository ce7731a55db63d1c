"""Pins of the warm-start network's oracle: gradients against central
finite differences, the symmetric aggregation, and a decreasing loss."""
import numpy as np

from oracle import gnn
from paper_1811_07717_amd import headmodel as hm


def _graph():
    import scipy.sparse as sp
    H = hm.make_head(8.0, L=4, m=1, seed=3)
    t = H.tets.astype(np.int64)
    A = sp.coo_matrix((np.ones(16 * H.e), (np.repeat(t, 4, 1).ravel(),
                                           np.tile(t, (1, 4)).ravel())),
                      shape=(H.n, H.n)).tocsr()
    A.sort_indices()
    return gnn.normalized_adjacency(A.indptr, A.indices, H.n), H


def test_aggregation_is_symmetric_and_normalised():
    Ah, H = _graph()
    assert abs(Ah - Ah.T).max() == 0.0
    assert Ah.diagonal().max() == 0.0
    # Ahat D^1/2 1 = D^1/2 1: the D^1/2-weighted constant is a fixed vector
    deg = np.diff(Ah.indptr).astype(float)
    np.testing.assert_allclose(Ah @ np.sqrt(deg), np.sqrt(deg), rtol=1e-12)


def test_gradients_match_finite_differences():
    Ah, H = _graph()
    rng = np.random.default_rng(0)
    n = H.n
    X = rng.normal(size=(n, 5))
    t = rng.normal(size=n)
    params = gnn.init_params([5, 8, 8, 1], seed=1)
    y, cache = gnn.forward(params, Ah, X)
    grads = gnn.backward(params, Ah, cache, y, t)
    for k in range(3):
        for name in ("Ws", "Wn", "b"):
            P = params[k][name]
            G = grads[k][name]
            for idx in [tuple(rng.integers(0, s) for s in P.shape) for _ in range(4)]:
                old = P[idx]
                h = 1e-6 * max(1.0, abs(old))
                P[idx] = old + h
                lp = gnn.loss(gnn.forward(params, Ah, X)[0], t)
                P[idx] = old - h
                lm = gnn.loss(gnn.forward(params, Ah, X)[0], t)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
                # ReLU kinks crossed by the +-h probe limit the agreement to ~1e-5
                assert abs(fd - G[idx]) <= 1e-4 * max(1e-3, abs(fd)), (k, name, idx, fd, G[idx])


def test_adam_training_reduces_loss():
    Ah, H = _graph()
    rng = np.random.default_rng(2)
    X = np.concatenate([H.nodes / 0.092, rng.normal(size=(H.n, 1))], axis=1)
    t = np.sin(4 * H.nodes[:, 0] / 0.092) + X[:, 3] * 0.1
    params = gnn.init_params([4, 16, 16, 1], seed=3)
    state = {}
    l0 = gnn.loss(gnn.forward(params, Ah, X)[0], t)
    for _ in range(60):
        y, cache = gnn.forward(params, Ah, X)
        gnn.adam_step(params, gnn.backward(params, Ah, cache, y, t), state, lr=1e-2)
    l1 = gnn.loss(gnn.forward(params, Ah, X)[0], t)
    assert l1 < 0.5 * l0
