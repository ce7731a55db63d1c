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


def test_multi_hop_gradients_and_power():
    # Layers aggregating over several hops: the aggregation equals the dense
    # matrix power, and the gradients match central finite differences.
    Ah, H = _graph()
    rng = np.random.default_rng(4)
    n = H.n
    Hm = rng.normal(size=(n, 3))
    dense = np.linalg.matrix_power(Ah.toarray(), 5)
    np.testing.assert_allclose(gnn.aggregate(Ah, Hm, 5), dense @ Hm, rtol=1e-10, atol=1e-12)
    hops = [1, 4, 2]
    X = rng.normal(size=(n, 5))
    t = rng.normal(size=n)
    params = gnn.init_params([5, 8, 8, 1], seed=6)
    y, cache = gnn.forward(params, Ah, X, hops)
    grads = gnn.backward(params, Ah, cache, y, t, hops)
    # a dropped hop in the backward pass would change these
    y1, c1 = gnn.forward(params, Ah, X)
    assert np.abs(y1 - y).max() > 1e-3
    for k in range(3):
        for name in ("Ws", "Wn", "b"):
            P = params[k][name]
            G = grads[k][name]
            for idx in [tuple(rng.integers(0, s) for s in P.shape) for _ in range(4)]:
                old = P[idx]
                h = 1e-6 * max(1.0, abs(old))
                P[idx] = old + h
                lp = gnn.loss(gnn.forward(params, Ah, X, hops)[0], t)
                P[idx] = old - h
                lm = gnn.loss(gnn.forward(params, Ah, X, hops)[0], t)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
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


def _adam_params(shape_seed=5):
    rng = np.random.default_rng(shape_seed)
    return [dict(Ws=rng.normal(size=(3, 4)), Wn=rng.normal(size=(3, 4)), b=rng.normal(size=4))]


def _grads_like(params, rng, scale):
    # magnitudes spread over many decades, down to the size of eps, both signs
    out = []
    for p in params:
        g = {}
        for name, a in p.items():
            mag = 10.0 ** rng.uniform(-9, 1, size=a.shape)
            g[name] = scale * mag * rng.choice([-1.0, 1.0], size=a.shape)
        out.append(g)
    return out


def test_adam_first_step_closed_form():
    """Kingma & Ba, Algorithm 1: from zero moments the bias-corrected
    moments of the first step are m_hat = g and v_hat = g^2, so every
    parameter moves by exactly -lr g / (|g| + eps), whatever beta1, beta2."""
    rng = np.random.default_rng(11)
    for b1, b2 in [(0.9, 0.999), (0.5, 0.75)]:
        params = _adam_params()
        p0 = [{k: v.copy() for k, v in p.items()} for p in params]
        g = _grads_like(params, rng, 1.0)
        lr, eps = 3e-3, 1e-8
        gnn.adam_step(params, g, {}, lr=lr, b1=b1, b2=b2, eps=eps)
        for p, q, gg in zip(params, p0, g):
            for name in p:
                want = q[name] - lr * gg[name] / (np.abs(gg[name]) + eps)
                np.testing.assert_allclose(p[name], want, rtol=1e-13, atol=1e-16)


def test_adam_two_steps_closed_form():
    """Two steps with gradients g1, g2 from zero moments: the moments are
    m2 = (1-b1)(b1 g1 + g2) and v2 = (1-b2)(b2 g1^2 + g2^2), and the bias
    corrections 1 - b^2 = (1-b)(1+b) leave m_hat = (b1 g1 + g2)/(1 + b1) and
    v_hat = (b2 g1^2 + g2^2)/(1 + b2).  Unequal betas and unequal gradients
    make a swapped pair of betas or a missing correction fail."""
    rng = np.random.default_rng(12)
    b1, b2, lr, eps = 0.9, 0.999, 1e-2, 1e-8
    params = _adam_params()
    p0 = [{k: v.copy() for k, v in p.items()} for p in params]
    g1 = _grads_like(params, rng, 1.0)
    g2 = _grads_like(params, rng, 1.0)
    state = {}
    gnn.adam_step(params, g1, state, lr=lr, b1=b1, b2=b2, eps=eps)
    gnn.adam_step(params, g2, state, lr=lr, b1=b1, b2=b2, eps=eps)
    assert state["t"] == 2
    for p, q, a, b in zip(params, p0, g1, g2):
        for name in p:
            mh = (b1 * a[name] + b[name]) / (1.0 + b1)
            vh = (b2 * a[name] ** 2 + b[name] ** 2) / (1.0 + b2)
            first = a[name] / (np.abs(a[name]) + eps)
            want = q[name] - lr * first - lr * mh / (np.sqrt(vh) + eps)
            np.testing.assert_allclose(p[name], want, rtol=1e-12, atol=1e-15)


def test_adam_constant_gradient_closed_form():
    """With the same gradient g at every step the bias-corrected moments stay
    m_hat = g and v_hat = g^2 for every t, so T steps move a parameter by
    exactly -T lr g / (|g| + eps)."""
    rng = np.random.default_rng(13)
    params = _adam_params()
    p0 = [{k: v.copy() for k, v in p.items()} for p in params]
    g = _grads_like(params, rng, 1.0)
    state = {}
    T, lr, eps = 25, 1e-3, 1e-8
    for _ in range(T):
        gnn.adam_step(params, g, state, lr=lr, eps=eps)
    for p, q, gg in zip(params, p0, g):
        for name in p:
            want = q[name] - T * lr * gg[name] / (np.abs(gg[name]) + eps)
            np.testing.assert_allclose(p[name], want, rtol=1e-11, atol=1e-14)
