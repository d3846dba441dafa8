"""Pins of the fp64 MLP reference: the chain-rule gradient against central
finite differences, closed forms of the forward pass and of Adam's first step,
and the mask's effect on loss and gradient."""
import numpy as np

from oracle import mlp


def rand_problem(seed, batch=12):
    rng = np.random.default_rng(seed)
    flat = rng.normal(0, 0.3, mlp.N_PARAMS)
    X = rng.normal(0, 1, (batch, mlp.N_IN))
    T = rng.normal(0, 1, (batch, mlp.N_OUT))
    M = (rng.random((batch, mlp.N_OUT)) < 0.7).astype(np.float64)
    return flat, X, T, M


def test_param_count():
    assert mlp.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 64 * 16 + 16 == 6288


def test_gradient_matches_central_differences():
    flat, X, T, M = rand_problem(1)
    g = mlp.gradient(flat, X, T, M)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, 300, replace=False)
    h = 1e-6
    fd = np.empty(len(idx))
    for t, i in enumerate(idx):
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd[t] = (mlp.loss(flat + e, X, T, M) - mlp.loss(flat - e, X, T, M)) / (2 * h)
    assert np.linalg.norm(fd - g[idx]) <= 1e-6 * max(1.0, np.linalg.norm(g[idx]))


def test_forward_closed_form_zero_hidden_weights():
    """With W3 = 0 the output is b3 for every row, whatever the input."""
    parts = mlp.unpack(np.random.default_rng(3).normal(size=mlp.N_PARAMS))
    parts["W3"][:] = 0
    flat = mlp.pack(parts)
    Y, _, _ = mlp.forward(flat, np.random.default_rng(4).normal(size=(5, 16)))
    assert np.array_equal(Y, np.tile(parts["b3"], (5, 1)))


def test_forward_closed_form_linear_region():
    """Positive weights and inputs keep every ReLU active: the net is the product
    of its affine maps."""
    rng = np.random.default_rng(5)
    parts = {k: np.abs(rng.normal(size=s)) for k, s in mlp.SHAPES}
    flat = mlp.pack(parts)
    X = np.abs(rng.normal(size=(3, 16)))
    Y, _, _ = mlp.forward(flat, X)
    W = parts["W1"] @ parts["W2"] @ parts["W3"]
    b = (parts["b1"] @ parts["W2"] + parts["b2"]) @ parts["W3"] + parts["b3"]
    assert np.allclose(Y, X @ W + b, rtol=1e-12)


def test_mask_removes_entries():
    flat, X, T, M = rand_problem(6)
    T2 = T.copy()
    T2[M == 0] += 100.0
    assert mlp.loss(flat, X, T, M) == mlp.loss(flat, X, T2, M)
    assert np.array_equal(mlp.gradient(flat, X, T, M), mlp.gradient(flat, X, T2, M))
    assert mlp.loss(flat, X, T, np.zeros_like(M)) == 0.0
    assert not mlp.gradient(flat, X, T, np.zeros_like(M)).any()


def test_loss_zero_at_target():
    flat, X, _, M = rand_problem(7)
    Y, _, _ = mlp.forward(flat, X)
    assert mlp.loss(flat, X, Y, M) == 0.0


def test_adam_first_step_closed_form():
    """At t = 1 the corrected moments are g and g^2: each parameter moves by
    -lr * g / (|g| + eps)."""
    rng = np.random.default_rng(8)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = mlp.adam_step(p, np.zeros(50), np.zeros(50), g, lr=0.01, t=1)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_planted_mistake_is_caught():
    """A gradient missing the ReLU mask on the first layer fails the
    finite-difference check."""
    flat, X, T, M = rand_problem(9)
    P = mlp.unpack(flat)
    Y, H1, H2 = mlp.forward(flat, X)
    dY = 2.0 * M * (Y - T) / M.sum()
    dZ2 = (dY @ P["W3"].T) * (H2 > 0)
    bad_W1 = X.T @ (dZ2 @ P["W2"].T)  # mask dropped
    good = mlp.unpack(mlp.gradient(flat, X, T, M))["W1"]
    assert not np.allclose(bad_W1, good, rtol=1e-3)
