"""Pins of the warm-start network's CPU reference: GELU against values of
the normal distribution function, the backward pass and the loss gradient
against central finite differences (float64, no rounding), Adam's first
steps against their closed form, the rank-4 head and the features on cases
worked by hand."""
import numpy as np

from oracle import mlp_oracle as M
from paper_2106_03508_amd import synthetic as syn


def test_gelu_values():
    # Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    z = np.array([0.0, 1.0, -1.0, 2.0, 10.0, -10.0])
    g = M.gelu(z)
    assert g[0] == 0.0
    assert abs(g[1] - 0.8413447460685429) < 1e-15
    assert abs(g[2] + 0.15865525393145707) < 1e-15
    assert abs(g[3] - 2.0 * 0.9772498680518208) < 1e-15
    assert abs(g[4] - 10.0) < 1e-15 and abs(g[5]) < 1e-15
    # derivative: 1/2 at zero, finite differences elsewhere
    assert abs(M.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    zz = np.linspace(-4, 4, 41)
    fd = (M.gelu(zz + 1e-6) - M.gelu(zz - 1e-6)) / 2e-6
    assert np.max(np.abs(fd - M.gelu_grad(zz))) < 1e-8


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = syn.mlp_init(7, out_scale=1.0).astype(np.float64)
    X = rng.standard_normal((7, M.NF))
    dY = rng.standard_normal((7, M.NO))
    Y, cache = M.forward(theta, X, fp16=False)
    g = M.backward(theta, cache, dY)
    assert g.shape == (M.NPARAM,)
    # sample parameters of every block
    offs, k = [], 0
    for _, shape in M.LAYOUT:
        n = int(np.prod(shape))
        offs += list(k + rng.choice(n, size=8, replace=False))
        k += n
    h = 1e-6
    for i in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fp = np.sum(M.forward(tp, X, fp16=False)[0] * dY)
        fm = np.sum(M.forward(tm, X, fp16=False)[0] * dY)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_loss_grad_matches_finite_differences():
    rng = np.random.default_rng(2)
    N = 6
    Y = rng.standard_normal((N, M.NO)) * 0.3
    a = rng.standard_normal((4, N, N))
    m0 = a + a.transpose(0, 2, 1)
    b = rng.standard_normal((4, N, N))
    mconv = m0 + 0.1 * (b + b.transpose(0, 2, 1))
    s = np.array([0.5, 2.0, 1.0, 3.0])
    loss, dY = M.loss_grad(Y, m0, mconv, s)
    T = (mconv - m0) / s[:, None, None]
    assert abs(loss - np.sum((M.head(Y, m0, s) - T) ** 2) / N) < 1e-12
    h = 1e-6
    for i in range(N):
        for j in range(M.NO):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, j] += h
            Ym[i, j] -= h
            fd = (M.loss_grad(Yp, m0, mconv, s)[0] - M.loss_grad(Ym, m0, mconv, s)[0]) / (2 * h)
            assert abs(fd - dY[i, j]) < 1e-7 * max(1.0, abs(dY[i, j]))


def test_adam_closed_form():
    g = np.array([0.3, -2.0, 1e-3, -5e-2])
    theta = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 0.01
    # with a constant gradient every bias-corrected step is -lr g / (|g| + eps)
    t1, m, v = M.adam(theta, m, v, g, 1, lr, eps=0.0)
    assert np.allclose(t1, theta - lr * np.sign(g), rtol=0, atol=1e-15)
    t2, m, v = M.adam(t1, m, v, g, 2, lr, eps=0.0)
    assert np.allclose(t2, theta - 2 * lr * np.sign(g), rtol=0, atol=1e-14)
    # a zero gradient leaves a parameter in place at the first step (eps > 0)
    t3, _, _ = M.adam(theta, np.zeros(4), np.zeros(4), np.zeros(4), 1, lr)
    assert np.array_equal(t3, theta)


def test_head_structure():
    N = 5
    rng = np.random.default_rng(9)
    a = rng.standard_normal((4, N, N))
    m0 = a + a.transpose(0, 2, 1)
    s = np.array([1.0, 2.0, 4.0, 0.5])
    Y = np.zeros((N, M.NO))
    r = np.arange(1.0, N + 1)
    Y[:, 0] = r
    P = M.head(Y, m0, s)
    assert np.array_equal(P[0], np.diag(r)) and not P[1:].any()
    w = np.array([1.0, -2.0, 0.5, 0.0, 3.0])
    for m in range(4):
        Y = np.zeros((N, M.NO))
        Y[:, 5 * 2 + 1 + m] = w           # moment 2, scaling of iteration-0 moment m
        P = M.head(Y, m0, s)
        assert np.allclose(P[2], (w[:, None] + w[None, :]) * m0[m] / s[m], rtol=0, atol=1e-15)
        assert not P[[0, 1, 3]].any()
    # a constant coefficient c on moment n itself rescales it by (1 + 2c)
    Y = np.zeros((N, M.NO))
    Y[:, 5 * 1 + 1 + 1] = 0.25
    assert np.allclose(s[1] * M.head(Y, m0, s)[1], 0.5 * m0[1], rtol=0, atol=1e-14)


def test_features_hand_case():
    e = np.array([-1.0, 0.5, 2.0])
    m0 = np.zeros((4, 3, 3))
    for n in range(4):
        m0[n] = np.diag([1.0, -2.0, 3.0]) * (n + 1) + 0.25   # off-diagonals do not enter
    X, s = M.features(e, 1, m0)
    # mu0 = -0.25, gap = 1.5; mean |diag| of diag(1, -2, 3)(n+1) + 0.25:
    # (1.25 + 1.75 + 3.25) / 3 = 6.25 / 3 for n = 0
    assert np.allclose(X[:, 0], e) and np.allclose(X[:, 1], [-0.75, 0.75, 2.25])
    assert np.allclose(X[:, 2], 1.5) and np.allclose(X[:, 3], [1, -1, -1])
    assert abs(s[0] - 6.25 / 3) < 1e-15
    assert np.allclose(X[:, 4], np.array([1.25, -1.75, 3.25]) / (6.25 / 3))
    # moment n is (n + 1) diag(1, -2, 3) + 0.25: mean |diag| = (1.25 + 1.75 + 3.25) / 3
    # for n = 0, (2.25 + 3.75 + 6.25) / 3 for n = 1, (3.25 + 5.75 + 9.25) / 3,
    # (4.25 + 7.75 + 12.25) / 3
    assert abs(s[1] - 12.25 / 3) < 1e-15 and abs(s[3] - 24.25 / 3) < 1e-15
    assert np.allclose(X[:, 8], np.log(12.25 / 6.25))
    assert np.allclose(X[:, 9], np.log(18.25 / 6.25))
    assert np.allclose(X[:, 10], np.log(24.25 / 18.25))
    assert np.allclose(X[:, 11], np.array([-0.75, 0.75, 2.25]) / 1.5)


def test_zero_last_layer_gives_zero_correction():
    theta = syn.mlp_init(3).astype(np.float64)
    p = M.unpack(theta)
    p["W3"][:] = 0.0
    p["b3"][:] = 0.0
    e = syn.orbital_energies(3, 10, 2)
    m0 = np.stack([np.eye(10) * (k + 1) for k in range(4)])
    dm = M.predict_correction(theta, e, 2, m0)
    assert dm.shape == (4, 10, 10) and not dm.any()
