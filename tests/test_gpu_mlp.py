"""Warm-start network on the GPU against its CPU reference (oracle/mlp_oracle):
features, the FP16-MFMA forward pass, the loss head, the backward pass,
three full training steps (forward, loss, backward, Adam), the predicted
moment correction, and a short training run that must reduce the loss.

Tolerances. The reference rounds the same operands to half precision but
accumulates in float64 and evaluates GELU in float64; the GPU accumulates in
float32. Pre-activations therefore agree to ~1e-6 relative, and an activation
whose float32 and float64 values straddle a half-precision rounding boundary
differs by one half-precision unit (2^-11 relative) in a small fraction of
entries. Outputs and gradients are compared to 2e-3 of their largest entry
(element-wise) and 5e-4 relative Frobenius; quantities computed from float32
inputs in float64 (features, the loss and its gradient) to 1e-6 relative."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def sym(rng, n, N):
    a = rng.standard_normal((n, N, N))
    return a + a.transpose(0, 2, 1)


def close_outputs(got, ref, label):
    scale = np.abs(ref).max()
    amax = np.abs(got - ref).max()
    frob = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"{label}: max abs diff {amax:.2e} (max |ref| {scale:.2e}), rel Frobenius {frob:.2e}",
          flush=True)
    assert amax <= 2e-3 * scale
    assert frob <= 5e-4


def test_features_match_oracle(h):
    from paper_2106_03508_amd import agf2
    rng = np.random.default_rng(3)
    N, nocc = 70, 13
    e = syn.orbital_energies(3, N, nocc)
    m0 = sym(rng, 4, N) + 5.0 * np.eye(N)
    m0[1] *= -1.0
    X, s = agf2.agf2_mlp_features(h, dev(e), nocc, dev(m0))
    Xr, sr = M.features(e, nocc, m0)
    assert np.allclose(s.cpu().numpy(), sr, rtol=1e-14, atol=0)
    np.testing.assert_allclose(X.cpu().numpy(), Xr, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("rows", [1, 64, 150])
def test_forward_matches_oracle(h, rows):
    from paper_2106_03508_amd import agf2
    theta = syn.mlp_init(11, out_scale=1.0)
    rng = np.random.default_rng(rows)
    X = rng.standard_normal((rows, M.NF)).astype(np.float32)
    net = agf2.Mlp(h, theta)
    Y = agf2.agf2_mlp_forward(h, net, dev(X, torch.float32)).cpu().numpy()
    Yr, _ = M.forward(theta.astype(np.float64), X.astype(np.float64), fp16=True)
    close_outputs(Y, Yr, f"forward rows={rows}")
    net.close()


def test_loss_grad_matches_oracle(h):
    from paper_2106_03508_amd import agf2
    rng = np.random.default_rng(5)
    N = 37
    Y = (0.3 * rng.standard_normal((N, M.NO))).astype(np.float32)
    m0 = sym(rng, 4, N)
    mconv = m0 + 0.1 * sym(rng, 4, N)
    s = np.array([0.5, 2.0, 1.0, 3.0])
    dY, loss = agf2.agf2_mlp_loss_grad(h, dev(Y, torch.float32), dev(m0), dev(mconv), dev(s))
    lr, dYr = M.loss_grad(Y.astype(np.float64), m0, mconv, s)
    assert abs(loss.item() - lr) <= 1e-12 * abs(lr)
    np.testing.assert_allclose(dY.cpu().numpy(), dYr, rtol=1e-6, atol=1e-7 * np.abs(dYr).max())
    # the loss accumulates over calls
    agf2.agf2_mlp_loss_grad(h, dev(Y, torch.float32), dev(m0), dev(mconv), dev(s), loss=loss)
    assert abs(loss.item() - 2 * lr) <= 1e-12 * abs(lr)


def test_backward_matches_oracle(h):
    from paper_2106_03508_amd import agf2
    theta = syn.mlp_init(12, out_scale=1.0)
    rng = np.random.default_rng(6)
    rows = 700     # splits the weight-gradient reductions
    X = rng.standard_normal((rows, M.NF)).astype(np.float32)
    dY = rng.standard_normal((rows, M.NO)).astype(np.float32)
    net = agf2.Mlp(h, theta)
    agf2.agf2_mlp_forward(h, net, dev(X, torch.float32))
    agf2.agf2_mlp_backward(h, net, dev(dY, torch.float32))
    g = net.get_grad().astype(np.float64)
    _, cache = M.forward(theta.astype(np.float64), X.astype(np.float64), fp16=True)
    gr = M.backward(theta.astype(np.float64), cache, dY.astype(np.float64))
    gp, grp = M.unpack(g), M.unpack(gr)
    for name, _ in M.LAYOUT:
        close_outputs(gp[name], grp[name], f"grad {name}")
    net.close()


def test_training_steps_match_oracle(h):
    """Three steps of forward, loss, backward and Adam on two systems stacked
    (eps = 0.1 keeps the Adam update a smooth function of the gradient, so the
    two sides' small gradient differences cannot flip an update's sign; the
    step size keeps the loss decreasing, since a diverging run would amplify
    rounding differences without bound)."""
    from paper_2106_03508_amd import agf2
    rng = np.random.default_rng(7)
    theta = syn.mlp_init(13)
    systems = []
    for N, nocc in [(30, 6), (45, 9)]:
        e = syn.orbital_energies(N, N, nocc)
        m0 = sym(rng, 4, N) + 4.0 * np.eye(N)
        mconv = m0 + 0.2 * sym(rng, 4, N)
        systems.append((e, nocc, m0, mconv))
    lr, b1, b2, eps = 1e-4, 0.9, 0.999, 0.1
    # GPU
    net = agf2.Mlp(h, theta)
    feats = [agf2.agf2_mlp_features(h, dev(e), nocc, dev(m0)) for e, nocc, m0, _ in systems]
    X = torch.cat([f[0] for f in feats]).contiguous()
    losses = []
    for _ in range(3):
        Y = agf2.agf2_mlp_forward(h, net, X)
        dY = torch.empty_like(Y)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        r0 = 0
        for (e, nocc, m0, mconv), (_, s) in zip(systems, feats):
            N = e.shape[0]
            agf2.agf2_mlp_loss_grad(h, Y[r0:r0 + N], dev(m0), dev(mconv), s, dY[r0:r0 + N], loss)
            r0 += N
        losses.append(loss.item())
        agf2.agf2_mlp_backward(h, net, dY)
        agf2.agf2_mlp_adam_step(h, net, lr, b1, b2, eps)
    assert losses[2] < losses[1] < losses[0]
    got = net.get_params().astype(np.float64)
    net.close()
    # reference
    t = theta.astype(np.float64)
    m = np.zeros_like(t)
    v = np.zeros_like(t)
    Xr = np.concatenate([M.features(e, nocc, m0)[0] for e, nocc, m0, _ in systems])
    Xr = Xr.astype(np.float32).astype(np.float64)   # the GPU features are float32
    for step in range(1, 4):
        Yr, cache = M.forward(t, Xr, fp16=True)
        dYr = np.zeros_like(Yr)
        r0 = 0
        for e, nocc, m0, mconv in systems:
            N = e.shape[0]
            _, s = M.features(e, nocc, m0)
            dYr[r0:r0 + N] = M.loss_grad(Yr[r0:r0 + N], m0, mconv, s)[1]
            r0 += N
        g = M.backward(t, cache, dYr)
        t, m, v = M.adam(t, m, v, g, step, lr, b1, b2, eps)
    diff = np.abs(got - t).max()
    print(f"params after 3 steps: max abs diff {diff:.2e} (lr {lr})", flush=True)
    assert diff <= 0.01 * lr


def test_predict_correction_matches_oracle(h):
    from paper_2106_03508_amd import agf2
    from oracle import agf2_oracle as O
    N, nocc, naux = 24, 5, 80
    L = syn.df_tensor(0, N, naux, nocc)
    e = syn.orbital_energies(0, N, nocc)
    m0 = np.stack(O.se_moments(L, e, np.eye(N), nocc))
    theta = syn.mlp_init(14, out_scale=1.0)
    net = agf2.Mlp(h, theta)
    dm = agf2.agf2_mlp_predict_correction(h, net, dev(e), nocc, dev(m0)).cpu().numpy()
    net.close()
    ref = M.predict_correction(theta.astype(np.float64), e, nocc, m0, fp16=True)
    assert np.array_equal(dm, dm.transpose(0, 2, 1))
    for n in range(4):
        close_outputs(dm[n], ref[n], f"correction {n}")


def test_short_training_reduces_loss(h):
    from paper_2106_03508_amd import agf2
    rng = np.random.default_rng(8)
    systems = []
    for N, nocc in [(40, 8), (50, 10), (60, 12)]:
        e = syn.orbital_energies(N + 1, N, nocc)
        m0 = sym(rng, 4, N) * 0.05 + np.diag(1.0 + np.abs(e))[None]
        mconv = m0 + np.diag(0.1 * (1.0 + np.abs(e)) + 0.05 * e)[None]   # learnable
        systems.append((dev(e), nocc, dev(m0), dev(mconv)))
    net = agf2.Mlp(h, syn.mlp_init(15))
    feats = [agf2.agf2_mlp_features(h, e, nocc, m0) for e, nocc, m0, _ in systems]
    X = torch.cat([f[0] for f in feats]).contiguous()
    losses = []
    for _ in range(150):
        Y = agf2.agf2_mlp_forward(h, net, X)
        dY = torch.empty_like(Y)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        r0 = 0
        for (e, nocc, m0, mconv), (_, s) in zip(systems, feats):
            N = e.shape[0]
            agf2.agf2_mlp_loss_grad(h, Y[r0:r0 + N], m0, mconv, s, dY[r0:r0 + N], loss)
            r0 += N
        losses.append(loss.item())
        agf2.agf2_mlp_backward(h, net, dY)
        agf2.agf2_mlp_adam_step(h, net, 1e-3)
    net.close()
    print(f"loss {losses[0]:.4e} -> {losses[-1]:.4e}", flush=True)
    assert losses[-1] < 0.1 * losses[0]


def test_mlp_argument_errors(h):
    from paper_2106_03508_amd import agf2
    net = agf2.Mlp(h)
    with pytest.raises(agf2.Agf2Error, match="AGF2_ERR_ARG"):
        agf2.agf2_mlp_backward(h, net, torch.zeros(5, 20, dtype=torch.float32, device="cuda"))
    with pytest.raises(agf2.Agf2Error, match="AGF2_ERR_ARG"):
        agf2.agf2_mlp_features(h, dev(np.arange(4.0)), 4, dev(np.zeros((4, 4, 4))))
    with pytest.raises(agf2.Agf2Error, match="AGF2_ERR_ARG"):
        agf2.agf2_mlp_adam_step(h, net, 0.0)
    net.close()
