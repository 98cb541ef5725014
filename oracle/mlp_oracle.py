"""CPU reference of the learned warm start: the per-orbital network, its
loss head, its gradients and the Adam update. TEST INFRASTRUCTURE ONLY: used
by tests/, the smoke check and the benchmark's CPU baseline, never by the
GPU library or its binding.

What it computes. The warm start corrects the iteration-0 self-energy
moments U_n (n = 0<, 1<, 0>, 1>; zeroth and first moments of the lesser and
greater parts) towards the converged ones before the first compression. A
small network sees each physical orbital x on its own and emits, for every
moment n, a diagonal entry r_n(x) and four scaling coefficients c_nm(x), one
per iteration-0 moment m, so that

    Delta U_n = s_n * P_n,
    P_n[x, y] = delta_xy r_n(x) + sum_m (c_nm(x) + c_nm(y)) U_m[x, y] / s_m,

i.e. a diagonal correction plus a symmetric per-orbital rescaling of the
four iteration-0 moments; s_n is the mean absolute diagonal of U_n (a scale
that makes outputs and targets dimensionless). Output column 5n holds r_n,
columns 5n+1 .. 5n+4 hold c_n0 .. c_n3. Per-orbital features:
    0  e_x                        orbital energy
    1  e_x - mu0                  mu0 = (e_HOMO + e_LUMO) / 2
    2  e_LUMO - e_HOMO            the gap (same for every orbital)
    3  +1 occupied, -1 virtual
    4..7   U_n[x, x] / s_n
    8  log(s_1 / s_0)   9  log(s_2 / s_0)   10  log(s_3 / s_2)
    11 (e_x - mu0) / gap
(no absolute scale of the moments enters, so the features do not drift with
the size of the system)
The network: three linear maps with GELU after the first two,
    Z1 = X W1 + b1, A1 = gelu(Z1), Z2 = A1 W2 + b2, A2 = gelu(Z2),
    Y = A2 W3 + b3,
with gelu(z) = z Phi(z) (Phi the standard normal distribution function).
With fp16=True the operands of the three products (X, A1, A2 and the
weights) are rounded to IEEE half precision first and everything else is
float64, mirroring a network with FP16 weights and FP32 accumulation.

Loss of one system (targets from a converged run):
    T_n = (U_n(converged) - U_n(iteration 0)) / s_n,
    loss = sum_n ||P_n - T_n||_F^2 / N.
Adam (Kingma and Ba) with bias-corrected first and second moments.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NF, NH, NO, NMOM = 12, 256, 20, 4
LAYOUT = [("W1", (NF, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NO)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in LAYOUT)


def unpack(theta):
    """Flat parameter vector -> dict of arrays (views)."""
    out, k = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = theta[k:k + n].reshape(shape)
        k += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in LAYOUT])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def _h(x, fp16):
    return x.astype(np.float16).astype(np.float64) if fp16 else np.asarray(x, dtype=np.float64)


def features(e_mf, nocc, m0):
    """Per-orbital features [N, 12] and moment scales s [4] from the
    mean-field energies and the iteration-0 moments m0 [4, N, N]."""
    e = np.asarray(e_mf, dtype=np.float64)
    N = e.shape[0]
    homo, lumo = e[nocc - 1], e[nocc]
    mu0, gap = 0.5 * (homo + lumo), lumo - homo
    s = np.array([max(np.mean(np.abs(np.diag(m0[n]))), 1e-30) for n in range(NMOM)])
    X = np.empty((N, NF))
    X[:, 0] = e
    X[:, 1] = e - mu0
    X[:, 2] = gap
    X[:, 3] = np.where(np.arange(N) < nocc, 1.0, -1.0)
    for n in range(NMOM):
        X[:, 4 + n] = np.diag(m0[n]) / s[n]
    X[:, 8] = np.log(s[1] / s[0])
    X[:, 9] = np.log(s[2] / s[0])
    X[:, 10] = np.log(s[3] / s[2])
    X[:, 11] = (e - mu0) / gap
    return X, s


def forward(theta, X, fp16=True):
    """Network outputs Y [rows, 20] and the activations the gradient needs."""
    p = unpack(theta)
    W1, W2, W3 = _h(p["W1"], fp16), _h(p["W2"], fp16), _h(p["W3"], fp16)
    X0 = _h(X, fp16)
    Z1 = X0 @ W1 + p["b1"]
    A1 = _h(gelu(Z1), fp16)
    Z2 = A1 @ W2 + p["b2"]
    A2 = _h(gelu(Z2), fp16)
    Y = A2 @ W3 + p["b3"]
    return Y, dict(X0=X0, Z1=Z1, A1=A1, Z2=Z2, A2=A2, W1=W1, W2=W2, W3=W3)


def head(Y, m0, s):
    """Normalised corrections P [4, N, N] from the outputs Y [N, 20], the
    iteration-0 moments m0 [4, N, N] and their scales s [4]."""
    N = Y.shape[0]
    Ut = np.asarray(m0) / s[:, None, None]
    P = np.empty((NMOM, N, N))
    for n in range(NMOM):
        P[n] = np.diag(Y[:, 5 * n])
        for m in range(NMOM):
            c = Y[:, 5 * n + 1 + m]
            P[n] += (c[:, None] + c[None, :]) * Ut[m]
    return P


def loss_grad(Y, m0, mconv, s):
    """Loss of one system and its gradient with respect to Y."""
    N = Y.shape[0]
    P = head(Y, m0, s)
    T = (np.asarray(mconv) - np.asarray(m0)) / s[:, None, None]
    Ut = np.asarray(m0) / s[:, None, None]
    R = P - T
    loss = float(np.sum(R * R)) / N
    dY = np.zeros_like(Y)
    for n in range(NMOM):
        dP = 2.0 * R[n] / N                       # symmetric
        dY[:, 5 * n] = np.diag(dP)
        for m in range(NMOM):
            dY[:, 5 * n + 1 + m] = 2.0 * np.sum(dP * Ut[m], axis=1)
    return loss, dY


def backward(theta, cache, dY):
    """Gradient of sum(Y * dY) with respect to the parameters (flat), the
    products' operands taken as rounded in the forward pass."""
    c = cache
    g = {}
    g["W3"] = c["A2"].T @ dY
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ c["W3"].T) * gelu_grad(c["Z2"])
    g["W2"] = c["A1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ c["W2"].T) * gelu_grad(c["Z1"])
    g["W1"] = c["X0"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def adam(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1). Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict_correction(theta, e_mf, nocc, m0, fp16=True):
    """Delta U [4, N, N] to add to the iteration-0 moments."""
    X, s = features(e_mf, nocc, m0)
    Y, _ = forward(theta, X, fp16)
    return head(Y, m0, s) * s[:, None, None]
