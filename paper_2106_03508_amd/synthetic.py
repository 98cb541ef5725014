"""Seeded synthetic closed-shell systems for the AGF2 moment build.

This module holds random draws and nothing else: no part of the AGF2 method
(no Fock build, no moments, no compression) lives here. Both the GPU library's
callers and the CPU oracle take their inputs from these functions, so a bug in
the method cannot hide in shared code.

A system is (eps, L, nocc):

* eps  -- nmo orbital energies of the mean-field reference. The nocc occupied
          ones are uniform in [-1.5, -0.3] Ha, the virtual ones uniform in
          [0.1, 3.0] Ha, each sorted ascending.
* L    -- density-fitting tensor L[Q, p, q], symmetric in (p, q), such that the
          electron repulsion integrals are (pq|rs) = sum_Q L[Q,p,q] L[Q,r,s]
          (positive semidefinite by construction). Row Q is
          c * s_Q * unpack(b_Q) where b_Q has one N(0, 1/npair) entry per pair
          p <= q, s_Q = exp(-Q/20), and c = (nocc/5)**(1/4) keeps the
          second-order correlation energy roughly proportional to nocc.
* nocc -- doubly occupied orbitals; nelec = 2 * nocc.

Every Q row is drawn from its own PCG64 stream keyed by (seed, 1, Q), so any
slice of L can be regenerated on its own and the draw does not depend on how
the tensor is chunked.
"""
from __future__ import annotations

import numpy as np

EPS_OCC_RANGE = (-1.5, -0.3)
EPS_VIR_RANGE = (0.1, 3.0)
S_DECAY = 20.0


def orbital_energies(seed: int, nmo: int, nocc: int) -> np.ndarray:
    """Sorted occupied energies followed by sorted virtual energies (Ha)."""
    if not (0 < nocc < nmo):
        raise ValueError("need 0 < nocc < nmo")
    rng = np.random.Generator(np.random.PCG64([seed, 0]))
    eo = np.sort(rng.uniform(*EPS_OCC_RANGE, size=nocc))
    ev = np.sort(rng.uniform(*EPS_VIR_RANGE, size=nmo - nocc))
    return np.concatenate([eo, ev])


def df_scale(nocc: int) -> float:
    """Global amplitude c of the synthetic DF tensor."""
    return (nocc / 5.0) ** 0.25


def df_tensor(seed: int, nmo: int, naux: int, nocc: int, q0: int = 0,
              q1: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Rows q0..q1-1 of the synthetic DF tensor, float64 [q1-q0, nmo, nmo]."""
    q1 = naux if q1 is None else q1
    if not (0 <= q0 <= q1 <= naux):
        raise ValueError("bad Q range")
    npair = nmo * (nmo + 1) // 2
    iu = np.triu_indices(nmo)
    c = df_scale(nocc)
    if out is None:
        out = np.empty((q1 - q0, nmo, nmo), dtype=np.float64)
    m = np.empty((nmo, nmo), dtype=np.float64)
    for q in range(q0, q1):
        rng = np.random.Generator(np.random.PCG64([seed, 1, q]))
        b = rng.standard_normal(npair)
        b *= c * np.exp(-q / S_DECAY) / np.sqrt(npair)
        m[iu] = b
        m.T[iu] = b
        out[q - q0] = m
    return out


def system(seed: int, nmo: int, nocc: int, naux: int) -> dict:
    """Full synthetic system as a dict of float64 numpy arrays."""
    return {
        "seed": seed, "nmo": nmo, "nocc": nocc, "naux": naux,
        "eps": orbital_energies(seed, nmo, nocc),
        "L": df_tensor(seed, nmo, naux, nocc),
    }


def random_poles(seed: int, nmo: int, npole: int, nocc_pole: int):
    """A random Green's function pole set (energies ascending, amplitudes
    [nmo, npole]) for exercising the moment build away from the mean-field
    reference. Energies below zero for the first nocc_pole poles."""
    rng = np.random.Generator(np.random.PCG64([seed, 2]))
    eo = np.sort(rng.uniform(-2.0, -0.2, size=nocc_pole))
    ev = np.sort(rng.uniform(0.05, 4.0, size=npole - nocc_pole))
    u = rng.standard_normal((nmo, npole)) / np.sqrt(npole / nmo)
    return np.concatenate([eo, ev]), u


# Workload shapes (nmo, nocc, naux) of the synthetic systems used by tests
# and benchmarks.
SMALL = dict(nmo=24, nocc=5, naux=80)          # oracle runs to convergence in seconds
MEDIUM = dict(nmo=200, nocc=40, naux=700)      # double-zeta-molecule-like
LARGE = dict(nmo=1000, nocc=76, naux=3500)     # ~1000 orbitals, artemisinin-like nocc
EVAL400 = dict(nmo=400, nocc=80, naux=1400)    # warm-start evaluation size
# the orbital and correlated-electron counts of the paper's timed runs
# (aug-cc-pVDZ guanine and artemisinin); naux = 3.5 nmo assumed
GUANINE = dict(nmo=298, nocc=39, naux=1043)
ARTEMISININ = dict(nmo=658, nocc=76, naux=2303)


def batch_shapes(nsys: int = 64, seed0: int = 1000, nmo_lo: int = 40, nmo_hi: int = 160):
    """Shapes of a batch of systems of uneven size: a list of dicts with seed
    (seed0 + k), nmo uniform over the integers [nmo_lo, nmo_hi] (PCG64 keyed
    by (seed0, 3)), nocc = nmo / 5 rounded half up and naux = 3.5 nmo rounded
    half up."""
    rng = np.random.Generator(np.random.PCG64([seed0, 3]))
    nmo = rng.integers(nmo_lo, nmo_hi, endpoint=True, size=nsys)
    out = []
    for k, n in enumerate(nmo.tolist()):
        out.append(dict(seed=seed0 + k, nmo=n, nocc=max(1, int(np.floor(n / 5 + 0.5))),
                        naux=int(np.floor(3.5 * n + 0.5))))
    return out


BATCH64 = dict(nsys=64, seed0=1000, nmo_lo=40, nmo_hi=160)   # batched moment build


MLP_SHAPES = [(12, 256), (256,), (256, 256), (256,), (256, 20), (20,)]   # W1 b1 W2 b2 W3 b3


def mlp_init(seed: int, out_scale: float = 0.1) -> np.ndarray:
    """Initial parameters of the warm-start network, flat float32 in the
    order W1, b1, W2, b2, W3, b3 (weights [fan_in, fan_out], row-major):
    weights normal with variance 2 / fan_in (the last layer's scaled by
    out_scale so the first predictions are small), biases zero. PCG64 keyed
    by (seed, 4)."""
    rng = np.random.Generator(np.random.PCG64([seed, 4]))
    parts = []
    for k, shape in enumerate(MLP_SHAPES):
        if len(shape) == 1:
            parts.append(np.zeros(shape))
        else:
            w = rng.standard_normal(shape) * np.sqrt(2.0 / shape[0])
            parts.append(w * (out_scale if k == len(MLP_SHAPES) - 2 else 1.0))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
