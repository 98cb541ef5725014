"""GPU parity of the broadened spectral function against the oracle, on the
poles of a converged small system and at the pole count of the nmo=1000
iteration >= 1 shape (3N poles), with and without a projection weight."""
import time

import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu

ETA = 0.2 / 27.211386   # 0.2 eV


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def close(got, ref):
    return np.abs(got - ref).max() / np.abs(ref).max()


def test_spectrum_of_converged_poles_matches_oracle(h):
    from paper_2106_03508_amd import agf2
    nmo, nocc, naux = 24, 5, 80
    eps = syn.orbital_energies(0, nmo, nocc)
    L = syn.df_tensor(0, nmo, naux, nocc)
    hc = O.synthetic_hcore(eps, L, nocc)
    m = O.se_moments(L, eps, np.eye(nmo), nocc)
    eo, vo = O.compress(m[0], m[1])
    ev, vv = O.compress(m[2], m[3])
    fl = O.fock_loop(hc, L, 2 * nocc, np.concatenate([eo, ev]), np.hstack([vo, vv]),
                     O.reference_density(nmo, nocc))
    lam, u = fl["e_pole"], fl["u_pole"]           # 72 poles: one partial LDS block
    omega = np.linspace(lam.min() - 0.5, lam.max() + 0.5, 1000)   # ragged last block
    weight = np.linspace(0.0, 2.0, nmo)
    for wt in (None, weight):
        ref = O.spectral_function(lam, u, omega, ETA, wt)
        got = agf2.agf2_spectral_function(h, dev(lam), dev(u), dev(omega), ETA,
                                          None if wt is None else dev(wt)).cpu().numpy()
        print("converged poles", "total" if wt is None else "projected",
              f"{close(got, ref):.2e}", flush=True)
        assert close(got, ref) < 1e-12


def test_spectrum_at_the_nmo1000_pole_count(h):
    from paper_2106_03508_amd import agf2
    nmo, npole = 1000, 3000
    lam, u = syn.random_poles(3, nmo, npole, nmo + 76)
    omega = np.linspace(lam.min() - 0.2, lam.max() + 0.2, 4000)
    ref = O.spectral_function(lam, u, omega, ETA)
    el, ul, om = dev(lam), dev(u), dev(omega)
    out = agf2.agf2_spectral_function(h, el, ul, om, ETA)
    assert close(out.cpu().numpy(), ref) < 1e-12
    torch.cuda.synchronize()
    agf2.agf2_profile_enable(h, True)
    t = time.perf_counter()
    for _ in range(20):
        agf2.agf2_spectral_function(h, el, ul, om, ETA, out=out)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / 20 * 1e3
    rec = agf2.agf2_profile_read(h)["spectrum"]
    agf2.agf2_profile_enable(h, False)
    print(f"spectrum: {npole} poles x {omega.size} frequencies, {wall:.3f} ms per call, "
          f"{rec['ms'] / rec['launches']:.3f} ms on the device", flush=True)


def test_spectrum_single_pole_and_edge_arguments(h):
    from paper_2106_03508_amd import agf2
    lam, u = np.array([0.25]), np.array([[0.6]])
    omega = np.linspace(-1.0, 1.5, 11)
    got = agf2.agf2_spectral_function(h, dev(lam), dev(u), dev(omega), 0.05).cpu().numpy()
    assert close(got, O.spectral_function(lam, u, omega, 0.05)) < 1e-14
    empty = agf2.agf2_spectral_function(h, dev(lam), dev(u), dev(np.zeros(0)), 0.05)
    assert empty.numel() == 0
    for eta in (0.0, -1.0, float("nan")):
        with pytest.raises(agf2.Agf2Error) as ei:
            agf2.agf2_spectral_function(h, dev(lam), dev(u), dev(omega), eta)
        assert ei.value.status == -1
