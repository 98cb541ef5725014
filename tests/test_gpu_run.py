"""The full self-consistent AGF2 loop on the GPU (agf2_run) against the
oracle's run_agf2 on the same synthetic systems. Both stop when the energy
changes by less than 1e-8 Ha and IP/EA by less than 1e-7 Ha; the Fock loop
fits the electron count to 1e-10, so converged values agree to ~1e-8."""
import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def gpu_run(h, eps, L, nocc, **kw):
    from paper_2106_03508_amd import agf2
    N = eps.shape[0]
    Ld = dev(L)
    D0 = dev(O.reference_density(N, nocc))
    hc = agf2.agf2_fock_build(h, Ld, dev(np.diag(eps)), D0, -1.0)
    return agf2.agf2_run(h, Ld, hc, dev(eps), nocc, agf2.run_opts(**kw))


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


@pytest.mark.parametrize("diis", [8, 0])
def test_agf2_run_matches_oracle_small(h, diis):
    sysd = syn.system(0, **syn.SMALL)
    eps, L, nocc = sysd["eps"], sysd["L"], sysd["nocc"]
    ref = O.run_agf2(O.synthetic_hcore(eps, L, nocc), L, eps, nocc, diis_space=diis,
                     max_iter=40)
    got = gpu_run(h, eps, L, nocc, diis_space=diis, max_iter=40)
    assert ref["converged"] and got["converged"]
    r, g = ref["history"], got["history"]
    assert len(r) == len(g)
    for a, b in zip(r, g):
        assert a["nocc_pole"] == b["nocc_pole"]
        assert abs(a["etot"] - b["e_tot"]) < 1e-8
        assert abs(a["ip"] - b["ip"]) < 1e-8 and abs(a["ea"] - b["ea"]) < 1e-8
    print("iterations", len(g) - 1, "E", g[-1]["e_tot"], "IP", g[-1]["ip"], "EA", g[-1]["ea"])


def test_agf2_run_split_precision_small(h):
    """Reduced-precision moments: converged IP/EA within 1e-5 Ha and total
    energy within 1e-6 Ha of the FP64 oracle."""
    sysd = syn.system(0, **syn.SMALL)
    eps, L, nocc = sysd["eps"], sysd["L"], sysd["nocc"]
    ref = O.run_agf2(O.synthetic_hcore(eps, L, nocc), L, eps, nocc)["history"][-1]
    for prec in ("split_fp16", "split_bf16"):
        g = gpu_run(h, eps, L, nocc, prec=prec)["history"][-1]
        dip, dea, de = abs(g["ip"] - ref["ip"]), abs(g["ea"] - ref["ea"]), abs(g["e_tot"] - ref["etot"])
        print(prec, f"dIP {dip:.2e} dEA {dea:.2e} dE {de:.2e}")
        assert dip < 1e-5 and dea < 1e-5 and de < 1e-6


def test_agf2_run_warm_start_hook(h):
    """A zero correction leaves the trajectory unchanged; a correction that
    breaks positive definiteness falls back to the cold start."""
    from paper_2106_03508_amd import agf2
    sysd = syn.system(0, **syn.SMALL)
    eps, L, nocc = sysd["eps"], sysd["L"], sysd["nocc"]
    N = eps.shape[0]
    Ld = dev(L)
    hc = agf2.agf2_fock_build(h, Ld, dev(np.diag(eps)), dev(O.reference_density(N, nocc)), -1.0)
    cold = agf2.agf2_run(h, Ld, hc, dev(eps), nocc)
    zero = agf2.agf2_run(h, Ld, hc, dev(eps), nocc,
                         dm_init=torch.zeros(4, N, N, dtype=torch.float64, device="cuda"))
    assert zero["history"][0]["warm"] == 1
    assert abs(zero["history"][-1]["e_tot"] - cold["history"][-1]["e_tot"]) < 1e-12
    bad = torch.zeros(4, N, N, dtype=torch.float64, device="cuda")
    bad[0] = -1e3 * torch.eye(N, dtype=torch.float64, device="cuda")
    fb = agf2.agf2_run(h, Ld, hc, dev(eps), nocc, dm_init=bad)
    assert fb["history"][0]["warm"] == 0
    assert abs(fb["history"][-1]["e_tot"] - cold["history"][-1]["e_tot"]) < 1e-12
