"""Higher-moment compression on the GPU against the oracle: moments
0 .. nmom-1 of both parts (FP64, 1e-10 relative Frobenius per moment), the
block-Lanczos compression to nmom/2 blocks (moments conserved, the same
compressed self-energy as the oracle's), and AGF2 with two Lanczos blocks
to self-consistency (converged results, tolerances as for one block)."""
import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# mean-field poles; ragged tiles with dressed poles; several slab chunks
CASES = [
    ("hf_small", 24, 80, ("hf", 5), 6),
    ("dressed_ragged", 70, 90, ("dressed", 210, 81), 4),
    ("dressed_tiles", 130, 100, ("dressed", 150, 40), 6),
    ("single_occ", 20, 33, ("hf", 1), 4),
]


def inputs(nmo, naux, poles, seed=11):
    if poles[0] == "hf":
        nocc = poles[1]
        L = syn.df_tensor(seed, nmo, naux, max(nocc, 1))
        return L, syn.orbital_energies(seed, nmo, nocc), np.eye(nmo), nocc
    npole, nocc = poles[1], poles[2]
    L = syn.df_tensor(seed, nmo, naux, 5)
    e, u = syn.random_poles(seed, nmo, npole, nocc)
    return L, e, u, nocc


@pytest.mark.parametrize("name,nmo,naux,poles,nmom", CASES, ids=[c[0] for c in CASES])
def test_higher_moments_match_oracle(h, name, nmo, naux, poles, nmom):
    from paper_2106_03508_amd import agf2
    L, e, u, nocc = inputs(nmo, naux, poles)
    ref_o, ref_v = O.se_moments_n(L, e, u, nocc, nmom)
    mo, mv = agf2.agf2_build_moments_n(h, dev(L), dev(e), dev(u), nocc, nmom)
    mo, mv = host(mo), host(mv)
    errs = [rel(mo[n], ref_o[n]) for n in range(nmom)] + [rel(mv[n], ref_v[n])
                                                          for n in range(nmom)]
    print(name, "rel err", [f"{x:.1e}" for x in errs], flush=True)
    assert max(errs) < 1e-10
    for x in list(mo) + list(mv):
        assert np.array_equal(x, x.T)
    # the first two are the moment build's own, bitwise
    m = [host(x) for x in agf2.agf2_build_moments(h, dev(L), dev(e), dev(u), nocc)]
    assert np.array_equal(mo[0], m[0]) and np.array_equal(mo[1], m[1])
    assert np.array_equal(mv[0], m[2]) and np.array_equal(mv[1], m[3])


@pytest.mark.parametrize("nblock", [2, 3])
def test_block_lanczos_compression_matches_oracle(h, nblock):
    from paper_2106_03508_amd import agf2
    nmo = 40
    L = syn.df_tensor(5, nmo, 60, 5)
    e, u = syn.random_poles(5, nmo, 120, 45)
    mo, mv = O.se_moments_n(L, e, u, 45, 2 * nblock)
    for mm in (mo, mv):
        n, ea, va = agf2.agf2_compress_lanczos(h, dev(mm))
        assert n == nblock * nmo
        ea, va = host(ea), host(va)
        assert np.all(np.diff(ea) >= 0)
        for k in range(2 * nblock):
            assert rel((va * ea ** k) @ va.T, mm[k]) < 1e-10, k
        er, vr = O.block_lanczos(list(mm))
        assert np.abs(ea - er).max() < 1e-10 * np.abs(er).max()
        for w in (-4.0 + 0.2j, 0.3 + 0.4j, 5.0 - 0.1j):
            ref = (vr / (w - er)) @ vr.T
            got = (va / (w - ea)) @ va.T
            assert np.abs(got - ref).max() < 1e-10 * np.abs(ref).max()


def test_block_lanczos_errors(h):
    from paper_2106_03508_amd import agf2
    m = np.zeros((4, 3, 3))
    m[0] = np.diag([1.0, 0.0, 2.0])
    with pytest.raises(agf2.Agf2Error) as ei:
        agf2.agf2_compress_lanczos(h, dev(m))
    assert ei.value.status == -4
    L = syn.df_tensor(1, 10, 20, 3)
    with pytest.raises(agf2.Agf2Error) as ei:
        agf2.agf2_build_moments_n(h, dev(L), dev(syn.orbital_energies(1, 10, 3)),
                                  dev(np.eye(10)), 3, 4, prec="split_fp16")
    assert ei.value.status == -1
    with pytest.raises(agf2.Agf2Error) as ei:
        agf2.agf2_build_moments_n(h, dev(L), dev(syn.orbital_energies(1, 10, 3)),
                                  dev(np.eye(10)), 3, 3)
    assert ei.value.status == -1


def test_agf2_two_blocks_matches_oracle(h):
    """AGF2 with two Lanczos blocks per part (moments 0..3 conserved, N + 4N
    poles) to self-consistency on the GPU and in the oracle: converged E,
    IP, EA and density within 1e-8, every pole within 1e-7."""
    from paper_2106_03508_amd import agf2
    sysd = syn.system(0, **syn.SMALL)
    eps, L, nocc = sysd["eps"], sysd["L"], sysd["nocc"]
    ref = O.run_agf2(O.synthetic_hcore(eps, L, nocc), L, eps, nocc, nblock=2)
    Ld = dev(L)
    hc = agf2.agf2_fock_build(h, Ld, dev(np.diag(eps)), dev(O.reference_density(24, nocc)), -1.0)
    got = agf2.agf2_run(h, Ld, hc, dev(eps), nocc, agf2.run_opts(nblock=2))
    assert ref["converged"] and got["converged"]
    r, g = ref["history"][-1], got["history"][-1]
    print("two blocks: iterations", len(got["history"]) - 1, "oracle", len(ref["history"]) - 1,
          "E", g["e_tot"], "IP", g["ip"], "EA", g["ea"], flush=True)
    assert g["npole"] == r["npole"] == 5 * 24 and g["nocc_pole"] == r["nocc_pole"]
    assert abs(r["etot"] - g["e_tot"]) < 1e-8
    assert abs(r["ip"] - g["ip"]) < 1e-8 and abs(r["ea"] - g["ea"]) < 1e-8
    assert np.abs(host(got["rdm1"]) - ref["rdm1"]).max() < 1e-8
    assert np.abs(host(got["e_pole"]) - ref["e_pole"]).max() < 1e-7
    with pytest.raises(agf2.Agf2Error) as ei:
        agf2.agf2_run(h, Ld, hc, dev(eps), nocc, agf2.run_opts(nblock=2, prec="split_fp16"))
    assert ei.value.status == -1
