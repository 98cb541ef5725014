"""Split-precision moment builds against the FP64 oracle.

split_fp16 (fp16 hi/lo pairs with power-of-two scaling: 22 significant bits
per operand, float32 accumulation) is held to the reduced-precision bar of
1e-7 relative Frobenius on every moment, with one exception: the single
occupied pole case, whose lesser moments sum only 19 Z columns. There the
operands' own 22-bit rounding (relative error up to 2^-22 per operand) does
not average out; a CPU emulation of the scheme with exact operands and the
same float32 accumulation reaches 4e-8 where the scheme gives 1.2e-7, so the
floor is the representation, not the kernels. That case is held to 2e-7 and
does not meet the bar.

split_bf16 (bf16 hi/lo pairs, 16 significant bits) carries ~2^-16 error per
operand and does not meet the 1e-7 bar at any size (measured 1e-6 - 1e-5);
it is held to its own bound of 1.5e-5 and the errors are printed."""
import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu

TOL = {"split_fp16": 1e-7, "split_bf16": 1.5e-5}
# the few-term case below the bar (see the module docstring)
TOL_FEW_TERMS = {"split_fp16": 2e-7, "split_bf16": 1.5e-5}


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


CASES = [
    ("hf_small", 24, 80, ("hf", 5)),
    ("hf_ragged", 70, 90, ("hf", 13)),
    ("dressed_ragged", 70, 90, ("dressed", 210, 81)),
    ("dressed_tiles", 130, 100, ("dressed", 150, 40)),
    ("single_occ", 20, 33, ("hf", 1)),
    ("medium_hf", 200, 700, ("hf", 40)),
    # lesser inner pole count 63: its pair column blocks are padded to 64
    # (odd count, one zero column each); greater 57 is not padded
    ("padded_pairs", 40, 70, ("dressed", 120, 57)),
]


def inputs(nmo, naux, poles, seed=11):
    if poles[0] == "hf":
        nocc = poles[1]
        L = syn.df_tensor(seed, nmo, naux, max(nocc, 1))
        e = syn.orbital_energies(seed, nmo, nocc)
        u = np.eye(nmo)
    else:
        npole, nocc = poles[1], poles[2]
        L = syn.df_tensor(seed, nmo, naux, 5)
        e, u = syn.random_poles(seed, nmo, npole, nocc)
    return L, e, u, nocc


_REF = {}


def reference(name, nmo, naux, poles):
    if name not in _REF:
        L, e, u, nocc = inputs(nmo, naux, poles)
        _REF[name] = (L, e, u, nocc, O.se_moments(L, e, u, nocc))
    return _REF[name]


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
@pytest.mark.parametrize("name,nmo,naux,poles", CASES, ids=[c[0] for c in CASES])
def test_moments_split_match_oracle(h, name, nmo, naux, poles, prec):
    from paper_2106_03508_amd import agf2
    L, e, u, nocc, ref = reference(name, nmo, naux, poles)
    got = agf2.agf2_build_moments(h, dev(L), dev(e), dev(u), nocc, prec=prec)
    got = [g.cpu().numpy() for g in got]
    errs = [rel(g, r) for g, r in zip(got, ref)]
    print(name, prec, "rel err", [f"{x:.2e}" for x in errs], flush=True)
    for g in got:
        assert np.array_equal(g, g.T)
    assert max(errs) < (TOL_FEW_TERMS if name == "single_occ" else TOL)[prec]


@pytest.mark.parametrize("prec", ["split_fp16", "split_bf16"])
def test_split_deterministic(h, prec):
    from paper_2106_03508_amd import agf2
    L, e, u, nocc = inputs(70, 90, ("dressed", 120, 50), seed=3)
    a = [x.cpu().numpy() for x in agf2.agf2_build_moments(h, dev(L), dev(e), dev(u), nocc,
                                                           prec=prec)]
    b = [x.cpu().numpy() for x in agf2.agf2_build_moments(h, dev(L), dev(e), dev(u), nocc,
                                                           prec=prec)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
