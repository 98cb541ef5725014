"""Checks at the medium and large sizes, against stored oracle values
(tests/golden/, written by tests/golden/make_golden.py from the CPU oracle
only) and, where the oracle finishes in seconds, against the oracle itself.

- nmo=200, nocc=40, naux=700 (the double-zeta-like system): the whole FP64
  moment build against the oracle (1e-10 relative Frobenius), and AGF2 to
  self-consistency on the GPU against the oracle's converged run (FP64: the
  converged-result tolerances of the small-system loop test; split fp16: IP
  and EA within 1e-5 Ha, energy within 1e-6 Ha).
- nmo=400, 1200 dressed poles (480 occupied: the pole shape of every
  iteration after the first at the warm-start evaluation size) and nmo=1000
  mean-field poles (the benchmark's launch configuration): moment elements
  sampled by the oracle in every lower-triangle 64 x 64 block of the output,
  per element within 1e-10 * sqrt(U0_pp U0_qq) (Cauchy-Schwarz bound of the
  element's summands; times the largest |weight| for U1), and the split
  builds against the FP64 build (relative Frobenius, error stated per
  moment)."""
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
sys.path.insert(0, ROOT)


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


def wmax(e, nocc_pole):
    """Largest |e_i + e_j - e_a| (lesser) and |e_a + e_b - e_i| (greater)."""
    eo, ev = e[:nocc_pole], e[nocc_pole:]
    lo = max(abs(2 * eo.min() - ev.max()), abs(2 * eo.max() - ev.min()))
    gr = max(abs(2 * ev.max() - eo.min()), abs(2 * ev.min() - eo.max()))
    return lo, gr


def check_samples(m, fix, e, nocc_pole, label):
    """m: the four FP64 GPU moments; fix: a sampled-elements fixture."""
    pairs = [tuple(p) for p in fix["pairs"]]
    vals = np.array(fix["values"])
    diag = {p: vals[k] for k, (p, q) in enumerate(pairs) if p == q}
    wl, wg = wmax(e, nocc_pole)
    worst = 0.0
    for k, (p, q) in enumerate(pairs):
        for i, (mom, w) in enumerate(((0, 1.0), (1, wl), (0, 1.0), (1, wg))):
            base = 2 * (i // 2)   # U0 of the same part
            scale = np.sqrt(diag[p][base] * diag[q][base]) * w
            err = abs(m[i][p, q] - vals[k, i]) / scale
            worst = max(worst, err)
            assert err <= 1e-10, (label, p, q, i, err)
    print(label, len(pairs), "sampled elements, worst error / bound scale", f"{worst:.1e}",
          flush=True)


def test_medium_fp64_moments_whole(h):
    from paper_2106_03508_amd import agf2
    s = syn.system(1, **syn.MEDIUM)
    eps, L, nocc = s["eps"], s["L"], s["nocc"]
    ref = O.se_moments(L, eps, np.eye(200), nocc)
    got = [x.cpu().numpy() for x in agf2.agf2_build_moments(h, dev(L), dev(eps),
                                                            dev(np.eye(200)), nocc)]
    errs = [rel(g, r) for g, r in zip(got, ref)]
    print("nmo=200 FP64 moments rel err", [f"{x:.1e}" for x in errs], flush=True)
    assert max(errs) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "split_fp16"])
def test_config2_agf2_to_convergence(h, prec):
    """AGF2 on the nmo=200 system from the mean-field reference to
    self-consistency, against the oracle's converged run (stored)."""
    from paper_2106_03508_amd import agf2
    ref = golden("config2_nmo200.json")
    s = syn.system(ref["system"]["seed"], **syn.MEDIUM)
    eps, L, nocc = s["eps"], s["L"], s["nocc"]
    Ld = dev(L)
    hc = agf2.agf2_fock_build(h, Ld, dev(np.diag(eps)), dev(O.reference_density(200, nocc)),
                              -1.0)
    r = agf2.agf2_run(h, Ld, hc, dev(eps), nocc, agf2.run_opts(prec=prec))
    g = r["history"][-1]
    de, dip, dea = (abs(g["e_tot"] - ref["e_tot"]), abs(g["ip"] - ref["ip"]),
                    abs(g["ea"] - ref["ea"]))
    print(prec, "iterations", len(r["history"]) - 1, "oracle", ref["iterations"],
          f"dE {de:.1e} dIP {dip:.1e} dEA {dea:.1e}", flush=True)
    assert r["converged"]
    assert g["npole"] == ref["npole"] and g["nocc_pole"] == ref["nocc_pole"]
    assert abs(float(r["rdm1"].trace()) - 80.0) < 1e-8
    if prec == "fp64":
        assert de < 1e-8 and dip < 1e-8 and dea < 1e-8
        assert abs(g["shift"] - ref["shift"]) < 1e-7
        assert abs(len(r["history"]) - 1 - ref["iterations"]) <= 1
        lam = r["e_pole"].cpu().numpy()
        n = g["nocc_pole"]
        front = lam[max(0, n - 8):n + 8]
        assert np.abs(front - np.array(ref["pole_energies_frontier"])).max() < 1e-7
    else:
        assert dip < 1e-5 and dea < 1e-5 and de < 1e-6


def test_dressed400_moments(h):
    """Moments at the 3N-pole shape of nmo=400: FP64 against sampled oracle
    elements; split builds against the FP64 build."""
    from paper_2106_03508_amd import agf2
    fix = golden("dressed400_samples.json")
    sy, po = fix["system"], fix["poles"]
    L = syn.df_tensor(sy["seed"], sy["nmo"], sy["naux"], sy["nocc"])
    e, u = syn.random_poles(po["seed"], sy["nmo"], po["npole"], po["nocc_pole"])
    Ld, ed, ud = dev(L), dev(e), dev(u)
    res = {}
    for prec in ("fp64", "split_fp16", "split_bf16"):
        res[prec] = [x.cpu().numpy() for x in agf2.agf2_build_moments(h, Ld, ed, ud,
                                                                      po["nocc_pole"],
                                                                      prec=prec)]
    check_samples(res["fp64"], fix, e, po["nocc_pole"], "nmo=400 3N poles FP64")
    for prec in ("split_fp16", "split_bf16"):
        errs = [rel(a, b) for a, b in zip(res[prec], res["fp64"])]
        print("nmo=400 3N poles", prec, "rel err vs FP64", [f"{x:.2e}" for x in errs],
              flush=True)
        assert max(errs) < (1e-7 if prec == "split_fp16" else 1.5e-5)


def test_large_moments_fp64_and_split():
    """nmo=1000, nocc=76, naux=3500 in the benchmark's launch configuration."""
    from bench import generate
    from paper_2106_03508_amd import agf2
    fix = golden("large1000_samples.json")
    sy = fix["system"]
    eps, L = generate(sy["seed"], sy["nmo"], sy["nocc"], sy["naux"])
    print("generated", flush=True)
    N = sy["nmo"]
    with agf2.Handle(0) as h:
        Ld = torch.from_numpy(L).cuda()
        del L
        ed = torch.from_numpy(eps).cuda()
        u = torch.eye(N, dtype=torch.float64, device="cuda")
        res = {}
        for prec in ("fp64", "split_fp16", "split_bf16"):
            m = agf2.agf2_build_moments(h, Ld, ed, u, sy["nocc"], prec=prec)
            res[prec] = [x.cpu().numpy() for x in m]
            print(prec, "done", flush=True)
    check_samples(res["fp64"], fix, eps, sy["nocc"], "nmo=1000 FP64")
    ref = res["fp64"]
    for prec in ("split_fp16", "split_bf16"):
        errs = [np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(res[prec], ref)]
        print(prec, "rel Frobenius err vs FP64", [f"{x:.2e}" for x in errs], flush=True)
        assert max(errs) < (1e-7 if prec == "split_fp16" else 5e-6)
