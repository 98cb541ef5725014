"""Full-size checks at nmo=1000, nocc=76, naux=3500 (the ~1000-orbital
workload), in the launch configuration the benchmark times: moment elements
sampled from the oracle (computed one by one), the FP64 build against them
at 1e-10, and the split builds against the FP64 build (relative Frobenius,
the reduced-precision error stated per moment) and against the samples."""
import os
import sys

import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

PAIRS = [(0, 0), (76, 76), (999, 999), (640, 77)]


@pytest.fixture(scope="module")
def large():
    from bench import generate
    wl = syn.LARGE
    eps, L = generate(2, wl["nmo"], wl["nocc"], wl["naux"])
    print("generated", flush=True)
    samples = O.se_moment_elements(L, eps, np.eye(wl["nmo"]), wl["nocc"], PAIRS,
                                   progress=lambda t: print(t, flush=True))
    print("oracle samples done", flush=True)
    return eps, L, wl["nocc"], samples


def test_large_moments_fp64_and_split(large):
    from paper_2106_03508_amd import agf2
    eps, L, nocc, samples = large
    N = eps.shape[0]
    with agf2.Handle(0) as h:
        Ld = torch.from_numpy(L).cuda()
        ed = torch.from_numpy(eps).cuda()
        u = torch.eye(N, dtype=torch.float64, device="cuda")
        res = {}
        for prec in ("fp64", "split_fp16", "split_bf16"):
            m = agf2.agf2_build_moments(h, Ld, ed, u, nocc, prec=prec)
            res[prec] = [x.cpu().numpy() for x in m]
            print(prec, "done", flush=True)
    ref = res["fp64"]
    scale = [np.abs(r).max() for r in ref]
    for k, (p, q) in enumerate(PAIRS):
        for m in range(4):
            assert abs(ref[m][p, q] - samples[k, m]) <= 1e-10 * scale[m]
    for prec in ("split_fp16", "split_bf16"):
        errs = [np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(res[prec], ref)]
        samp = max(abs(res[prec][m][p, q] - samples[k, m]) / scale[m]
                   for k, (p, q) in enumerate(PAIRS) for m in range(4))
        print(prec, "rel Frobenius err vs FP64", [f"{x:.2e}" for x in errs],
              f"max sampled err / max|U| {samp:.2e}", flush=True)
        if prec == "split_fp16":
            assert max(errs) < 1e-7
        else:
            assert max(errs) < 5e-6
