"""The trained warm-start network against the plain cold start: held-out
synthetic systems (seeds never used in training) are converged by agf2_run
twice, cold and with the network's correction as dm_init. The converged
spectrum must be the cold start's (IP/EA within 1e-5 Ha, total energy within
1e-6 Ha; the fixed point is the same, so the differences are at the
convergence threshold), and the warm start must save iterations on average.
Also: the correction of a network with zero output layer is exactly zero, so
such a warm start reproduces the cold history."""
import os

import numpy as np
import pytest
import torch

from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu

HELDOUT = dict(n=8, seed0=21000, nmo_lo=80, nmo_hi=160)


@pytest.fixture(scope="module")
def h():
    from paper_2106_03508_amd import agf2
    hd = agf2.Handle(0)
    yield hd
    hd.close()


def test_trained_network_saves_iterations(h):
    from paper_2106_03508_amd import warmstart as W
    assert os.path.exists(W.PARAMS_PATH), "trained parameters are missing"
    params = W.load_params()
    shapes = syn.batch_shapes(HELDOUT["n"], HELDOUT["seed0"], HELDOUT["nmo_lo"],
                              HELDOUT["nmo_hi"])
    rows = W.evaluate(h, params, shapes)
    summ = W.summarize(rows)
    print(summ, flush=True)
    for r in rows:
        assert r["cold"]["converged"] and r["warm_fp64"]["converged"]
        assert r["warm_fp64"]["warm"] == 1
        assert abs(r["warm_fp64"]["d_ip"]) < 1e-5 and abs(r["warm_fp64"]["d_ea"]) < 1e-5
        assert abs(r["warm_fp64"]["d_e"]) < 1e-6
    assert summ["iterations_saved"] >= 0.5
    assert summ["more"] == 0


def test_zero_network_is_the_cold_start(h):
    from paper_2106_03508_amd import agf2
    from paper_2106_03508_amd import warmstart as W
    s = W.System(h, 5, 40, 8, 140)
    net = agf2.Mlp(h, np.zeros(agf2.MLP_NPARAM, dtype=np.float32))
    m0 = s.moments0(h)
    dm = agf2.agf2_mlp_predict_correction(h, net, s.eps, s.nocc, m0)
    net.close()
    assert not torch.any(dm).item()
    cold = s.run(h)
    warm = s.run(h, dm_init=dm)
    assert warm["warm"] == 1
    assert cold["iterations"] == warm["iterations"]
    assert abs(cold["e_tot"] - warm["e_tot"]) < 1e-12
