"""The allocation-free spectral function (agf2_spectral_function_noalloc)
called through the C ABI against the allocating entry point on the same
inputs: two calls in a row on the same handle, the second with fewer poles
and frequencies (the static scratch keeps the first call's contents), and
the size limit. Both entry points run the same kernels in the same order,
so their results are bitwise equal; the oracle bounds both."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import agf2_oracle as O
from paper_2106_03508_amd import synthetic as syn

pytestmark = pytest.mark.gpu

ETA = 0.2 / 27.211386   # 0.2 eV


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def noalloc(h, lam, u, omega, weight):
    nphys, npole = u.shape
    A = torch.full((omega.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    st = h.lib.agf2_spectral_function_noalloc(
        h.h, nphys, npole, lam.data_ptr(), u.data_ptr(),
        None if weight is None else weight.data_ptr(), omega.shape[0], omega.data_ptr(),
        ctypes.c_double(ETA), A.data_ptr())
    return st, A


def test_noalloc_matches_allocating_entry_point_twice():
    from paper_2106_03508_amd import agf2
    with agf2.Handle(0) as h:
        cases = [(1000, 3000, 4000, 5), (200, 650, 333, 6)]   # second call smaller
        for nmo, npole, nomega, seed in cases:
            lam, u = syn.random_poles(seed, nmo, npole, nmo // 2)
            omega = np.linspace(lam.min() - 0.3, lam.max() + 0.3, nomega)
            weight = np.linspace(0.2, 1.7, nmo)
            for wt in (None, weight):
                ld, ud, od = dev(lam), dev(u), dev(omega)
                wd = None if wt is None else dev(wt)
                st, got = noalloc(h, ld, ud, od, wd)
                assert st == 0, agf2.load_library().agf2_last_error(h.h)
                ref = agf2.agf2_spectral_function(h, ld, ud, od, ETA, wd)
                torch.cuda.synchronize()
                assert torch.equal(got, ref)
                o = O.spectral_function(lam, u, omega, ETA, wt)
                err = np.abs(got.cpu().numpy() - o).max() / np.abs(o).max()
                print(nmo, npole, nomega, "weighted" if wt is not None else "total",
                      f"vs oracle {err:.1e}", flush=True)
                assert err < 1e-12


def test_noalloc_rejects_more_poles_than_its_scratch():
    """The size check runs before any array is touched, so small buffers
    stand in for the arrays of the rejected size."""
    from paper_2106_03508_amd import agf2
    with agf2.Handle(0) as h:
        buf = dev(np.zeros(16))
        st = h.lib.agf2_spectral_function_noalloc(h.h, 4, 32769, buf.data_ptr(),
                                                  buf.data_ptr(), None, 4, buf.data_ptr(),
                                                  ctypes.c_double(ETA), buf.data_ptr())
        assert st == -1
        assert b"AGF2_SPECTRUM_NOALLOC_MAX_POLE" in agf2.load_library().agf2_last_error(h.h)
