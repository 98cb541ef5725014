"""Thin ctypes binding of libagf2.so (C ABI declared in include/agf2.h).

Argument marshalling only: every function checks that its tensors are
float64, contiguous and on the handle's GPU, allocates outputs with torch
(device memory), and passes raw pointers to the library. No arithmetic of the
method happens here. The library must be built (``python -m
paper_2106_03508_amd.build`` or ``__graft_entry__.build()``); importing the
binding without it, or calling it without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagf2.so")

AGF2_FP64 = 0
AGF2_SPLIT_BF16 = 1
AGF2_SPLIT_FP16 = 2
PRECISIONS = {"fp64": AGF2_FP64, "split_bf16": AGF2_SPLIT_BF16, "split_fp16": AGF2_SPLIT_FP16}

STATUS = {0: "AGF2_OK", -1: "AGF2_ERR_ARG", -2: "AGF2_ERR_HIP", -3: "AGF2_ERR_NOMEM",
          -4: "AGF2_ERR_NOT_PD", -5: "AGF2_ERR_NO_CONVERGE", -6: "AGF2_ERR_NELEC"}

# exported entry points (name -> (restype, argtypes))
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)


class FockOpts(ctypes.Structure):
    _fields_ = [("tol_rdm1", _D), ("tol_nelec", _D), ("bracket", _D), ("step0", _D),
                ("max_cycle", _I), ("diis_space", _I)]


class RunOpts(ctypes.Structure):
    _fields_ = [("max_iter", _I), ("conv_tol", _D), ("conv_tol_ipea", _D), ("diis_space", _I),
                ("damping", _D), ("prec", _I), ("compress_tol", _D), ("fock", FockOpts),
                ("nblock", _I)]


class IterRecord(ctypes.Structure):
    _fields_ = [("iter", _I), ("nocc_pole", _I), ("npole", _I), ("fock_cycles", _I),
                ("warm", _I), ("fock_converged", _I), ("e_1b", _D), ("e_2b", _D), ("e_tot", _D), ("ip", _D),
                ("ea", _D), ("w_ip", _D), ("w_ea", _D), ("mu", _D), ("shift", _D),
                ("t_moments", _D), ("t_compress", _D), ("t_fock", _D), ("t_energy", _D)]


class System(ctypes.Structure):
    _fields_ = [("nphys", _I), ("naux", _I), ("Lpq", _P), ("npole", _I), ("nocc_pole", _I),
                ("e_pole", _P), ("u_pole", _P), ("m0_occ", _P), ("m1_occ", _P),
                ("m0_vir", _P), ("m1_vir", _P)]


SIGNATURES = {
    "agf2_create": (_I, [ctypes.POINTER(_P), _I, _P]),
    "agf2_destroy": (_I, [_P]),
    "agf2_last_error": (ctypes.c_char_p, [_P]),
    "agf2_synchronize": (_I, [_P]),
    "agf2_build_moments": (_I, [_P, _I, _I, _I, _P, _I, _I, _P, _P, _P, _P, _P, _P]),
    "agf2_build_moments_batched": (_I, [_P, _I, ctypes.POINTER(System), _IP]),
    "agf2_build_moments_n": (_I, [_P, _I, _I, _I, _I, _P, _I, _I, _P, _P, _P, _P]),
    "agf2_compress_lanczos": (_I, [_P, _I, _I, _P, _IP, _P, _P]),
    "agf2_fock_build": (_I, [_P, _I, _I, _P, _P, _P, _D, _P]),
    "agf2_compress": (_I, [_P, _I, _P, _P, _D, _IP, _P, _P]),
    "agf2_fock_opts_default": (None, [ctypes.POINTER(FockOpts)]),
    "agf2_fock_loop": (_I, [_P, _I, _I, _P, _P, _I, _I, _P, _P, _P, _P, _P, _P, _IP, _DP,
                            _DP, _IP, ctypes.POINTER(FockOpts)]),
    "agf2_energy_gf": (_I, [_P, _I, _P, _P, _P, _I, _I, _P, _P, _I, _P, _P, _I, _P, _P,
                            _DP, _DP]),
    "agf2_spectral_function": (_I, [_P, _I, _I, _P, _P, _P, _I, _P, _D, _P]),
    "agf2_spectral_function_noalloc": (_I, [_P, _I, _I, _P, _P, _P, _I, _P, _D, _P]),
    "agf2_run_opts_default": (None, [ctypes.POINTER(RunOpts)]),
    "agf2_run": (_I, [_P, ctypes.POINTER(RunOpts), _I, _I, _P, _P, _P, _I, _P,
                      ctypes.POINTER(IterRecord), _IP, _IP, _P, _P, _IP, _P]),
    "agf2_run_state_bytes": (ctypes.c_long, [_I, ctypes.POINTER(RunOpts)]),
    "agf2_run_resume": (_I, [_P, ctypes.POINTER(RunOpts), _I, _I, _P, _P, _P, _I, _P, _P, _P,
                             _I, ctypes.POINTER(IterRecord), _IP, _IP, _P, _P, _IP, _P]),
    "agf2_mlp_create": (_I, [_P, ctypes.POINTER(_P)]),
    "agf2_mlp_destroy": (_I, [_P]),
    "agf2_mlp_set_params": (_I, [_P, _P, _P]),
    "agf2_mlp_get_params": (_I, [_P, _P, _P]),
    "agf2_mlp_get_grad": (_I, [_P, _P, _P]),
    "agf2_mlp_features": (_I, [_P, _I, _I, _P, _P, _P, _P]),
    "agf2_mlp_forward": (_I, [_P, _P, _I, _P, _P]),
    "agf2_mlp_loss_grad": (_I, [_P, _I, _P, _P, _P, _P, _P, _P]),
    "agf2_mlp_backward": (_I, [_P, _P, _I, _P]),
    "agf2_mlp_adam_step": (_I, [_P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float]),
    "agf2_mlp_predict_correction": (_I, [_P, _P, _I, _I, _P, _P, _P]),
    "agf2_profile_enable": (_I, [_P, _I]),
    "agf2_profile_count": (_I, [_P]),
    "agf2_profile_get": (_I, [_P, _I, ctypes.POINTER(ctypes.c_char_p),
                              ctypes.POINTER(ctypes.c_long), _DP, _DP, _DP]),
}

_lib = None


class Agf2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libagf2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t: torch.Tensor, name: str, dev: torch.device) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if t.device != dev:
        raise ValueError(f"{name} must be on {dev}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _ptr32(t: torch.Tensor, name: str, dev: torch.device) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.device != dev:
        raise ValueError(f"{name} must be on {dev}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


class Handle:
    """An agf2 handle bound to a GPU and to torch's current stream there."""

    def __init__(self, device: int = 0, stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("agf2 needs a ROCm GPU; none is visible")
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _P()
        self._check(self.lib.agf2_create(ctypes.byref(h), device, _P(stream.cuda_stream)), None)
        self.h = h

    def _check(self, status, h=None):
        if status != 0:
            msg = self.lib.agf2_last_error(h if h is not None else self.h)
            raise Agf2Error(status, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.agf2_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def synchronize(self):
        self._check(self.lib.agf2_synchronize(self.h))

    def empty(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.device)


def agf2_create(device: int = 0, stream=None) -> Handle:
    return Handle(device, stream)


def agf2_build_moments(h: Handle, L, e_pole, u_pole, nocc_pole: int, prec="fp64", out=None):
    """Moments (m0_occ, m1_occ, m0_vir, m1_vir) of the poles (e_pole, u_pole)."""
    naux, nphys, _ = L.shape
    npole = e_pole.shape[0]
    if out is None:
        out = tuple(h.empty(nphys, nphys) for _ in range(4))
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    d = h.device
    h._check(h.lib.agf2_build_moments(
        h.h, p, nphys, naux, _ptr(L, "L", d), npole, nocc_pole, _ptr(e_pole, "e_pole", d),
        _ptr(u_pole, "u_pole", d), *[_ptr(m, "moment", d) for m in out]))
    return out


def agf2_build_moments_n(h: Handle, L, e_pole, u_pole, nocc_pole: int, nmom: int, prec="fp64"):
    """Moments 0..nmom-1 of each part: (m_occ [nmom, N, N], m_vir [nmom, N, N])."""
    naux, nphys, _ = L.shape
    npole = e_pole.shape[0]
    mo = h.empty(nmom, nphys, nphys)
    mv = h.empty(nmom, nphys, nphys)
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    d = h.device
    h._check(h.lib.agf2_build_moments_n(
        h.h, p, int(nmom), nphys, naux, _ptr(L, "L", d), npole, nocc_pole,
        _ptr(e_pole, "e_pole", d), _ptr(u_pole, "u_pole", d), _ptr(mo, "m_occ", d),
        _ptr(mv, "m_vir", d)))
    return mo, mv


def agf2_compress_lanczos(h: Handle, m):
    """Compression of one part to nmom/2 Lanczos blocks from its moments m
    [nmom, N, N]: (naux, e_aux [naux], v_aux [N, naux])."""
    nmom, nphys, _ = m.shape
    nb = nmom // 2
    e = h.empty(nb * nphys)
    v = h.empty(nphys, nb * nphys if nb > 1 else nphys)
    n = ctypes.c_int(0)
    d = h.device
    h._check(h.lib.agf2_compress_lanczos(h.h, nphys, int(nmom), _ptr(m, "m", d), ctypes.byref(n),
                                         _ptr(e, "e_aux", d), _ptr(v, "v_aux", d)))
    return n.value, e[:n.value], v[:, :n.value]


def agf2_build_moments_batched(h: Handle, systems, outs=None):
    """FP64 moments of a batch of systems in one replayed HIP graph.

    ``systems`` is a sequence of (L, e_pole, u_pole, nocc_pole). Returns
    (outs, tile_width): outs[s] = (m0_occ, m1_occ, m0_vir, m1_vir) and
    tile_width[s] the slab inner-tile width the library chose for system s.
    The library reuses its captured graph while the sizes and the buffers are
    the same as in the previous call, so pass the same tensors (and ``outs``)
    again to replay it with new values.
    """
    d = h.device
    n = len(systems)
    if outs is None:
        outs = [tuple(h.empty(L.shape[1], L.shape[1]) for _ in range(4)) for L, *_ in systems]
    arr = (System * n)()
    for k, ((L, e, u, nocc), out) in enumerate(zip(systems, outs)):
        naux, nphys, _ = L.shape
        arr[k] = System(nphys, naux, _ptr(L, "L", d), e.shape[0], int(nocc), _ptr(e, "e_pole", d),
                        _ptr(u, "u_pole", d), *[_ptr(m, "moment", d) for m in out])
    tw = (_I * n)()
    h._check(h.lib.agf2_build_moments_batched(h.h, n, arr, tw))
    return outs, list(tw)


def agf2_fock_build(h: Handle, L, hcore, rdm1, alpha=1.0, out=None):
    naux, nphys, _ = L.shape
    out = h.empty(nphys, nphys) if out is None else out
    d = h.device
    h._check(h.lib.agf2_fock_build(h.h, nphys, naux, _ptr(L, "L", d), _ptr(hcore, "hcore", d),
                                   _ptr(rdm1, "rdm1", d), float(alpha), _ptr(out, "fock", d)))
    return out


def agf2_compress(h: Handle, m0, m1, tol=0.0):
    """Returns (naux, e_aux[nphys], v_aux[nphys, nphys]); columns >= naux are zero."""
    nphys = m0.shape[0]
    e = h.empty(nphys)
    v = h.empty(nphys, nphys)
    n = ctypes.c_int(0)
    d = h.device
    h._check(h.lib.agf2_compress(h.h, nphys, _ptr(m0, "m0", d), _ptr(m1, "m1", d), float(tol),
                                 ctypes.byref(n), _ptr(e, "e_aux", d), _ptr(v, "v_aux", d)))
    return n.value, e, v


def fock_opts(**kw) -> FockOpts:
    o = FockOpts()
    load_library().agf2_fock_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def agf2_fock_loop(h: Handle, L, hcore, nelec: int, e_se, v_se, rdm1, opts: FockOpts = None,
                   raise_on_no_converge=True):
    """Fock loop. e_se (shifted in place) and rdm1 (updated in place) are
    modified. Returns a dict with fock, e_pole, u_pole, nocc_pole, mu, shift,
    n_cycle, converged."""
    naux, nphys, _ = L.shape
    naux_se = e_se.shape[0]
    npole = nphys + naux_se
    fock = h.empty(nphys, nphys)
    e_pole = h.empty(npole)
    u_pole = h.empty(nphys, npole)
    nocc = ctypes.c_int(0)
    mu = ctypes.c_double(0.0)
    shift = ctypes.c_double(0.0)
    ncyc = ctypes.c_int(0)
    d = h.device
    st = h.lib.agf2_fock_loop(
        h.h, nphys, naux, _ptr(L, "L", d), _ptr(hcore, "hcore", d), int(nelec), naux_se,
        _ptr(e_se, "e_se", d), _ptr(v_se, "v_se", d), _ptr(rdm1, "rdm1", d),
        _ptr(fock, "fock", d), _ptr(e_pole, "e_pole", d), _ptr(u_pole, "u_pole", d),
        ctypes.byref(nocc), ctypes.byref(mu), ctypes.byref(shift), ctypes.byref(ncyc),
        ctypes.byref(opts) if opts is not None else None)
    converged = st == 0
    if st != 0 and (st != -5 or raise_on_no_converge):
        h._check(st)
    return dict(fock=fock, e_pole=e_pole, u_pole=u_pole, nocc_pole=nocc.value, mu=mu.value,
                shift=shift.value, n_cycle=ncyc.value, converged=converged, rdm1=rdm1)


def agf2_spectral_function(h: Handle, e_pole, u_pole, omega, eta, weight=None, out=None):
    """A[k] = -1/pi Im Tr[P G(omega_k + i eta)] of the poles; weight [nphys]
    (a projection) or None for the total spectrum."""
    nphys, npole = u_pole.shape
    out = h.empty(omega.shape[0]) if out is None else out
    d = h.device
    wp = None if weight is None else _ptr(weight, "weight", d)
    h._check(h.lib.agf2_spectral_function(h.h, nphys, npole, _ptr(e_pole, "e_pole", d),
                                          _ptr(u_pole, "u_pole", d), wp, omega.shape[0],
                                          _ptr(omega, "omega", d), float(eta),
                                          _ptr(out, "A", d)))
    return out


def agf2_energy_gf(h: Handle, hcore, fock, rdm1, e_pole, u_pole, nocc_pole, e_se_occ, v_se_occ,
                   e_se_vir, v_se_vir):
    """(e_1b, e_2b). v_se_* are [nphys, naux_*] contiguous."""
    nphys = hcore.shape[0]
    npole = e_pole.shape[0]
    e1 = ctypes.c_double(0.0)
    e2 = ctypes.c_double(0.0)
    d = h.device
    h._check(h.lib.agf2_energy_gf(
        h.h, nphys, _ptr(hcore, "hcore", d), _ptr(fock, "fock", d), _ptr(rdm1, "rdm1", d),
        npole, int(nocc_pole), _ptr(e_pole, "e_pole", d), _ptr(u_pole, "u_pole", d),
        e_se_occ.shape[0], _ptr(e_se_occ, "e_se_occ", d), _ptr(v_se_occ, "v_se_occ", d),
        e_se_vir.shape[0], _ptr(e_se_vir, "e_se_vir", d), _ptr(v_se_vir, "v_se_vir", d),
        ctypes.byref(e1), ctypes.byref(e2)))
    return e1.value, e2.value


def agf2_profile_enable(h: Handle, enable: bool = True):
    h._check(h.lib.agf2_profile_enable(h.h, 1 if enable else 0))


def agf2_profile_read(h: Handle) -> dict:
    """{kernel class: dict(launches, ms, flops, bytes)} accumulated since the
    profiler was enabled."""
    n = h.lib.agf2_profile_count(h.h)
    if n < 0:
        h._check(n)
    out = {}
    for i in range(n):
        name = ctypes.c_char_p()
        launches = ctypes.c_long(0)
        ms = ctypes.c_double(0.0)
        fl = ctypes.c_double(0.0)
        by = ctypes.c_double(0.0)
        h._check(h.lib.agf2_profile_get(h.h, i, ctypes.byref(name), ctypes.byref(launches),
                                        ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(by)))
        out[name.value.decode()] = dict(launches=launches.value, ms=ms.value, flops=fl.value,
                                        bytes=by.value)
    return out


def run_opts(**kw) -> RunOpts:
    """agf2_run options: the library defaults, overridden by keyword (prec may
    be a name such as "split_fp16"; fock_* keys set Fock-loop options)."""
    o = RunOpts()
    load_library().agf2_run_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "prec":
            v = PRECISIONS[v] if isinstance(v, str) else int(v)
        if k.startswith("fock_"):
            setattr(o.fock, k[5:], v)
        else:
            setattr(o, k, v)
    return o


def agf2_run(h: Handle, L, hcore, e_mf, nocc: int, opts: RunOpts = None, dm_init=None,
             raise_on_no_converge=False):
    """AGF2 to self-consistency. Returns a dict with the per-iteration records
    (list of dicts), converged flag, final e_pole, u_pole, nocc_pole and rdm1."""
    naux, nphys, _ = L.shape
    opts = run_opts() if opts is None else opts
    recs = (IterRecord * (opts.max_iter + 1))()
    nrec = ctypes.c_int(0)
    conv = ctypes.c_int(0)
    nocc_pole = ctypes.c_int(0)
    npmax = nphys * (1 + 2 * max(1, opts.nblock))
    e_pole = h.empty(npmax)
    u_pole = h.empty(nphys, npmax)
    rdm1 = h.empty(nphys, nphys)
    d = h.device
    st = h.lib.agf2_run(h.h, ctypes.byref(opts), nphys, naux, _ptr(L, "L", d),
                        _ptr(hcore, "hcore", d), _ptr(e_mf, "e_mf", d), int(nocc),
                        None if dm_init is None else _ptr(dm_init, "dm_init", d), recs,
                        ctypes.byref(nrec), ctypes.byref(conv), _ptr(e_pole, "e_pole", d),
                        _ptr(u_pole, "u_pole", d), ctypes.byref(nocc_pole), _ptr(rdm1, "rdm1", d))
    if st != 0 and (st != -5 or raise_on_no_converge):
        h._check(st)
    history = [{f: getattr(recs[i], f) for f, _ in IterRecord._fields_} for i in range(nrec.value)]
    npole = history[-1]["npole"] if history else nphys
    return dict(history=history, converged=bool(conv.value), e_pole=e_pole[:npole],
                u_pole=u_pole.view(-1)[:nphys * npole].view(nphys, npole),
                nocc_pole=nocc_pole.value, rdm1=rdm1)


def agf2_run_resume(h: Handle, L, hcore, e_mf, nocc: int, opts: RunOpts = None, dm_init=None,
                    state_in=None, save_state=True, max_iter_call=0,
                    raise_on_no_converge=False):
    """agf2_run continued from a saved state (state_in: numpy uint8 array from
    an earlier call, or None to start at iteration 0), stopping after
    max_iter_call iterations (0: no limit). Returns the agf2_run dict plus
    "state" (numpy uint8, the state after this call's last iteration) and
    "status"."""
    import numpy as np
    naux, nphys, _ = L.shape
    opts = run_opts() if opts is None else opts
    nbytes = h.lib.agf2_run_state_bytes(nphys, ctypes.byref(opts))
    if nbytes < 0:
        raise ValueError("bad nphys or run options")
    sin = None
    if state_in is not None:
        sin = np.ascontiguousarray(state_in, dtype=np.uint8)
        if sin.shape != (nbytes,):
            raise ValueError(f"state_in must hold {nbytes} bytes")
    sout = np.empty(nbytes, dtype=np.uint8) if save_state else None
    recs = (IterRecord * (opts.max_iter + 1))()
    nrec = ctypes.c_int(0)
    conv = ctypes.c_int(0)
    nocc_pole = ctypes.c_int(0)
    npmax = nphys * (1 + 2 * max(1, opts.nblock))
    e_pole = h.empty(npmax)
    u_pole = h.empty(nphys, npmax)
    rdm1 = h.empty(nphys, nphys)
    d = h.device
    st = h.lib.agf2_run_resume(
        h.h, ctypes.byref(opts), nphys, naux, _ptr(L, "L", d), _ptr(hcore, "hcore", d),
        _ptr(e_mf, "e_mf", d), int(nocc), None if dm_init is None else _ptr(dm_init, "dm_init", d),
        None if sin is None else sin.ctypes.data, None if sout is None else sout.ctypes.data,
        int(max_iter_call), recs, ctypes.byref(nrec), ctypes.byref(conv),
        _ptr(e_pole, "e_pole", d), _ptr(u_pole, "u_pole", d), ctypes.byref(nocc_pole),
        _ptr(rdm1, "rdm1", d))
    if st != 0 and (st != -5 or raise_on_no_converge):
        h._check(st)
    history = [{f: getattr(recs[i], f) for f, _ in IterRecord._fields_} for i in range(nrec.value)]
    npole = history[-1]["npole"] if history else nphys
    return dict(history=history, converged=bool(conv.value), e_pole=e_pole[:npole],
                u_pole=u_pole.view(-1)[:nphys * npole].view(nphys, npole),
                nocc_pole=nocc_pole.value, rdm1=rdm1, state=sout, status=st)


# ---------------------------------------------------------------- warm start
MLP_FEATURES, MLP_HIDDEN, MLP_OUTPUTS, MLP_NPARAM = 12, 256, 20, 74260


class Mlp:
    """A warm-start network on the handle's device (see agf2_mlp_* in the
    header). Parameters move in and out as float32 numpy arrays."""

    def __init__(self, h: Handle, params=None):
        self.h = h
        p = _P()
        h._check(h.lib.agf2_mlp_create(h.h, ctypes.byref(p)))
        self.p = p
        if params is not None:
            self.set_params(params)

    def set_params(self, params):
        import numpy as np
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.shape != (MLP_NPARAM,):
            raise ValueError(f"parameters must have shape ({MLP_NPARAM},)")
        self.h._check(self.h.lib.agf2_mlp_set_params(self.h.h, self.p, a.ctypes.data))

    def get_params(self):
        import numpy as np
        a = np.empty(MLP_NPARAM, dtype=np.float32)
        self.h._check(self.h.lib.agf2_mlp_get_params(self.h.h, self.p, a.ctypes.data))
        return a

    def get_grad(self):
        import numpy as np
        a = np.empty(MLP_NPARAM, dtype=np.float32)
        self.h._check(self.h.lib.agf2_mlp_get_grad(self.h.h, self.p, a.ctypes.data))
        return a

    def close(self):
        if getattr(self, "p", None):
            self.h.lib.agf2_mlp_destroy(self.p)
            self.p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def agf2_mlp_features(h: Handle, e_mf, nocc: int, m0):
    """(X float32 [N, 12], scale float64 [4]) of one system; m0 [4, N, N]."""
    N = e_mf.shape[0]
    X = torch.empty(N, MLP_FEATURES, dtype=torch.float32, device=h.device)
    s = h.empty(4)
    h._check(h.lib.agf2_mlp_features(h.h, N, nocc, _ptr(e_mf, "e_mf", h.device),
                                     _ptr(m0, "m0", h.device), _ptr32(X, "X", h.device),
                                     _ptr(s, "scale", h.device)))
    return X, s


def agf2_mlp_forward(h: Handle, net: Mlp, X, Y=None):
    rows = X.shape[0]
    if Y is None:
        Y = torch.empty(rows, MLP_OUTPUTS, dtype=torch.float32, device=h.device)
    h._check(h.lib.agf2_mlp_forward(h.h, net.p, rows, _ptr32(X, "X", h.device),
                                    _ptr32(Y, "Y", h.device)))
    return Y


def agf2_mlp_loss_grad(h: Handle, Y, m0, mconv, scale, dY=None, loss=None):
    """dY of one system; adds its loss into the device scalar `loss`."""
    N = Y.shape[0]
    if dY is None:
        dY = torch.empty_like(Y)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float64, device=h.device)
    h._check(h.lib.agf2_mlp_loss_grad(h.h, N, _ptr32(Y, "Y", h.device),
                                      _ptr(m0, "m0", h.device), _ptr(mconv, "mconv", h.device),
                                      _ptr(scale, "scale", h.device), _ptr32(dY, "dY", h.device),
                                      _ptr(loss, "loss", h.device)))
    return dY, loss


def agf2_mlp_backward(h: Handle, net: Mlp, dY):
    h._check(h.lib.agf2_mlp_backward(h.h, net.p, dY.shape[0], _ptr32(dY, "dY", h.device)))


def agf2_mlp_adam_step(h: Handle, net: Mlp, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    h._check(h.lib.agf2_mlp_adam_step(h.h, net.p, lr, beta1, beta2, eps))


def agf2_mlp_predict_correction(h: Handle, net: Mlp, e_mf, nocc: int, m0, out=None):
    """Delta U [4, N, N] for agf2_run's dm_init."""
    N = e_mf.shape[0]
    if out is None:
        out = h.empty(4, N, N)
    h._check(h.lib.agf2_mlp_predict_correction(h.h, net.p, N, nocc, _ptr(e_mf, "e_mf", h.device),
                                               _ptr(m0, "m0", h.device),
                                               _ptr(out, "dm", h.device)))
    return out
