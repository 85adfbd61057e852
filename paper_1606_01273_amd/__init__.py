"""MI355X-native hot path of internally contracted (X)MS-CASPT2.

Python front end over the C ABI in include/caspt2.h.  PyTorch provides device
memory and streams only; every arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib
from ._lib import (E_ARG, E_DEVICE, E_INDEFINITE, E_NOCONV, E_NOMEM, E_NOTIMPL, E_STATE, ENTRY_NAMES,
                   FP64, MIXED, MSMR, OK, SSSR, Caspt2Error)

__all__ = ["Caspt2", "Caspt2Error", "batch_solve", "residual_all_many", "xms_rotate", "lib", "MSMR", "SSSR", "FP64",
           "MIXED", "ENTRY_NAMES"]

_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _lib.load()
    return _LIB


def _ptr(t) -> int:
    return int(t.data_ptr())


def _marshal(nclosed, nact, nvirt, naux, nstates, nelec, fock, hcore, dfB, ci, eref, shift, scheme, xms, thresh,
             precision):
    """caspt2_dims and caspt2_inputs of one problem, and the host arrays the
    inputs point to (to be kept alive until the creation returns)."""
    d = _lib.Dims(nclosed, nact, nvirt, naux, nstates, nelec, scheme, 1 if xms else 0, int(precision), 0,
                  float(shift), float(thresh))
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (fock, hcore, dfB, ci, eref)]
    return d, _lib.Inputs(*[a.ctypes.data for a in arrs]), arrs


def _check(rc: int, where: str, allow=(OK,)):
    if rc not in allow:
        L = lib()
        raise Caspt2Error(rc, where, f"{L.caspt2_strerror(rc).decode()}: {L.caspt2_last_error().decode()}")
    return rc


class Caspt2:
    """One problem on the current HIP device (device memory held by the
    library handle).  Host numpy inputs are copied at creation."""

    def __init__(self, nclosed, nact, nvirt, naux, nstates, nelec, fock, hcore, dfB, ci, eref,
                 shift=0.0, scheme=MSMR, xms=True, thresh=1e-9, precision=FP64, stream=None):
        import torch
        L = lib()
        d, inp, keep = _marshal(nclosed, nact, nvirt, naux, nstates, nelec, fock, hcore, dfB, ci, eref,
                                shift, scheme, xms, thresh, precision)
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(L.caspt2_create(ctypes.byref(d), ctypes.byref(inp), 0, ctypes.c_void_p(stream.cuda_stream),
                               ctypes.byref(h)), "caspt2_create")
        del keep
        self._attach(h, nstates, nclosed, nact, nvirt, stream)

    def _attach(self, h, nstates, nclosed, nact, nvirt, stream):
        self.nst = nstates
        self.nc, self.na, self.nv = nclosed, nact, nvirt
        self.nmo = nclosed + nact + nvirt
        self._stream = stream
        self._h = h
        self.length = int(lib().caspt2_vector_length(h))

    @classmethod
    def from_problem(cls, prob, scheme=MSMR, xms=True, thresh=1e-9, **kw):
        return cls(prob.nc, prob.na, prob.nv, prob.naux, prob.nst, prob.nelec, prob.fock, prob.hcore,
                   prob.B, prob.ci, prob.eref, shift=prob.shift, scheme=scheme, xms=xms,
                   thresh=thresh, **kw)

    @classmethod
    def create_many(cls, probs, threads=8, streams=None, scheme=MSMR, xms=True, thresh=1e-9, precision=FP64):
        """Set up every problem of probs (objects with the fields from_problem
        reads) with caspt2_create_many, `threads` creations at a time on the
        library's host threads; problem k runs on streams[k] (default: one new
        stream per thread, assigned round-robin).  Returns the handles in
        order; raises on the first failed problem (the others are released)."""
        import torch
        L = lib()
        n = len(probs)
        if n == 0:
            return []
        if streams is None:
            pool = [torch.cuda.Stream() for _ in range(max(1, min(threads, n)))]
            streams = [pool[k % len(pool)] for k in range(n)]
        ds = (_lib.Dims * n)()
        ins = (_lib.Inputs * n)()
        keep = []
        for k, p in enumerate(probs):
            d, inp, kp = _marshal(p.nc, p.na, p.nv, p.naux, p.nst, p.nelec, p.fock, p.hcore, p.B, p.ci, p.eref,
                                  p.shift, scheme, xms, thresh, precision)
            ds[k], ins[k] = d, inp
            keep.append(kp)
        sp = (ctypes.c_void_p * n)(*[s.cuda_stream for s in streams])
        hs = (ctypes.c_void_p * n)()
        st = (ctypes.c_int32 * n)()
        rc = L.caspt2_create_many(n, ds, ins, 0, sp, int(threads), hs, st)
        del keep
        if rc != OK:
            for k in range(n):
                if hs[k]:
                    L.caspt2_destroy(ctypes.c_void_p(hs[k]))
            _check(rc, "caspt2_create_many")
        out = []
        for k, p in enumerate(probs):
            g = cls.__new__(cls)
            g._attach(ctypes.c_void_p(hs[k]), p.nst, p.nc, p.na, p.nv, streams[k])
            out.append(g)
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().caspt2_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self):
        out = []
        for k in range(len(ENTRY_NAMES)):
            o, r, a = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            _check(lib().caspt2_layout(self._h, k, ctypes.byref(o), ctypes.byref(r), ctypes.byref(a)),
                   "caspt2_layout")
            out.append((ENTRY_NAMES[k], o.value, r.value, a.value))
        return out

    def set_streams(self, n):
        _check(lib().caspt2_set_streams(self._h, int(n)), "caspt2_set_streams")

    def set_precision(self, precision):
        _check(lib().caspt2_set_precision(self._h, int(precision)), "caspt2_set_precision")

    def autotune(self, cache_path=None, force=False):
        """Time the launch candidates of every residual entry and keep the
        fastest; returns {entry name: (splitk, order, grid, tile, kb, occ, plain, breg, rule_ms, tuned_ms)}."""
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().caspt2_autotune(self._h, path, 1 if force else 0), "caspt2_autotune")
        out = {}
        for k, name in enumerate(ENTRY_NAMES):
            c = (ctypes.c_int32 * 8)()
            r, t = ctypes.c_double(), ctypes.c_double()
            _check(lib().caspt2_tune_entry(self._h, k, c, ctypes.byref(r), ctypes.byref(t)), "caspt2_tune_entry")
            out[name] = (c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], r.value, t.value)
        return out

    def profile(self, enable=True):
        _check(lib().caspt2_profile(self._h, 1 if enable else 0), "caspt2_profile")

    def profile_entry(self, k):
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().caspt2_profile_entry(self._h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)),
               "caspt2_profile_entry")
        return ms.value, n.value, b.value

    def profile_stages(self):
        """{stage name: ms per residual evaluation} of the Fock couplings
        timed while profiling was on."""
        out = {}
        k = 0
        while True:
            buf = ctypes.create_string_buffer(64)
            ms, n = ctypes.c_double(), ctypes.c_int64()
            if lib().caspt2_profile_stage(self._h, k, buf, 64, ctypes.byref(ms), ctypes.byref(n)) != OK:
                break
            out[buf.value.decode()] = ms.value
            k += 1
        return out

    def residual(self, L, x, sigma, with_source=True):
        _check(lib().caspt2_residual(self._h, L, 1 if with_source else 0, _ptr(x), _ptr(sigma)),
               "caspt2_residual")

    def residual_all(self, x, sigma, with_source=True):
        _check(lib().caspt2_residual_all(self._h, 1 if with_source else 0, _ptr(x), _ptr(sigma)),
               "caspt2_residual_all")

    def solve_amplitudes(self, tol=1e-10, maxiter=200, T0=None):
        """T0: optional device tensor [nst][length] of starting amplitudes."""
        info = (_lib.Info * self.nst)()
        p0 = None if T0 is None else _ptr(T0)
        rc = _check(lib().caspt2_solve_amplitudes(self._h, tol, maxiter, p0, info),
                    "caspt2_solve_amplitudes", allow=(OK, E_NOCONV))
        return rc, [i.as_dict() for i in info]

    def amplitudes(self, L):
        import torch
        t = torch.empty(self.length, dtype=torch.float64, device="cuda")
        _check(lib().caspt2_get_amplitudes(self._h, L, _ptr(t)), "caspt2_get_amplitudes")
        return t

    def xms_rotate(self):
        """The XMS rotation U and E^(0) the handle applied at creation."""
        U = np.zeros((self.nst, self.nst))
        e0 = np.zeros(self.nst)
        _check(lib().caspt2_get_xms(self._h, U.ctypes.data_as(_lib._D), e0.ctypes.data_as(_lib._D)),
               "caspt2_get_xms")
        return U, e0

    def heff(self):
        n = self.nst
        H, w, R = np.zeros((n, n)), np.zeros(n), np.zeros((n, n))
        _check(lib().xms_heff(self._h, H.ctypes.data_as(_lib._D), w.ctypes.data_as(_lib._D),
                              R.ctypes.data_as(_lib._D)), "xms_heff")
        return H, w, R

    def solve_lambda(self, target=0, tol=1e-10, maxiter=200, lam0=None):
        """lam0: optional device tensor [nst][length] of starting multipliers."""
        info = (_lib.Info * self.nst)()
        p0 = None if lam0 is None else _ptr(lam0)
        rc = _check(lib().caspt2_solve_lambda(self._h, target, tol, maxiter, p0, info),
                    "caspt2_solve_lambda", allow=(OK, E_NOCONV))
        return rc, [i.as_dict() for i in info]

    def densities(self):
        """Correlated densities of the target state of the last lambda solve:
        dict with d1, dbar2, d2 ([nmo][nmo] numpy), NL ([nst]) and D1
        ({(spaces of x, y, z, w): device tensor [x][y][z][w]}, spaces 'c',
        'a', 'v')."""
        import torch
        L = lib()
        nmo = self.nmo
        d1, db, d2 = np.zeros((nmo, nmo)), np.zeros((nmo, nmo)), np.zeros((nmo, nmo))
        NL = np.zeros(self.nst)
        n2 = int(L.caspt2_density2_length(self._h))
        D1 = torch.empty(max(n2, 1), dtype=torch.float64, device="cuda")
        _check(L.caspt2_densities(self._h, d1.ctypes.data_as(_lib._D), _ptr(D1), db.ctypes.data_as(_lib._D),
                                  d2.ctypes.data_as(_lib._D), NL.ctypes.data_as(_lib._D)), "caspt2_densities")
        dims = {"c": self.nc, "a": self.na, "v": self.nv}
        out = {}
        for k in range(15):
            o = ctypes.c_int64()
            sp = (ctypes.c_int32 * 4)()
            _check(L.caspt2_density2_layout(self._h, k, ctypes.byref(o), sp), "caspt2_density2_layout")
            key = tuple("cav"[sp[a]] for a in range(4))
            shape = tuple(dims[c] for c in key)
            n = int(np.prod(shape))
            out[key] = D1[o.value:o.value + n].view(shape)
        return dict(d1=d1, D1=out, dbar2=db, d2=d2, NL=NL)

    def lam(self, L):
        import torch
        t = torch.empty(self.length, dtype=torch.float64, device="cuda")
        _check(lib().caspt2_get_lambda(self._h, L, _ptr(t)), "caspt2_get_lambda")
        return t


def xms_rotate(f_act, rdm1):
    """Standalone XMS rotation (Eqs. 3-5) on the current device: f_act
    [na][na], rdm1 [nst][nst][na][na] = <M|E_rs|N>; returns (U, E~)."""
    f = np.ascontiguousarray(f_act, dtype=np.float64)
    g = np.ascontiguousarray(rdm1, dtype=np.float64)
    nst, na = g.shape[0], f.shape[0]
    U = np.zeros((nst, nst))
    e0 = np.zeros(nst)
    _check(lib().xms_rotate(na, nst, f.ctypes.data_as(_lib._D), g.ctypes.data_as(_lib._D),
                            U.ctypes.data_as(_lib._D), e0.ctypes.data_as(_lib._D)), "xms_rotate")
    return U, e0


def batch_solve(problems, targets=None, tol=1e-10, maxiter=200):
    """caspt2_batch_solve over a list of FP64 Caspt2 objects (distinct).
    Returns (status, amplitude infos, lambda infos), one list per problem;
    results are read afterwards from each object (amplitudes, heff, lam)."""
    n = len(problems)
    if targets is None:
        targets = [0] * n
    hs = (ctypes.c_void_p * n)(*[p._h.value for p in problems])
    tg = (ctypes.c_int32 * n)(*targets)
    tot = sum(p.nst for p in problems)
    ai, li = (_lib.Info * tot)(), (_lib.Info * tot)()
    rc = _check(lib().caspt2_batch_solve(hs, n, tg, tol, maxiter, ai, li), "caspt2_batch_solve",
                allow=(OK, E_NOCONV, E_INDEFINITE))
    out_a, out_l, k = [], [], 0
    for p in problems:
        out_a.append([ai[k + L].as_dict() for L in range(p.nst)])
        out_l.append([li[k + L].as_dict() for L in range(p.nst)])
        k += p.nst
    return rc, out_a, out_l


def residual_all_many(handles, xs, sigmas, with_source=True, threads=8):
    """caspt2_residual_all of every handle (xs[k], sigmas[k]: device tensors
    [nst][length]), `threads` calls at a time on the library's host threads."""
    n = len(handles)
    if n == 0:
        return
    hs = (ctypes.c_void_p * n)(*[g._h.value for g in handles])
    xp = (ctypes.c_void_p * n)(*[_ptr(x) for x in xs])
    sp = (ctypes.c_void_p * n)(*[_ptr(s) for s in sigmas])
    st = (ctypes.c_int32 * n)()
    _check(lib().caspt2_residual_all_many(n, hs, 1 if with_source else 0, xp, sp, int(threads), st),
           "caspt2_residual_all_many")
