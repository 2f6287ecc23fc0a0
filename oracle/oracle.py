"""ctypes wrapper around ``libctmhd_oracle.so``.  TEST INFRASTRUCTURE ONLY.

The library is a plain scalar FP64 implementation of one second-order CT-MHD
step (RK2-SSP with first-order flux correction), written from the paper's
Sec. 2; see ``ctmhd_oracle.cpp`` for the per-function citations and the
readings taken where the paper is silent.

Array conventions (shared with the tests, not with the GPU path): ``cons`` is
``(5, n2, n1, n0)`` = (rho, m0, m1, m2, e_tot) and ``bface`` is
``(3, n2, n1, n0)`` = b_a on the lower x_a face of each cell, float64,
interior cells only (periodic box).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ctmhd_oracle.cpp")
LIB = os.environ.get("CTMHD_ORACLE_LIB", os.path.join(_HERE, "libctmhd_oracle.so"))

RECON = {"pc": 0, "plm": 1, "plm_mc": 1, "plm_minmod": 2, "ppm": 3}
RIEMANN = {"hlld": 0, "llf": 1}
EMF = {"q26": 0, "b25a": 1, "fs18": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no FMA contraction)."""
    if force or not os.path.exists(LIB):
        subprocess.check_call([
            "g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
            "-o", LIB, SRC])
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("eta", ctypes.c_double),
                ("cfl", ctypes.c_double), ("recon", ctypes.c_int),
                ("riemann", ctypes.c_int), ("emf", ctypes.c_int),
                ("fofc", ctypes.c_int), ("flag_mask", ctypes.c_int),
                ("pad_", ctypes.c_int)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)
_up = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER(_Params)
        L.oracle_step.argtypes = [P, _ip, _dp, _dp, _dp, ctypes.c_int, _dp, _dp, _lp, _up]
        L.oracle_step_dual.argtypes = [P, _ip, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, _dp]
        L.oracle_count_step.argtypes = [P, _ip, _dp, _dp, _dp, _lp, _lp]
        L.oracle_recon1d.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        L.oracle_hlld.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
        L.oracle_hlld_fan.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_llf.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_llf.restype = ctypes.c_double
        L.oracle_hll.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_double, _dp]
        L.oracle_fast_speed.argtypes = [ctypes.c_double] * 6
        L.oracle_fast_speed.restype = ctypes.c_double
        L.oracle_dt.argtypes = [P, _ip, _dp, _dp, _dp]
        L.oracle_dt.restype = ctypes.c_double
        L.oracle_fluxes.argtypes = [P, _ip, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp]
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only; the
    results do not depend on it)."""
    lib().oracle_set_threads(int(n))


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def make_params(gamma=5.0 / 3.0, eta=0.0, cfl=0.3, recon="plm", riemann="hlld", emf="q26",
                fofc=True, flag_mask=7) -> _Params:
    return _Params(float(gamma), float(eta), float(cfl), RECON[recon], RIEMANN[riemann],
                   EMF[emf], int(bool(fofc)), int(flag_mask), 0)


def _params(p):
    if isinstance(p, _Params):
        return p
    return make_params(**p)


def _dims(cons):
    n2, n1, n0 = cons.shape[1:]
    return (ctypes.c_int * 3)(n0, n1, n2)


def step(params, cons, bface, dx, nsteps=1, dt_fixed=None, force=None):
    """Advance ``nsteps``.  Returns (cons, bface, dts, diag) as new arrays.

    diag = [flagged cells stage 1, flagged cells stage 2, HLL fallbacks,
    non-finite dt].  ``force`` is an optional (2, n2, n1, n0) uint8 mask
    OR-ed into the FOFC flags of each stage of every step.
    """
    P = _params(params)
    c = np.ascontiguousarray(cons, dtype=np.float64).copy()
    b = np.ascontiguousarray(bface, dtype=np.float64).copy()
    dxa = (ctypes.c_double * 3)(*[float(v) for v in dx])
    dts = np.zeros(nsteps, np.float64)
    diag = np.zeros(4, np.int64)
    dtf = None
    if dt_fixed is not None:
        dtf = np.ascontiguousarray(np.broadcast_to(np.asarray(dt_fixed, np.float64), (nsteps,)))
    fm = None
    if force is not None:
        fm = np.ascontiguousarray(force, dtype=np.uint8)
        assert fm.shape == (2,) + c.shape[1:]
    lib().oracle_step(ctypes.byref(P), _dims(c), dxa, _ptr(c), _ptr(b), int(nsteps),
                      _ptr(dtf) if dtf is not None else None, _ptr(dts), _ptr(diag, _lp),
                      _ptr(fm, _up) if fm is not None else None)
    return c, b, dts, diag


def step_dual(params, cons, bface, tcons, tbface, dx, dts):
    """Forward-mode derivative through len(dts) steps with frozen dt values.

    Returns (cons, bface, tcons, tbface) after the steps."""
    P = _params(params)
    c = np.ascontiguousarray(cons, dtype=np.float64).copy()
    b = np.ascontiguousarray(bface, dtype=np.float64).copy()
    tc = np.ascontiguousarray(tcons, dtype=np.float64).copy()
    tb = np.ascontiguousarray(tbface, dtype=np.float64).copy()
    d = np.ascontiguousarray(np.asarray(dts, np.float64))
    dxa = (ctypes.c_double * 3)(*[float(v) for v in dx])
    lib().oracle_step_dual(ctypes.byref(P), _dims(c), dxa, _ptr(c), _ptr(b), _ptr(tc),
                           _ptr(tb), len(d), _ptr(d))
    return c, b, tc, tb


PHASES = ("dt", "prim", "face", "emf", "update", "fofc", "recon")
OPS = ("add", "mul", "div", "sqrt", "cmp")


def count_step(params, cons, bface, dx):
    """Arithmetic of one step, as a dict phase -> dict op -> count (whole box),
    plus "recon_calls": the number of 1D reconstructions performed."""
    P = _params(params)
    c = np.ascontiguousarray(cons, dtype=np.float64)
    b = np.ascontiguousarray(bface, dtype=np.float64)
    out = np.zeros((len(PHASES), len(OPS)), np.int64)
    dxa = (ctypes.c_double * 3)(*[float(v) for v in dx])
    calls = np.zeros(1, np.int64)
    lib().oracle_count_step(ctypes.byref(P), _dims(c), dxa, _ptr(c), _ptr(b), _ptr(out, _lp),
                            _ptr(calls, _lp))
    res = {ph: {op: int(out[i, j]) for j, op in enumerate(OPS)} for i, ph in enumerate(PHASES)}
    res["recon_calls"] = int(calls[0])
    return res


def recon1d(method, q5):
    q = np.ascontiguousarray(q5, np.float64)
    qm = ctypes.c_double()
    qp = ctypes.c_double()
    lib().oracle_recon1d(RECON[method], _ptr(q), ctypes.byref(qm), ctypes.byref(qp))
    return qm.value, qp.value


def hlld(L, R, bn, gamma):
    """Face-local states (rho, un, ut1, ut2, p, bt1, bt2).  Returns (F, SL, SR, fallback)."""
    a = np.ascontiguousarray(L, np.float64)
    b = np.ascontiguousarray(R, np.float64)
    F = np.zeros(5)
    SL = ctypes.c_double()
    SR = ctypes.c_double()
    fb = lib().oracle_hlld(_ptr(a), _ptr(b), float(bn), float(gamma), _ptr(F),
                           ctypes.byref(SL), ctypes.byref(SR))
    return F, SL.value, SR.value, fb


def hlld_fan(L, R, bn, gamma):
    """Subsonic HLLD wave fan: (speeds dict, states (4, 7)) with the states
    U*_L, U**_L, U**_R, U*_R as (rho, u_n, u_t1, u_t2, b_t1, b_t2, e_tot)."""
    a = np.ascontiguousarray(L, np.float64)
    b = np.ascontiguousarray(R, np.float64)
    fan = np.full(34, np.nan)
    fb = lib().oracle_hlld_fan(_ptr(a), _ptr(b), float(bn), float(gamma), _ptr(fan))
    names = ("SL", "SM", "SR", "SsL", "SsR", "pTs")
    return {k: fan[i] for i, k in enumerate(names)}, fan[6:].reshape(4, 7), fb


def llf(L, R, bn, gamma):
    a = np.ascontiguousarray(L, np.float64)
    b = np.ascontiguousarray(R, np.float64)
    F = np.zeros(5)
    s = lib().oracle_llf(_ptr(a), _ptr(b), float(bn), float(gamma), _ptr(F))
    return F, s


def hll(L, R, bn, gamma):
    a = np.ascontiguousarray(L, np.float64)
    b = np.ascontiguousarray(R, np.float64)
    F = np.zeros(5)
    lib().oracle_hll(_ptr(a), _ptr(b), float(bn), float(gamma), _ptr(F))
    return F


def fast_speed(rho, p, bn, bt1, bt2, gamma):
    return lib().oracle_fast_speed(rho, p, bn, bt1, bt2, gamma)


def cfl_dt(params, cons, bface, dx):
    P = _params(params)
    c = np.ascontiguousarray(cons, dtype=np.float64)
    b = np.ascontiguousarray(bface, dtype=np.float64)
    dxa = (ctypes.c_double * 3)(*[float(v) for v in dx])
    return lib().oracle_dt(ctypes.byref(P), _dims(c), dxa, _ptr(c), _ptr(b))


def fluxes(params, cons, bface, dx, recon=None, riemann=None):
    """Face fluxes (3, 5, n2, n1, n0) and edge EMFs (3, n2, n1, n0) of one state."""
    P = _params(params)
    c = np.ascontiguousarray(cons, dtype=np.float64)
    b = np.ascontiguousarray(bface, dtype=np.float64)
    F = np.zeros((3, 5) + c.shape[1:])
    E = np.zeros((3,) + c.shape[1:])
    dxa = (ctypes.c_double * 3)(*[float(v) for v in dx])
    r = P.recon if recon is None else RECON[recon]
    s = P.riemann if riemann is None else RIEMANN[riemann]
    nfb = lib().oracle_fluxes(ctypes.byref(P), _dims(c), dxa, _ptr(c), _ptr(b), r, s,
                              _ptr(F), _ptr(E))
    return F, E, nfb
