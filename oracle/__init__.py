"""FP64 CPU oracle of the entropic anisotropic ADE lattice Boltzmann scheme.

TEST INFRASTRUCTURE ONLY: the independent, plain reference implementation (C++, FP64) that
the GPU library is checked against. Only tests/, the smoke check and the CPU-baseline leg of
bench.py may import it; the product path never does. It shares no code with the GPU library.

Functions here are argument marshalling around oracle/elbm_oracle.cpp plus the closed-form
pins in oracle/symbol.py. Populations use the oracle's own velocity order (velocities()).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

# Default ghost floor of the FP64 reference (the same reading the GPU path uses in FP64). At
# a node whose ghost part is at rounding level h ~ 1e-16 phi (an equilibrium start), the
# floor turns the closed-form amplitude into (lambda - 1) h ~ |ln E| (h / tau)^2 phi; with
# tau = 1e-9 that is ~1e-14 of phi, with 1e-10 it reaches 1e-12 at |u| ~ 0.14.
TAU64 = 1e-9


class Params(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("bc_x", ctypes.c_int32), ("d_uniform", ctypes.c_int32),
        ("u_uniform", ctypes.c_int32), ("r_mode", ctypes.c_int32),
        ("tensor_is_log", ctypes.c_int32), ("nthreads", ctypes.c_int32),
        ("phi_lo", ctypes.c_double), ("phi_hi", ctypes.c_double),
        ("eps", ctypes.c_double), ("tau", ctypes.c_double), ("root_rho", ctypes.c_double),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_velocities.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), dp]
        L.oracle_s_from_d.argtypes = [dp, dp]
        L.oracle_expm_sym.argtypes = [dp, dp]
        L.oracle_collide.argtypes = [ctypes.POINTER(Params), ctypes.c_int64, dp, dp, dp, dp, dp]
        L.oracle_run.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp, ctypes.c_int32, dp, dp,
                                 ctypes.POINTER(ctypes.c_int64)]
        L.oracle_run_tangent.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp, dp, dp,
                                         ctypes.c_int32]
        L.oracle_moments.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp, dp, dp]
        L.oracle_init_equilibrium.argtypes = [ctypes.POINTER(Params), dp, dp, dp, dp]
        _LIB = L
    return _LIB


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def velocities(q: int = 19):
    """(c[q][3] int, W[q]) in the oracle's order."""
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    rc = lib().oracle_velocities(q, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(w))
    assert rc == q
    return c.astype(np.int64), w


def s_from_d(d6) -> np.ndarray:
    d = _f64(d6)
    s = np.zeros(9)
    lib().oracle_s_from_d(_p(d), _p(s))
    return s.reshape(3, 3)


def expm_sym(l6) -> np.ndarray:
    l = _f64(l6)
    d = np.zeros(6)
    lib().oracle_expm_sym(_p(l), _p(d))
    return d


def make_params(prob=None, *, q=19, shape=(1, 1, 1), bc_x="periodic", phi_lo=0.0, phi_hi=0.0,
                eps=0.0, tau=0.0, root_rho=-1.0, d_uniform=True, u_uniform=True, r_mode=0,
                tensor_is_log=False, nthreads=0) -> Params:
    """Params from a Problem (inputs.Problem) or from keywords. shape = (nx, ny, nz)."""
    if prob is not None:
        shape = (prob.nx, prob.ny, prob.nz)
        bc_x, phi_lo, phi_hi = prob.bc_x, prob.phi_lo, prob.phi_hi
        eps = prob.eps
        d_uniform, u_uniform = prob.d_uniform, prob.u_uniform
        r_mode = 0 if prob.r is None else (1 if np.ndim(prob.r) == 0 else 2)
        tensor_is_log = prob.tensor_is_log
    p = Params()
    p.q = q
    p.nx, p.ny, p.nz = (int(v) for v in shape)
    p.bc_x = {"periodic": 0, "dirichlet": 1}[bc_x]
    p.d_uniform, p.u_uniform, p.r_mode = int(d_uniform), int(u_uniform), int(r_mode)
    p.tensor_is_log = int(tensor_is_log)
    p.nthreads = int(nthreads)
    p.phi_lo, p.phi_hi, p.eps, p.tau, p.root_rho = phi_lo, phi_hi, eps, tau, root_rho
    return p


def _r_array(prob):
    if prob.r is None:
        return None
    return _f64(np.atleast_1d(prob.r))


def init_equilibrium(prob, q: int = 19, j0=None) -> np.ndarray:
    """f = g_eq(phi0, u) (+ P(j0)), shape (q, nz, ny, nx)."""
    p = make_params(prob, q=q)
    f = np.zeros((q, prob.nz, prob.ny, prob.nx))
    rc = lib().oracle_init_equilibrium(ctypes.byref(p), _p(_f64(prob.u)), _p(_f64(prob.phi0)),
                                       _p(None if j0 is None else _f64(j0)), _p(f))
    assert rc == 0
    return f


def run(prob, f: np.ndarray, nsteps: int, *, q: int = 19, tau: float = TAU64,
        root_rho: float = -1.0, nthreads: int = 0, want_last: bool = False):
    """Advance a copy of f by nsteps. Returns f_new (and lambda/alpha of the last step and
    the counters {alpha<1 nodes, flagged nodes} if want_last)."""
    p = make_params(prob, q=q, tau=tau, root_rho=root_rho, nthreads=nthreads)
    p.tau, p.root_rho, p.nthreads = tau, root_rho, nthreads
    out = _f64(f).copy()
    lam = np.zeros((prob.nz, prob.ny, prob.nx)) if want_last else None
    alp = np.zeros((prob.nz, prob.ny, prob.nx)) if want_last else None
    cnt = (ctypes.c_int64 * 2)()
    rc = lib().oracle_run(ctypes.byref(p), _p(_f64(prob.d6)), _p(_f64(prob.u)),
                          _p(_r_array(prob)), _p(out), int(nsteps), _p(lam), _p(alp), cnt)
    assert rc == 0
    if want_last:
        return out, lam, alp, (cnt[0], cnt[1])
    return out


def run_tangent(prob, f: np.ndarray, df: Optional[np.ndarray], dd6: Optional[np.ndarray],
                nsteps: int, *, q: int = 19, tau: float = TAU64, nthreads: int = 0):
    """Forward-mode derivative: returns (f_N, df_N) for the tangent (df, dd6)."""
    p = make_params(prob, q=q, tau=tau, nthreads=nthreads)
    p.tau = tau
    out = _f64(f).copy()
    dout = np.zeros_like(out) if df is None else _f64(df).copy()
    rc = lib().oracle_run_tangent(ctypes.byref(p), _p(_f64(prob.d6)),
                                  _p(None if dd6 is None else _f64(dd6)), _p(_f64(prob.u)),
                                  _p(_r_array(prob)), _p(out), _p(dout), int(nsteps))
    assert rc == 0
    return out, dout


def moments(prob, f: np.ndarray, q: int = 19):
    """(phi, j, q_flux) at the current time, shapes (nz,ny,nx), (3,nz,ny,nx), (3,nz,ny,nx)."""
    p = make_params(prob, q=q)
    n3 = (prob.nz, prob.ny, prob.nx)
    phi = np.zeros(n3)
    j = np.zeros((3,) + n3)
    qf = np.zeros((3,) + n3)
    rc = lib().oracle_moments(ctypes.byref(p), _p(_f64(prob.d6)), _p(_f64(prob.u)), _p(_f64(f)),
                              _p(phi), _p(j), _p(qf))
    assert rc == 0
    return phi, j, qf


def collide(g: np.ndarray, d6, u, *, q: int = 19, eps: float = 0.0, tau: float = TAU64,
            root_rho: float = -1.0, tensor_is_log: bool = False):
    """Collide m independent nodes: g (m, q); d6 (6,) or (m, 6); u (3,) or (m, 3).
    Returns (post (m, q), info (m, 4) = lambda used, closed-form lambda, alpha, flagged)."""
    g = _f64(np.atleast_2d(g))
    m = g.shape[0]
    d6 = _f64(d6)
    u = _f64(u)
    p = make_params(q=q, eps=eps, tau=tau, root_rho=root_rho, d_uniform=(d6.ndim == 1),
                    u_uniform=(u.ndim == 1), tensor_is_log=tensor_is_log)
    out = np.zeros_like(g)
    info = np.zeros((m, 4))
    rc = lib().oracle_collide(ctypes.byref(p), m, _p(g), _p(d6), _p(u), _p(out), _p(info))
    assert rc == 0
    return out, info
