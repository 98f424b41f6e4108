"""CPU oracle for the Kuramoto model on graphs -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct FP64 implementation of what the GPU library computes, written
from the paper (Boehle, Kuehn, Thalhammer, arXiv 2102.07167) and pinned by the tests in
``tests/test_oracle_pins.py``. Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it. It shares no code with the library in
``paper_2102_07167_amd``; the only module both sides use is the input generator ``gen``.

Functions (all FP64; graphs are ``gen.Graph`` objects in user order):
  rhs(graph, omega, K, theta)            Sec. 3 eq. KuramotoGraph, straightforward summation
  rhs_rows(graph, omega, K, theta, rows) the same on a subset of rows
  rk4(graph, omega, K, theta0, dt, n)    classical RK4, unwrapped phases, r(t) sampling
  midpoint(graph, omega, K, theta0, dt, n, iters)  implicit midpoint rule, fixed-point iterations
  rkf45(graph, omega, K, theta0, t_end, dt0, atol)  variable-step embedded RK pair of orders 4(5)
  order_parameter(theta)                 Sec. 2 eq. OrderParameter
  vjp(graph, K, theta, lam)              J(theta)^T lam
  adjoint_rk4(...)                       discrete adjoint of ``rk4``
  potential(graph, omega, K, theta)      Sec. 3 eq. ExtendedPotentialConservation
  loss_and_seed(theta_T, target)         (1 - r)^2 + (1/N) sum 2 (1 - cos(theta - target))
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libkur_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile kur_oracle.c with gcc -O2 -fopenmp (no fast-math: plain IEEE double)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp,
                               os.path.join(_HERE, "kur_oracle.c"), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P, i64, f64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        lib.orc_rhs.restype = None
        lib.orc_rhs.argtypes = [i64, ci, P, P, P, ci, P, f64, P, P]
        lib.orc_rhs_rows.restype = None
        lib.orc_rhs_rows.argtypes = [i64, ci, P, P, P, ci, P, f64, P, i64, P, P]
        lib.orc_order_parameter.restype = None
        lib.orc_order_parameter.argtypes = [i64, P, P, P]
        lib.orc_rk4.restype = ci
        lib.orc_rk4.argtypes = [i64, ci, P, P, P, ci, P, f64, f64, i64, i64, P, P, P]
        lib.orc_rkf45.restype = ci
        lib.orc_rkf45.argtypes = [i64, ci, P, P, P, ci, P, f64, f64, f64, f64, i64, P, P]
        lib.orc_rkf45_tableau.restype = None
        lib.orc_rkf45_tableau.argtypes = [P, P, P]
        lib.orc_midpoint.restype = ci
        lib.orc_midpoint.argtypes = [i64, ci, P, P, P, ci, P, f64, f64, i64, ctypes.c_int32, i64, P, P, P]
        lib.orc_vjp.restype = None
        lib.orc_vjp.argtypes = [i64, ci, P, P, P, ci, f64, P, P, P]
        lib.orc_adjoint_rk4.restype = ci
        lib.orc_adjoint_rk4.argtypes = [i64, ci, P, P, P, ci, P, f64, f64, i64, P, P, P, P, P]
        lib.orc_potential.restype = f64
        lib.orc_potential.argtypes = [i64, ci, P, P, P, ci, P, f64, P]
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ci
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _g(graph):
    if graph.complete:
        return graph.n, 1, None, None, None
    w = getattr(graph, "weight", None)
    return graph.n, 0, _p(graph.row_ptr), _p(graph.col), None if w is None else _p(w)


def rhs(graph, omega, K, theta, scaling: int = 0) -> np.ndarray:
    """F_m = omega_m + K/Mscale_m sum_{A_ml=1} sin(theta_l - theta_m) (Sec. 3, eq. KuramotoGraph;
    scaling 0: Mscale = N, 1: Mscale = row degree)."""
    omega, theta = _f64(omega), _f64(theta)
    out = np.empty(graph.n)
    _load().orc_rhs(*_g(graph), scaling, _p(omega), float(K), _p(theta), _p(out))
    return out


def rhs_rows(graph, omega, K, theta, rows, scaling: int = 0) -> np.ndarray:
    omega, theta = _f64(omega), _f64(theta)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(len(rows))
    _load().orc_rhs_rows(*_g(graph), scaling, _p(omega), float(K), _p(theta), len(rows), _p(rows), _p(out))
    return out


def order_parameter(theta):
    """(r, psi) with r e^{i psi} = (1/N) sum_m e^{i theta_m} (Sec. 2, eq. OrderParameter)."""
    theta = _f64(theta)
    r, psi = ctypes.c_double(), ctypes.c_double()
    _load().orc_order_parameter(len(theta), _p(theta), ctypes.byref(r), ctypes.byref(psi))
    return r.value, psi.value


def rk4(graph, omega, K, theta0, dt, nsteps, r_every: int = 0, scaling: int = 0):
    """Classical RK4 with fixed step on unwrapped phases. Returns (theta(T), r, psi) where r/psi
    hold the samples at steps 0, r_every, ... (empty when r_every == 0)."""
    omega = _f64(omega)
    theta = _f64(theta0).copy()
    nr = nsteps // r_every + 1 if r_every > 0 else 0
    r = np.empty(nr)
    psi = np.empty(nr)
    rc = _load().orc_rk4(*_g(graph), scaling, _p(omega), float(K), float(dt), int(nsteps), int(r_every),
                         _p(theta), _p(r) if nr else None, _p(psi) if nr else None)
    if rc != 0:
        raise MemoryError("oracle rk4")
    return theta, r, psi


def midpoint(graph, omega, K, theta0, dt, nsteps, iters, r_every: int = 0, scaling: int = 0):
    """Implicit midpoint rule by `iters` fixed-point iterations per step on unwrapped phases;
    returns (theta(T), r, psi) as rk4."""
    omega = _f64(omega)
    theta = _f64(theta0).copy()
    nr = nsteps // r_every + 1 if r_every > 0 else 0
    r = np.empty(nr)
    psi = np.empty(nr)
    rc = _load().orc_midpoint(*_g(graph), scaling, _p(omega), float(K), float(dt), int(nsteps), int(iters),
                              int(r_every), _p(theta), _p(r) if nr else None, _p(psi) if nr else None)
    if rc != 0:
        raise MemoryError("oracle midpoint")
    return theta, r, psi


def rkf45(graph, omega, K, theta0, t_end, dt0, atol, max_steps: int = 1000000, scaling: int = 0):
    """Variable-step embedded RK pair of orders 4(5) over [0, t_end]; returns (theta(T), stats)
    with stats = (t reached, next dt, accepted, rejected)."""
    omega = _f64(omega)
    theta = _f64(theta0).copy()
    stats = np.zeros(4)
    rc = _load().orc_rkf45(*_g(graph), scaling, _p(omega), float(K), float(t_end), float(dt0), float(atol),
                           int(max_steps), _p(theta), _p(stats))
    if rc != 0:
        raise ArithmeticError("oracle rkf45 failed (%d)" % rc)
    return theta, stats


def rkf45_tableau():
    """(a 6x6, b4, b5) of the oracle's embedded pair."""
    a, b4, b5 = np.zeros(36), np.zeros(6), np.zeros(6)
    _load().orc_rkf45_tableau(_p(a), _p(b4), _p(b5))
    return a.reshape(6, 6), b4, b5


def vjp(graph, K, theta, lam, scaling: int = 0) -> np.ndarray:
    theta, lam = _f64(theta), _f64(lam)
    out = np.empty(graph.n)
    _load().orc_vjp(*_g(graph), scaling, float(K), _p(theta), _p(lam), _p(out))
    return out


def adjoint_rk4(graph, omega, K, theta0, dt, nsteps, dl_dthetaT, scaling: int = 0):
    """Discrete adjoint of ``rk4``: returns (dL/dtheta0, dL/domega, dL/dK)."""
    omega, theta0, lam = _f64(omega), _f64(theta0), _f64(dl_dthetaT)
    gt = np.empty(graph.n)
    gw = np.empty(graph.n)
    gk = ctypes.c_double()
    rc = _load().orc_adjoint_rk4(*_g(graph), scaling, _p(omega), float(K), float(dt), int(nsteps),
                                 _p(theta0), _p(lam), _p(gt), _p(gw), ctypes.byref(gk))
    if rc != 0:
        raise MemoryError("oracle adjoint")
    return gt, gw, gk.value


def potential(graph, omega, K, theta, scaling: int = 0) -> float:
    omega, theta = _f64(omega), _f64(theta)
    return _load().orc_potential(*_g(graph), scaling, _p(omega), float(K), _p(theta))


def threads() -> int:
    """Threads the oracle's parallel row loops run on (OpenMP)."""
    return int(_load().orc_threads())


def loss_and_seed(theta_T, target):
    """L = (1 - r)^2 + (1/N) sum_m 2 (1 - cos(theta_m - target_m)) at the final phases, and
    dL/dtheta_m = -2 (1 - r) sin(psi - theta_m)/N + 2 sin(theta_m - target_m)/N
    (the derivative of r is taken as 0 when r == 0)."""
    theta_T, target = _f64(theta_T), _f64(target)
    n = len(theta_T)
    c = math.fsum(np.cos(theta_T)) / n
    s = math.fsum(np.sin(theta_T)) / n
    r = math.hypot(c, s)
    psi = math.atan2(s, c)
    L = (1.0 - r) ** 2 + 2.0 * math.fsum(1.0 - np.cos(theta_T - target)) / n
    dr = np.sin(psi - theta_T) / n if r > 0 else np.zeros(n)
    seed = -2.0 * (1.0 - r) * dr + 2.0 * np.sin(theta_T - target) / n
    return L, seed
