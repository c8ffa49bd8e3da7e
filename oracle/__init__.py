"""CPU FP64 oracle for the BSSN right-hand side and the RK4 and RK3 steps.

TEST INFRASTRUCTURE ONLY.  Loaded by the test suite, the smoke check and the
benchmark's CPU-baseline leg; the HIP library and its Python binding never
import it.  The arithmetic lives in ``bssn_oracle.cpp`` (plain C++, g++,
no FP contraction); this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bssn_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

NGF = 24


class _Params(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int32), ("ghost", ctypes.c_int32), ("upwind", ctypes.c_int32),
                ("ko_radius", ctypes.c_int32), ("eps_diss", ctypes.c_double), ("lapse", ctypes.c_int32),
                ("shift", ctypes.c_int32), ("eta", ctypes.c_double), ("bc", ctypes.c_int32),
                ("nthreads", ctypes.c_int32)]


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("ghost", ctypes.c_int32), ("sy", ctypes.c_int64),
                ("sz", ctypes.c_int64), ("sf", ctypes.c_int64), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3)]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", _SRC, "-o", _LIB_PATH + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P, G = ctypes.POINTER(_Params), ctypes.POINTER(_Grid)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_rhs.argtypes = [P, G, dp, dp]
        L.oracle_rk4.argtypes = [P, G, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_rk3.argtypes = [P, G, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_rk4_timed.argtypes = [P, G, ctypes.c_double, ctypes.c_int, dp, dp]
        L.oracle_rk3_ext.argtypes = [P, G, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_enforce_algebraic.argtypes = [P, G, dp]
        L.oracle_momentum.argtypes = [P, G, dp, dp]
        L.oracle_mom_point.argtypes = [dp, dp, dp]
        L.oracle_psi4.argtypes = [P, G, dp, dp]
        pdp = ctypes.POINTER(dp)
        L.oracle_sync_ghosts.argtypes = [P, G, pdp, ctypes.c_int]
        L.oracle_restrict.argtypes = [P, G, pdp, ctypes.c_int]
        L.oracle_steps_synced.argtypes = [P, G, pdp, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.oracle_psi4_point.argtypes = [dp, dp, dp, dp, dp]
        L.oracle_rhs_ext.argtypes = [P, G, dp, dp]
        L.oracle_rk4_ext.argtypes = [P, G, ctypes.c_double, ctypes.c_int, dp]
        L.oracle_fill_periodic.argtypes = [G, dp]
        L.oracle_hamiltonian.argtypes = [P, G, dp, dp]
        L.oracle_rhs_point.argtypes = [P, dp, dp, dp, dp, dp, dp]
        L.oracle_ham_point.argtypes = [dp, dp, dp, dp]
        L.oracle_apply_op.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, G, dp, dp]
        L.oracle_count_rhs_flops.argtypes = [P, G, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_longlong)]
        L.oracle_required_ghost.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(p, nthreads: int = 0) -> _Params:
    return _Params(p.fd_order, p.ghost, p.upwind, p.ko_radius, p.eps_diss, p.lapse, p.shift, p.eta,
                   p.bc, nthreads)


def _grid(g) -> _Grid:
    return _Grid((ctypes.c_int32 * 3)(*g.n), g.ghost, g.sy, g.sz, g.sf, g.h,
                 (ctypes.c_double * 3)(*getattr(g, "origin", (0.0, 0.0, 0.0))))


def _ok(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what}: invalid arguments")


def rhs(params, grid, u: np.ndarray, nthreads: int = 0, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Right-hand side at the interior points, and at the ghost points with the
    radiative boundary (other entries of the result are NaN unless ``out`` is
    given)."""
    out = np.full(grid.shape, np.nan) if out is None else out
    _ok(lib().oracle_rhs(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), _ptr(u),
                         _ptr(out)), "rhs")
    return out


def rk4(params, grid, u: np.ndarray, dt: float, nsteps: int = 1, nthreads: int = 0) -> np.ndarray:
    """Return a copy of u advanced by nsteps classic RK4 steps."""
    v = np.ascontiguousarray(u.copy())
    _ok(lib().oracle_rk4(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), dt, nsteps,
                         _ptr(v)), "rk4")
    return v


def rk4_timed(params, grid, u: np.ndarray, dt: float, nsteps: int = 1, nthreads: int = 0):
    """(copy of u advanced by nsteps RK4 steps, wall seconds of the step loop
    alone): the allocation of the oracle's stage vectors is not timed."""
    v = np.ascontiguousarray(u.copy())
    sec = np.zeros(1)
    _ok(lib().oracle_rk4_timed(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), dt, nsteps,
                               _ptr(v), _ptr(sec)), "rk4_timed")
    return v, float(sec[0])


def rk3(params, grid, u: np.ndarray, dt: float, nsteps: int = 1, nthreads: int = 0) -> np.ndarray:
    """Return a copy of u advanced by nsteps third-order SSP Runge-Kutta
    (Shu-Osher) steps."""
    v = np.ascontiguousarray(u.copy())
    _ok(lib().oracle_rk3(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), dt, nsteps,
                         _ptr(v)), "rk3")
    return v


def enforce_algebraic(params, grid, u: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Return a copy of u with det(gt) = 1 and gt^ij At_ij = 0 restored at
    every interior point (periodic ghosts refilled)."""
    v = np.ascontiguousarray(u.copy())
    _ok(lib().oracle_enforce_algebraic(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)),
                                       _ptr(v)), "enforce_algebraic")
    return v


def rhs_ext(params, grid, u: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """rhs() evaluated in x87 extended precision (64-bit significand), rounded
    to FP64: the reference against which FP64 rounding error is measured."""
    out = np.full(grid.shape, np.nan)
    _ok(lib().oracle_rhs_ext(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), _ptr(u),
                             _ptr(out)), "rhs_ext")
    return out


def ext_mantissa_bits() -> int:
    return int(lib().oracle_ext_mant_dig())


def rk4_ext(params, grid, u: np.ndarray, dt: float, nsteps: int = 1, nthreads: int = 0) -> np.ndarray:
    """rk4() evaluated in x87 extended precision, rounded to FP64 at the end."""
    v = np.ascontiguousarray(u.copy())
    _ok(lib().oracle_rk4_ext(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), dt, nsteps,
                             _ptr(v)), "rk4_ext")
    return v


def rk3_ext(params, grid, u: np.ndarray, dt: float, nsteps: int = 1, nthreads: int = 0) -> np.ndarray:
    """rk3() evaluated in x87 extended precision, rounded to FP64 at the end."""
    v = np.ascontiguousarray(u.copy())
    _ok(lib().oracle_rk3_ext(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), dt, nsteps,
                             _ptr(v)), "rk3_ext")
    return v


def fill_periodic(grid, u: np.ndarray) -> None:
    _ok(lib().oracle_fill_periodic(ctypes.byref(_grid(grid)), _ptr(u)), "fill_periodic")


def hamiltonian(params, grid, u: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Hamiltonian constraint at interior points, shape (nz, ny, nx)."""
    H = np.full(grid.shape[1:], np.nan)
    _ok(lib().oracle_hamiltonian(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)),
                                 _ptr(u), _ptr(H)), "hamiltonian")
    return H[grid.interior()]


def rhs_point(params, u, d1, d2, adv, diss) -> np.ndarray:
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (u, d1, d2, adv, diss)]
    assert arrs[0].size == NGF and arrs[1].size == NGF * 3 and arrs[2].size == NGF * 6
    out = np.zeros(NGF)
    _ok(lib().oracle_rhs_point(ctypes.byref(_params(params)), *[_ptr(a) for a in arrs], _ptr(out)), "rhs_point")
    return out


def momentum(params, grid, u: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Momentum constraint M_i at interior points, shape (3, nz, ny, nx)."""
    M = np.full((3,) + grid.shape[1:], np.nan)
    _ok(lib().oracle_momentum(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), _ptr(u),
                              _ptr(M)), "momentum")
    return M[(slice(None),) + grid.interior()]


def _many(grids, states):
    gs = (_Grid * len(grids))(*[_grid(g) for g in grids])
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(states))(*[_ptr(s) for s in states])
    return gs, ptrs


def sync_ghosts(params, grids, states, nthreads: int = 0) -> None:
    """Refill the ghost points of several patches in place from the patches of
    the same and the next coarser refinement level."""
    gs, ptrs = _many(grids, states)
    _ok(lib().oracle_sync_ghosts(ctypes.byref(_params(params, nthreads)), gs, ptrs, len(grids)), "sync_ghosts")


def restrict(params, grids, states) -> None:
    """Finer interior values injected into coincident coarse interior points, in place."""
    gs, ptrs = _many(grids, states)
    _ok(lib().oracle_restrict(ctypes.byref(_params(params)), gs, ptrs, len(grids)), "restrict")


def steps_synced(params, grids, states, dt: float, nsteps: int, integrator: int = 4, nthreads: int = 0):
    """Copies of the patch states advanced together by nsteps RK4 (integrator
    4) or SSP RK3 (3) steps with one dt, ghosts refilled after every stage."""
    out = [np.ascontiguousarray(s.copy()) for s in states]
    gs, ptrs = _many(grids, out)
    _ok(lib().oracle_steps_synced(ctypes.byref(_params(params, nthreads)), gs, ptrs, len(grids), dt, nsteps,
                                  integrator), "steps_synced")
    return out


def psi4(params, grid, u: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Psi4 at interior points, shape (2, nz, ny, nx): real and imaginary part."""
    out = np.full((2,) + grid.shape[1:], np.nan)
    _ok(lib().oracle_psi4(ctypes.byref(_params(params, nthreads)), ctypes.byref(_grid(grid)), _ptr(u),
                          _ptr(out)), "psi4")
    return out[(slice(None),) + grid.interior()]


def psi4_point(u, d1, d2, xyz):
    """(psi4 as complex, E 3x3, B 3x3, tetrad rows e_r, e_theta, e_phi) at one
    point from exact values and derivatives."""
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (u, d1, d2, xyz)]
    assert arrs[0].size == NGF and arrs[1].size == NGF * 3 and arrs[2].size == NGF * 6 and arrs[3].size == 3
    res = np.zeros(29)
    _ok(lib().oracle_psi4_point(*[_ptr(a) for a in arrs], _ptr(res)), "psi4_point")
    return complex(res[0], res[1]), res[2:11].reshape(3, 3), res[11:20].reshape(3, 3), res[20:29].reshape(3, 3)


def mom_point(u, d1) -> np.ndarray:
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (u, d1)]
    assert arrs[0].size == NGF and arrs[1].size == NGF * 3
    out = np.zeros(3)
    _ok(lib().oracle_mom_point(*[_ptr(a) for a in arrs], _ptr(out)), "mom_point")
    return out


def ham_point(u, d1, d2) -> float:
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64)) for a in (u, d1, d2)]
    out = np.zeros(1)
    _ok(lib().oracle_ham_point(*[_ptr(a) for a in arrs], _ptr(out)), "ham_point")
    return float(out[0])


OP_D1, OP_D2, OP_D11, OP_UP_PLUS, OP_UP_MINUS, OP_KO = range(6)


def apply_op(op: int, grid, f: np.ndarray, order: int, a: int = 0, b: int = 0, r: int = 0,
             eps: float = 0.0) -> np.ndarray:
    """One stencil operator on a single grid function f of shape grid.shape[1:];
    returns the interior values (nz, ny, nx)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.full(grid.shape[1:], np.nan)
    _ok(lib().oracle_apply_op(op, a, b, order, r, eps, ctypes.byref(_grid(grid)), _ptr(f), _ptr(out)),
        "apply_op")
    return out[grid.interior()]


def count_rhs_flops(params, grid, u: np.ndarray, point=(0, 0, 0)):
    """(adds, muls, divs) of one right-hand-side evaluation at one interior point."""
    c = (ctypes.c_longlong * 3)()
    _ok(lib().oracle_count_rhs_flops(ctypes.byref(_params(params)), ctypes.byref(_grid(grid)), _ptr(u),
                                     point[0], point[1], point[2], c), "count")
    return int(c[0]), int(c[1]), int(c[2])


def required_ghost(order: int, upwind: int, ko_radius: int) -> int:
    return int(lib().oracle_required_ghost(order, upwind, ko_radius))
