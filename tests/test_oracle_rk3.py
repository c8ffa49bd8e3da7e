"""Pins of the oracle's third-order Runge-Kutta step.

The paper's production runs use a third-order Runge-Kutta integrator
(section "Binary Black Hole Simulations"); which one is a reading (the
strong-stability-preserving scheme of Shu and Osher).  What the mathematics
fixes for any three-stage third-order method is pinned here:

* Uniform data turns the PDE into an ODE.  For the linear Gamma-driver pair
  beta' = 3/4 B, B' = -eta B one step must apply exactly the degree-3 Taylor
  polynomial of exp(dt M) (the stability function of every three-stage
  third-order Runge-Kutta method).
* Nonlinear uniform data (1+log lapse): third-order convergence to the exact
  ODE solution computed with a high-order Taylor integrator in 30 digits.
* Static ghosts never change; periodic ghosts hold the periodic images.
"""
import math

import numpy as np
import pytest

from paper_1307_6488_amd import inputs as I

from test_oracle_rk4 import _flat_values, _ode_exact, _uniform


@pytest.mark.parametrize("dt", [0.1, 0.37])
def test_rk3_linear_gamma_driver_step_is_taylor3_of_exp(orc, dt):
    v = _flat_values()
    v[18:21] = (0.1, -0.2, 0.05)
    v[21:24] = (0.3, 0.1, -0.2)
    eta = 2.0
    grid, u = _uniform(v)
    p = I.Params(fd_order=4, ghost=2, upwind=0, ko_radius=2, eps_diss=0.1, eta=eta, bc=I.BC_PERIODIC)
    out = orc.rk3(p, grid, u, dt, 1)
    M = np.array([[0.0, 0.75], [0.0, -eta]])
    P = sum(np.linalg.matrix_power(dt * M, k) / math.factorial(k) for k in range(4))
    for i in range(3):
        want = P @ np.array([v[18 + i], v[21 + i]])
        got = out[[18 + i, 21 + i]][(slice(None),) + grid.interior()]
        assert np.max(np.abs(got[0] - want[0])) < 1e-15
        assert np.max(np.abs(got[1] - want[1])) < 1e-15
    inner = out[(slice(None),) + grid.interior()]
    for f in range(0, 18):
        assert np.all(inner[f] == v[f])


def test_rk3_nonlinear_uniform_converges_at_third_order(orc):
    v = _flat_values()
    v[0], v[7], v[17] = 0.9, 0.4, 0.8
    T = 0.8
    exact = _ode_exact(v[0], v[7], v[17], T)
    p = I.Params(fd_order=4, ghost=2, upwind=0, ko_radius=2, eps_diss=0.1, bc=I.BC_PERIODIC)
    errs = []
    for nsteps in (8, 16, 32):
        grid, u = _uniform(v)
        out = orc.rk3(p, grid, u, T / nsteps, nsteps)
        c = (slice(None), grid.ghost + 1, grid.ghost + 2, grid.ghost + 3)
        got = out[c][[0, 7, 17]]
        errs.append(float(np.max(np.abs(got - np.array(exact)))))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.8 < q < 3.3 for q in rates), (errs, rates)
    assert errs[-1] < 1e-5


def test_rk3_static_ghosts_unchanged_and_periodic_ghosts_are_images(orc):
    w = I.workload(2, n_override=10)
    u = w.make_state()
    out = orc.rk3(w.params, w.grid, u, w.dt, 2)
    mask = np.ones(w.grid.shape, dtype=bool)
    mask[(slice(None),) + w.grid.interior()] = False
    mask[:, :, :, w.grid.ext[0]:] = False
    assert np.array_equal(out[mask], u[mask])
    assert not np.array_equal(out[(slice(None),) + w.grid.interior()], u[(slice(None),) + w.grid.interior()])

    w1 = I.workload(1, n_override=8)
    u1 = w1.make_state()
    o1 = orc.rk3(w1.params, w1.grid, u1, w1.dt, 1)
    g, n = w1.grid.ghost, w1.grid.n
    core = o1[(slice(None),) + w1.grid.interior()]
    ext = core
    for ax in (1, 2, 3):
        idx = np.arange(-g, n[3 - ax] + g) % n[3 - ax]
        ext = np.take(ext, idx, axis=ax)
    assert np.array_equal(o1[:, :, :, : w1.grid.ext[0]], ext)


def test_extended_precision_rk3_step_is_the_exact_step_rounded(orc):
    """The extended-precision RK3 path (the FP64-rounding reference of the GPU
    tests) on uniform data: one step of the ODE the system reduces to, worked
    out in 40-digit arithmetic with the same three stages, comes back
    correctly rounded to FP64 (within 0.51 ulp); pins its 3/4, 1/4, 1/3 and
    2/3 in its own precision."""
    import mpmath
    assert orc.ext_mantissa_bits() >= 64
    v = _flat_values()
    v[0], v[7], v[17] = 0.9, 0.3, 0.8
    v[18:21] = (0.1, -0.2, 0.05)
    v[21:24] = (0.3, 0.1, -0.2)
    eta, dt = 2.0, 0.37
    grid, u = _uniform(v)
    p = I.Params(fd_order=4, ghost=2, upwind=0, ko_radius=2, eps_diss=0.1, eta=eta, bc=I.BC_PERIODIC)
    out = orc.rk3_ext(p, grid, u, dt, 1)
    inner = out[(slice(None),) + grid.interior()]
    with mpmath.workdps(40):
        def f(y):
            chi, K, a = y[0], y[1], y[2]
            d = [mpmath.mpf(2) / 3 * chi * a * K, a * K * K / 3, -2 * a * K]
            d += [mpmath.mpf(3) / 4 * y[6 + i] for i in range(3)]
            d += [-mpmath.mpf(eta) * y[6 + i] for i in range(3)]
            return d
        h = mpmath.mpf(dt)
        y0 = [mpmath.mpf(float(v[i])) for i in (0, 7, 17, 18, 19, 20, 21, 22, 23)]
        y1 = [a + h * b for a, b in zip(y0, f(y0))]
        y2 = [mpmath.mpf(3) / 4 * a + (b + h * c) / 4 for a, b, c in zip(y0, y1, f(y1))]
        y3 = [a / 3 + 2 * (b + h * c) / 3 for a, b, c in zip(y0, y2, f(y2))]
    for slot, gf in enumerate((0, 7, 17, 18, 19, 20, 21, 22, 23)):
        want = y3[slot]
        ulp = np.spacing(abs(float(want)))
        err = float(abs(mpmath.mpf(float(inner[gf].flat[0])) - want))
        assert err <= 0.51 * ulp, (gf, err / ulp)
