"""Pins of the oracle's momentum constraint M_i.

* An exact vacuum slice (Minkowski space in deformed coordinates, with
  nonzero At, d K and d chi): M_i = 0, every term nonzero.
* Curved random metrics with random extrinsic curvature (not a solution):
  the oracle's conformal M_i equals the textbook ADM momentum constraint
  D_j K^j_i - d_i K of the physical metric and curvature, computed here from
  their exact jets and the physical Christoffel symbols.
* On the grid: flat space gives exactly zero, and polynomial data of degree
  within the stencils' exactness give the pointwise constraint of the exact
  derivatives.
"""
import numpy as np
import pytest

import exact_solutions as E
from paper_1307_6488_amd import inputs as I
from test_oracle_algebra import POINTS, _random_metric_fields


@pytest.mark.parametrize("pt", POINTS)
def test_exact_vacuum_slice_has_zero_momentum_constraint(orc, pt):
    pd = E.extract(E.bssn_from_adm(*E.adm_from_4metric(E.minkowski_deformed(pt))))
    assert np.max(np.abs(pd["u"][8:14])) > 1e-3 and np.max(np.abs(pd["d1"][7])) > 1e-3
    M = orc.mom_point(pd["u"], pd["d1"])
    scale = max(np.max(np.abs(pd["d1"][8:14])), np.max(np.abs(pd["d1"][7])))
    assert np.max(np.abs(M)) < 1e-13 * scale


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_conformal_momentum_constraint_equals_adm_one(orc, seed):
    rng = np.random.default_rng(100 + seed)
    pt = (0.0, 0.31, -0.17, 0.23)
    gam, _, _ = _random_metric_fields(rng, pt)
    X = E.coords(pt)
    sp = X[1:]

    def field():
        c = rng.uniform(-0.5, 0.5, 7)
        return c[0] + c[1] * sp[0] + c[2] * sp[1] + c[3] * sp[2] + c[4] * sp[0] * sp[1] \
            + c[5] * sp[1] * sp[2] + c[6] * sp[2] * sp[2]

    K = [[None] * 3 for _ in range(3)]
    for a in range(3):
        for b in range(a, 3):
            K[a][b] = field()
            K[b][a] = K[a][b]
    zero = E.Jet.const(0)
    pd = E.extract(E.bssn_from_adm(gam, K, E.Jet.const(1), [zero, zero, zero]))
    gamu, _ = E.inv3(gam)
    G = E.christoffel(gam, gamu)
    trK = sum((gamu[i][j] * K[i][j] for i in range(3) for j in range(3)), zero)
    want = []
    for i in range(3):
        s = zero
        for j in range(3):
            for k in range(3):
                t = K[i][j].d(1 + k)
                for l in range(3):
                    t = t - G[l][k][i] * K[l][j] - G[l][k][j] * K[i][l]
                s = s + gamu[j][k] * t
        want.append(float((s - trK.d(1 + i)).val()))
    got = orc.mom_point(pd["u"], pd["d1"])
    assert np.max(np.abs(want)) > 0.1
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.max(np.abs(want)))


def test_grid_momentum_flat_zero_and_polynomial_data(orc):
    grid = I.Grid((6, 5, 4), 2, 0.25)
    p = I.config_params(4, 0, 2, 2, I.BC_STATIC)
    u = I.flat(grid)
    assert np.all(orc.momentum(p, grid, u) == 0.0)
    # quadratic fields: 4th-order centred first derivatives are exact
    z, y, x = np.meshgrid(*[grid.origin[a] + grid.h * (np.arange(grid.shape[3 - a]) - grid.ghost)
                            for a in (2, 1, 0)], indexing="ij")
    coef = np.random.default_rng(4).uniform(-0.1, 0.1, (24, 6))

    def q(f):
        c = coef[f]
        return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * z * z

    def dq(f):
        c = coef[f]
        return [c[1] + c[4] * y, c[2] + c[4] * x, c[3] + 2 * c[5] * z]

    for f in range(24):
        u[f] = u[f] + q(f)
    M = orc.momentum(p, grid, u)
    s = grid.interior()
    for (kk, jj, ii) in [(0, 0, 0), (1, 2, 3), (3, 4, 5)]:
        at = (s[0].start + kk, s[1].start + jj, s[2].start + ii)
        d1 = np.array([[dq(f)[a][at] for a in range(3)] for f in range(24)])
        want = orc.mom_point(u[(slice(None),) + at], d1)
        np.testing.assert_allclose(M[:, kk, jj, ii], want, rtol=0, atol=1e-13)
