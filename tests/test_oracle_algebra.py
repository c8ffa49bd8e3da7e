"""Pins of the oracle's pointwise BSSN algebra against exact solutions.

The oracle exposes its pointwise right-hand side with caller-supplied
derivatives.  Feeding it the exact derivatives of an exact solution of the
Einstein equations (computed by Taylor-mode differentiation in extended
precision, no finite differences) must reproduce the exact time derivatives.
None of these expected values comes from re-typing the BSSN equations: they
are the time derivatives of a known spacetime, textbook Ricci tensors of a
3-metric, or ADM (York) evolution equations.
"""
import math

import numpy as np
import pytest

import exact_solutions as E
from paper_1307_6488_amd import inputs as I

LD = np.longdouble
EVOLVED_GEOMETRY = list(range(0, 17))   # chi, gt, K, At, Gt


def _rhs(orc, params, pd, B=None):
    u = pd["u"].copy()
    if B is not None:
        u[21:24] = B
    beta = u[18:21]
    adv = pd["d1"] @ beta                  # exact advection beta^k d_k u
    return orc.rhs_point(params, u, pd["d1"], pd["d2"], adv, np.zeros(24))


POINTS = [(0.2, 0.3, -0.25, 0.4), (0.0, -0.7, 0.45, 0.15), (0.35, 0.1, 0.6, -0.5)]


@pytest.mark.parametrize("pt", POINTS)
def test_deformed_minkowski_rhs_is_exact_time_derivative(orc, pt):
    """Minkowski space in deformed coordinates has nonzero lapse gradients,
    shift, shift gradients and K, so every term of the chi, gt, K, At and Gt
    equations (incl. all shift terms) is exercised; the right-hand side must
    equal the exact d_t of each BSSN variable and H must vanish."""
    fields = E.bssn_from_adm(*E.adm_from_4metric(E.minkowski_deformed(pt)))
    pd = E.extract(fields)
    assert np.max(np.abs(pd["dt"][EVOLVED_GEOMETRY])) > 1e-3     # nontrivial
    for lapse in (0, 1, 2):
        p = I.Params(lapse=lapse, shift=0, eps_diss=0.0)
        rhs = _rhs(orc, p, pd)
        scale = np.max(np.abs(pd["dt"][EVOLVED_GEOMETRY]))
        np.testing.assert_allclose(rhs[EVOLVED_GEOMETRY], pd["dt"][EVOLVED_GEOMETRY], rtol=0,
                                   atol=1e-13 * scale)
    H = orc.ham_point(pd["u"], pd["d1"], pd["d2"])
    assert abs(H) < 1e-14


@pytest.mark.parametrize("pt", POINTS[:2])
def test_gamma_driver_couples_to_exact_gt_source(orc, pt):
    """Gamma-driver shift: d_t beta^i = beta^j d_j beta^i + 3/4 B^i and
    d_t B^i = beta^j d_j B^i + (d_t Gt^i - beta^j d_j Gt^i) - eta B^i, where the
    Gt source is the exact one of the spacetime.  The 1+log lapse is
    d_t alpha = beta^j d_j alpha - 2 alpha K."""
    pd = E.extract(E.bssn_from_adm(*E.adm_from_4metric(E.minkowski_deformed(pt))))
    B = np.array([0.3, -0.2, 0.1])              # uniform: d B = 0
    eta = 2.0
    p = I.Params(lapse=0, shift=0, eta=eta, eps_diss=0.0)
    rhs = _rhs(orc, p, pd, B=B)
    beta = pd["u"][18:21]
    adv_beta = pd["d1"][18:21] @ beta
    adv_gt = pd["d1"][14:17] @ beta
    np.testing.assert_allclose(rhs[18:21], adv_beta + 0.75 * B, rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(rhs[21:24], pd["dt"][14:17] - adv_gt - eta * B, rtol=0, atol=1e-15)
    K, alpha = pd["u"][7], pd["u"][17]
    np.testing.assert_allclose(rhs[17], pd["d1"][17] @ beta - 2.0 * alpha * K, rtol=1e-13)
    # frozen gauge: no evolution of alpha, beta, B
    rhs_f = _rhs(orc, I.Params(lapse=2, shift=1, eps_diss=0.0), pd, B=B)
    assert np.all(rhs_f[17:24] == 0.0)


@pytest.mark.parametrize("pt", [(0.13, 0.21, 0.0, 0.0), (0.7, -0.33, 0.1, 0.2)])
def test_gauge_wave_harmonic_lapse_exact(orc, pt):
    """The gauge wave is an exact solution with harmonic slicing
    (d_t alpha = -alpha^2 K) and zero shift; every right-hand side, the lapse
    included, must equal its exact time derivative."""
    pd = E.extract(E.bssn_from_adm(*E.adm_from_4metric(E.gauge_wave_metric(pt, A=0.1))))
    p = I.Params(lapse=1, shift=1, eps_diss=0.0)
    rhs = _rhs(orc, p, pd)
    idx = EVOLVED_GEOMETRY + [17]
    scale = np.max(np.abs(pd["dt"][idx]))
    assert scale > 0.1
    np.testing.assert_allclose(rhs[idx], pd["dt"][idx], rtol=0, atol=1e-13 * scale)


def _random_metric_fields(rng, pt):
    """gt = L L^T with L unit lower triangular (det gt = 1) and chi > 0, both
    low-degree polynomials; everything else zero, alpha = 1, Gt^i = -d_j gt^ij."""
    X = E.coords(pt)
    sp = X[1:]

    def lin(c):
        return c[0] + c[1] * sp[0] + c[2] * sp[1] + c[3] * sp[2] + c[4] * sp[0] * sp[1]

    one = E.Jet.const(1)
    zero = E.Jet.const(0)
    Lm = [[one, zero, zero], [None, one, zero], [None, None, one]]
    for (i, j) in [(1, 0), (2, 0), (2, 1)]:
        Lm[i][j] = lin(rng.uniform(-0.3, 0.3, 5))
    gt = [[sum((Lm[i][k] * Lm[j][k] for k in range(3)), zero) for j in range(3)] for i in range(3)]
    chi = lin(np.concatenate([[0.8], rng.uniform(-0.2, 0.2, 4)])) * lin(
        np.concatenate([[1.1], rng.uniform(-0.1, 0.1, 4)]))
    inv_chi = chi.pow(-1)
    gam = [[gt[i][j] * inv_chi for j in range(3)] for i in range(3)]
    return gam, gt, chi


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ricci_of_random_metric(orc, seed):
    """With alpha = 1 and zero shift, K and At, the At right-hand side is
    chi R^TF_ij and H = R (the scalar curvature), so the oracle's full Ricci
    tensor R_ij = rhs_At/chi + gt_ij R/(3 chi) must equal the textbook Ricci
    tensor of gamma_ij = gt_ij / chi computed from its Christoffel symbols."""
    rng = np.random.default_rng(seed)
    pt = (0.0, 0.31, -0.17, 0.23)
    gam, gt, chi = _random_metric_fields(rng, pt)
    zero = E.Jet.const(0)
    K = [[zero] * 3 for _ in range(3)]
    fields = E.bssn_from_adm(gam, K, E.Jet.const(1), [zero, zero, zero])
    pd = E.extract(fields)
    # the change of variables must reproduce the constructed gt (det 1)
    np.testing.assert_allclose(pd["u"][1:7], [float(gt[a][b].val()) for (a, b) in E.PAIRS], rtol=1e-14)
    p = I.Params(lapse=2, shift=1, eps_diss=0.0)
    rhs = _rhs(orc, p, pd)
    Hs = orc.ham_point(pd["u"], pd["d1"], pd["d2"])
    Ric, _ = E.ricci(gam, E.inv3(gam)[0])
    chi0 = pd["u"][0]
    gt0 = pd["u"][1:7]
    R_or = rhs[8:14] / chi0 + gt0 * Hs / (3.0 * chi0)
    R_ex = np.array([float(Ric[a][b].val()) for (a, b) in E.PAIRS])
    gamu, _ = E.inv3(gam)
    R_scalar = float(sum((gamu[i][j] * Ric[i][j] for i in range(3) for j in range(3)), E.Jet.const(0)).val())
    assert np.max(np.abs(R_ex)) > 1e-2
    np.testing.assert_allclose(R_or, R_ex, rtol=0, atol=1e-13 * np.max(np.abs(R_ex)))
    assert abs(Hs - R_scalar) < 1e-13 * max(1.0, abs(R_scalar))


def _bl_fields(pt, masses=(0.5, 0.5), centres=((3.0, 0, 0), (-3.0, 0, 0))):
    X = E.coords(pt)
    sp = X[1:]
    psi = E.Jet.const(1)
    for m, c in zip(masses, centres):
        r = ((sp[0] - c[0]) * (sp[0] - c[0]) + (sp[1] - c[1]) * (sp[1] - c[1])
             + (sp[2] - c[2]) * (sp[2] - c[2])).sqrt()
        psi = psi + r.pow(-1) * (m / 2.0)
    return psi


@pytest.mark.parametrize("pt", [(0.0, 2.7, 0.2, -0.1), (0.0, 0.3, 1.1, 0.4), (0.0, -3.2, -0.15, 0.25)])
def test_brill_lindquist_initial_time_derivatives(orc, pt):
    """Two-puncture Brill-Lindquist data with precollapsed lapse alpha = psi^-2
    and zero shift, at t = 0 (K_ij = 0).  ADM (York) evolution gives
    d_t gamma_ij = 0 and d_t K_ij = -D_i D_j alpha + alpha R_ij, hence
    d_t K = -D^2 alpha (R = 0 since psi is harmonic) and
    d_t At_ij = chi [-D_i D_j alpha + alpha R_ij]^TF; all other variables are
    stationary at t = 0.  Also d_t K = -2 psi^-8 |grad psi|^2 in closed form."""
    psi = _bl_fields(pt)
    zero = E.Jet.const(0)
    psi4 = psi * psi * psi * psi
    gam = [[psi4 if i == j else zero for j in range(3)] for i in range(3)]
    alpha = psi.pow(-2)
    K = [[zero] * 3 for _ in range(3)]
    fields = E.bssn_from_adm(gam, K, alpha, [zero, zero, zero])
    pd = E.extract(fields)
    gamu, _ = E.inv3(gam)
    Ric, G = E.ricci(gam, gamu)
    DDa = [[alpha.d(1 + i).d(1 + j) - sum((G[k][i][j] * alpha.d(1 + k) for k in range(3)), zero)
            for j in range(3)] for i in range(3)]
    dtK = [[-DDa[i][j] + alpha * Ric[i][j] for j in range(3)] for i in range(3)]
    trdt = sum((gamu[i][j] * dtK[i][j] for i in range(3) for j in range(3)), zero)
    chi = fields[0]
    dtAt = np.array([float(((dtK[a][b] - gam[a][b] * trdt * (1.0 / 3.0)) * chi).val()) for (a, b) in E.PAIRS])
    lap = sum((gamu[i][j] * DDa[i][j] for i in range(3) for j in range(3)), zero)
    grad2 = sum((psi.d(1 + i) * psi.d(1 + i) for i in range(3)), zero)
    closed = float((-2.0 * psi.pow(-8) * grad2).val())
    assert abs(float((-lap).val()) - closed) < 1e-14 * abs(closed)
    p = I.Params(lapse=0, shift=0, eps_diss=0.0)
    rhs = _rhs(orc, p, pd)
    assert abs(rhs[7] - closed) < 1e-13 * abs(closed)
    np.testing.assert_allclose(rhs[8:14], dtAt, rtol=0, atol=1e-13 * np.max(np.abs(dtAt)))
    for f in [0, 1, 2, 3, 4, 5, 6, 14, 15, 16, 17, 18, 19, 20, 21, 22, 23]:
        assert rhs[f] == 0.0 or abs(rhs[f]) < 1e-15 * abs(closed), (f, rhs[f])
    assert abs(orc.ham_point(pd["u"], pd["d1"], pd["d2"])) < 1e-13 * abs(float(grad2.val()))


def test_gauge_wave_inputs_match_exact(orc):
    """The numpy gauge-wave generator agrees with the 3+1 split of the metric."""
    A = 0.1
    for xv in (-0.4, 0.05, 0.33):
        pd = E.extract(E.bssn_from_adm(*E.adm_from_4metric(E.gauge_wave_metric((0.0, xv, 0.0, 0.0), A=A))))
        f = I.gauge_wave_fields(np.array([xv]), 0.0, A, 1.0)
        for gf, val in f.items():
            assert abs(val[0] - pd["u"][gf]) < 1e-14, (gf, val[0], pd["u"][gf])
