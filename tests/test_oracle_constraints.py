"""Pins of the oracle's algebraic-constraint enforcement (det gt = 1,
gt^ij At_ij = 0), against numpy's determinant and inverse and closed forms:

* after it, det(gt) = 1 and the trace of At vanishes at every interior point;
* the result is invariant under gt -> lambda gt of the input (the rescaling
  divides out) and idempotent, and leaves constrained data as it is;
* diagonal metric and curvature: the closed form
  gt_ii -> gt_ii / (g00 g11 g22)^(1/3),  At_ii -> At_ii - gt_ii / 3 * sum_k At_kk / gt_kk;
* the other 12 grid functions, static ghosts and row padding are untouched;
  periodic ghosts are the images of the interior.
"""
import numpy as np

from paper_1307_6488_amd import inputs as I

SYM = [[0, 1, 2], [1, 3, 4], [2, 4, 5]]


def _random_state(grid, seed=5, amp=0.25):
    """Random symmetric positive metrics gt = s B B^T (B = 1 + amp N, s in
    [0.5, 2]) and random symmetric At; K random too."""
    rng = np.random.default_rng(seed)
    u = I.flat(grid)
    nz, ny, nx = grid.shape[1], grid.shape[2], grid.ext[0]
    B = np.eye(3) + amp * rng.standard_normal((nz, ny, nx, 3, 3))
    gt = np.einsum("...ik,...jk->...ij", B, B) * rng.uniform(0.5, 2.0, (nz, ny, nx, 1, 1))
    At = rng.standard_normal((nz, ny, nx, 3, 3))
    At = 0.5 * (At + np.swapaxes(At, -1, -2))
    for a in range(3):
        for b in range(a, 3):
            u[I.GT + SYM[a][b], :, :, :nx] = gt[..., a, b]
            u[I.AT + SYM[a][b], :, :, :nx] = At[..., a, b]
    u[I.TRK] = rng.standard_normal(u[I.TRK].shape)
    return u


def _tensors(u, grid):
    s = grid.interior()
    g = np.empty(u[(0,) + s].shape + (3, 3))
    A = np.empty_like(g)
    for a in range(3):
        for b in range(3):
            g[..., a, b] = u[(I.GT + SYM[a][b],) + s]
            A[..., a, b] = u[(I.AT + SYM[a][b],) + s]
    return g, A


def _params(bc=I.BC_STATIC):
    return I.config_params(4, 1, 3, 3, bc)


def test_enforced_state_has_unit_determinant_and_traceless_curvature(orc):
    grid = I.Grid((7, 5, 6), 3, 0.25)
    u = _random_state(grid)
    out = orc.enforce_algebraic(_params(), grid, u)
    g, A = _tensors(out, grid)
    assert np.max(np.abs(np.linalg.det(g) - 1.0)) < 1e-14
    tr = np.einsum("...ij,...ij->...", np.linalg.inv(g), A)
    assert np.max(np.abs(tr)) < 1e-13 * np.max(np.abs(A))
    g0, A0 = _tensors(u, grid)
    assert np.max(np.abs(np.linalg.det(g0) - 1.0)) > 0.1           # the input was far from it
    # the other grid functions, the ghosts and the row padding are untouched
    keep = np.ones(u.shape, dtype=bool)
    for f in list(range(I.GT, I.GT + 6)) + list(range(I.AT, I.AT + 6)):
        keep[(f,) + grid.interior()] = False
    assert np.array_equal(out[keep], u[keep], equal_nan=True)


def test_rescaling_invariance_idempotence_and_fixed_points(orc):
    grid = I.Grid((5, 4, 3), 3, 0.25)
    u = _random_state(grid, seed=9)
    once = orc.enforce_algebraic(_params(), grid, u)
    v = u.copy()
    for s in range(6):
        v[(I.GT + s,) + grid.interior()] *= 2.7
    scaled = orc.enforce_algebraic(_params(), grid, v)
    twice = orc.enforce_algebraic(_params(), grid, once)
    inner = (slice(None),) + grid.interior()
    scale = np.max(np.abs(once[inner]))
    assert np.max(np.abs(scaled[inner] - once[inner])) < 1e-14 * scale
    assert np.max(np.abs(twice[inner] - once[inner])) < 1e-14 * scale


def test_diagonal_closed_form(orc):
    grid = I.Grid((3, 3, 3), 3, 0.25)
    u = I.flat(grid)
    a, b, c = 1.7, 0.6, 2.3
    p, q, r = 0.4, -1.1, 0.25
    for s, val in zip((0, 3, 5), (a, b, c)):
        u[I.GT + s] = val
    for s, val in zip((0, 3, 5), (p, q, r)):
        u[I.AT + s] = val
    out = orc.enforce_algebraic(_params(), grid, u)
    inner = grid.interior()
    sc = (a * b * c) ** (1.0 / 3.0)
    t = p / a + q / b + r / c
    for s, gval, aval in ((0, a, p), (3, b, q), (5, c, r)):
        assert np.allclose(out[(I.GT + s,) + inner], gval / sc, rtol=1e-15, atol=0)
        assert np.allclose(out[(I.AT + s,) + inner], aval - gval * t / 3.0, rtol=1e-14, atol=1e-15)
    for s in (1, 2, 4):
        assert np.all(out[(I.GT + s,) + inner] == 0.0)
        assert np.all(out[(I.AT + s,) + inner] == 0.0)


def test_periodic_ghosts_are_images(orc):
    grid = I.Grid((6, 5, 4), 2, 0.25)
    u = _random_state(grid, seed=3)
    p = I.config_params(4, 0, 2, 2, I.BC_PERIODIC)
    out = orc.enforce_algebraic(p, grid, u)
    g, n = grid.ghost, grid.n
    ext = out[(slice(None),) + grid.interior()]
    for ax in (1, 2, 3):
        ext = np.take(ext, np.arange(-g, n[3 - ax] + g) % n[3 - ax], axis=ax)
    assert np.array_equal(out[:, :, :, : grid.ext[0]], ext)
