"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Error metric per grid function f (max-norm normalised, interior points):
    err_f = max |x_f - x_f^oracle| / max |x_f^oracle|
and for a function the oracle gives as exactly zero, |x_f| <= 1e-14 times the
largest magnitude over all functions, whatever the bar of the others
(tests/parity_metrics.py).  Bars: 1e-12 after one right-hand side
or one RK4 step, 1e-10 after 100 RK4 steps.  The GPU is free to contract to
FMA and to reorder sums; bitwise checks only compare the GPU with itself
(translation, determinism) or exact zeros.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1307_6488_amd import inputs as I
from parity_metrics import ZERO_BAR, gf_errors, parity_failures

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_1307_6488_amd import chemora
    chemora.lib()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_parity(got, ref, grid, tol, what, zero_tol=ZERO_BAR):
    e = gf_errors(got, ref, grid)
    worst = int(np.argmax(e))
    say(f"{what}: max err {e[worst]:.3e} ({I.GF_NAMES[worst]}); per GF: "
        + " ".join(f"{v:.1e}" for v in e))
    assert np.all(np.isfinite(got[(slice(None),) + grid.interior()])), what
    bad = parity_failures(got, ref, grid, tol, zero_tol)
    assert not bad, (what, {I.GF_NAMES[f]: v for f, v in bad.items()})


def assert_fp64_accuracy(got, orc, ext, grid, what, factor=4.0, floor=1e-14, cap=1e-10):
    """FP64 rounding bar: against the oracle's extended-precision evaluation of
    the same scheme (ext), the GPU's error per GF (max-norm, normalised by the
    GF's max |ext|) is at most `factor` times the FP64 oracle's own error, or
    `floor`, and never above `cap`.  Long evolutions of functions that start
    near zero are dominated by the rounding of large cancelling terms, which
    no FP64 evaluation avoids; this bar separates that from a wrong path."""
    e_gpu = gf_errors(got, ext, grid)
    e_orc = gf_errors(orc, ext, grid)
    bar = np.minimum(np.maximum(factor * e_orc, floor), cap)
    worst = int(np.argmax(e_gpu / bar))
    say(f"{what}: GPU err {e_gpu.max():.2e}, FP64 oracle err {e_orc.max():.2e}; worst ratio "
        f"{e_gpu[worst] / max(e_orc[worst], 1e-300):.2f} ({I.GF_NAMES[worst]})")
    assert np.all(np.isfinite(got[(slice(None),) + grid.interior()])), what
    bad = {I.GF_NAMES[f]: (float(e_gpu[f]), float(e_orc[f])) for f in range(24) if e_gpu[f] > bar[f]}
    assert not bad, (what, bad)


def gpu_rhs(torch, params, grid, u, fill=np.nan):
    from paper_1307_6488_amd.chemora import Patch
    P = Patch(params, grid, u)
    out = torch.full_like(P.u, fill)
    P.rhs(out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gpu_rk4(torch, params, grid, u, dt, nsteps):
    from paper_1307_6488_amd.chemora import Patch
    P = Patch(params, grid, u)
    P.rk4_step(dt, nsteps)
    torch.cuda.synchronize()
    return P.u.cpu().numpy()


def bl_grid(n, ghost, h=1.0 / 8.0):
    return I.centred_grid(n, ghost, h)


CASES_RHS = [
    # (name, params, grid, state maker)
    ("sinusoid-32^3-o4-centred", lambda: I.workload(1)),
    ("bl-ragged-o4-upwind", lambda: I.Workload("bl", I.workload(2).params, bl_grid((70, 37, 19), 3),
                                               None, 1 / 32, 1)),
    ("bl-pert-ragged-o8-upwind", lambda: I.Workload("blp", I.workload(3).params, bl_grid((45, 20, 13), 5),
                                                    None, 1 / 32, 1)),
    # a 3-column last tile in x at either tile width
    ("bl-pert-ragged-o8-narrow-tail", lambda: I.Workload("blp", I.workload(3).params, bl_grid((67, 11, 9), 5),
                                                         None, 1 / 32, 1)),
]


def _state(w):
    if w.make_state is not None:
        return w.make_state()
    u = I.brill_lindquist(w.grid)
    if w.params.fd_order == 8:
        I.add_sinusoids(u, w.grid, np.random.default_rng(1310), 1e-4, [I.GT + s for s in range(6)] + [I.TRK],
                        periodic_ghosts=False)
    return u


@pytest.mark.parametrize("name,mk", CASES_RHS, ids=[c[0] for c in CASES_RHS])
def test_rhs_parity(torch_cuda, name, mk):
    w = mk()
    u = _state(w)
    say(f"rhs parity {name} n={w.grid.n} order={w.params.fd_order}")
    got = gpu_rhs(torch_cuda, w.params, w.grid, u)
    ref = oracle.rhs(w.params, w.grid, u, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-12, f"rhs {name}")


@pytest.mark.parametrize("index", [2, 3])
def test_rhs_parity_full_size(torch_cuda, index):
    """Full-size grids (128^3 order 4, 192^3 order 8) in the benchmark's
    launch configuration, compared at every interior point."""
    w = I.workload(index)
    u = w.make_state()
    say(f"full-size rhs parity workload {index} n={w.grid.n}")
    got = gpu_rhs(torch_cuda, w.params, w.grid, u)
    ref = oracle.rhs(w.params, w.grid, u, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-12, f"rhs full {index}")


def test_rhs_leaves_ghosts_and_ignores_poisoned_points(torch_cuda):
    w = I.workload(2, n_override=20)
    u = w.make_state()
    I.poison_padding(u, w.grid)
    I.poison_corners(u, w.grid)
    got = gpu_rhs(torch_cuda, w.params, w.grid, u, fill=7.0)
    inner = (slice(None),) + w.grid.interior()
    assert np.all(np.isfinite(got[inner]))
    mask = np.ones(w.grid.shape, dtype=bool)
    mask[inner] = False
    assert np.all(got[mask] == 7.0)
    ref = oracle.rhs(w.params, w.grid, u, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-12, "rhs poisoned")


@pytest.mark.parametrize("index", [1, 2, 3])
def test_flat_space_is_exactly_zero(torch_cuda, index):
    w = I.workload(index, n_override=16)
    u = I.flat(w.grid)
    got = gpu_rhs(torch_cuda, w.params, w.grid, u)
    assert np.all(got[(slice(None),) + w.grid.interior()] == 0.0)
    after = gpu_rk4(torch_cuda, w.params, w.grid, u, w.dt, 3)
    assert np.array_equal(after[:, :, :, : w.grid.ext[0]], u[:, :, :, : w.grid.ext[0]])


def test_periodic_translation_is_bitwise(torch_cuda):
    w = I.workload(1, n_override=24)
    u = w.make_state()
    g, gr = w.grid.ghost, w.grid
    inner = u[(slice(None),) + gr.interior()]
    r1 = gpu_rhs(torch_cuda, w.params, gr, u)[(slice(None),) + gr.interior()]
    for ax, shift in ((3, 1), (2, 5), (1, -3)):
        rolled = np.roll(inner, -shift, axis=ax)
        ext = rolled
        for a in (1, 2, 3):
            n = rolled.shape[a]
            ext = np.take(ext, np.arange(-g, n + g) % n, axis=a)
        u2 = I.alloc_state(gr)
        u2[:, :, :, : gr.ext[0]] = ext
        r2 = gpu_rhs(torch_cuda, w.params, gr, u2)[(slice(None),) + gr.interior()]
        assert np.array_equal(np.roll(r1, -shift, axis=ax), r2), (ax, shift)


def test_determinism(torch_cuda):
    w = I.workload(2, n_override=40)
    u = w.make_state()
    a = gpu_rhs(torch_cuda, w.params, w.grid, u)
    b = gpu_rhs(torch_cuda, w.params, w.grid, u)
    assert np.array_equal(a, b, equal_nan=True)
    x = gpu_rk4(torch_cuda, w.params, w.grid, u, w.dt, 2)
    y = gpu_rk4(torch_cuda, w.params, w.grid, u, w.dt, 2)
    assert np.array_equal(x, y, equal_nan=True)


def test_rk4_one_step_periodic(torch_cuda):
    w = I.workload(1)
    u = w.make_state()
    got = gpu_rk4(torch_cuda, w.params, w.grid, u, w.dt, 1)
    ref = oracle.rk4(w.params, w.grid, u, w.dt, 1, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-12, "rk4 1 step periodic")
    # ghosts hold the periodic images of the interior, bitwise
    g, n = w.grid.ghost, w.grid.n
    core = got[(slice(None),) + w.grid.interior()]
    ext = core
    for a in (1, 2, 3):
        ext = np.take(ext, np.arange(-g, n[3 - a] + g) % n[3 - a], axis=a)
    assert np.array_equal(got[:, :, :, : w.grid.ext[0]], ext)


def test_rk4_100_steps_brill_lindquist(torch_cuda):
    w = I.workload(2, n_override=24)
    u = w.make_state()
    say("rk4 100 steps BL 24^3")
    got = gpu_rk4(torch_cuda, w.params, w.grid, u, w.dt, 100)
    ref = oracle.rk4(w.params, w.grid, u, w.dt, 100, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-10, "rk4 100 steps BL")
    mask = np.ones(w.grid.shape, dtype=bool)
    mask[(slice(None),) + w.grid.interior()] = False
    mask[:, :, :, w.grid.ext[0]:] = False
    assert np.array_equal(got[mask], u[mask])        # static ghosts untouched


def test_rk4_order8_steps(torch_cuda):
    w = I.workload(3, n_override=18)
    u = w.make_state()
    say("rk4 20 steps order 8 18^3")
    got = gpu_rk4(torch_cuda, w.params, w.grid, u, w.dt, 20)
    ref = oracle.rk4(w.params, w.grid, u, w.dt, 20, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-10, "rk4 20 steps order 8")


def test_gauge_wave_harmonic_periodic(torch_cuda):
    grid = I.gauge_wave_grid(32, 3)
    u = I.gauge_wave(grid, A=0.1)
    p = I.Params(fd_order=4, ghost=3, upwind=1, ko_radius=3, eps_diss=0.1, lapse=1, shift=1,
                 bc=I.BC_PERIODIC)
    dt = 0.25 * grid.h
    got = gpu_rk4(torch_cuda, p, grid, u, dt, 16)
    ref = oracle.rk4(p, grid, u, dt, 16, nthreads=NTHREADS)
    assert_parity(got, ref, grid, 1e-12, "gauge wave 16 steps")


@pytest.mark.parametrize("order,ghost,n", [(8, 5, (21, 14, 11)), (4, 3, (19, 12, 9))])
def test_periodic_ragged_steps_against_oracle(torch_cuda, order, ghost, n):
    """Periodic boundaries on ragged, odd extents (every ghost row kind of the
    ghost kernel: whole y/z ghost rows, x ghosts of interior rows, 2g = 6 and
    10): RK4 steps against the oracle, and the ghosts hold the periodic
    images of the interior, bitwise."""
    grid = I.centred_grid(n, ghost, 0.25)
    p = I.config_params(order, 1, ghost, ghost, I.BC_PERIODIC)
    u = I.flat(grid)
    I.add_sinusoids(u, grid, np.random.default_rng(1312), 1e-3, range(I.NGF))
    dt = 0.25 * grid.h
    say(f"periodic ragged order {order} n={n}")
    got = gpu_rk4(torch_cuda, p, grid, u, dt, 3)
    ref = oracle.rk4(p, grid, u, dt, 3, nthreads=NTHREADS)
    assert_parity(got, ref, grid, 1e-10, f"periodic ragged order {order}")
    core = got[(slice(None),) + grid.interior()]
    ext = core
    for a in (1, 2, 3):
        ext = np.take(ext, np.arange(-ghost, n[3 - a] + ghost) % n[3 - a], axis=a)
    assert np.array_equal(got[:, :, :, : grid.ext[0]], ext)


def gpu_rk3(torch, params, grid, u, dt, nsteps):
    from paper_1307_6488_amd.chemora import Patch
    P = Patch(params, grid, u)
    P.rk3_step(dt, nsteps)
    torch.cuda.synchronize()
    return P.u.cpu().numpy()


@pytest.mark.parametrize("case", ["bl24-o4-static", "sinusoid32-o4-periodic", "blpert18-o8-static"])
def test_rk3_steps_against_oracle(torch_cuda, case):
    """Third-order SSP Runge-Kutta steps through the C ABI against the
    oracle's; static ghosts stay untouched, periodic ghosts are images."""
    if case == "bl24-o4-static":
        w, nsteps, bar = I.workload(2, n_override=24), 40, 1e-10
    elif case == "sinusoid32-o4-periodic":
        w, nsteps, bar = I.workload(1), 4, 1e-10
    else:
        w, nsteps, bar = I.workload(3, n_override=18), 10, 1e-10
    u = w.make_state()
    say(f"rk3 {case} {nsteps} steps")
    got = gpu_rk3(torch_cuda, w.params, w.grid, u, w.dt, nsteps)
    ref = oracle.rk3(w.params, w.grid, u, w.dt, nsteps, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, bar, f"rk3 {case}")
    if case == "bl24-o4-static":
        # functions that start at zero (shift, B) end as small remainders:
        # against the extended-precision RK3, the GPU's error is held to the
        # FP64 oracle's own
        ext = oracle.rk3_ext(w.params, w.grid, u, w.dt, nsteps, nthreads=NTHREADS)
        assert_fp64_accuracy(got, ref, ext, w.grid, f"rk3 {case}")
    if w.params.bc == I.BC_PERIODIC:
        g, n = w.grid.ghost, w.grid.n
        ext = got[(slice(None),) + w.grid.interior()]
        for a in (1, 2, 3):
            ext = np.take(ext, np.arange(-g, n[3 - a] + g) % n[3 - a], axis=a)
        assert np.array_equal(got[:, :, :, : w.grid.ext[0]], ext)
    else:
        mask = np.ones(w.grid.shape, dtype=bool)
        mask[(slice(None),) + w.grid.interior()] = False
        mask[:, :, :, w.grid.ext[0]:] = False
        assert np.array_equal(got[mask], u[mask])


@pytest.mark.parametrize("bc", ["static", "periodic"])
def test_enforce_constraints_against_oracle(torch_cuda, bc):
    """Algebraic-constraint enforcement through the C ABI on random metrics
    (within about 30 % of the identity, as conformal metrics are; nearly
    singular ones would make det's rounding, not the kernel, decide) and
    curvatures of a ragged patch: equal to the oracle's to rounding,
    det(gt) = 1 by numpy's determinant; ghosts as the boundary says."""
    from paper_1307_6488_amd.chemora import Patch
    from test_oracle_constraints import _random_state
    grid = I.Grid((37, 21, 9), 3, 0.25)
    p = I.config_params(4, 1, 3, 3, I.BC_STATIC if bc == "static" else I.BC_PERIODIC)
    u = _random_state(grid, seed=21, amp=0.1)
    if bc == "periodic":
        oracle.fill_periodic(grid, u)
    say(f"enforce constraints {bc}")
    P = Patch(p, grid, u)
    P.enforce_constraints()
    torch_cuda.cuda.synchronize()
    got = P.u.cpu().numpy()
    ref = oracle.enforce_algebraic(p, grid, u)
    inner = (slice(None),) + grid.interior()
    for f in range(24):
        scale = max(float(np.max(np.abs(ref[f][inner[1:]]))), 1e-300)
        err = float(np.max(np.abs(got[f][inner[1:]] - ref[f][inner[1:]]))) / scale
        assert err <= 1e-14, (I.GF_NAMES[f], err)
    g = np.stack([np.stack([got[(I.GT + [[0, 1, 2], [1, 3, 4], [2, 4, 5]][a][b],) + grid.interior()]
                            for b in range(3)], -1) for a in range(3)], -2)
    assert np.max(np.abs(np.linalg.det(g) - 1.0)) < 1e-14
    if bc == "static":
        mask = np.ones(grid.shape, dtype=bool)
        mask[inner] = False
        mask[:, :, :, grid.ext[0]:] = False
        assert np.array_equal(got[mask], u[mask])
    else:
        gg, n = grid.ghost, grid.n
        ext = got[inner]
        for a in (1, 2, 3):
            ext = np.take(ext, np.arange(-gg, n[3 - a] + gg) % n[3 - a], axis=a)
        assert np.array_equal(got[:, :, :, : grid.ext[0]], ext)


@pytest.mark.parametrize("order,ghost,n", [(4, 3, (37, 21, 13)), (8, 5, (29, 17, 11))])
def test_momentum_constraint_against_oracle(torch_cuda, order, ghost, n):
    """Momentum constraint through the C ABI on perturbed Brill-Lindquist data
    (sinusoids on chi, gt, K and At so that every term is nonzero) of a ragged
    patch, against the oracle's, per component to 1e-12 of its max."""
    from paper_1307_6488_amd.chemora import Patch
    grid = I.Grid(n, ghost, 0.125, (1.1, -0.6, 0.35))
    p = I.config_params(order, 1, ghost, ghost, I.BC_STATIC)
    u = I.brill_lindquist(grid)
    I.add_sinusoids(u, grid, np.random.default_rng(77), 1e-2, [I.CHI] + [I.GT + s for s in range(6)] + [I.TRK] +
                    [I.AT + s for s in range(6)], periodic_ghosts=False)
    say(f"momentum constraint order {order} n={n}")
    got = Patch(p, grid, u).momentum_constraint().cpu().numpy()
    torch_cuda.cuda.synchronize()
    ref = oracle.momentum(p, grid, u, nthreads=NTHREADS)
    for a in range(3):
        scale = float(np.max(np.abs(ref[a])))
        assert scale > 1e-3
        err = float(np.max(np.abs(got[a] - ref[a]))) / scale
        say(f"  M_{'xyz'[a]}: max |M| {scale:.3e}, rel err {err:.2e}")
        assert err <= 1e-12, (a, err)


def test_check_finite(torch_cuda):
    from paper_1307_6488_amd import chemora as C
    w = I.workload(2, n_override=12)
    u = w.make_state()
    P = C.Patch(w.params, w.grid, u)
    assert C.chemora_check_finite(P.params, P.patch) == 0
    P.u[5, w.grid.ghost + 3, w.grid.ghost + 2, w.grid.ghost + 1] = float("nan")
    P.u[0, w.grid.ghost, w.grid.ghost, w.grid.ghost] = float("inf")
    P.u[0, 0, 0, 0] = float("nan")                     # a ghost: not counted
    assert C.chemora_check_finite(P.params, P.patch) == 2


def _small_patches(count=6, seed=5, off_axis=False):
    rng = np.random.default_rng(seed)
    grids = []
    for p in range(count):
        n = [int(v) for v in rng.integers(9, 40, size=3)]
        h = 1.0 / 8.0 if p % 2 else 1.0 / 16.0
        c = rng.uniform(-4, 4, size=3)
        if off_axis:            # keep the patch at least ~1 M away from the punctures
            c[1] = rng.uniform(3.5, 5.0)
        grids.append(I.Grid(tuple(n), 3, h, tuple(float(c[a] - (n[a] - 1) * h / 2) for a in range(3))))
    return grids


def test_batched_plan_equals_per_patch_steps(torch_cuda):
    """One plan over uneven patches (each its own h and dt = courant h)
    advances every patch exactly as per-patch rk4_step calls do (bitwise:
    the same tile code runs in both), and graph replays are deterministic."""
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    params = I.workload(2).params
    grids = _small_patches()
    states = [I.brill_lindquist(g) for g in grids]
    say("batched plan: " + " ".join(str(g.n) for g in grids))
    courant = 0.25
    B = C.Batch(params, grids, states, courant)
    assert B.points() == sum(g.npoints for g in grids)
    B.step(3)
    torch.cuda.synchronize()
    got = [p.u.cpu().numpy() for p in B.patches]
    B2 = C.Batch(params, grids, states, courant)
    B2.step(1)
    B2.step(2)
    torch.cuda.synchronize()
    again = [p.u.cpu().numpy() for p in B2.patches]
    for g, u0, a, b in zip(grids, states, got, again):
        ref = gpu_rk4(torch, params, g, u0, courant * g.h, 3)
        assert np.array_equal(a, ref, equal_nan=True)
        assert np.array_equal(b, ref, equal_nan=True)
    B.close()
    B2.close()


@pytest.mark.parametrize("integrator", ["rk4", "rk3"])
def test_persistent_plan_equals_per_tile_dispatch(torch_cuda, integrator):
    """Plans launch each stage persistently by default: resident work-groups
    pull tiles from per-XCD queues that every launch leaves zeroed for the
    next.  The same plan dispatched one work-group per tile computes the
    same bits, and so do per-patch steps, over several graph replays, with
    two tile-variant groups (two launches and two queue sets per stage) of
    which one has fewer tiles than there are XCDs (its work-groups pull from
    other XCDs' queues)."""
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    params = I.workload(2).params
    grids = _small_patches(count=5, seed=31) + [bl_grid((9, 3, 3), 3)]
    states = [I.brill_lindquist(g) for g in grids]
    P = C.make_params(params)
    tiny = C.make_patch(grids[-1], 0x7F0000001000)   # class key only
    before = C.chemora_tile_variant(P, tiny)
    C.chemora_set_tile_variant(P, tiny, 0)            # 64x4: 3 tiles for the tiny patch
    try:
        out = {}
        for mode in (C.DISPATCH_PERSISTENT, C.DISPATCH_PER_TILE):
            B = C.Batch(params, grids, states, 0.25, integrator=integrator, dispatch=mode)
            assert B.dispatch() == mode
            variants = B.variants()
            B.step(2)
            B.step(3)
            torch.cuda.synchronize()
            out[mode] = [p.u.cpu().numpy() for p in B.patches]
            B.close()
        say(f"persistent vs per-tile {integrator}: variants {variants}")
        assert variants[-1] == 0 and len(set(variants)) == 2, variants
        step = gpu_rk3 if integrator == "rk3" else gpu_rk4
        for g, u0, a, b in zip(grids, states, out[C.DISPATCH_PERSISTENT], out[C.DISPATCH_PER_TILE]):
            assert np.array_equal(a, b, equal_nan=True), g.n
            assert np.array_equal(a, step(torch, params, g, u0, 0.25 * g.h, 5), equal_nan=True), g.n
    finally:
        C.chemora_set_tile_variant(P, tiny, before)


@pytest.mark.parametrize("bc", ["static", "periodic"])
def test_rk3_plan_equals_per_patch_steps_and_oracle(torch_cuda, bc):
    """An RK3 plan over uneven patches advances every patch exactly as
    per-patch rk3_step calls do (bitwise), and one patch matches the
    oracle's RK3 (evolution bar)."""
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    params = I.workload(2).params if bc == "static" else I.config_params(4, 1, 3, 3, I.BC_PERIODIC)
    # static: patches kept ~1 M from the punctures and 1e-4 sinusoids in every
    # grid function, as in the RK4 plan test, so that no function starts at
    # zero and the FP64 bar applies (near a puncture only the FP64-accuracy
    # bar does)
    grids = _small_patches(count=4, seed=8, off_axis=bc == "static")
    if bc == "static":
        states = []
        for q, g in enumerate(grids):
            u = I.brill_lindquist(g)
            I.add_sinusoids(u, g, np.random.default_rng(50 + q), 1e-4, range(24), periodic_ghosts=False)
            states.append(u)
    else:
        states = []
        for q, g in enumerate(grids):
            u = I.flat(g)
            I.add_sinusoids(u, g, np.random.default_rng(30 + q), 1e-3, range(24))
            states.append(u)
    say(f"rk3 plan {bc}: " + " ".join(str(g.n) for g in grids))
    courant = 0.25
    B = C.Batch(params, grids, states, courant, integrator="rk3")
    B.step(3)
    torch.cuda.synchronize()
    got = [p.u.cpu().numpy() for p in B.patches]
    B.close()
    for g, u0, a in zip(grids, states, got):
        ref = gpu_rk3(torch, params, g, u0, courant * g.h, 3)
        assert np.array_equal(a, ref, equal_nan=True)
    g0 = grids[0]
    orc = oracle.rk3(params, g0, states[0], courant * g0.h, 3, nthreads=NTHREADS)
    assert_parity(got[0], orc, g0, 1e-10, f"rk3 plan {bc} vs oracle")


def test_batched_plan_matches_oracle(torch_cuda):
    """Per-patch spacing and time step in the batched path against the oracle
    (FP64 bar 1e-10, and the FP64-accuracy bar against the extended-precision
    oracle).  Brill-Lindquist data plus seeded 1e-4 sinusoids in every grid
    function, so that no function starts identically zero."""
    from paper_1307_6488_amd import chemora as C
    params = I.workload(2).params
    grids = _small_patches(count=3, seed=9, off_axis=True)
    states = []
    for n, g in enumerate(grids):
        u = I.brill_lindquist(g)
        I.add_sinusoids(u, g, np.random.default_rng(40 + n), 1e-4, range(24), periodic_ghosts=False)
        states.append(u)
    B = C.Batch(params, grids, states, 0.25)
    B.step(4)
    torch_cuda.cuda.synchronize()
    for g, u0, P in zip(grids, states, B.patches):
        ref = oracle.rk4(params, g, u0, 0.25 * g.h, 4, nthreads=NTHREADS)
        ext = oracle.rk4_ext(params, g, u0, 0.25 * g.h, 4, nthreads=NTHREADS)
        got = P.u.cpu().numpy()
        assert_parity(got, ref, g, 1e-10, f"batched {g.n}")
        assert_fp64_accuracy(got, ref, ext, g, f"batched {g.n}")
    B.close()


@pytest.mark.parametrize("index,n", [(2, (70, 37, 19)), (2, (33, 9, 7)), (3, (45, 20, 13)), (3, (67, 11, 9)),
                                     (3, (36, 17, 6))])
def test_tile_variants_are_bitwise_identical(torch_cuda, index, n):
    """Every tile variant computes every point with the same arithmetic in
    the same order: the right-hand side and two RK4 steps agree bitwise with
    variant 0 (ragged extents in x and y, odd nx, both orders).  At order 8
    the x-outer mixed derivatives move inner stencils across lanes, with the
    halo columns held by the row-edge lanes of the same row (64-wide tiles)
    or of the other row of the wave (32-wide tiles); the extents put valid
    points next to both tile edges and leave narrow last tiles of 3 and 4
    columns."""
    from paper_1307_6488_amd import chemora as C
    w = I.workload(index)
    grid = bl_grid(n, w.params.ghost)
    u = I.brill_lindquist(grid)
    I.add_sinusoids(u, grid, np.random.default_rng(77), 1e-4, range(24), periodic_ghosts=False)
    P, X = C.make_params(w.params), C.make_patch(grid, 0x7F0000001000)   # class key only
    built = [v for v in range(6) if w.params.fd_order == 4 or v in (0, 2)]
    before = C.chemora_tile_variant(P, X)
    ref = None
    try:
        for v in built:
            C.chemora_set_tile_variant(P, X, v)
            assert C.chemora_tile_variant(P, X) == v
            r = gpu_rhs(torch_cuda, w.params, grid, u)
            e = gpu_rk4(torch_cuda, w.params, grid, u, 0.25 * grid.h, 2)
            say(f"variant {v} {C.chemora_tile_variant_shape(v)} x {C.chemora_tile_variant_depth(v)} on {n}: done")
            if ref is None:
                ref = (r, e)
                continue
            assert np.array_equal(r, ref[0], equal_nan=True), v
            assert np.array_equal(e, ref[1], equal_nan=True), v
    finally:
        C.chemora_set_tile_variant(P, X, before)


def test_tuned_plan_matches_per_patch_steps_and_writes_cache(torch_cuda, tmp_path):
    """A plan created with a tune cache times the classes of its patches,
    records them in the cache file, groups the patches by variant, and still
    advances every patch bitwise as per-patch rk4_step calls do."""
    import json
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    params = I.workload(2).params
    grids = _small_patches(count=6, seed=21) + [bl_grid((96, 40, 24), 3), bl_grid((30, 70, 16), 3)]
    states = [I.brill_lindquist(g) for g in grids]
    path = tmp_path / "tiles.json"
    B = C.Batch(params, grids, states, 0.25, tune_cache_path=str(path))
    variants = B.variants()
    say(f"tuned variants: {variants}")
    d = json.loads(path.read_text())
    # each patch runs its class's tuned variant, or (the plan's own timing of
    # the whole pass) one variant for every patch
    table = [C.chemora_tile_variant(C.make_params(params), C.make_patch(g, 0x7F0000001000)) for g in grids]
    assert variants == table or len(set(variants)) == 1, (variants, table)
    assert all(e["variant"] in range(6) and "ms" in e for e in d["entries"].values() if e.get("ms") is not None)
    assert len(d["entries"]) >= len({tuple(v for v in (g.n[0] <= 32, g.n[1] <= 16)) for g in grids})
    B.step(2)
    torch.cuda.synchronize()
    for g, u0, p in zip(grids, states, B.patches):
        ref = gpu_rk4(torch, params, g, u0, 0.25 * g.h, 2)
        assert np.array_equal(p.u.cpu().numpy(), ref, equal_nan=True)
    B.close()
    # a second plan reads the classes from the file (no class is timed again)
    B2 = C.Batch(params, grids[:2], states[:2], 0.25, tune_cache_path=str(path))
    v2 = B2.variants()
    assert v2 == table[:2] or len(set(v2)) == 1, (v2, table[:2])
    B2.close()


def _split_params(chi_split):
    p = I.Params(**vars(I.workload(5, n_override=16).params))
    p.chi_split = chi_split
    return p


def _bl_pert(n, seed):
    g = bl_grid(n, 3)
    u = I.brill_lindquist(g)
    I.add_sinusoids(u, g, np.random.default_rng(seed), 1e-4, range(24), periodic_ghosts=False)
    return g, u


# Split precision.  FP32 unit roundoff is u32 = 2^-24 = 6e-8.  A stencil rounds
# each FP64 difference once (relative u32) and combines <= 20 of them with
# cancellation <= 2; the algebra chains <= ~50 FP32 operations over terms up
# to ~10x the right-hand side they sum to; so a right-hand side is off by
# <~ 100 u32 ~ 6e-6 of its max-norm, and an RK4 step mixes those with weight
# dt.  Bars: 1e-5 for one right-hand side and for 20 steps of evolution (the
# FP64 path meets 1e-12 on the same data).
@pytest.mark.parametrize("n", [(70, 37, 19), (48, 48, 48)])
def test_split_rhs_against_oracle(torch_cuda, n):
    g, u = _bl_pert(n, 5)
    ref = oracle.rhs(I.workload(2).params, g, u, nthreads=NTHREADS)
    errs = {}
    for cs in (0.0, 0.1, float("inf")):
        got = gpu_rhs(torch_cuda, _split_params(cs), g, u)
        e = gf_errors(got, ref, g)
        errs[cs] = e
        say(f"split chi_split={cs} {n}: max err {e.max():.2e} ({I.GF_NAMES[int(np.argmax(e))]})")
        assert np.all(np.isfinite(got[(slice(None),) + g.interior()]))
        assert e.max() <= 1e-5, dict(zip(I.GF_NAMES, e.tolist()))
    # the FP64 chi phase (chi_split = inf) is at least as accurate on chi as
    # the FP32 one (chi_split = 0) near the punctures, where 1/chi is large
    assert errs[float("inf")][I.CHI] <= errs[0.0][I.CHI]


def test_split_evolution_against_fp64(torch_cuda):
    g = bl_grid((48, 48, 48), 3)
    u = I.brill_lindquist(g)
    fp64 = gpu_rk4(torch_cuda, I.workload(2).params, g, u, 0.25 * g.h, 20)
    split = gpu_rk4(torch_cuda, _split_params(0.1), g, u, 0.25 * g.h, 20)
    e = gf_errors(split, fp64, g)
    say(f"split vs FP64, 20 steps 48^3: max {e.max():.2e} ({I.GF_NAMES[int(np.argmax(e))]})")
    assert np.all(np.isfinite(split[(slice(None),) + g.interior()]))
    assert e.max() <= 1e-5, dict(zip(I.GF_NAMES, e.tolist()))


def test_split_rk3_evolution_against_fp64(torch_cuda):
    """The RK3 step in split precision against the FP64 RK3 step (split bar)."""
    g = bl_grid((40, 36, 32), 3)
    u = I.brill_lindquist(g)
    fp64 = gpu_rk3(torch_cuda, I.workload(2).params, g, u, 0.25 * g.h, 20)
    split = gpu_rk3(torch_cuda, _split_params(0.1), g, u, 0.25 * g.h, 20)
    e = gf_errors(split, fp64, g)
    say(f"split vs FP64 RK3, 20 steps: max {e.max():.2e} ({I.GF_NAMES[int(np.argmax(e))]})")
    assert np.all(np.isfinite(split[(slice(None),) + g.interior()]))
    assert e.max() <= 1e-5, dict(zip(I.GF_NAMES, e.tolist()))


def test_split_tile_variants_agree_and_plans_are_bitwise(torch_cuda):
    """Split precision in every tile variant agrees within the split bar (the
    FP32 kernels of different tile shapes and occupancies are compiled
    separately and may form FMAs differently), and a plan advances each
    patch bitwise as per-patch calls with the same variant do."""
    from paper_1307_6488_amd import chemora as C
    p = _split_params(0.1)
    g, u = _bl_pert((33, 9, 7), 8)
    P, X = C.make_params(p), C.make_patch(g, 0x7F0000001000)
    before = C.chemora_tile_variant(P, X)
    ref = None
    try:
        for v in range(4):
            C.chemora_set_tile_variant(P, X, v)
            r = gpu_rhs(torch_cuda, p, g, u)
            if ref is None:
                ref = r
                continue
            e = gf_errors(r, ref, g)
            say(f"split variant {v} vs 0: max {e.max():.2e} ({I.GF_NAMES[int(np.argmax(e))]})")
            assert e.max() <= 1e-5, v
    finally:
        C.chemora_set_tile_variant(P, X, before)
    grids = _small_patches(count=4, seed=33)
    states = [I.brill_lindquist(gg) for gg in grids]
    B = C.Batch(p, grids, states, 0.25)
    B.step(2)
    torch_cuda.cuda.synchronize()
    for gg, u0, pp in zip(grids, states, B.patches):
        assert np.array_equal(pp.u.cpu().numpy(), gpu_rk4(torch_cuda, p, gg, u0, 0.25 * gg.h, 2), equal_nan=True)
    B.close()


@pytest.mark.parametrize("n", [(48, 40, 36), (33, 9, 7)])
def test_hamiltonian_constraint_against_oracle(torch_cuda, n):
    """The GPU Hamiltonian-constraint diagnostic against the oracle's on
    Brill-Lindquist data with 1e-3 sinusoids in every GF (so that H is far
    from zero); bar 1e-10 of max |H| (the same arithmetic as one RHS, whose
    terms cancel into H), and exactly 0 in flat space."""
    from paper_1307_6488_amd.chemora import Patch
    g = bl_grid(n, 3)
    u = I.brill_lindquist(g)
    I.add_sinusoids(u, g, np.random.default_rng(12), 1e-3, range(24), periodic_ghosts=False)
    params = I.workload(2).params
    ref = oracle.hamiltonian(params, g, u, nthreads=NTHREADS)
    got = Patch(params, g, u).hamiltonian().cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say(f"H {n}: max |H| {np.max(np.abs(ref)):.3e}, normalised err {err:.2e}")
    assert np.all(np.isfinite(got)) and err <= 1e-10
    assert np.all(Patch(params, g, I.flat(g)).hamiltonian().cpu().numpy() == 0.0)


def test_periodic_plan_equals_per_patch_steps(torch_cuda):
    """Plans with periodic ghosts: the graph refills every patch's ghosts after
    each stage; bitwise equal to per-patch rk4_step calls, over two graph
    launches, for patches of different shapes and spacings."""
    from paper_1307_6488_amd import chemora as C
    params = I.workload(1).params                       # periodic, centred order 4, KO r=2
    grids = [I.Grid((32, 24, 20), params.ghost, 0.25), I.Grid((17, 40, 9), params.ghost, 0.125),
             I.Grid((64, 8, 12), params.ghost, 0.5)]
    states = []
    for n, g in enumerate(grids):
        u = I.flat(g)
        I.add_sinusoids(u, g, np.random.default_rng(60 + n), 1e-3, range(24), periodic_ghosts=True)
        states.append(u)
    B = C.Batch(params, grids, states, 0.25)
    B.step(1)
    B.step(2)
    torch_cuda.cuda.synchronize()
    for g, u0, p in zip(grids, states, B.patches):
        ref = gpu_rk4(torch_cuda, params, g, u0, 0.25 * g.h, 3)
        got = p.u.cpu().numpy()
        assert np.array_equal(got, ref, equal_nan=True), g.n
        # the ghosts hold periodic images of the interior
        full = got[:, :, :, :g.ext[0]]
        gz, gy, gx = g.ghost, g.ghost, g.ghost
        assert np.array_equal(full[:, :, :, :gx], full[:, :, :, g.n[0]:g.n[0] + gx])
    B.close()


@pytest.mark.parametrize("n", [(1, 1, 1), (1, 5, 3), (65, 1, 2), (2, 33, 1)])
def test_degenerate_extents_against_oracle(torch_cuda, n):
    """Patches one point thick (and a single point): every tile is ragged in
    x and y, the staging clamps almost everything into the ghost box.  The
    patch sits off the symmetry point of the two punctures (at the origin
    K's right-hand side is a near-total cancellation, and one point's
    max-norm would normalise by that remainder)."""
    g = I.Grid(n, 3, 1.0 / 8.0, (1.3, 0.7, -0.4))
    u = I.brill_lindquist(g)
    I.add_sinusoids(u, g, np.random.default_rng(90), 1e-4, range(24), periodic_ghosts=False)
    params = I.workload(2).params
    ref = oracle.rhs(params, g, u, nthreads=NTHREADS)
    assert_parity(gpu_rhs(torch_cuda, params, g, u), ref, g, 1e-12, f"degenerate {n}")
    ref = oracle.rk4(params, g, u, 0.25 * g.h, 2, nthreads=NTHREADS)
    assert_parity(gpu_rk4(torch_cuda, params, g, u, 0.25 * g.h, 2), ref, g, 1e-10, f"degenerate rk4 {n}")


def test_rhs_parity_largest_workload(torch_cuda):
    """The largest single-patch workload (256^3, 3 ghosts, order 4 upwind,
    FP64): the full right-hand side against the oracle's, element by element."""
    w = I.workload(5)
    params = I.Params(**vars(w.params))
    params.precision = I.PREC_FP64
    u = w.make_state()
    say(f"rhs parity at {w.grid.n}")
    got = gpu_rhs(torch_cuda, params, w.grid, u)
    ref = oracle.rhs(params, w.grid, u, nthreads=NTHREADS)
    assert_parity(got, ref, w.grid, 1e-12, "rhs 256^3")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name,index", [("bl128_o4_100steps", 2), ("blpert192_o8_50steps", 3)])
def test_full_size_evolution_against_oracle_samples(torch_cuda, name, index):
    """Full-size multi-step evolution in the benchmark's launch configuration,
    compared at the oracle's sampled points (tests/golden, written by
    make_golden.py from the oracle alone), normalised per GF by the oracle's
    max-norm over the whole grid; bar 1e-10."""
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"{name}.npz not generated")
    z = np.load(path)
    w = I.workload(index)
    steps = int(z["steps"])
    say(f"full-size evolution {name}: {steps} steps on {w.grid.n}")
    got = gpu_rk4(torch_cuda, w.params, w.grid, w.make_state(), float(z["dt"]), steps)
    g = w.grid.ghost
    idx = z["idx"]
    samp = got[:, idx[:, 2] + g, idx[:, 1] + g, idx[:, 0] + g]
    ref = z["samples"]
    err = np.max(np.abs(samp - ref), axis=1) / np.maximum(z["maxabs"], 1e-300)
    say(f"{name}: max err {err.max():.3e} ({I.GF_NAMES[int(np.argmax(err))]})")
    assert np.all(np.isfinite(samp))
    assert err.max() <= 1e-10, dict(zip(I.GF_NAMES, err.tolist()))


# The ABI's least strides: sy = nx + 2g (even nx; + 1 for odd nx), sz and sf
# without padding, odd sy / sz / sf, and ghost wider than the stencils reach
# (g - R odd), so that the staged pairs of doubles sit only 8-byte aligned.
MIN_STRIDE_CASES = [
    # (id, order, upwind, ko_radius, ghost, n, row_pad)
    ("o4-upwind-g4-odd-strides", 4, 1, 3, 4, (22, 13, 9), 1),
    ("o4-upwind-g3-odd-nx-least-sy", 4, 1, 3, 3, (21, 14, 11), 1),
    ("o4-centred-r2-g3-even-nx", 4, 0, 2, 3, (26, 11, 8), 0),
    ("o8-upwind-g6-odd-strides", 8, 1, 5, 6, (18, 11, 9), 1),
]


@pytest.mark.parametrize("case", MIN_STRIDE_CASES, ids=[c[0] for c in MIN_STRIDE_CASES])
def test_least_strides_and_wide_ghosts_against_oracle(torch_cuda, case):
    name, order, upwind, ko, ghost, n, pad = case
    g = I.Grid(n, ghost, 1.0 / 8.0, tuple(-(v - 1) / 16.0 + 0.37 for v in n), row_align=1, row_pad=pad)
    assert g.sy == n[0] + 2 * ghost + pad
    if n[0] % 2:
        assert g.sy >= n[0] + 2 * ghost + 1
    p = I.config_params(order, upwind, ghost, ko, I.BC_STATIC)
    u = I.brill_lindquist(g)
    I.add_sinusoids(u, g, np.random.default_rng(1330 + order + ghost), 1e-4, range(I.NGF), periodic_ghosts=False)
    I.poison_padding(u, g)
    say(f"least strides {name}: n={n} g={ghost} sy={g.sy} sz={g.sz} sf={g.sf}")
    got = gpu_rhs(torch_cuda, p, g, u)
    ref = oracle.rhs(p, g, u, nthreads=NTHREADS)
    assert_parity(got, ref, g, 1e-12, f"least strides rhs {name}")
    dt = 0.25 * g.h
    got = gpu_rk4(torch_cuda, p, g, u, dt, 2)
    ref = oracle.rk4(p, g, u, dt, 2, nthreads=NTHREADS)
    assert_parity(got, ref, g, 1e-10, f"least strides rk4 {name}")


def test_split_precision_bar_against_fp64_oracle(torch_cuda):
    """The split-precision bar at a small size of the 256^3 workload's data
    (Brill-Lindquist, order 4 upwinded, chi_split = 0.1): after 20 RK4 steps
    at 48^3 the split state is within 1e-5 of the FP64 oracle's per GF
    (max-norm normalised), and the RMS of its Hamiltonian constraint (the
    oracle's H of each final state) is at most twice that of the FP64
    oracle's state."""
    g = bl_grid((48, 48, 48), 3)
    u = I.brill_lindquist(g)
    p64 = I.workload(2).params
    dt, nsteps = 0.25 * g.h, 20
    say("split precision bar 48^3, 20 steps")
    split = gpu_rk4(torch_cuda, _split_params(0.1), g, u, dt, nsteps)
    fp64 = gpu_rk4(torch_cuda, p64, g, u, dt, nsteps)
    ref = oracle.rk4(p64, g, u, dt, nsteps, nthreads=NTHREADS)
    assert_parity(fp64, ref, g, 1e-10, "fp64 48^3 20 steps")
    e = gf_errors(split, ref, g)
    say(f"split vs FP64 oracle: max {e.max():.2e} ({I.GF_NAMES[int(np.argmax(e))]})")
    assert np.all(np.isfinite(split[(slice(None),) + g.interior()]))
    assert e.max() <= 1e-5, dict(zip(I.GF_NAMES, e.tolist()))
    h_ref = float(np.sqrt(np.mean(oracle.hamiltonian(p64, g, ref, nthreads=NTHREADS) ** 2)))
    h_split = float(np.sqrt(np.mean(oracle.hamiltonian(p64, g, split, nthreads=NTHREADS) ** 2)))
    say(f"H rms: FP64 oracle {h_ref:.6e}, split {h_split:.6e}, ratio {h_split / h_ref:.6f}")
    assert h_split <= 2.0 * h_ref


# ---- radiative (Sommerfeld) outer boundary: every ghost point evolves ------

class _WholeBox:
    """A grid view whose 'interior' is every stored point of the box (ghosts
    included, row padding not): the points the radiative boundary evolves."""

    def __init__(self, g):
        self.g = g

    def interior(self):
        e = self.g.ext
        return (slice(0, e[2]), slice(0, e[1]), slice(0, e[0]))


RADIATIVE_CASES = [
    # (id, order, upwind, ko, ghost, n, lapse, shift)
    ("o4-upwind-1+log", 4, 1, 3, 3, (37, 22, 15), I.LAPSE_ONE_PLUS_LOG, I.SHIFT_GAMMA_DRIVER),
    ("o8-upwind-1+log", 8, 1, 5, 5, (20, 14, 11), I.LAPSE_ONE_PLUS_LOG, I.SHIFT_GAMMA_DRIVER),
    ("o4-centred-harmonic-frozen-shift", 4, 0, 2, 2, (17, 19, 9), I.LAPSE_HARMONIC, I.SHIFT_FROZEN),
]


def _radiative_case(case):
    name, order, upwind, ko, ghost, n, lapse, shift = case
    h = 1.0 / 8.0
    # off-centre and off every axis: all gradient components, both face ends
    g = I.Grid(n, ghost, h, (0.9, -1.7, 0.6))
    p = I.config_params(order, upwind, ghost, ko, I.BC_RADIATIVE)
    p.lapse, p.shift = lapse, shift
    u = I.brill_lindquist(g)
    I.add_sinusoids(u, g, np.random.default_rng(1360 + order + ghost), 1e-3, range(I.NGF), periodic_ghosts=False)
    return p, g, u


@pytest.mark.parametrize("case", RADIATIVE_CASES, ids=[c[0] for c in RADIATIVE_CASES])
def test_radiative_boundary_rhs_and_steps_against_oracle(torch_cuda, case):
    """Right-hand side at interior and ghost points, 3 RK4 steps and 3 RK3
    steps (ghosts evolved by the boundary condition), per GF over every stored
    point, against the oracle."""
    p, g, u = _radiative_case(case)
    box = _WholeBox(g)
    say(f"radiative {case[0]}: n={g.n} g={g.ghost}")
    got = gpu_rhs(torch_cuda, p, g, u)
    ref = oracle.rhs(p, g, u, nthreads=NTHREADS)
    assert np.all(np.isfinite(ref[(slice(None),) + box.interior()]))
    assert_parity(got, ref, box, 1e-12, f"radiative rhs {case[0]}")
    dt = 0.25 * g.h
    got = gpu_rk4(torch_cuda, p, g, u, dt, 3)
    ref = oracle.rk4(p, g, u, dt, 3, nthreads=NTHREADS)
    assert_parity(got, ref, box, 1e-10, f"radiative rk4 {case[0]}")
    got = gpu_rk3(torch_cuda, p, g, u, dt, 3)
    ref = oracle.rk3(p, g, u, dt, 3, nthreads=NTHREADS)
    assert_parity(got, ref, box, 1e-10, f"radiative rk3 {case[0]}")


def test_radiative_plan_equals_per_patch_steps(torch_cuda):
    """Plans launch the boundary kernel per patch and stage: the same state
    as per-patch RK4 and RK3 steps, bitwise."""
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    p = I.config_params(4, 1, 3, 3, I.BC_RADIATIVE)
    grids = _small_patches(count=3, seed=11, off_axis=True)
    states = []
    for q, g in enumerate(grids):
        u = I.brill_lindquist(g)
        I.add_sinusoids(u, g, np.random.default_rng(60 + q), 1e-3, range(24), periodic_ghosts=False)
        states.append(u)
    say("radiative plans: " + " ".join(str(g.n) for g in grids))
    for integ, step in (("rk4", gpu_rk4), ("rk3", gpu_rk3)):
        B = C.Batch(p, grids, states, 0.25, integrator=integ)
        B.step(2)
        torch.cuda.synchronize()
        got = [q.u.cpu().numpy() for q in B.patches]
        B.close()
        for g, u0, a in zip(grids, states, got):
            ref = step(torch, p, g, u0, 0.25 * g.h, 2)
            assert np.array_equal(a, ref, equal_nan=True), integ
            assert not np.array_equal(a[:, :3], u0[:, :3]), integ     # ghost planes moved


# ---- Psi4 (Weyl scalar of outgoing radiation) ------------------------------

PSI4_CASES = [
    # (id, order, ghost, n, origin): odd extents of a grid centred on the
    # coordinate origin put points on the z axis and at the origin itself
    ("o4-ragged-offcentre", 4, 3, (37, 22, 15), (0.9, -1.7, 0.6)),
    ("o4-through-origin-and-z-axis", 4, 3, (21, 19, 17), None),
    ("o8-ragged", 8, 5, (20, 14, 11), (1.3, 0.4, -0.9)),
]


@pytest.mark.parametrize("case", PSI4_CASES, ids=[c[0] for c in PSI4_CASES])
def test_psi4_against_oracle(torch_cuda, case):
    """Psi4 (real and imaginary part) at every interior point of perturbed
    Brill-Lindquist data with nonzero K and At, against the oracle, per part
    (max-norm normalised, bar 1e-12)."""
    from paper_1307_6488_amd import chemora as C
    name, order, ghost, n, origin = case
    h = 1.0 / 8.0
    g = I.centred_grid(n, ghost, h) if origin is None else I.Grid(n, ghost, h, origin)
    p = I.config_params(order, 1, ghost, ghost, I.BC_STATIC)
    u = I.brill_lindquist(g, centres=((2.05, 0.3, -0.2), (-2.1, -0.25, 0.15)))
    I.add_sinusoids(u, g, np.random.default_rng(1370 + order), 1e-3, range(I.NGF), periodic_ghosts=False)
    say(f"psi4 {name}: n={g.n} order={order}")
    P = C.Patch(p, g, u)
    got = P.psi4().cpu().numpy()
    torch_cuda.cuda.synchronize()
    ref = oracle.psi4(p, g, u, nthreads=NTHREADS)
    assert np.all(np.isfinite(ref)) and np.all(np.isfinite(got))
    for part, what in ((0, "re"), (1, "im")):
        scale = np.max(np.abs(ref[part]))
        err = np.max(np.abs(got[part] - ref[part])) / scale
        say(f"psi4 {name} {what}: max |ref| {scale:.3e}, err {err:.2e}")
        assert scale > 1e-6 and err <= 1e-12, (what, err)


# ---- synchronised plans: ghost exchange, prolongation, restriction ---------

def _split_x(g, cut):
    a = I.Grid((cut, g.n[1], g.n[2]), g.ghost, g.h, g.origin)
    b = I.Grid((g.n[0] - cut, g.n[1], g.n[2]), g.ghost, g.h, (g.origin[0] + cut * g.h, g.origin[1], g.origin[2]))
    return a, b


def _sub_state(u, sub, off):
    v = I.alloc_state(sub)
    e = sub.ext
    v[:, :, :, :e[0]] = u[:, :, :, off:off + e[0]]
    return v


@pytest.mark.parametrize("integ", ["rk4", "rk3"])
def test_synced_plan_two_patch_split_equals_single_grid(torch_cuda, integ):
    """One grid split into two abutting patches in a synchronised plan is
    bitwise the single grid stepped alone (same kernels, ghost exchange after
    every stage)."""
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    p = I.config_params(4, 1, 3, 3, I.BC_STATIC)
    g = I.Grid((45, 20, 14), 3, 0.125, (1.1, -1.3, 0.4))
    u = I.brill_lindquist(g)
    I.add_sinusoids(u, g, np.random.default_rng(1400), 1e-3, range(I.NGF), periodic_ghosts=False)
    a, b = _split_x(g, 19)
    dt = 0.25 * g.h
    say(f"synced split {integ}: {g.n} -> {a.n} + {b.n}")
    B = C.Batch(p, [a, b], [_sub_state(u, a, 0), _sub_state(u, b, 19)], integrator=integ, synced_dt=dt)
    B.step(3)
    torch.cuda.synchronize()
    got = [q.u.cpu().numpy() for q in B.patches]
    B.close()
    ref = (gpu_rk4 if integ == "rk4" else gpu_rk3)(torch, p, g, u, dt, 3)
    assert np.array_equal(got[0][:, :, :, :a.ext[0]], ref[:, :, :, :a.ext[0]])
    assert np.array_equal(got[1][:, :, :, :b.ext[0]], ref[:, :, :, 19:19 + b.ext[0]])


def _two_level(order, ghost, bc):
    """Two abutting coarse patches (h = 1/4) and one refined patch (h = 1/8)
    straddling their interface: Brill-Lindquist data (punctures outside the
    patches, so that the FP64 evolution bar applies) plus 1e-3 sinusoids."""
    hc = 0.25
    c0 = I.Grid((14, 22, 20), ghost, hc, (-3.5, -2.75, -2.5))
    c1 = I.Grid((12, 22, 20), ghost, hc, (-3.5 + 14 * hc, -2.75, -2.5))
    hf = hc / 2
    f = I.Grid((21, 18, 15), ghost, hf, (-3.5 + 19 * hf, -2.75 + 13 * hf, -2.5 + 17 * hf))
    grids = [c0, c1, f]
    p = I.config_params(order, 1, ghost, ghost, bc)
    states = []
    for q, g in enumerate(grids):
        u = I.brill_lindquist(g, centres=((4.5, 0.3, -0.2), (-5.0, -0.25, 0.15)))
        I.add_sinusoids(u, g, np.random.default_rng(1410 + q), 1e-3, range(I.NGF), periodic_ghosts=False)
        states.append(u)
    return p, grids, states


@pytest.mark.parametrize("order,ghost,bc,integ", [(4, 3, I.BC_STATIC, 4), (4, 3, I.BC_RADIATIVE, 4),
                                                  (4, 3, I.BC_STATIC, 3), (8, 5, I.BC_STATIC, 4)],
                         ids=["o4-static-rk4", "o4-radiative-rk4", "o4-static-rk3", "o8-static-rk4"])
def test_synced_plan_two_levels_against_oracle(torch_cuda, order, ghost, bc, integ):
    """A refined patch across the interface of two coarse patches, stepped in
    a synchronised plan, against the oracle's synchronised steps: every stored
    point of every patch (evolution bar)."""
    from paper_1307_6488_amd import chemora as C
    torch = torch_cuda
    p, grids, states = _two_level(order, ghost, bc)
    dt = 0.25 * grids[2].h
    say(f"synced two-level order {order} bc {bc} integrator {integ}: " + " ".join(str(g.n) for g in grids))
    B = C.Batch(p, grids, states, integrator="rk4" if integ == 4 else "rk3", synced_dt=dt)
    B.step(3)
    torch.cuda.synchronize()
    got = [q.u.cpu().numpy() for q in B.patches]
    B.close()
    ref = oracle.steps_synced(p, grids, states, dt, 3, integ, nthreads=NTHREADS)
    for q, (g, a, r) in enumerate(zip(grids, got, ref)):
        assert_parity(a, r, _WholeBox(g), 1e-10, f"synced patch {q}")


def test_bbh_share_rk3_step_against_oracle(torch_cuda):
    """The paper's production shape on one GPU -- 90^3 interior points, 5
    ghost zones, 8th-order partially upwinded stencils, third-order
    Runge-Kutta, the share holding a puncture -- in the launch configuration
    the benchmark times: one step against the oracle (evolution bar) and the
    FP64-accuracy bar against the extended-precision oracle (near the puncture
    the FP64 oracle itself is off by up to ~3e-12 after one step)."""
    w = I.bbh_share()
    u = w.make_state()
    say(f"bbh share {w.name}: one RK3 step")
    got = gpu_rk3(torch_cuda, w.params, w.grid, u, w.dt, 1)
    orc = oracle.rk3(w.params, w.grid, u, w.dt, 1, nthreads=NTHREADS)
    assert_parity(got, orc, w.grid, 1e-10, "bbh share rk3")
    ext = oracle.rk3_ext(w.params, w.grid, u, w.dt, 1, nthreads=NTHREADS)
    assert_fp64_accuracy(got, orc, ext, w.grid, "bbh share rk3 fp64 accuracy")
