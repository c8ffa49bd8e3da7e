"""Host-only checks of the C ABI (no GPU needed).

The library must load, export every function include/chemora.h declares, and
reject every invalid argument on the host with CHEMORA_EINVAL (or
EUNSUPPORTED) before any HIP call -- so these run without a GPU.
"""
import ctypes
import os
import re

import pytest

from paper_1307_6488_amd import chemora as C
from paper_1307_6488_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x7F0000001000          # never dereferenced: validation fails first


def header_functions():
    text = open(os.path.join(ROOT, "include", "chemora.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chemora_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = C.lib()
    declared = header_functions()
    assert set(declared) == set(C.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name
    assert C.chemora_abi_version() == 103


def test_plan_dispatch_mode_checks():
    L = C.lib()
    assert L.chemora_set_plan_dispatch(3) == C.EINVAL
    assert L.chemora_set_plan_dispatch(-1) == C.EINVAL
    assert L.chemora_plan_dispatch(None) == C.EINVAL
    assert L.chemora_set_plan_dispatch(C.DISPATCH_PER_TILE) == C.OK
    assert L.chemora_set_plan_dispatch(C.DISPATCH_PERSISTENT) == C.OK
    assert L.chemora_set_plan_dispatch(C.DISPATCH_AUTO) == C.OK


def test_required_ghost_matches_inputs():
    for o, u, r in [(4, 0, 2), (4, 1, 3), (8, 1, 5), (8, 0, 0), (4, 0, 0)]:
        assert C.chemora_required_ghost(o, u, r) == I.required_ghost(o, u, r)
    assert C.chemora_required_ghost(6, 0, 0) < 0


def _good():
    w = I.workload(2, n_override=16)
    return I.Params(**vars(w.params)), w.grid


def _call_rhs(p, g, u=FAKE, rhs=FAKE + (1 << 34)):
    P = C.make_params(p)
    X = C.make_patch(g, u)
    return C.lib().chemora_bssn_rhs(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(rhs), None)


def _call_rk4(p, g, dt=0.01, scratch=FAKE + (1 << 34), u=FAKE):
    P = C.make_params(p)
    X = C.make_patch(g, u)
    return C.lib().chemora_rk4_step(ctypes.byref(P), ctypes.byref(X), dt, ctypes.c_void_p(scratch), None)


BAD_PARAMS = [
    ("fd_order", 6, C.EINVAL, "fd_order"),
    ("ghost", 2, C.EINVAL, "ghost"),
    ("upwind", 2, C.EINVAL, "upwind"),
    ("ko_radius", 4, C.EUNSUPPORTED, "ko_radius"),
    ("eps_diss", -0.1, C.EINVAL, "eps_diss"),
    ("eps_diss", float("nan"), C.EINVAL, "eps_diss"),
    ("lapse", 3, C.EINVAL, "lapse"),
    ("shift", 2, C.EINVAL, "shift"),
    ("eta", float("inf"), C.EINVAL, "eta"),
    ("bc", 5, C.EINVAL, "bc"),
    ("precision", 7, C.EUNSUPPORTED, "precision"),
]


def test_split_precision_validation_on_host():
    p, g = _good()
    p.precision = I.PREC_SPLIT
    for bad in (-1.0, float("nan")):
        p.chi_split = bad
        assert _call_rhs(p, g) == C.EINVAL and "chi_split" in C.last_error()
    w8 = I.workload(3, n_override=16)
    p8 = I.Params(**vars(w8.params))
    p8.precision = I.PREC_SPLIT
    assert _call_rhs(p8, w8.grid) == C.EUNSUPPORTED and "fd_order 4 only" in C.last_error()


@pytest.mark.parametrize("field,value,code,word", BAD_PARAMS)
def test_invalid_params_rejected_on_host(field, value, code, word):
    p, g = _good()
    setattr(p, field, value)
    assert _call_rhs(p, g) == code
    assert word in C.last_error()
    assert _call_rk4(p, g) == code


def test_invalid_patch_rejected_on_host():
    p, g = _good()
    for n in [(0, 16, 16), (16, -1, 16)]:
        gg = I.Grid(n, g.ghost, g.h)
        X = C.make_patch(gg, FAKE)
        X.n[0], X.n[1], X.n[2] = n
        P = C.make_params(p)
        assert C.lib().chemora_bssn_rhs(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 34)),
                                        None) == C.EINVAL
    P = C.make_params(p)
    for field, value in [("sy", g.n[0]), ("sz", g.sy), ("sf", g.sz), ("h", 0.0), ("h", float("nan")),
                         ("reserved", 1)]:
        X = C.make_patch(g, FAKE)
        setattr(X, field, value)
        assert C.lib().chemora_bssn_rhs(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 34)),
                                        None) == C.EINVAL, field
    # null / misaligned / aliased pointers
    assert _call_rhs(p, g, u=0) == C.EINVAL
    assert _call_rhs(p, g, rhs=0) == C.EINVAL
    assert _call_rhs(p, g, u=FAKE + 4) == C.EINVAL
    assert _call_rhs(p, g, rhs=FAKE + 8 * 100) == C.EINVAL
    assert "overlaps" in C.last_error()
    assert C.lib().chemora_bssn_rhs(None, None, None, None) == C.EINVAL
    # odd nx needs one element of row padding
    go = I.Grid((17, 16, 16), g.ghost, g.h)
    X = C.make_patch(go, FAKE)
    X.sy = 17 + 2 * g.ghost
    X.sz = X.sy * (16 + 2 * g.ghost)
    X.sf = X.sz * (16 + 2 * g.ghost)
    assert C.lib().chemora_bssn_rhs(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 34)),
                                    None) == C.EINVAL
    assert "row padding" in C.last_error()
    # periodic boundary needs n >= ghost
    p.bc = I.BC_PERIODIC
    gg = I.Grid((2, 16, 16), p.ghost, g.h)
    assert _call_rhs(p, gg) == C.EINVAL


def test_size_limits_rejected_on_host():
    """A 24-GF state over 4 GiB (32-bit byte offsets) is EUNSUPPORTED with a
    hint to split the patch; extents beyond the launch geometry are EINVAL."""
    p, _ = _good()
    P = C.make_params(p)
    big = I.Grid((300, 300, 300), p.ghost, 0.125)             # 306^3 padded: 5.2 GB of state
    X = C.make_patch(big, FAKE)
    assert C.lib().chemora_bssn_rhs(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 40)),
                                    None) == C.EUNSUPPORTED
    assert "4 GiB" in C.last_error()
    ok = I.Grid((280, 280, 256), p.ghost, 0.125)              # just under the limit
    X = C.make_patch(ok, FAKE)
    assert 24 * ok.sf * 8 + 64 <= 1 << 32
    assert C.lib().chemora_rk4_scratch_elems(ctypes.byref(X)) == 3 * 24 * ok.sf
    tall = I.Grid((8, 70000, 1), p.ghost, 0.125)
    X = C.make_patch(tall, FAKE)
    assert C.lib().chemora_bssn_rhs(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 40)),
                                    None) == C.EINVAL
    assert "launch geometry" in C.last_error()


def test_rk4_argument_checks_on_host():
    p, g = _good()
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        assert _call_rk4(p, g, dt=dt) == C.EINVAL
    assert _call_rk4(p, g, scratch=0) == C.EINVAL
    assert _call_rk4(p, g, scratch=FAKE + 8 * 5) == C.EINVAL      # overlaps u
    X = C.make_patch(g, FAKE)
    assert C.chemora_rk4_scratch_elems(X) == 3 * 24 * g.sf
    assert C.lib().chemora_rk4_scratch_elems(None) == 0


def test_radiative_boundary_needs_finite_origin_on_host():
    p, g = _good()
    p.bc = I.BC_RADIATIVE
    bad = I.Grid(g.n, g.ghost, g.h, (0.0, float("nan"), 0.0))
    assert _call_rhs(p, bad) == C.EINVAL and "origin" in C.last_error()
    assert _call_rk4(p, bad) == C.EINVAL and "origin" in C.last_error()
    # the same origin is metadata for the other boundaries
    p.bc = I.BC_STATIC
    assert _call_rhs(p, bad, u=0) == C.EINVAL and "origin" not in C.last_error()


def test_rk4_noalloc_argument_checks_on_host():
    p, g = _good()

    def call(p, g, dt=0.01, u=FAKE):
        P = C.make_params(p)
        X = C.make_patch(g, u)
        return C.lib().chemora_rk4_step_noalloc(ctypes.byref(P), ctypes.byref(X), dt, None)

    for dt in (0.0, -1.0, float("nan"), float("inf")):
        assert call(p, g, dt=dt) == C.EINVAL and "dt" in C.last_error()
    assert call(p, g, u=0) == C.EINVAL
    bad = I.Params(**vars(p))
    bad.fd_order = 6
    assert call(bad, g) == C.EINVAL
    # a patch whose three scratch states exceed the per-GPU buffer (128^3:
    # 3 * 24 * 134^2 * 136 doubles) is refused before any HIP call
    big = I.workload(2).grid
    X = C.make_patch(big, FAKE)
    assert C.chemora_rk4_scratch_elems(X) > C.NOALLOC_SCRATCH_ELEMS
    assert call(p, big) == C.EINVAL and "scratch" in C.last_error()
    # the header's limit is the binding's
    text = open(os.path.join(ROOT, "include", "chemora.h")).read()
    assert "#define CHEMORA_NOALLOC_SCRATCH_ELEMS ((size_t)8 << 20)" in text
    assert C.NOALLOC_SCRATCH_ELEMS == 8 << 20


def test_rk3_argument_checks_on_host():
    p, g = _good()
    P = C.make_params(p)

    def call(dt=0.01, scratch=FAKE + (1 << 34), u=FAKE, params=P):
        X = C.make_patch(g, u)
        return C.lib().chemora_rk3_step(ctypes.byref(params), ctypes.byref(X), dt, ctypes.c_void_p(scratch), None)
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        assert call(dt=dt) == C.EINVAL
    assert call(scratch=0) == C.EINVAL
    assert call(scratch=FAKE + 4) == C.EINVAL                         # misaligned
    state = 24 * g.sf * 8
    assert call(scratch=FAKE - 2 * state + 8) == C.EINVAL            # second stage buffer overlaps u
    assert "overlaps" in C.last_error()
    bad = C.make_params(p)
    bad.fd_order = 6
    assert call(params=bad) == C.EINVAL
    X = C.make_patch(g, FAKE)
    assert C.chemora_rk3_scratch_elems(X) == 2 * 24 * g.sf
    assert C.lib().chemora_rk3_scratch_elems(None) == 0


def test_momentum_constraint_argument_checks_on_host():
    p, g = _good()
    P = C.make_params(p)
    X = C.make_patch(g, FAKE)

    def call(M):
        return C.lib().chemora_momentum_constraint(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(M), None)
    assert call(0) == C.EINVAL
    assert call(FAKE + (1 << 34) + 4) == C.EINVAL                     # misaligned
    assert call(FAKE + 8) == C.EINVAL                                  # overlaps u
    assert "overlaps" in C.last_error()


def test_enforce_constraints_argument_checks_on_host():
    p, g = _good()
    bad = C.make_params(p)
    bad.fd_order = 6
    X = C.make_patch(g, FAKE)
    assert C.lib().chemora_enforce_constraints(ctypes.byref(bad), ctypes.byref(X), None) == C.EINVAL
    P = C.make_params(p)
    X = C.make_patch(g, 0)
    assert C.lib().chemora_enforce_constraints(ctypes.byref(P), ctypes.byref(X), None) == C.EINVAL


def test_hamiltonian_argument_checks_on_host():
    p, g = _good()
    P, X = C.make_params(p), C.make_patch(g, FAKE)
    assert C.lib().chemora_hamiltonian(ctypes.byref(P), ctypes.byref(X), None, None) == C.EINVAL
    assert C.lib().chemora_hamiltonian(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + 8 * 7),
                                       None) == C.EINVAL
    assert "overlaps" in C.last_error()
    assert C.lib().chemora_hamiltonian(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 34) + 4),
                                       None) == C.EINVAL


def test_check_finite_argument_checks_on_host():
    p, g = _good()
    P, X = C.make_params(p), C.make_patch(g, FAKE)
    assert C.lib().chemora_check_finite(ctypes.byref(P), ctypes.byref(X), None, None) == C.EINVAL
    X0 = C.make_patch(g, 0)
    n = ctypes.c_int64(0)
    assert C.lib().chemora_check_finite(ctypes.byref(P), ctypes.byref(X0), ctypes.byref(n), None) == C.EINVAL


def test_binding_refuses_to_run_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(C, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(C, "_lib", None)
    with pytest.raises(RuntimeError):
        C.lib()


def test_plan_argument_checks_on_host():
    p, g = _good()
    P = C.make_params(p)
    X = C.make_patch(g, FAKE)
    out = ctypes.c_void_p(0)
    sc = (ctypes.c_void_p * 1)(ctypes.c_void_p(FAKE + (1 << 34)))
    arr = (C.chemora_patch * 1)(X)
    L = C.lib()
    assert L.chemora_plan_create(ctypes.byref(P), arr, sc, 0, 0.25, None, None, ctypes.byref(out)) == C.EINVAL
    assert L.chemora_plan_create(ctypes.byref(P), arr, sc, 1, 0.0, None, None, ctypes.byref(out)) == C.EINVAL
    assert L.chemora_plan_create(ctypes.byref(P), arr, sc, 1, 0.25, None, None, None) == C.EINVAL
    bad = (C.chemora_patch * 2)(X, C.make_patch(g, 0))
    sc2 = (ctypes.c_void_p * 2)(ctypes.c_void_p(FAKE + (1 << 34)), ctypes.c_void_p(FAKE + (1 << 35)))
    assert L.chemora_plan_create(ctypes.byref(P), bad, sc2, 2, 0.25, None, None, ctypes.byref(out)) == C.EINVAL
    assert "patch 1" in C.last_error()
    assert out.value is None
    assert L.chemora_batch_step(None, 1, None) == C.EINVAL
    assert L.chemora_plan_destroy(None) == C.OK
    assert L.chemora_plan_points(None) == 0


def test_plan_rejects_aliased_buffers_on_host():
    """Two patches sharing a state, or a scratch buffer reaching into another
    patch's state or scratch, are rejected before any HIP call."""
    p, g = _good()
    P = C.make_params(p)
    L = C.lib()
    state = 24 * g.sf * 8
    out = ctypes.c_void_p(0)

    def create(us, scs):
        arr = (C.chemora_patch * len(us))(*[C.make_patch(g, u) for u in us])
        sc = (ctypes.c_void_p * len(scs))(*[ctypes.c_void_p(v) for v in scs])
        return L.chemora_plan_create(ctypes.byref(P), arr, sc, len(us), 0.25, None, None, ctypes.byref(out))

    base = FAKE
    far = FAKE + (1 << 36)
    # shared state
    assert create([base, base], [far, far + 4 * state]) == C.EINVAL
    assert "overlaps" in C.last_error()
    # scratch of patch 0 runs into the state of patch 1
    assert create([base, far + 2 * state], [far, far + 8 * state]) == C.EINVAL
    assert "overlaps" in C.last_error()
    # scratch buffers of two patches overlap by one element
    assert create([base, base + state], [far, far + 3 * state - 8]) == C.EINVAL
    assert out.value is None


def test_synced_plan_checks_on_host():
    """Bad dt / integrator, periodic ghosts, spacings that are not a
    power-of-two hierarchy, origins off their lattice and refined patches
    whose ghosts no coarser patch covers are refused before any HIP call."""
    p, _ = _good()
    L = C.lib()
    out = ctypes.c_void_p(0)

    def create(params, grids, dt=0.01, integ=4):
        P = C.make_params(params)
        state = max(24 * g.sf * 8 for g in grids)
        us = [FAKE + q * 4 * state for q in range(len(grids))]
        scs = [FAKE + (1 << 36) + q * 4 * state for q in range(len(grids))]
        arr = (C.chemora_patch * len(grids))(*[C.make_patch(g, u) for g, u in zip(grids, us)])
        sc = (ctypes.c_void_p * len(grids))(*[ctypes.c_void_p(v) for v in scs])
        return L.chemora_plan_create_synced(ctypes.byref(P), arr, sc, len(grids), dt, integ, None, None,
                                            ctypes.byref(out))

    coarse = I.Grid((8, 8, 8), 3, 0.5, (0.0, 0.0, 0.0))
    fine_ok = I.Grid((6, 6, 6), 3, 0.25, (1.0, 1.0, 1.0))
    for dt in (0.0, -1.0, float("nan")):
        assert create(p, [coarse, fine_ok], dt=dt) == C.EINVAL and "dt" in C.last_error()
    assert create(p, [coarse, fine_ok], integ=5) == C.EINVAL and "integrator" in C.last_error()
    per = I.Params(**vars(p))
    per.bc = I.BC_PERIODIC
    assert create(per, [coarse, fine_ok]) == C.EUNSUPPORTED
    # a fine patch reaching past the coarse stored box
    assert create(p, [coarse, I.Grid((20, 6, 6), 3, 0.25, (1.0, 1.0, 1.0))]) == C.EINVAL
    assert "no patch" in C.last_error()
    # origin off the fine lattice; spacing ratio 3
    assert create(p, [coarse, I.Grid((4, 4, 4), 3, 0.25, (1.1, 1.0, 1.0))]) == C.EINVAL
    assert "lattice" in C.last_error()
    assert create(p, [coarse, I.Grid((4, 4, 4), 3, 0.5 / 3, (1.0, 1.0, 1.0))]) == C.EINVAL
    assert "spacing" in C.last_error()
    assert out.value is None


def test_tile_variant_shapes_and_table_on_host():
    assert [C.chemora_tile_variant_shape(v) for v in range(6)] == [(64, 4), (64, 8), (32, 8), (32, 16), (32, 8),
                                                                   (32, 4)]
    assert [C.chemora_tile_variant_depth(v) for v in range(6)] == [1, 1, 1, 1, 2, 4]
    assert C.lib().chemora_tile_variant_shape(6, None, None) == C.EINVAL
    assert C.lib().chemora_tile_variant_depth(6) == C.EINVAL and C.lib().chemora_tile_variant_depth(-1) == C.EINVAL
    p, g = _good()
    P, X = C.make_params(p), C.make_patch(g, FAKE)
    before = C.chemora_tile_variant(P, X)
    try:
        for v in range(6):
            C.chemora_set_tile_variant(P, X, v)
            assert C.chemora_tile_variant(P, X) == v
        assert C.lib().chemora_set_tile_variant(ctypes.byref(P), ctypes.byref(X), 7) == C.EINVAL
        p8 = I.workload(3, n_override=16).params
        P8, X8 = C.make_params(p8), C.make_patch(I.workload(3, n_override=16).grid, FAKE)
        for v in (1, 3, 4, 5):
            assert C.lib().chemora_set_tile_variant(ctypes.byref(P8), ctypes.byref(X8), v) == C.EUNSUPPORTED
        assert "not built for order 8" in C.last_error()
        bad = C.make_params(p)
        bad.fd_order = 6
        assert C.lib().chemora_set_tile_variant(ctypes.byref(bad), ctypes.byref(X), 0) == C.EINVAL
        assert C.lib().chemora_tile_variant(ctypes.byref(bad), ctypes.byref(X)) == C.EINVAL
    finally:
        C.chemora_set_tile_variant(P, X, before)


def test_tune_reads_and_rewrites_the_cache_without_timing_cached_classes(tmp_path):
    """A class with a cache entry is taken from the file, not timed (no HIP
    call), and the file is rewritten as valid JSON holding every entry."""
    import json
    p, _ = _good()
    g = I.Grid((40, 20, 12), p.ghost, 0.125)         # a class no other test touches: buckets x1 y1
    key = f"unknown/o4/u1/r{p.ghost}/fp64/x1/y1"
    path = tmp_path / "tiles.json"
    path.write_text(json.dumps({"format": "chemora tile-variant cache", "version": 1,
                                "entries": {key: {"variant": 2, "tile": "32x8"},
                                            "other/o8/u1/r5/fp64/x4/y3": {"variant": 0}}}, indent=1))
    P, X = C.make_params(p), C.make_patch(g, FAKE)
    assert C.chemora_tile_variant(P, X) == 2          # order-4 default before the cache is read
    v = ctypes.c_int32(-1)
    rc = C.lib().chemora_tune(ctypes.byref(P), ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 34)),
                              str(path).encode(), None, ctypes.byref(v))
    try:
        assert rc == C.OK, C.last_error()
        assert v.value == 2 and C.chemora_tile_variant(P, X) == 2
        d = json.loads(path.read_text())
        assert d["entries"][key]["variant"] == 2 and d["entries"][key]["tile"] == "32x8"
        assert d["entries"]["other/o8/u1/r5/fp64/x4/y3"]["variant"] == 0
    finally:
        C.chemora_set_tile_variant(P, X, 2)


def test_tune_argument_checks_on_host():
    p, g = _good()
    P, X = C.make_params(p), C.make_patch(g, FAKE)
    assert C.lib().chemora_tune(ctypes.byref(P), ctypes.byref(X), None, None, None, None) == C.EINVAL
    assert C.lib().chemora_tune(None, ctypes.byref(X), ctypes.c_void_p(FAKE + (1 << 34)), None, None,
                                None) == C.EINVAL
    assert C.lib().chemora_plan_patch_variant(None, 0) == C.EINVAL
