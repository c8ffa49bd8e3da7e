"""ctypes binding of libchemora.so (the gfx950 BSSN library).

Argument marshalling only: every step of the right-hand side and of the RK4
step runs in the library's HIP kernels.  The functions carry the C names and
take the same arguments (structs by value are built from Python objects).
The library must be built (``python -m paper_1307_6488_amd.build``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; CHEMORA_LIB names another build of the same library
LIB_PATH = os.environ.get("CHEMORA_LIB") or os.path.join(_HERE, "libchemora.so")

OK, EINVAL, EDEVICE, ENOMEM, EUNSUPPORTED, ENOTFINITE = 0, -1, -2, -3, -4, -5
NGF = 24

# Every symbol include/chemora.h declares.
EXPORTS = (
    "chemora_required_ghost", "chemora_bssn_rhs", "chemora_rk4_scratch_elems", "chemora_rk4_step",
    "chemora_rk4_stage", "chemora_check_finite", "chemora_last_error", "chemora_abi_version",
    "chemora_plan_create", "chemora_batch_step", "chemora_plan_points", "chemora_plan_destroy",
    "chemora_plan_patch_variant", "chemora_tune", "chemora_tile_variant", "chemora_set_tile_variant",
    "chemora_tile_variant_shape", "chemora_hamiltonian", "chemora_rk3_scratch_elems", "chemora_rk3_step",
    "chemora_enforce_constraints", "chemora_momentum_constraint", "chemora_plan_create_rk3",
    "chemora_rk4_step_noalloc", "chemora_psi4", "chemora_plan_create_synced", "chemora_tile_variant_depth",
    "chemora_set_plan_dispatch", "chemora_plan_dispatch",
)
# CHEMORA_NOALLOC_SCRATCH_ELEMS of include/chemora.h
NOALLOC_SCRATCH_ELEMS = 8 << 20


class chemora_params(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int32), ("ghost", ctypes.c_int32), ("upwind", ctypes.c_int32),
                ("ko_radius", ctypes.c_int32), ("eps_diss", ctypes.c_double), ("lapse", ctypes.c_int32),
                ("shift", ctypes.c_int32), ("eta", ctypes.c_double), ("bc", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("chi_split", ctypes.c_double)]


class chemora_patch(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("reserved", ctypes.c_int32), ("sy", ctypes.c_int64),
                ("sz", ctypes.c_int64), ("sf", ctypes.c_int64), ("h", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("u", ctypes.c_void_p)]


class ChemoraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chemora error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1307_6488_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, X = ctypes.POINTER(chemora_params), ctypes.POINTER(chemora_patch)
        L.chemora_required_ghost.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.chemora_required_ghost.restype = ctypes.c_int
        L.chemora_bssn_rhs.argtypes = [P, X, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_bssn_rhs.restype = ctypes.c_int
        L.chemora_rk4_scratch_elems.argtypes = [X]
        L.chemora_rk4_scratch_elems.restype = ctypes.c_size_t
        L.chemora_rk4_step.argtypes = [P, X, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_rk4_step.restype = ctypes.c_int
        L.chemora_rk4_step_noalloc.argtypes = [P, X, ctypes.c_double, ctypes.c_void_p]
        L.chemora_rk4_step_noalloc.restype = ctypes.c_int
        L.chemora_rk4_stage.argtypes = [P, X, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_rk4_stage.restype = ctypes.c_int
        L.chemora_rk3_scratch_elems.argtypes = [X]
        L.chemora_rk3_scratch_elems.restype = ctypes.c_size_t
        L.chemora_rk3_step.argtypes = [P, X, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_rk3_step.restype = ctypes.c_int
        L.chemora_enforce_constraints.argtypes = [P, X, ctypes.c_void_p]
        L.chemora_enforce_constraints.restype = ctypes.c_int
        L.chemora_momentum_constraint.argtypes = [P, X, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_momentum_constraint.restype = ctypes.c_int
        L.chemora_psi4.argtypes = [P, X, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_psi4.restype = ctypes.c_int
        L.chemora_check_finite.argtypes = [P, X, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]
        L.chemora_check_finite.restype = ctypes.c_int
        L.chemora_last_error.argtypes = []
        L.chemora_last_error.restype = ctypes.c_char_p
        L.chemora_plan_create.argtypes = [P, X, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_char_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
        L.chemora_plan_create.restype = ctypes.c_int
        L.chemora_plan_create_rk3.argtypes = L.chemora_plan_create.argtypes
        L.chemora_plan_create_rk3.restype = ctypes.c_int
        L.chemora_plan_create_synced.argtypes = [P, X, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                                 ctypes.c_double, ctypes.c_int32, ctypes.c_char_p, ctypes.c_void_p,
                                                 ctypes.POINTER(ctypes.c_void_p)]
        L.chemora_plan_create_synced.restype = ctypes.c_int
        L.chemora_batch_step.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
        L.chemora_batch_step.restype = ctypes.c_int
        L.chemora_plan_points.argtypes = [ctypes.c_void_p]
        L.chemora_plan_points.restype = ctypes.c_int64
        L.chemora_plan_destroy.argtypes = [ctypes.c_void_p]
        L.chemora_plan_destroy.restype = ctypes.c_int
        L.chemora_hamiltonian.argtypes = [P, X, ctypes.c_void_p, ctypes.c_void_p]
        L.chemora_hamiltonian.restype = ctypes.c_int
        L.chemora_set_plan_dispatch.argtypes = [ctypes.c_int32]
        L.chemora_set_plan_dispatch.restype = ctypes.c_int
        L.chemora_plan_dispatch.argtypes = [ctypes.c_void_p]
        L.chemora_plan_dispatch.restype = ctypes.c_int
        L.chemora_plan_patch_variant.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.chemora_plan_patch_variant.restype = ctypes.c_int
        L.chemora_tune.argtypes = [P, X, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_int32)]
        L.chemora_tune.restype = ctypes.c_int
        L.chemora_tile_variant.argtypes = [P, X]
        L.chemora_tile_variant.restype = ctypes.c_int
        L.chemora_set_tile_variant.argtypes = [P, X, ctypes.c_int32]
        L.chemora_set_tile_variant.restype = ctypes.c_int
        L.chemora_tile_variant_shape.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32)]
        L.chemora_tile_variant_shape.restype = ctypes.c_int
        L.chemora_tile_variant_depth.argtypes = [ctypes.c_int32]
        L.chemora_tile_variant_depth.restype = ctypes.c_int
        L.chemora_abi_version.argtypes = []
        L.chemora_abi_version.restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().chemora_last_error().decode()


def _check(rc: int) -> int:
    if rc != OK:
        raise ChemoraError(rc, last_error())
    return rc


def _check_id(rc: int) -> int:
    """For calls that return a non-negative value or a negative status."""
    if rc < 0:
        raise ChemoraError(rc, last_error())
    return rc


def make_params(p) -> chemora_params:
    """From an object with the chemora_params field names (e.g. inputs.Params)."""
    return chemora_params(p.fd_order, p.ghost, p.upwind, p.ko_radius, p.eps_diss, p.lapse, p.shift, p.eta,
                          p.bc, getattr(p, "precision", 0), getattr(p, "chi_split", 0.1))


def make_patch(grid, u_ptr: int) -> chemora_patch:
    """From an object with n, h, origin, sy, sz, sf (e.g. inputs.Grid) and a
    device address."""
    return chemora_patch((ctypes.c_int32 * 3)(*grid.n), 0, grid.sy, grid.sz, grid.sf, grid.h,
                         (ctypes.c_double * 3)(*grid.origin), ctypes.c_void_p(u_ptr))


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)      # torch.cuda.Stream


# --- the C entry points, same names -------------------------------------------------

def chemora_required_ghost(fd_order: int, upwind: int, ko_radius: int) -> int:
    return lib().chemora_required_ghost(fd_order, upwind, ko_radius)


def chemora_bssn_rhs(params: chemora_params, patch: chemora_patch, rhs_ptr: int, stream=None) -> int:
    return _check(lib().chemora_bssn_rhs(ctypes.byref(params), ctypes.byref(patch), ctypes.c_void_p(rhs_ptr),
                                         _stream(stream)))


def chemora_rk4_scratch_elems(patch: chemora_patch) -> int:
    return int(lib().chemora_rk4_scratch_elems(ctypes.byref(patch)))


def chemora_rk4_step(params: chemora_params, patch: chemora_patch, dt: float, scratch_ptr: int,
                     stream=None) -> int:
    return _check(lib().chemora_rk4_step(ctypes.byref(params), ctypes.byref(patch), dt,
                                         ctypes.c_void_p(scratch_ptr), _stream(stream)))


def chemora_rk4_step_noalloc(params: chemora_params, patch: chemora_patch, dt: float, stream=None) -> int:
    return _check(lib().chemora_rk4_step_noalloc(ctypes.byref(params), ctypes.byref(patch), dt,
                                                 _stream(stream)))


def chemora_rk3_scratch_elems(patch: chemora_patch) -> int:
    return int(lib().chemora_rk3_scratch_elems(ctypes.byref(patch)))


def chemora_rk3_step(params: chemora_params, patch: chemora_patch, dt: float, scratch_ptr: int,
                     stream=None) -> int:
    return _check(lib().chemora_rk3_step(ctypes.byref(params), ctypes.byref(patch), dt,
                                         ctypes.c_void_p(scratch_ptr), _stream(stream)))


def chemora_momentum_constraint(params: chemora_params, patch: chemora_patch, M_ptr: int, stream=None) -> int:
    return _check(lib().chemora_momentum_constraint(ctypes.byref(params), ctypes.byref(patch), ctypes.c_void_p(M_ptr),
                                                    _stream(stream)))


def chemora_psi4(params: chemora_params, patch: chemora_patch, psi4_ptr: int, stream=None) -> int:
    return _check(lib().chemora_psi4(ctypes.byref(params), ctypes.byref(patch), ctypes.c_void_p(psi4_ptr),
                                     _stream(stream)))


def chemora_enforce_constraints(params: chemora_params, patch: chemora_patch, stream=None) -> int:
    return _check(lib().chemora_enforce_constraints(ctypes.byref(params), ctypes.byref(patch), _stream(stream)))


def chemora_rk4_stage(params: chemora_params, patch: chemora_patch, stage: int, dt: float, scratch_ptr: int,
                      stream=None) -> int:
    return _check(lib().chemora_rk4_stage(ctypes.byref(params), ctypes.byref(patch), stage, dt,
                                          ctypes.c_void_p(scratch_ptr), _stream(stream)))


def chemora_check_finite(params: chemora_params, patch: chemora_patch, stream=None) -> int:
    """Number of non-finite interior values (0 when all are finite)."""
    n = ctypes.c_int64(0)
    rc = lib().chemora_check_finite(ctypes.byref(params), ctypes.byref(patch), ctypes.byref(n), _stream(stream))
    if rc not in (OK, ENOTFINITE):
        raise ChemoraError(rc, last_error())
    return int(n.value)


def chemora_plan_create(params: chemora_params, patches, scratch_ptrs, courant: float, tune_cache_path=None,
                        stream=None, rk3: bool = False) -> int:
    """Returns the opaque plan handle (an int).  patches: sequence of
    chemora_patch; scratch_ptrs: device addresses, one per patch; rk3 selects
    chemora_plan_create_rk3."""
    n = len(patches)
    arr = (chemora_patch * n)(*patches)
    sc = (ctypes.c_void_p * n)(*[ctypes.c_void_p(p) for p in scratch_ptrs])
    out = ctypes.c_void_p(0)
    path = tune_cache_path.encode() if tune_cache_path else None
    fn = lib().chemora_plan_create_rk3 if rk3 else lib().chemora_plan_create
    _check(fn(ctypes.byref(params), arr, sc, n, courant, path, _stream(stream), ctypes.byref(out)))
    return out.value


def chemora_plan_create_synced(params: chemora_params, patches, scratch_ptrs, dt: float, integrator: int = 4,
                               tune_cache_path=None, stream=None) -> int:
    """A synchronised plan (one dt, ghosts exchanged between the patches and
    refinement levels); returns the opaque plan handle."""
    n = len(patches)
    arr = (chemora_patch * n)(*patches)
    sc = (ctypes.c_void_p * n)(*[ctypes.c_void_p(p) for p in scratch_ptrs])
    out = ctypes.c_void_p(0)
    path = tune_cache_path.encode() if tune_cache_path else None
    _check(lib().chemora_plan_create_synced(ctypes.byref(params), arr, sc, n, dt, integrator, path, _stream(stream),
                                            ctypes.byref(out)))
    return out.value


def chemora_batch_step(plan: int, nsteps: int, stream=None) -> int:
    return _check(lib().chemora_batch_step(ctypes.c_void_p(plan), nsteps, _stream(stream)))


def chemora_plan_points(plan: int) -> int:
    return int(lib().chemora_plan_points(ctypes.c_void_p(plan)))


def chemora_plan_destroy(plan: int) -> int:
    return _check(lib().chemora_plan_destroy(ctypes.c_void_p(plan)))


def chemora_hamiltonian(params: chemora_params, patch: chemora_patch, h_ptr: int, stream=None) -> int:
    return _check(lib().chemora_hamiltonian(ctypes.byref(params), ctypes.byref(patch), ctypes.c_void_p(h_ptr),
                                            _stream(stream)))


DISPATCH_PERSISTENT, DISPATCH_PER_TILE, DISPATCH_AUTO = 0, 1, 2


def chemora_set_plan_dispatch(mode: int) -> int:
    return _check(lib().chemora_set_plan_dispatch(mode))


def chemora_plan_dispatch(plan: int) -> int:
    return _check_id(lib().chemora_plan_dispatch(ctypes.c_void_p(plan)))


def chemora_plan_patch_variant(plan: int, p: int) -> int:
    return _check_id(lib().chemora_plan_patch_variant(ctypes.c_void_p(plan), p))


def chemora_tune(params: chemora_params, patch: chemora_patch, scratch_ptr: int, cache_path=None,
                 stream=None) -> int:
    """Tile variant of the patch's class (timed on this patch unless known)."""
    v = ctypes.c_int32(-1)
    _check(lib().chemora_tune(ctypes.byref(params), ctypes.byref(patch), ctypes.c_void_p(scratch_ptr),
                              cache_path.encode() if cache_path else None, _stream(stream), ctypes.byref(v)))
    return int(v.value)


def chemora_tile_variant(params: chemora_params, patch: chemora_patch) -> int:
    return _check_id(lib().chemora_tile_variant(ctypes.byref(params), ctypes.byref(patch)))


def chemora_set_tile_variant(params: chemora_params, patch: chemora_patch, variant: int) -> int:
    return _check(lib().chemora_set_tile_variant(ctypes.byref(params), ctypes.byref(patch), variant))


def chemora_tile_variant_shape(variant: int):
    """(tile_x, tile_y) of a tile variant."""
    tx, ty = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().chemora_tile_variant_shape(variant, ctypes.byref(tx), ctypes.byref(ty)))
    return int(tx.value), int(ty.value)


def chemora_tile_variant_depth(variant: int) -> int:
    return _check_id(lib().chemora_tile_variant_depth(variant))


def chemora_abi_version() -> int:
    return lib().chemora_abi_version()


# --- torch conveniences (device memory and streams only) ----------------------------

class Patch:
    """A device-resident patch: torch tensor of the state plus the C structs."""

    def __init__(self, params, grid, state, device="cuda"):
        import torch
        self.params_py, self.grid = params, grid
        self.params = make_params(params)
        if isinstance(state, torch.Tensor):
            self.u = state
        else:
            self.u = torch.from_numpy(state).to(device)
        assert self.u.dtype == torch.float64 and self.u.is_contiguous()
        assert tuple(self.u.shape) == tuple(grid.shape)
        self.patch = make_patch(grid, self.u.data_ptr())
        self._scratch = None

    def scratch(self):
        import torch
        if self._scratch is None:
            n = chemora_rk4_scratch_elems(self.patch)
            self._scratch = torch.empty(n, dtype=torch.float64, device=self.u.device)
        return self._scratch

    def rhs(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.full_like(self.u, float("nan"))
        chemora_bssn_rhs(self.params, self.patch, out.data_ptr(), stream or torch.cuda.current_stream())
        return out

    def hamiltonian(self, stream=None):
        """H at the interior points, as a (nz, ny, nx) torch tensor view."""
        import torch
        h = torch.full((self.grid.sf,), float("nan"), dtype=torch.float64, device=self.u.device)
        chemora_hamiltonian(self.params, self.patch, h.data_ptr(), stream or torch.cuda.current_stream())
        g = self.grid.ghost
        n = self.grid.n
        v = h[: self.grid.sz * (n[2] + 2 * g)].view(n[2] + 2 * g, n[1] + 2 * g, self.grid.sy)
        return v[g:g + n[2], g:g + n[1], g:g + n[0]]

    def momentum_constraint(self, stream=None):
        """M_i at the interior points, as a (3, nz, ny, nx) torch tensor view."""
        import torch
        m = torch.full((3 * self.grid.sf,), float("nan"), dtype=torch.float64, device=self.u.device)
        chemora_momentum_constraint(self.params, self.patch, m.data_ptr(), stream or torch.cuda.current_stream())
        g = self.grid.ghost
        n = self.grid.n
        v = m.view(3, self.grid.sf)[:, : self.grid.sz * (n[2] + 2 * g)].reshape(3, n[2] + 2 * g, n[1] + 2 * g,
                                                                                  self.grid.sy)
        return v[:, g:g + n[2], g:g + n[1], g:g + n[0]]

    def psi4(self, stream=None):
        """Psi4 at the interior points, as a (2, nz, ny, nx) torch tensor view
        (real and imaginary part)."""
        import torch
        m = torch.full((2 * self.grid.sf,), float("nan"), dtype=torch.float64, device=self.u.device)
        chemora_psi4(self.params, self.patch, m.data_ptr(), stream or torch.cuda.current_stream())
        g = self.grid.ghost
        n = self.grid.n
        v = m.view(2, self.grid.sf)[:, : self.grid.sz * (n[2] + 2 * g)].reshape(2, n[2] + 2 * g, n[1] + 2 * g,
                                                                                  self.grid.sy)
        return v[:, g:g + n[2], g:g + n[1], g:g + n[0]]

    def tune(self, cache_path=None, stream=None) -> int:
        import torch
        return chemora_tune(self.params, self.patch, self.scratch().data_ptr(), cache_path,
                            stream or torch.cuda.current_stream())

    def rk4_step(self, dt: float, nsteps: int = 1, stream=None):
        import torch
        s = stream or torch.cuda.current_stream()
        sc = self.scratch().data_ptr()
        for _ in range(nsteps):
            chemora_rk4_step(self.params, self.patch, dt, sc, s)
        return self.u

    def enforce_constraints(self, stream=None):
        """Restore det(gt) = 1 and gt^ij At_ij = 0 at every interior point."""
        import torch
        chemora_enforce_constraints(self.params, self.patch, stream or torch.cuda.current_stream())
        return self.u

    def rk3_step(self, dt: float, nsteps: int = 1, stream=None):
        """Third-order SSP Runge-Kutta steps (the RK4 scratch is large enough)."""
        import torch
        s = stream or torch.cuda.current_stream()
        sc = self.scratch().data_ptr()
        for _ in range(nsteps):
            chemora_rk3_step(self.params, self.patch, dt, sc, s)
        return self.u


class Batch:
    """Several device-resident patches advanced together through a plan."""

    def __init__(self, params, grids, states, courant: float = 0.0, device="cuda", tune_cache_path=None,
                 integrator: str = "rk4", synced_dt: float = 0.0, dispatch: int = DISPATCH_AUTO):
        """Independent patches with dt = courant * h each, or (synced_dt > 0)
        one synchronised grid hierarchy stepped with synced_dt.  dispatch:
        DISPATCH_AUTO, DISPATCH_PERSISTENT or DISPATCH_PER_TILE (the
        process-wide setting is restored to AUTO afterwards)."""
        import torch
        if integrator not in ("rk4", "rk3"):
            raise ValueError(f"integrator {integrator!r} is neither 'rk4' nor 'rk3'")
        self.plan = 0
        self.patches = [Patch(params, g, s, device=device) for g, s in zip(grids, states)]
        self.params = make_params(params)
        scr = [p.scratch().data_ptr() for p in self.patches]
        chemora_set_plan_dispatch(dispatch)
        try:
            if synced_dt > 0.0:
                self.plan = chemora_plan_create_synced(self.params, [p.patch for p in self.patches], scr, synced_dt,
                                                       3 if integrator == "rk3" else 4, tune_cache_path,
                                                       torch.cuda.current_stream())
            else:
                self.plan = chemora_plan_create(self.params, [p.patch for p in self.patches], scr, courant,
                                                tune_cache_path, torch.cuda.current_stream(),
                                                rk3=integrator == "rk3")
        finally:
            chemora_set_plan_dispatch(DISPATCH_AUTO)

    def dispatch(self) -> int:
        return chemora_plan_dispatch(self.plan)

    def variants(self):
        return [chemora_plan_patch_variant(self.plan, p) for p in range(len(self.patches))]

    def step(self, nsteps: int = 1, stream=None):
        import torch
        chemora_batch_step(self.plan, nsteps, stream or torch.cuda.current_stream())

    def points(self) -> int:
        return chemora_plan_points(self.plan)

    def close(self):
        if self.plan:
            chemora_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
