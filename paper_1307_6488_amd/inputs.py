"""Seeded synthetic inputs for the BSSN right-hand side and its RK4 step.

This module is the one piece shared by the HIP library's callers (tests, bench,
smoke) and by the CPU oracle's tests.  It holds grid geometry, run parameters
and closed-form initial data only; none of the evolution arithmetic (stencils,
right-hand side, Runge-Kutta, boundary filling) lives here.

State layout (used by every caller): one float64 array of shape
``(24, nz + 2g, ny + 2g, sy)`` in C order, i.e. element ``u[f, k, j, i]`` sits at
``f*sf + k*sz + j*sy + i`` with x fastest.  ``sy >= nx + 2g`` is padded to a
multiple of 8 doubles (64 B) and the padding is filled with NaN so that a
reader of padding is caught.  Interior point (i, j, k), 0 <= i < nx, is stored
at array index (i + g, j + g, k + g) and sits at ``origin + (i, j, k) * h``.

Grid-function order (the paper counts the BSSN variables in its section
"Scientific Motivation"; the library evolves the 24 of the moving-puncture
chi-BSSN system):

    0 chi | 1-6 gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz | 7 K |
    8-13 At_xx .. At_zz | 14-16 Gt^x Gt^y Gt^z | 17 alpha |
    18-20 beta^x beta^y beta^z | 21-23 B^x B^y B^z
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

NGF = 24
GF_NAMES = [
    "chi", "gt_xx", "gt_xy", "gt_xz", "gt_yy", "gt_yz", "gt_zz", "K",
    "At_xx", "At_xy", "At_xz", "At_yy", "At_yz", "At_zz",
    "Gt_x", "Gt_y", "Gt_z", "alpha", "beta_x", "beta_y", "beta_z",
    "B_x", "B_y", "B_z",
]
CHI, GT, TRK, AT, XT, ALPHA, BETA, BDRV = 0, 1, 7, 8, 14, 17, 18, 21
# packed symmetric index (xx, xy, xz, yy, yz, zz)
SYM = ((0, 1, 2), (1, 3, 4), (2, 4, 5))

LAPSE_ONE_PLUS_LOG, LAPSE_HARMONIC, LAPSE_FROZEN = 0, 1, 2
SHIFT_GAMMA_DRIVER, SHIFT_FROZEN = 0, 1
BC_STATIC, BC_PERIODIC, BC_RADIATIVE = 0, 1, 2
PREC_FP64, PREC_SPLIT = 0, 1


@dataclasses.dataclass
class Params:
    """Run parameters of the discrete BSSN operator (mirrors the C structs)."""
    fd_order: int = 4          # 4 or 8
    ghost: int = 3
    upwind: int = 1            # 1 = lopsided advection stencils, 0 = centred
    ko_radius: int = 3         # Kreiss-Oliger radius r (0 = off)
    eps_diss: float = 0.1
    lapse: int = LAPSE_ONE_PLUS_LOG
    shift: int = SHIFT_GAMMA_DRIVER
    eta: float = 2.0
    bc: int = BC_STATIC
    precision: int = PREC_FP64
    chi_split: float = 0.1


def required_ghost(fd_order: int, upwind: int, ko_radius: int) -> int:
    """Ghost width the stencils of one right-hand side reach."""
    g = fd_order // 2
    if upwind:
        g = max(g, fd_order // 2 + 1)
    return max(g, ko_radius)


@dataclasses.dataclass
class Grid:
    """One Cartesian patch: interior extents, ghost width, spacing, origin."""
    n: Tuple[int, int, int]
    ghost: int
    h: float
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    row_align: int = 8          # sy is rounded up to a multiple of this
    row_pad: int = 0            # ... then this many elements are added

    @property
    def ext(self) -> Tuple[int, int, int]:
        g = self.ghost
        return (self.n[0] + 2 * g, self.n[1] + 2 * g, self.n[2] + 2 * g)

    @property
    def sy(self) -> int:
        a = self.row_align
        return (self.ext[0] + a - 1) // a * a + self.row_pad

    @property
    def sz(self) -> int:
        return self.sy * self.ext[1]

    @property
    def sf(self) -> int:
        return self.sz * self.ext[2]

    @property
    def shape(self) -> Tuple[int, int, int, int]:
        return (NGF, self.ext[2], self.ext[1], self.sy)

    @property
    def npoints(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def axis_coords(self, axis: int) -> np.ndarray:
        """Coordinates of all stored points (ghosts included) along one axis."""
        idx = np.arange(-self.ghost, self.n[axis] + self.ghost, dtype=np.float64)
        return self.origin[axis] + idx * self.h

    def coords(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """Broadcastable (z, y, x)-ordered coordinate arrays, ghosts included."""
        x = self.axis_coords(0)[None, None, :]
        y = self.axis_coords(1)[None, :, None]
        z = self.axis_coords(2)[:, None, None]
        return x, y, z

    def interior(self) -> Tuple[slice, slice, slice]:
        g = self.ghost
        return (slice(g, g + self.n[2]), slice(g, g + self.n[1]), slice(g, g + self.n[0]))


def centred_grid(n: Sequence[int], ghost: int, h: float, **kw) -> Grid:
    """Grid symmetric about the origin: interior point 0 at -(n-1)h/2 per axis."""
    origin = tuple(-(ni - 1) * h / 2.0 for ni in n)
    return Grid(tuple(int(v) for v in n), ghost, h, origin, **kw)


def alloc_state(grid: Grid, fill: float = np.nan) -> np.ndarray:
    return np.full(grid.shape, fill, dtype=np.float64)


def set_field(u: np.ndarray, grid: Grid, f: int, values) -> None:
    """Write a (z, y, x)-broadcastable field into the unpadded part of GF f."""
    ex = grid.ext
    u[f, :, :, : ex[0]] = np.broadcast_to(values, (ex[2], ex[1], ex[0]))


def poison_padding(u: np.ndarray, grid: Grid) -> None:
    u[:, :, :, grid.ext[0]:] = np.nan


def poison_corners(u: np.ndarray, grid: Grid) -> None:
    """NaN in the 3-D ghost corners (points outside the interior along all
    three axes).  No stencil of the right-hand side reads them: mixed
    derivatives only reach points that are outside along at most two axes."""
    g, n = grid.ghost, grid.n
    for zs in (slice(0, g), slice(g + n[2], g + n[2] + g)):
        for ys in (slice(0, g), slice(g + n[1], g + n[1] + g)):
            for xs in (slice(0, g), slice(g + n[0], g + n[0] + g)):
                u[:, zs, ys, xs] = np.nan


# --------------------------------------------------------------------------
# initial data
# --------------------------------------------------------------------------

def flat(grid: Grid) -> np.ndarray:
    """Minkowski space in Cartesian coordinates: gt = delta, chi = alpha = 1."""
    u = alloc_state(grid)
    for f in range(NGF):
        set_field(u, grid, f, 0.0)
    for f in (CHI, GT + 0, GT + 3, GT + 5, ALPHA):
        set_field(u, grid, f, 1.0)
    return u


def _wrapped_coords(grid: Grid):
    """Coordinates of the periodic image inside the interior of every stored
    point, so that ghost values are bit-identical copies of interior values."""
    out = []
    for a in range(3):
        idx = np.arange(-grid.ghost, grid.n[a] + grid.ghost) % grid.n[a]
        out.append(grid.origin[a] + idx.astype(np.float64) * grid.h)
    x = out[0][None, None, :]
    y = out[1][None, :, None]
    z = out[2][:, None, None]
    return x, y, z


def add_sinusoids(u: np.ndarray, grid: Grid, rng: np.random.Generator, amp: float,
                  gfs: Sequence[int], nwaves: int = 4, periodic_ghosts: bool = True) -> None:
    """Add ``nwaves`` random low-frequency plane waves of amplitude ``amp`` to
    each listed GF.  Wave numbers n_q in {-2..2}^3 minus 0, phases U[0, 2pi);
    draws go GF by GF, then wave by wave, then (n_x, n_y, n_z, phase).  Each
    wave is periodic on the interior box L = n*h."""
    if periodic_ghosts:
        x, y, z = _wrapped_coords(grid)
    else:
        x, y, z = grid.coords()
    L = [grid.n[a] * grid.h for a in range(3)]
    x0 = grid.origin
    for f in gfs:
        acc = np.zeros((grid.ext[2], grid.ext[1], grid.ext[0]))
        for _ in range(nwaves):
            while True:
                kv = rng.integers(-2, 3, size=3)
                if np.any(kv != 0):
                    break
            phi = rng.uniform(0.0, 2.0 * np.pi)
            arg = (2.0 * np.pi * kv[0] * (x - x0[0]) / L[0]
                   + 2.0 * np.pi * kv[1] * (y - x0[1]) / L[1]
                   + 2.0 * np.pi * kv[2] * (z - x0[2]) / L[2] + phi)
            acc = acc + amp * np.sin(arg)
        u[f, :, :, : grid.ext[0]] += acc


def brill_lindquist(grid: Grid, masses=(0.5, 0.5), centres=((3.0, 0.0, 0.0), (-3.0, 0.0, 0.0)),
                    precollapsed: bool = True) -> np.ndarray:
    """Time-symmetric two-puncture data (Brill & Lindquist 1963):
    psi = 1 + sum m_a / (2 r_a) with r_a floored at h/2; chi = psi^-4,
    gt = delta, K = At = Gt = 0, alpha = psi^-2 (precollapsed) or 1, beta = B = 0.
    Ghost points take the same closed form."""
    x, y, z = grid.coords()
    psi = np.ones((grid.ext[2], grid.ext[1], grid.ext[0]))
    for m, c in zip(masses, centres):
        r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
        r = np.maximum(r, grid.h / 2.0)
        psi = psi + m / (2.0 * r)
    u = flat(grid)
    set_field(u, grid, CHI, psi ** -4)
    if precollapsed:
        set_field(u, grid, ALPHA, psi ** -2)
    return u


def gauge_wave_fields(x: np.ndarray, t: float, A: float, d: float):
    """Closed-form gauge wave (Alcubierre et al. 2004): metric
    -H dt^2 + H dx^2 + dy^2 + dz^2, H = 1 - A sin(2 pi (x - t)/d), in BSSN
    variables.  Returns a dict GF index -> array of x."""
    ph = 2.0 * np.pi * (x - t) / d
    H = 1.0 - A * np.sin(ph)
    dH = -A * np.cos(ph) * 2.0 * np.pi / d          # dH/dx
    Kxx = -(np.pi * A / d) * np.cos(ph) / np.sqrt(H)
    chi = H ** (-1.0 / 3.0)
    K = Kxx / H
    out = {
        CHI: chi,
        GT + 0: H ** (2.0 / 3.0), GT + 3: chi, GT + 5: chi,
        TRK: K,
        AT + 0: 2.0 / 3.0 * chi * Kxx, AT + 3: -chi * K / 3.0, AT + 5: -chi * K / 3.0,
        # Gt^x = -d_x (1/gt_xx) = -d_x H^(-2/3) = (2/3) H^(-5/3) H'
        XT + 0: (2.0 / 3.0) * H ** (-5.0 / 3.0) * dH,
        ALPHA: np.sqrt(H),
    }
    return out


def gauge_wave(grid: Grid, A: float = 0.01, d: float = 1.0, t: float = 0.0) -> np.ndarray:
    """Gauge-wave state on a grid periodic in x with period d (and in y, z)."""
    u = flat(grid)
    x, _, _ = _wrapped_coords(grid)
    fields = gauge_wave_fields(x, t, A, d)
    for f, v in fields.items():
        set_field(u, grid, f, v)
    return u


def gauge_wave_grid(nx: int, ghost: int, nyz: int = 8, d: float = 1.0) -> Grid:
    h = d / nx
    return Grid((nx, nyz, nyz), ghost, h, (-d / 2.0, -nyz * h / 2.0, -nyz * h / 2.0))


def uniform_state(grid: Grid, values: Sequence[float]) -> np.ndarray:
    u = alloc_state(grid)
    for f in range(NGF):
        set_field(u, grid, f, float(values[f]))
    return u


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    params: Params
    grid: Grid
    make_state: Callable[[], np.ndarray]
    dt: float
    steps: int


def config_params(order: int, upwind: int, ghost: int, ko_radius: int, bc: int,
                  precision: int = PREC_FP64) -> Params:
    return Params(fd_order=order, ghost=ghost, upwind=upwind, ko_radius=ko_radius,
                  eps_diss=0.1, lapse=LAPSE_ONE_PLUS_LOG, shift=SHIFT_GAMMA_DRIVER,
                  eta=2.0, bc=bc, precision=precision)


def workload(index: int, n_override: Optional[int] = None) -> Workload:
    """The single-patch workloads 1, 2, 3 and 5 (index as numbered in the
    workload table), optionally at a smaller grid for quick runs."""
    if index == 1:
        n = n_override or 32
        grid = centred_grid((n, n, n), 2, 0.25)
        p = config_params(4, 0, 2, 2, BC_PERIODIC)

        def mk():
            u = flat(grid)
            add_sinusoids(u, grid, np.random.default_rng(1308), 1e-3, range(NGF))
            return u
        return Workload("sinusoid-32^3-o4-centred-periodic", p, grid, mk, 0.25 * grid.h, 1)
    if index == 2:
        n = n_override or 128
        grid = centred_grid((n, n, n), 3, 1.0 / 8.0)
        p = config_params(4, 1, 3, 3, BC_STATIC)
        return Workload(f"brill-lindquist-{n}^3-o4-upwind", p, grid,
                        lambda: brill_lindquist(grid), 0.25 * grid.h, 100)
    if index == 3:
        n = n_override or 192
        grid = centred_grid((n, n, n), 5, 1.0 / 8.0)
        p = config_params(8, 1, 5, 5, BC_STATIC)

        def mk():
            u = brill_lindquist(grid)
            add_sinusoids(u, grid, np.random.default_rng(1310), 1e-4,
                          [GT + s for s in range(6)] + [TRK], periodic_ghosts=False)
            return u
        return Workload(f"brill-lindquist-pert-{n}^3-o8-upwind", p, grid, mk, 0.25 * grid.h, 50)
    if index == 5:
        n = n_override or 256
        grid = centred_grid((n, n, n), 3, 1.0 / 8.0)
        p = config_params(4, 1, 3, 3, BC_STATIC, precision=PREC_SPLIT)
        return Workload(f"brill-lindquist-{n}^3-o4-upwind-split", p, grid,
                        lambda: brill_lindquist(grid), 0.25 * grid.h, 100)
    raise ValueError(f"no single-patch workload {index}")


def bbh_share(n_override: Optional[int] = None) -> Workload:
    """One GPU's share of the paper's production binary-black-hole run: 90^3
    interior points with 5 ghost zones, 8th-order partially upwinded stencils
    (Kreiss-Oliger r = 5) and the third-order Runge-Kutta integrator (section
    "Binary Black Hole Simulations with Chemora": 270^3 over 27 GPUs on
    [-6.75, 6.75]^3).  h = 13.5 / 270; the share is the block x in
    [2.25, 6.75) of a 3 x 3 x 3 split, which holds the puncture at x = +3 of
    the Brill-Lindquist data standing in for the paper's QC-0 initial data;
    static ghosts, dt = h / 4."""
    n = n_override or 90
    h = 13.5 / 270.0
    grid = Grid((n, n, n), 5, h, (2.25 + h / 2, -2.25 + h / 2, -2.25 + h / 2))
    p = config_params(8, 1, 5, 5, BC_STATIC)
    return Workload(f"bbh-share-{n}^3-o8-upwind-rk3", p, grid, lambda: brill_lindquist(grid), 0.25 * h, 100)


def patch_list(seed: int = 1311, npatch: int = 64, nmin: int = 24, nmax: int = 96,
               refine: bool = True) -> List[Grid]:
    """Uneven patch set of the batched workload: even patches are cubes with
    edge U{nmin..nmax}; odd ones are boxes whose other edges are
    round(n0 * 2^U(-1,1)) clipped to [nmin, nmax] and to aspect ratio <= 2.
    Spacing M/8 or M/16 (uniform draw), centre U[-6, 6]^3, ghost 3."""
    rng = np.random.default_rng(seed)
    grids = []
    for p in range(npatch):
        n0 = int(rng.integers(nmin, nmax + 1))
        if p % 2 == 0:
            n = [n0, n0, n0]
        else:
            n = [n0]
            for _ in range(2):
                v = int(round(n0 * 2.0 ** rng.uniform(-1.0, 1.0)))
                n.append(v)
            n = [min(max(v, nmin), nmax) for v in n]
            lo = int(math.ceil(max(n) / 2))          # aspect ratio <= 2
            n = [max(v, lo) for v in n]
            perm = rng.permutation(3)
            n = [n[i] for i in perm]
        h = (1.0 / 8.0) if (not refine or rng.uniform() < 0.5) else (1.0 / 16.0)
        c = rng.uniform(-6.0, 6.0, size=3)
        origin = tuple(float(c[a] - (n[a] - 1) * h / 2.0) for a in range(3))
        grids.append(Grid(tuple(n), 3, h, origin))
    return grids
