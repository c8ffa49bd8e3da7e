"""Exact spacetimes and their BSSN data, by Taylor-mode differentiation (test helper).

Nothing here shares code with the oracle or the HIP library.  Every field is
a truncated multivariate Taylor series ("jet") in (t, x, y, z) about one point,
with numpy long-double coefficients, so derivatives are exact up to rounding
(about 1e-18 relative) -- no finite differences.

A spacetime is turned into BSSN data by the textbook 3+1 split:
gamma_ij = g_ij, beta_i = g_ti, alpha^2 = beta_i beta^i - g_tt,
K_ij = -(d_t gamma_ij - D_i beta_j - D_j beta_i) / (2 alpha), and then the BSSN
change of variables chi = det(gamma)^(-1/3), gt_ij = chi gamma_ij,
K = gamma^ij K_ij, At_ij = chi (K_ij - gamma_ij K / 3), Gt^i = -d_j gt^ij.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List, Sequence

import numpy as np

LD = np.longdouble
N = 3                        # truncation degree of every jet
PAIRS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))
NGF = 24
_IDX = [m for m in itertools.product(range(N + 1), repeat=4) if sum(m) <= N]
_MASK = np.zeros((N + 1,) * 4, dtype=bool)
for _m in _IDX:
    _MASK[_m] = True


class Jet:
    """Truncated Taylor series in (t, x, y, z), total degree <= N."""
    __slots__ = ("c",)

    def __init__(self, c):
        self.c = c

    @staticmethod
    def const(v) -> "Jet":
        c = np.zeros((N + 1,) * 4, dtype=LD)
        c[0, 0, 0, 0] = LD(v)
        return Jet(c)

    @staticmethod
    def var(axis: int, v0) -> "Jet":
        j = Jet.const(v0)
        m = [0, 0, 0, 0]
        m[axis] = 1
        j.c[tuple(m)] = LD(1)
        return j

    @staticmethod
    def lift(v) -> "Jet":
        return v if isinstance(v, Jet) else Jet.const(v)

    def __add__(self, o):
        return Jet(self.c + Jet.lift(o).c)
    __radd__ = __add__

    def __sub__(self, o):
        return Jet(self.c - Jet.lift(o).c)

    def __rsub__(self, o):
        return Jet(Jet.lift(o).c - self.c)

    def __neg__(self):
        return Jet(-self.c)

    def __mul__(self, o):
        if not isinstance(o, Jet):
            return Jet(self.c * LD(o))
        out = np.zeros_like(self.c)
        for (a, b, cc, d) in _IDX:
            v = self.c[a, b, cc, d]
            if v == 0:
                continue
            out[a:, b:, cc:, d:] += v * o.c[: N + 1 - a, : N + 1 - b, : N + 1 - cc, : N + 1 - d]
        out[~_MASK] = 0
        return Jet(out)
    __rmul__ = __mul__

    def __truediv__(self, o):
        if not isinstance(o, Jet):
            return Jet(self.c / LD(o))
        return self * o.pow(-1)

    def __rtruediv__(self, o):
        return Jet.lift(o) * self.pow(-1)

    def __pow__(self, p):
        if isinstance(p, int) and p >= 0:
            r = Jet.const(1)
            for _ in range(p):
                r = r * self
            return r
        return self.pow(p)

    def _series(self, derivs) -> "Jet":
        """f(a0 + D) = sum_n f^(n)(a0)/n! D^n with D nilpotent."""
        a0 = self.c[0, 0, 0, 0]
        D = Jet(self.c.copy())
        D.c[0, 0, 0, 0] = 0
        out = Jet.const(derivs[0])
        Dn = Jet.const(1)
        for n in range(1, N + 1):
            Dn = Dn * D
            out = out + Dn * (derivs[n] / LD(math.factorial(n)))
        return out

    def pow(self, p) -> "Jet":
        a0 = self.c[0, 0, 0, 0]
        p = LD(p)
        derivs, coef = [], LD(1)
        for n in range(N + 1):
            derivs.append(coef * a0 ** (p - n))
            coef = coef * (p - n)
        return self._series(derivs)

    def sqrt(self) -> "Jet":
        return self.pow(LD(1) / LD(2))

    def sin(self) -> "Jet":
        a0 = self.c[0, 0, 0, 0]
        s, c = np.sin(a0), np.cos(a0)
        return self._series([s, c, -s, -c][: N + 1] + [s] * max(0, N - 3))

    def cos(self) -> "Jet":
        a0 = self.c[0, 0, 0, 0]
        s, c = np.sin(a0), np.cos(a0)
        return self._series([c, -s, -c, s][: N + 1] + [c] * max(0, N - 3))

    def d(self, axis: int) -> "Jet":
        """Partial derivative along axis (0 t, 1 x, 2 y, 3 z); valid to degree N-1."""
        c = np.zeros_like(self.c)
        sl_src = [slice(None)] * 4
        sl_dst = [slice(None)] * 4
        sl_src[axis] = slice(1, None)
        sl_dst[axis] = slice(0, N)
        k = np.arange(1, N + 1, dtype=LD).reshape([-1 if a == axis else 1 for a in range(4)])
        c[tuple(sl_dst)] = self.c[tuple(sl_src)] * k
        return Jet(c)

    # values of derivatives at the expansion point
    def val(self) -> float:
        return self.c[0, 0, 0, 0]

    def dspace(self, i: int):
        m = [0, 0, 0, 0]
        m[1 + i] = 1
        return self.c[tuple(m)]

    def dspace2(self, i: int, j: int):
        m = [0, 0, 0, 0]
        m[1 + i] += 1
        m[1 + j] += 1
        fac = 2 if i == j else 1
        return self.c[tuple(m)] * fac

    def dtime(self):
        return self.c[1, 0, 0, 0]


def coords(pt):
    return [Jet.var(a, LD(pt[a])) for a in range(4)]


def det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def inv3(m):
    d = det3(m)
    inv_d = d.pow(-1)
    adj = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            r = [a for a in range(3) if a != j]
            c = [b for b in range(3) if b != i]
            minor = m[r[0]][c[0]] * m[r[1]][c[1]] - m[r[0]][c[1]] * m[r[1]][c[0]]
            adj[i][j] = minor * inv_d if (i + j) % 2 == 0 else -(minor * inv_d)
    return adj, d


def christoffel(gam, gamu):
    """Gamma^k_ij of a 3-metric."""
    dg = [[[gam[a][b].d(1 + m) for b in range(3)] for a in range(3)] for m in range(3)]
    G = [[[None] * 3 for _ in range(3)] for _ in range(3)]
    for k in range(3):
        for i in range(3):
            for j in range(3):
                s = Jet.const(0)
                for l in range(3):
                    s = s + gamu[k][l] * (dg[j][l][i] + dg[i][l][j] - dg[l][i][j])
                G[k][i][j] = s * 0.5
    return G


def ricci(gam, gamu):
    """R_ij = d_k G^k_ij - d_j G^k_ik + G^k_kl G^l_ij - G^k_jl G^l_ik."""
    G = christoffel(gam, gamu)
    R = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            s = Jet.const(0)
            for k in range(3):
                s = s + G[k][i][j].d(1 + k) - G[k][i][k].d(1 + j)
                for l in range(3):
                    s = s + G[k][k][l] * G[l][i][j] - G[k][j][l] * G[l][i][k]
            R[i][j] = s
    return R, G


def adm_from_4metric(g):
    gam = [[g[1 + i][1 + j] for j in range(3)] for i in range(3)]
    betal = [g[0][1 + i] for i in range(3)]
    gamu, _ = inv3(gam)
    betau = [gamu[i][0] * betal[0] + gamu[i][1] * betal[1] + gamu[i][2] * betal[2] for i in range(3)]
    alpha = (betal[0] * betau[0] + betal[1] * betau[1] + betal[2] * betau[2] - g[0][0]).sqrt()
    G = christoffel(gam, gamu)
    Db = [[betal[j].d(1 + i) - (G[0][i][j] * betal[0] + G[1][i][j] * betal[1] + G[2][i][j] * betal[2])
           for j in range(3)] for i in range(3)]
    inv2a = (alpha * 2).pow(-1)
    K = [[-(gam[i][j].d(0) - Db[i][j] - Db[j][i]) * inv2a for j in range(3)] for i in range(3)]
    return gam, K, alpha, betau


def bssn_from_adm(gam, K, alpha, betau, B=(0.0, 0.0, 0.0)) -> List[Jet]:
    gamu, det = inv3(gam)
    chi = det.pow(LD(-1) / LD(3))
    inv_chi = chi.pow(-1)
    gt = [[gam[i][j] * chi for j in range(3)] for i in range(3)]
    gtu = [[gamu[i][j] * inv_chi for j in range(3)] for i in range(3)]
    trK = Jet.const(0)
    for i in range(3):
        for j in range(3):
            trK = trK + gamu[i][j] * K[i][j]
    At = [[(K[i][j] - gam[i][j] * trK * (LD(1) / LD(3))) * chi for j in range(3)] for i in range(3)]
    Xt = [-(gtu[i][0].d(1) + gtu[i][1].d(2) + gtu[i][2].d(3)) for i in range(3)]
    out = [chi] + [gt[a][b] for (a, b) in PAIRS] + [trK] + [At[a][b] for (a, b) in PAIRS]
    out += Xt + [alpha] + list(betau) + [Jet.lift(v) for v in B]
    return out


def minkowski_deformed(pt):
    """Minkowski space in the polynomially deformed coordinates
    T = t + xy/10 + zt/20, X = x + tz/8 + y^2/30, Y = y + tx/12, Z = z + ty/15:
    an exact vacuum solution with nonzero lapse variation, shift and K."""
    t, x, y, z = coords(pt)
    F = [t + x * y * 0.1 + z * t * (1.0 / 20), x + t * z * 0.125 + y * y * (1.0 / 30),
         y + t * x * (1.0 / 12), z + t * y * (1.0 / 15)]
    J = [[F[a].d(b) for b in range(4)] for a in range(4)]
    eta = (-1.0, 1.0, 1.0, 1.0)
    g = [[sum((J[c][a] * J[c][b] * eta[c] for c in range(4)), Jet.const(0)) for b in range(4)] for a in range(4)]
    return g


def gauge_wave_metric(pt, A=0.1, d=1.0):
    """-H dt^2 + H dx^2 + dy^2 + dz^2, H = 1 - A sin(2 pi (x - t)/d)."""
    t, x, y, z = coords(pt)
    H = 1.0 - ((x - t) * (2.0 * math.pi / d)).sin() * A
    zero, one = Jet.const(0), Jet.const(1)
    return [[-H, zero, zero, zero], [zero, H, zero, zero], [zero, zero, one, zero], [zero, zero, zero, one]]


def extract(fields: Sequence[Jet]) -> Dict[str, np.ndarray]:
    """Values, first/second spatial and first time derivatives as float64."""
    u = np.array([float(f.val()) for f in fields])
    d1 = np.array([[float(f.dspace(i)) for i in range(3)] for f in fields])
    d2 = np.array([[float(f.dspace2(a, b)) for (a, b) in PAIRS] for f in fields])
    dt = np.array([float(f.dtime()) for f in fields])
    return {"u": u, "d1": d1, "d2": d2, "dt": dt}
