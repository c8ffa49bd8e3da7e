"""Error metric of the parity tests (max-norm normalised per grid function).

For grid function f over the interior points:
    err_f = max |x_f - x_f^ref| / max |x_f^ref|            if max |x_f^ref| > 0
    err_f = max |x_f| / max_g max |x_g^ref|                  if x_f^ref is exactly 0
A function the reference gives as exactly zero is held to ``ZERO_BAR`` of the
largest magnitude over all functions, whatever the bar of the others: a
leak into a function that must vanish is not excused by a loose tolerance.
"""
from __future__ import annotations

import numpy as np

ZERO_BAR = 1e-14


def gf_errors(got, ref, grid, zero_mask=False):
    """Per-GF error (shape (24,)); with zero_mask=True also the boolean mask
    of the functions whose reference is exactly zero."""
    s = (slice(None),) + grid.interior()
    a, b = got[s], ref[s]
    scale = np.max(np.abs(b), axis=(1, 2, 3))
    diff = np.max(np.abs(a - b), axis=(1, 2, 3))
    big = max(float(np.max(scale)), 1e-300)
    zero = scale == 0
    err = np.where(zero, diff / big, diff / np.where(zero, 1.0, scale))
    return (err, zero) if zero_mask else err


def parity_failures(got, ref, grid, tol, zero_tol=ZERO_BAR):
    """{gf index: (err, bar)} of every function above its bar: `tol` for
    functions with a nonzero reference, `zero_tol` for exactly-zero ones."""
    err, zero = gf_errors(got, ref, grid, zero_mask=True)
    bar = np.where(zero, zero_tol, tol)
    bad = np.nonzero(~(err <= bar))[0]
    return {int(f): (float(err[f]), float(bar[f])) for f in bad}
