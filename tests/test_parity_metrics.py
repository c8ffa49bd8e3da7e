"""The parity tests' error metric on synthetic arrays (no GPU): a function the
reference gives as exactly zero is held to 1e-14 of the largest magnitude,
independently of the bar of the nonzero functions."""
import numpy as np

from parity_metrics import ZERO_BAR, gf_errors, parity_failures
from paper_1307_6488_amd import inputs as I


def _pair():
    g = I.Grid((5, 4, 3), 2, 0.5)
    rng = np.random.default_rng(7)
    ref = rng.uniform(-2.0, 2.0, size=g.shape)
    ref[3] = 0.0                               # an exactly-zero function
    ref[5] *= 1e-6                             # a small but nonzero one
    return g, ref


def test_relative_error_of_nonzero_functions():
    g, ref = _pair()
    got = ref.copy()
    s = (0,) + tuple(x.start + 1 for x in g.interior())
    got[s] += 1e-9 * np.max(np.abs(ref[0][g.interior()]))
    got[(5,) + s[1:]] += 3e-7 * np.max(np.abs(ref[5][g.interior()]))
    e = gf_errors(got, ref, g)
    assert abs(e[0] - 1e-9) < 1e-15 and abs(e[5] - 3e-7) < 1e-13
    assert np.all(e[[f for f in range(24) if f not in (0, 5)]] == 0.0)


def test_zero_function_bar_is_absolute_fraction_of_largest():
    g, ref = _pair()
    big = np.max(np.abs(ref[(slice(None),) + g.interior()]))
    s = (3,) + tuple(x.start for x in g.interior())
    ok, leak = ref.copy(), ref.copy()
    ok[s] = 0.5 * ZERO_BAR * big
    leak[s] = 10.0 * ZERO_BAR * big
    # a loose bar for the nonzero functions does not excuse the leak
    assert parity_failures(ok, ref, g, 1e-5) == {}
    bad = parity_failures(leak, ref, g, 1e-5)
    assert list(bad) == [3] and bad[3][1] == ZERO_BAR
    assert parity_failures(leak, ref, g, 1e-5, zero_tol=1e-12) == {}


def test_ghosts_and_padding_are_ignored():
    g, ref = _pair()
    got = ref.copy()
    got[:, 0, :, :] = np.nan                  # a ghost plane
    got[:, :, :, -1] = 1e30                   # row padding / x ghosts
    assert parity_failures(got, ref, g, 1e-12) == {}


def test_nan_inside_fails():
    g, ref = _pair()
    got = ref.copy()
    got[(1,) + tuple(x.start for x in g.interior())] = np.nan
    assert 1 in parity_failures(got, ref, g, 1e-12)
