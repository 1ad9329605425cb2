"""Pins of the oracle's effective window and of its error against the position shift (§4.2, §4.3; CPU only).

* the effective window equals the taper at the sample points, where the phase
  gradient cancels (§4.2);
* the closed form a^T R(s) a of one shift's side-lobe energy against quadrature
  of |f(x, s)|^2 over the side lobes, for random tapers;
* R(s) averaged over |s| <= h is the appendix's Rbar;
* the error depends on the position as §4.3 describes: symmetric in s, lowest
  near the centre, largest where the main lobe wraps around (s = h);
* tests/golden/fig34_shift_error.txt (the data of the figures of the effective
  window and of the error against position) is what tests/golden/make_fig34.py
  computes from the oracle now.
"""

import importlib.util
import os

import numpy as np
import pytest

from oracle import taper as ot
from synth import pswf_taper_1d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _gl(a, b, step=1.0, order=8):
    x0, w0 = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(a, b, max(1, int(np.ceil((b - a) / step))) + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    return ((hi - lo) / 2 * x0 + (hi + lo) / 2).ravel(), ((hi - lo) / 2 * w0 + 0 * lo).ravel()


@pytest.mark.parametrize("L", [8, 24, 32])
def test_effective_window_is_the_taper_at_the_samples(L):
    rng = np.random.default_rng(L)
    a = rng.standard_normal(L)
    for s in (0.0, 1.7, -5.25, L / 2 - 0.5):
        f = ot.effective_window(a, s, np.arange(L))
        assert np.abs(f - a).max() < 1e-13
    # between the samples the phase gradient no longer cancels
    f = ot.effective_window(a, 3.0, np.arange(L) + 0.5)
    assert np.abs(f.imag).max() > 1e-3


def _side_lobe_energy_quadrature(a, s, X=2000.0):
    """int over x < 0 and x >= L of |f(x, s)|^2 dx (index units), plus the 1/x^2 tail beyond X."""
    L = a.size
    k = np.arange(L)
    total = 0.0
    for lo, hi in ((-X, 0.0), (float(L), L + X)):
        x, w = _gl(lo, hi, step=0.5)
        total += w @ np.abs(ot.effective_window(a, s, x)) ** 2
    # far from the field |f|^2 -> sin^2(pi x) |sum_k a_k (-1)^k exp(2 pi i k s / L)|^2 / (pi x)^2 on each side
    A = abs(np.exp(2j * np.pi * k * s / L) @ (a * (-1.0) ** k)) ** 2
    return total + 2 * A / (2 * np.pi ** 2 * X)


@pytest.mark.parametrize("L,s", [(8, 0.0), (8, 2.5), (16, -4.0), (16, 6.5)])
def test_side_lobe_energy_at_one_shift(L, s):
    rng = np.random.default_rng(100 + L)
    a = rng.standard_normal(L)
    a /= np.linalg.norm(a)
    closed = a @ ot.side_lobe_matrix_at_shift(L, s) @ a
    assert abs(closed / _side_lobe_energy_quadrature(a, s) - 1) < 2e-4


@pytest.mark.parametrize("L,beta", [(8, 3), (32, 7)])
def test_shift_matrices_average_to_rbar(L, beta):
    h = ot.shift_half_range(L, beta)
    s, w = _gl(-h, h, step=0.25, order=16)
    mean = sum(wi * ot.side_lobe_matrix_at_shift(L, si) for si, wi in zip(s, w)) / (2 * h)
    assert np.abs(mean - ot.idg_window_matrix(L, h)).max() < 1e-12


def test_error_against_position():
    L, beta = 32, 7
    h = ot.shift_half_range(L, beta)
    eps, a = ot.idg_optimal_window(L, h)
    ss = np.arange(0, h + 0.25, 0.25)
    e = np.array([ot.side_lobe_error_at_shift(a, s) for s in ss])
    assert np.allclose(e, [ot.side_lobe_error_at_shift(a, -s) for s in ss], rtol=1e-9)
    assert e[0] < eps < e[-1]                       # low in the centre, highest at the wrap-around bound
    # rising from the centre to the bound at whole-pixel shifts (between them it ripples by a few per cent
    # with the sub-pixel position), and everywhere in the inner half below the outer pixel
    whole = e[::4]
    assert np.all(np.diff(whole) > 0)
    assert e[ss <= h / 2].max() < e[ss >= h - 1].min()
    # the optimum minimises the mean over positions, not the error at each: the sampled PSWF does better at
    # middle shifts and much worse at the bound
    pswf = np.asarray(pswf_taper_1d(L, beta), np.float64)
    assert ot.side_lobe_error_at_shift(pswf, 10) < ot.side_lobe_error_at_shift(a, 10)
    assert ot.side_lobe_error_at_shift(pswf, h) > 2 * ot.side_lobe_error_at_shift(a, h)


def test_figure_data_is_current():
    spec = importlib.util.spec_from_file_location("make_fig34", os.path.join(GOLDEN, "make_fig34.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(GOLDEN, "fig34_shift_error.txt")) as f:
        stored = np.array([[float(v) for v in ln.split()] for ln in f if ln.strip() and not ln.startswith("#")])
    fresh = np.array(mod.rows(), np.float64)
    assert stored.shape == fresh.shape
    assert np.allclose(stored, fresh, rtol=1e-8, atol=0)
