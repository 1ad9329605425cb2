"""Plant plausible mistakes in the oracle (on the CPU) and check that a pin catches each.

The pins of test_oracle_pins must not pass for a wrong oracle: a flipped phase
sign, swapped A-term order, a dropped w-term, an off-by-one subgrid centre,
transposed l/m, a normalised or uncentred subgrid DFT, a degridder that
applies the wrong Jones product, the pixel spacing S/(L-1), column-major Jones
matrices, or a gridder that ignores the taper.
"""

import numpy as np
import pytest

from oracle import idg
from tests import test_oracle_pins as pins

PIN_TESTS = [
    pins.test_impulse_on_pixel,
    pins.test_lattice_identity_grid_vs_direct_image,
    pins.test_lattice_identity_degrid_vs_direct_prediction,
    pins.test_adjoint_identity,
    pins.test_classical_equivalence_single_sample,
    pins.test_integer_shift_moves_the_grid,
    pins.test_brute_force_loops_grid,
    pins.test_brute_force_loops_degrid,
    lambda: pins.test_image_between_lattice_points_matches_direct_image(24),
]


def _n_failing():
    n = 0
    for t in PIN_TESTS:
        try:
            t()
        except AssertionError:
            n += 1
    return n


def _flip_phase_sign(mp):
    orig = idg.phasor_matrix
    mp.setattr(idg, "phasor_matrix", lambda du, dv, w, l, m, n, sign: orig(du, dv, w, l, m, n, -sign))


def _drop_w(mp):
    orig = idg.phasor_matrix
    mp.setattr(idg, "phasor_matrix", lambda du, dv, w, l, m, n, sign: orig(du, dv, 0 * w, l, m, n, sign))


def _transpose_lm(mp):
    orig = idg.lmn
    mp.setattr(idg, "lmn", lambda L, S: (lambda l, m, n: (m, l, n))(*orig(L, S)))


def _centre_off_by_one(mp):
    orig = idg.subgrid_centre
    mp.setattr(idg, "subgrid_centre", lambda sub, N, L, S: tuple(c + 1.0 / S for c in orig(sub, N, L, S)))


def _normalised_dft(mp):
    orig = idg.centred_dft_matrix
    mp.setattr(idg, "centred_dft_matrix", lambda L, sign=-1: orig(L, sign) / L)


def _uncentred_dft(mp):
    def dft(L, sign=-1):
        k = np.arange(L)
        return np.exp(sign * 2j * np.pi * np.mod(np.outer(k, k), L) / L)
    mp.setattr(idg, "centred_dft_matrix", dft)


def _swap_stations(mp):
    # grid with A_s2^H Y A_s1 instead of A_s1^H Y A_s2
    orig = idg.grid_subgrid_image

    def grid_image(plan, p, *a, **k):
        sub = plan.subgrids[p].copy()
        plan.subgrids[p, [8, 9]] = sub[[9, 8]]
        try:
            return orig(plan, p, *a, **k)
        finally:
            plan.subgrids[p] = sub
    mp.setattr(idg, "grid_subgrid_image", grid_image)


def _degrid_wrong_jones(mp):
    orig = idg._jones

    def jones(aterms, slot, st, L):
        a = orig(aterms, slot, st, L)
        return np.conj(np.transpose(a, (0, 2, 1)))    # A^H where A is meant (and vice versa)
    orig_degrid = idg.degrid_subgrid

    def degrid_subgrid(*args, **kw):
        with pytest.MonkeyPatch.context() as inner:
            inner.setattr(idg, "_jones", jones)
            return orig_degrid(*args, **kw)
    mp.setattr(idg, "degrid_subgrid", degrid_subgrid)


def _pixel_spacing_over_l_minus_1(mp):
    # the spacing S/(L-1) that one of the algorithm listings suggests
    def lmn(L, S):
        idx = (np.arange(L, dtype=np.float64) - L // 2) * (S / (L - 1))
        l, m = idx[None, :], idx[:, None]
        return np.broadcast_to(l, (L, L)), np.broadcast_to(m, (L, L)), np.sqrt(1.0 - l * l - m * m) - 1.0
    mp.setattr(idg, "lmn", lmn)


def _jones_column_major(mp):
    orig = idg._jones
    mp.setattr(idg, "_jones", lambda aterms, slot, st, L: np.transpose(orig(aterms, slot, st, L), (0, 2, 1)))


def _taper_ignored_in_gridding(mp):
    orig = idg.grid_subgrid_image
    mp.setattr(idg, "grid_subgrid_image",
               lambda plan, p, uvw, freqs, vis, aterms, taper: orig(plan, p, uvw, freqs, vis, aterms,
                                                                    np.ones_like(taper)))


@pytest.mark.parametrize("mutation", [_flip_phase_sign, _drop_w, _transpose_lm, _centre_off_by_one,
                                      _normalised_dft, _uncentred_dft, _swap_stations, _degrid_wrong_jones,
                                      _pixel_spacing_over_l_minus_1, _jones_column_major,
                                      _taper_ignored_in_gridding],
                         ids=lambda f: f.__name__.strip("_"))
def test_pins_catch_planted_mistake(mutation, monkeypatch):
    mutation(monkeypatch)
    assert _n_failing() >= 1
