"""The library's optimal-window generator and rms correction (host code, no GPU) against the oracle."""

import numpy as np
import pytest

import paper_1909_07226_amd as idg
from oracle import taper as ot
from synth import pswf_taper_1d


@pytest.mark.parametrize("L,h", [(8, 3), (16, 6), (24, 9), (32, 13), (32, 12), (48, 20), (64, 29), (32, 11.5), (32, 11)])
def test_optimal_taper_matches_oracle(L, h):
    a, eps = idg.optimal_taper(L, h)
    eps_o, a_o = ot.idg_optimal_window(L, h)
    # both sides build Rbar in float64 (entries rounded to ~1e-17 absolute, with different Si/Ci
    # and eigensolvers), so eps^2 agrees to ~1e-17 absolute: eps to 1e-17 / eps^2 relative
    assert abs(eps / eps_o - 1) < 1e-9 + 2e-17 / eps_o ** 2
    assert np.abs(a - a_o).max() < 1e-6 * np.abs(a_o).max()
    assert a[L // 2] == 1.0


def test_optimal_taper_range_and_arguments():
    # eps^2 ~ 2e-16 at L = 32 with Table 1's bound for beta = 13: beyond float64, reported as IDG_ERANGE
    with pytest.raises(idg.IDGError) as e:
        idg.optimal_taper(32, ot.shift_half_range(32, 13))
    assert e.value.code == -4
    for L, h in ((2, 1), (300, 7), (16, 0.0), (16, 8.5), (16, float("nan"))):
        with pytest.raises(idg.IDGError) as e:
            idg.optimal_taper(L, h)
        assert e.value.code == -1
    assert idg.taper_shift_for_plan(32, 7) == 12.5


@pytest.mark.parametrize("taper_kind", ["optimal", "pswf"])
def test_taper_correction_matches_oracle(taper_kind):
    L, beta, N = 32, 7, 512
    h = idg.taper_shift_for_plan(L, beta)
    a = idg.optimal_taper(L, h)[0] if taper_kind == "optimal" else pswf_taper_1d(L, beta)
    corr = idg.taper_correction(a, h, N)
    ref = ot.taper_correction(a, h, N)
    assert corr.dtype == np.float32 and corr.shape == (N,)
    assert np.abs(corr / ref - 1).max() < 1e-6
    with pytest.raises(idg.IDGError):
        idg.taper_correction(a, h, 1)
