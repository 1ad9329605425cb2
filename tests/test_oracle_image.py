"""Pins of the oracle's master grid <-> image steps (CPU only).

* brute force: the grid's DTFT at the image pixels written out as a quadruple loop;
* adjoint: image_to_grid is the adjoint of grid_to_image;
* grid -> image of gridded point-source data matches the direct imaging
  equation (§2) to the window's aliasing level between the lattice points;
* the major cycle model image -> grid -> degrid matches the discrete
  measurement equation (§2 eq. DME) of a point source, to the same level.
"""

import numpy as np
import pytest
from scipy.special import pro_ang1

from oracle import idg
from oracle import image as oim
from synth import pswf_taper_2d
from tests.util import make_mini, plan_of


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _continuous_taper(L, beta, S, N):
    """corr[x] = L c(l_x): the separable continuous PSWF window at the master-grid image pixels."""
    alpha = beta * np.pi / 2
    lx = (np.arange(N) - N // 2) * S / N
    c = np.array([pro_ang1(0, 0, alpha, 2 * li / S)[0] if abs(2 * li / S) < 1 else np.nan for li in lx])
    return L * c / pro_ang1(0, 0, alpha, 0.0)[0], lx


def test_grid_to_image_brute_force():
    N = 8
    rng = np.random.default_rng(3)
    g = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    cl, cm = 0.5 + rng.random(N), 0.5 + rng.random(N)
    ref = np.zeros((4, N, N), np.complex128)
    for p in range(4):
        for y in range(N):
            for x in range(N):
                acc = 0j
                for v in range(N):
                    for u in range(N):
                        acc += g[p, v, u] * np.exp(2j * np.pi * ((u - N / 2) * (x - N / 2) + (v - N / 2) * (y - N / 2)) / N)
                ref[p, y, x] = acc / (cm[y] * cl[x])
    assert _rel(oim.grid_to_image(g, cl, cm), ref) < 1e-12


def test_image_to_grid_is_the_adjoint():
    N = 32
    rng = np.random.default_rng(4)
    g = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    im = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    cl, cm = 0.5 + rng.random(N), 0.5 + rng.random(N)
    lhs = np.vdot(oim.image_to_grid(im, cl, cm), g)        # <T^H im, g>
    rhs = np.vdot(im, oim.grid_to_image(g, cl, cm))        # <im, T g>
    assert abs(lhs - rhs) / abs(rhs) < 1e-12


def _tracks(rng, nbl, nt, N):
    uvw = np.zeros((nbl, nt, 3))
    t = np.arange(nt)
    for b in range(nbl):
        start = rng.uniform(-N / 4, N / 4, 2)
        vel = rng.uniform(-0.8, 0.8, 2)
        uvw[b, :, 0] = start[0] + vel[0] * t
        uvw[b, :, 1] = start[1] + vel[1] * t
    return uvw


@pytest.mark.parametrize("L", [24, 32])
def test_dirty_image_matches_direct_image(L):
    N, beta, S = 128, 7, 1.0
    rng = np.random.default_rng(21)
    uvw = _tracks(rng, 6, 40, N)
    l0, m0 = 0.11, -0.07
    y = np.exp(-2j * np.pi * (uvw[..., 0] * l0 + uvw[..., 1] * m0))       # measurement equation, 1 Jy
    vis = np.zeros(uvw.shape[:2] + (1, 4), np.complex64)
    vis[..., 0, 0] = y
    vis[..., 0, 3] = y
    wl = make_mini(uvw, N=N, L=L, beta=beta, S=S, vis=vis, taper=pswf_taper_2d(L, beta))
    plan = plan_of(wl)
    assert plan.nr_dropped == 0
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    corr, lx = _continuous_taper(L, beta, S, N)
    keep = np.abs(lx) <= 0.35 * S
    img = oim.grid_to_image(g[:, :, :], np.where(keep, corr, 1.0), np.where(keep, corr, 1.0))[0]
    u, v = uvw[..., 0].ravel(), uvw[..., 1].ravel()
    direct = (np.exp(2j * np.pi * np.outer(lx, v)) * y.ravel()[None, :]) @ np.exp(2j * np.pi * np.outer(u, lx))
    err = np.abs(img - direct)[np.ix_(keep, keep)].max() / np.abs(direct).max()
    assert err < 1e-4, err


@pytest.mark.parametrize("w_scale", [0.0, 1.0])
def test_major_cycle_predicts_the_measurement_equation(w_scale):
    # model image: a point source of flux 1 (XX = YY) on the image pixel (x0, y0); image -> grid
    # (divided by L c(l) c(m)) -> degrid must give the DME visibilities exp(-2 pi i (u l + v m + w n'))
    N, L, beta, S = 128, 32, 7, 1.0
    rng = np.random.default_rng(22)
    uvw = _tracks(rng, 5, 30, N)
    uvw[..., 2] = w_scale * rng.uniform(-1.5, 1.5, (5, 1))
    wl = make_mini(uvw, N=N, L=L, beta=beta, S=S, taper=pswf_taper_2d(L, beta))
    plan = plan_of(wl)
    assert plan.nr_dropped == 0
    x0, y0 = N // 2 + 17, N // 2 - 11                       # |l|, |m| < 0.35 S
    model = np.zeros((4, N, N), np.complex128)
    model[0, y0, x0] = model[3, y0, x0] = 1.0
    corr, lx = _continuous_taper(L, beta, S, N)
    corr = np.where(np.isfinite(corr), corr, 1.0)
    g = oim.image_to_grid(model, corr, corr)
    vis = idg.degrid(plan, wl.uvw, wl.freqs, g, wl.aterms, wl.taper)
    l0, m0 = lx[x0], lx[y0]
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0) - 1.0
    dme = np.exp(-2j * np.pi * (uvw[..., 0] * l0 + uvw[..., 1] * m0 + uvw[..., 2] * n0))
    err = np.abs(vis[..., 0, 0] - dme).max()
    assert err < 1e-4, err
    assert np.abs(vis[..., 0, 1]).max() < 1e-12 and np.abs(vis[..., 0, 3] - dme).max() < 1e-4


def test_one_pixel_forms_match_the_whole_transform():
    # the per-pixel forms used on grids too large for the whole transform give the same values
    N = 16
    rng = np.random.default_rng(5)
    g = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    cl, cm = 0.5 + rng.random(N), 0.5 + rng.random(N)
    xs, ys = rng.integers(0, N, 7), rng.integers(0, N, 7)
    full = oim.grid_to_image(g, cl, cm)
    assert _rel(oim.grid_to_image_at(g, xs, ys, cl, cm), full[:, ys, xs]) < 1e-12
    full = oim.image_to_grid(g, cl, cm)
    assert _rel(oim.image_to_grid_at(g, xs, ys, cl, cm), full[:, ys, xs]) < 1e-12
