"""Pins of the oracle's W-layers (w_0p of Algorithms 1 and 2; CPU only).

* with w so large that no block fits without an offset (|w| S^2 > L - 1 - beta),
  the plan without layers drops every sample and the layered plan none; every
  layered subgrid still satisfies the box rule with |w - w_0p|;
* data whose w stays in layer 0 give the same plan and grid with or without layers;
* the layered major cycle model image -> W-layer grids -> degrid matches the
  measurement equation of a point source, w-term included, to the window's
  aliasing level; the dirty image of the measurement equation matches direct
  imaging;
* the layered chain is adjoint: <degrid(image_to_wstack(I)), y> = <I, wstack_to_image(grid(y))>.
"""

import numpy as np
import pytest
from scipy.special import pro_ang1

from oracle import idg
from oracle import image as oim
from oracle.plan import F, make_plan
from synth import pswf_taper_2d
from tests.util import make_mini

N, L, BETA, S = 128, 32, 7, 1.0


def _corr(N):
    alpha = BETA * np.pi / 2
    lx = (np.arange(N) - N // 2) * S / N
    c = np.array([pro_ang1(0, 0, alpha, 2 * li / S)[0] if abs(2 * li / S) < 1 else 1.0 for li in lx])
    return L * c / pro_ang1(0, 0, alpha, 0.0)[0], lx


def _deep_w_workload(seed=31, nbl=5, nt=30):
    rng = np.random.default_rng(seed)
    uvw = np.zeros((nbl, nt, 3))
    t = np.arange(nt)
    for b in range(nbl):
        start = rng.uniform(-N / 4, N / 4, 2)
        vel = rng.uniform(-0.6, 0.6, 2)
        uvw[b, :, 0] = start[0] + vel[0] * t
        uvw[b, :, 1] = start[1] + vel[1] * t
        uvw[b, :, 2] = rng.choice([-1, 1]) * (rng.uniform(30, 40) + 0.3 * t)     # |w| S^2 > L - 1 - beta
    return make_mini(uvw, N=N, L=L, beta=BETA, S=S, taper=pswf_taper_2d(L, BETA))


def _plan(wl, w_step):
    return make_plan(wl.grid_size, wl.image_size, wl.subgrid_size, wl.kernel_size, wl.max_timesteps,
                     wl.aterm_timesteps, wl.baselines, wl.uvw, wl.freqs, wl.flags, w_step)


def test_layers_rescue_deep_w_samples():
    wl = _deep_w_workload()
    assert _plan(wl, 0.0).nr_gridded == 0
    plan = _plan(wl, 4.0)
    assert plan.nr_dropped == 0 and plan.nr_wlayers > 1
    for p in range(plan.nr_subgrids):
        sub = plan.subgrids[p]
        tc = plan.subgrid_samples(p)
        u, v, w = idg.sample_uvw(wl.uvw, wl.freqs, sub[F["bl"]], tc)
        x, y = u * S + N / 2, v * S + N / 2
        ext = BETA + np.ceil(np.abs(w - plan.w_offset(p)) * S * S).max()
        assert (x.max() - x.min()) + ext <= L - 1 and (y.max() - y.min()) + ext <= L - 1
        assert sub[F["x0"]] <= x.min() and x.max() <= sub[F["x0"]] + L - 1


def test_layer_zero_is_the_unlayered_plan():
    rng = np.random.default_rng(3)
    uvw = np.zeros((4, 20, 3))
    uvw[..., 0] = rng.uniform(-30, 30, (4, 1)) + 0.5 * np.arange(20)
    uvw[..., 1] = rng.uniform(-30, 30, (4, 1))
    uvw[..., 2] = rng.uniform(-1.5, 1.5, (4, 20))
    wl = make_mini(uvw, freqs=(299792458.0, 3.1e8), N=N, L=L, beta=BETA, S=S, random_aterms=True,
                   random_taper=True)
    p0, p1 = _plan(wl, 0.0), _plan(wl, 100.0)
    assert np.array_equal(p0.subgrids, p1.subgrids) and np.array_equal(p0.samples, p1.samples)
    g0 = idg.grid(p0, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    g1 = idg.grid(p1, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    assert g1.shape == (1, 4, N, N) and np.array_equal(g0, g1[0])


def _w0s(plan):
    return [(plan.wlayer_min + j) * plan.w_step for j in range(plan.nr_wlayers)]


def test_layered_major_cycle_predicts_the_measurement_equation():
    wl = _deep_w_workload()
    plan = _plan(wl, 4.0)
    corr, lx = _corr(N)
    x0, y0 = N // 2 + 36, N // 2 - 28                      # l = 0.28, m = -0.22
    model = np.zeros((4, N, N))
    model[0, y0, x0] = model[3, y0, x0] = 1.0
    grids = oim.image_to_wstack(model, _w0s(plan), S, corr, corr)
    vis = idg.degrid(plan, wl.uvw, wl.freqs, grids, wl.aterms, wl.taper)
    l0, m0 = lx[x0], lx[y0]
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0) - 1.0
    u, v, w = wl.uvw[..., 0], wl.uvw[..., 1], wl.uvw[..., 2]
    dme = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * n0))
    assert np.abs(w * n0).max() > 1.0                      # the w-term is several turns
    assert np.abs(vis[..., 0, 0] - dme).max() < 1e-4
    assert np.abs(vis[..., 0, 3] - dme).max() < 1e-4 and np.abs(vis[..., 0, 1]).max() < 1e-12


def test_layered_dirty_image_matches_direct_image():
    wl = _deep_w_workload(seed=32)
    plan = _plan(wl, 4.0)
    corr, lx = _corr(N)
    l0, m0 = 0.27, -0.21
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0) - 1.0
    u, v, w = wl.uvw[..., 0], wl.uvw[..., 1], wl.uvw[..., 2]
    y = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * n0))
    vis = np.zeros(wl.uvw.shape[:2] + (1, 4), np.complex64)
    vis[..., 0, 0] = vis[..., 0, 3] = y
    g = idg.grid(plan, wl.uvw, wl.freqs, vis, wl.aterms, wl.taper)
    img = oim.wstack_to_image(g, _w0s(plan), S, corr, corr)[0]
    keep = np.abs(lx) <= 0.35 * S
    n1 = oim.nprime_image(N, S)
    yv = vis[..., 0, 0].astype(np.complex128).ravel()
    ph = (u.ravel()[None, None, :] * lx[None, :, None] + v.ravel()[None, None, :] * lx[:, None, None]
          + w.ravel()[None, None, :] * n1[:, :, None])
    direct = np.exp(2j * np.pi * ph) @ yv
    err = np.abs(img - direct)[np.ix_(keep, keep)].max() / np.abs(direct).max()
    assert err < 1e-4, err


def test_layered_chain_is_adjoint():
    wl = _deep_w_workload(seed=33, nbl=3, nt=12)
    plan = _plan(wl, 4.0)
    rng = np.random.default_rng(9)
    cl, cm = 0.5 + rng.random(N), 0.5 + rng.random(N)
    im = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    yv = wl.vis.astype(np.complex128)
    w0s = _w0s(plan)
    lhs = np.vdot(idg.degrid(plan, wl.uvw, wl.freqs, oim.image_to_wstack(im, w0s, S, cl, cm), wl.aterms,
                             wl.taper), yv)
    rhs = np.vdot(im, oim.wstack_to_image(idg.grid(plan, wl.uvw, wl.freqs, yv, wl.aterms, wl.taper), w0s, S,
                                          cl, cm))
    assert abs(lhs - rhs) / abs(rhs) < 1e-11


def _w0_sign(mp):
    from oracle import plan as op
    orig = op.Plan.w_offset
    mp.setattr(op.Plan, "w_offset", lambda self, p: -orig(self, p))


def _correction_sign(mp):
    orig = oim.nprime_image
    mp.setattr(oim, "nprime_image", lambda N, S: -orig(N, S))


@pytest.mark.parametrize("mutation", [_w0_sign, _correction_sign])
def test_wstack_mutations_are_caught(mutation, monkeypatch):
    mutation(monkeypatch)
    with pytest.raises(AssertionError):
        test_layered_major_cycle_predicts_the_measurement_equation()
    with pytest.raises(AssertionError):
        test_layered_dirty_image_matches_direct_image()


def test_one_pixel_forms_match_the_whole_wstack():
    rng = np.random.default_rng(12)
    n = 32
    g = rng.standard_normal((3, 4, n, n)) + 1j * rng.standard_normal((3, 4, n, n))
    cl, cm = 0.5 + rng.random(n), 0.5 + rng.random(n)
    w0s, S = [-5.0, 0.0, 7.0], 1.0
    xs, ys = rng.integers(0, n, 6), rng.integers(0, n, 6)
    full = oim.wstack_to_image(g, w0s, S, cl, cm)
    assert np.allclose(oim.wstack_to_image_at(g, w0s, S, xs, ys, cl, cm), full[:, ys, xs], rtol=1e-12, atol=1e-9)
    full = oim.image_to_wstack(g[0], w0s, S, cl, cm)
    assert np.allclose(oim.image_to_wstack_at(g[0], w0s, S, xs, ys, cl, cm), full[:, :, ys, xs], rtol=1e-12,
                       atol=1e-9)
