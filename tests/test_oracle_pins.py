"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test checks the oracle against something the paper or plain mathematics
fixes, not against a retyped copy of its own formulas:

* Table 1 column 2 (classical PSWF aliasing) -> the taper / eigenvalue code;
* a sample exactly on a grid pixel must give a single pixel of value L^2 y
  (DFT sign, centring, normalisation, corner offsets);
* the grid's image at the subgrid lattice must equal the direct imaging
  equation (§2, eq. imaging) with A-terms and taper, for any plan;
* degridding a grid whose image lives on the lattice must equal the discrete
  measurement equation (§2, eq. DME) with A-terms and taper;
* degridding must be the adjoint of gridding (§2, eq. derivative: A and A^H);
* with identity A-terms and w = 0 one sample spreads as the sampled taper's
  DTFT, which approximates the continuous PSWF kernel within the Table 1
  aliasing level (classical-gridding equivalence, §2 eq. gridding, §4.2);
* shifting all samples by whole pixels shifts the grid (§3.3: the shifts
  cancel).
"""

import os

import numpy as np
import pytest
from scipy.special import pro_ang1

from oracle import direct, idg
from oracle.plan import F
from oracle.taper import classical_aliasing
from synth import C0, pswf_taper_1d, pswf_taper_2d
from tests.util import make_mini, plan_of, random_track_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b))


def _load_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_classical_pswf.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                b, e = line.split()
                rows.append((int(b), float(e)))
    return rows


@pytest.mark.parametrize("beta,eps_paper", _load_table1())
def test_table1_classical_pswf_column(beta, eps_paper):
    eps = classical_aliasing(beta)
    assert f"{eps:.2e}" == f"{eps_paper:.2e}", (beta, eps, eps_paper)


def test_synth_taper_is_the_pswf():
    # the generator's taper: unit centre, symmetric about L/2, equal to scipy's psi_0 at interior points
    for L, beta in [(24, 7), (32, 7), (16, 5)]:
        a = pswf_taper_1d(L, beta)
        assert a[L // 2] == pytest.approx(1.0, abs=1e-14)
        assert np.allclose(a[1:L // 2], a[L - 1:L // 2:-1], atol=1e-13)
        x = 2 * (-0.5 + np.arange(1, L) / L)
        ref = np.array([pro_ang1(0, 0, beta * np.pi / 2, xi)[0] for xi in x])
        assert np.max(np.abs(a[1:] - ref)) < 1e-8
    # the edge value quoted for L = 24, beta = 7
    assert pswf_taper_1d(24, 7)[0] == pytest.approx(1.924e-4, rel=1e-3)


def test_impulse_on_pixel():
    # a sample exactly on grid pixel (x, y) must give one pixel of value L^2 y there, nothing elsewhere
    N, L = 64, 16
    # (a) one sample at (x, y) = (37, 29)
    uvw = np.array([[[37.0 - N / 2, 29.0 - N / 2, 0.0]]])             # S = 1, f = c0: u = x - N/2
    wl = make_mini(uvw, N=N, L=L, beta=3)
    plan = plan_of(wl)
    assert plan.nr_subgrids == 1 and plan.nr_gridded == 1
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    y = wl.vis[0, 0, 0].astype(np.complex128)
    expect = np.zeros_like(g)
    expect[:, 29, 37] = L * L * y
    assert np.max(np.abs(g - expect)) < 1e-9 * L * L * np.abs(y).max()
    # (b) two channels of one sample on the v = 0 axis at x = 37 and x = 39 share a subgrid
    uvw = np.array([[[37.0 - N / 2, 0.0, 0.0]]])
    freqs = np.array([C0, C0 * (39.0 - N / 2) / (37.0 - N / 2)])
    wl = make_mini(uvw, freqs=freqs, N=N, L=L, beta=3, seed=1)
    plan = plan_of(wl)
    assert plan.nr_subgrids == 1 and plan.nr_gridded == 2
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    y = wl.vis[0, 0].astype(np.complex128)
    expect = np.zeros_like(g)
    expect[:, N // 2, 37] = L * L * y[0]
    expect[:, N // 2, 39] = L * L * y[1]
    assert np.max(np.abs(g - expect)) < 1e-9 * L * L * np.abs(y).max()


def test_lattice_identity_grid_vs_direct_image():
    wl = random_track_workload(seed=3, random_aterms=True, random_taper=True)
    plan = plan_of(wl)
    assert plan.nr_subgrids >= 4 and plan.nr_dropped == 0
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    img = direct.grid_image_at_lattice(g, plan.image_size, plan.subgrid_size)
    ref = direct.direct_image_lattice(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    assert _rel(img, ref) < 1e-12


def test_lattice_identity_degrid_vs_direct_prediction():
    wl = random_track_workload(seed=4, random_aterms=True, random_taper=True)
    plan = plan_of(wl)
    L, N, S = plan.subgrid_size, plan.grid_size, plan.image_size
    rng = np.random.default_rng(11)
    img = rng.standard_normal((4, L, L)) + 1j * rng.standard_normal((4, L, L))
    g = direct.grid_from_lattice_image(img, N, S)
    vis = idg.degrid(plan, wl.uvw, wl.freqs, g, wl.aterms, wl.taper)
    ref = direct.predict_direct_lattice(plan, wl.uvw, wl.freqs, img, wl.aterms, wl.taper)
    assert _rel(vis, ref) < 1e-12


def test_adjoint_identity():
    wl = random_track_workload(seed=5, random_aterms=True, random_taper=True, nbl=4)
    plan = plan_of(wl)
    N = plan.grid_size
    rng = np.random.default_rng(12)
    x = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    y = wl.vis.astype(np.complex128)
    gy = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    dx = idg.degrid(plan, wl.uvw, wl.freqs, x, wl.aterms, wl.taper)
    lhs = np.vdot(dx, y)                     # <degrid(x), y>
    rhs = np.vdot(x, gy)                     # <x, grid(y)>
    assert abs(lhs - rhs) / abs(rhs) < 1e-12


def test_classical_equivalence_single_sample():
    # identity A-terms, w = 0, PSWF taper: the oracle spreads one sample at a fractional pixel
    # position over its subgrid as y * K(dx) * K(dy), K being the continuous classical kernel
    # (the Fourier transform of the PSWF window, psi_0(2 d / beta) inside the support |d| < beta/2),
    # to within the aliasing level Table 1 gives for beta = 7; outside the support the response
    # stays below that level (image-domain gridding reduces to classical gridding, §2 eq. gridding).
    N, L, beta = 128, 32, 7
    eps = 7.96e-5                                      # Table 1, beta = 7, classical PSWF
    for xk, yk in [(70.37, 51.81), (64.0, 64.5), (81.93, 40.02)]:
        uvw = np.array([[[xk - N / 2, yk - N / 2, 0.0]]])
        wl = make_mini(uvw, N=N, L=L, beta=beta, taper=pswf_taper_2d(L, beta))
        plan = plan_of(wl)
        g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
        sub = plan.subgrids[0]
        x0, y0 = sub[F["x0"]], sub[F["y0"]]
        outside = g.copy()
        outside[:, y0:y0 + L, x0:x0 + L] = 0
        assert np.all(outside == 0)
        y = wl.vis[0, 0, 0].astype(np.complex128)
        resp = g[:, y0:y0 + L, x0:x0 + L] / (y[:, None, None] * wl.taper.astype(np.float64).sum())
        dx = x0 + np.arange(L) - xk
        dy = y0 + np.arange(L) - yk

        def kern(d):
            d = np.asarray(d, np.float64)
            out = np.zeros_like(d)
            inside = np.abs(d) < beta / 2
            out[inside] = [pro_ang1(0, 0, beta * np.pi / 2, 2 * di / beta)[0] for di in d[inside]]
            return out

        ref = kern(dy)[:, None] * kern(dx)[None, :]
        # the truncated classical kernel jumps from psi_0(1) to 0 at |d| = beta/2: skip that edge
        keep = (np.abs(np.abs(dy) - beta / 2) > 0.1)[:, None] & (np.abs(np.abs(dx) - beta / 2) > 0.1)[None, :]
        assert np.max(np.abs(resp - ref[None])[:, keep]) < 2 * eps, (xk, yk)
        assert np.max(np.abs(resp)) == pytest.approx(np.max(ref), abs=2 * eps)


def test_integer_shift_moves_the_grid():
    wl = random_track_workload(seed=6, random_aterms=True, nch=1, N=96)
    plan = plan_of(wl)
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    sx, sy = 7, -5
    wl2 = make_mini(wl.uvw + np.array([sx, sy, 0.0]), freqs=wl.freqs, N=wl.grid_size, L=wl.subgrid_size,
                    beta=wl.kernel_size, vis=wl.vis, aterms=wl.aterms, taper=wl.taper)
    plan2 = plan_of(wl2)
    assert np.array_equal(plan2.subgrids[:, F["x0"]], plan.subgrids[:, F["x0"]] + sx)
    assert np.array_equal(plan2.subgrids[:, F["y0"]], plan.subgrids[:, F["y0"]] + sy)
    g2 = idg.grid(plan2, wl2.uvw, wl2.freqs, wl2.vis, wl2.aterms, wl2.taper)
    shifted = np.roll(np.roll(g, sy, axis=1), sx, axis=2)
    assert _rel(g2, shifted) < 1e-10


# ---------------------------------------------------------------------------
# brute force: the algorithms written out as plain loops on a tiny case

def _brute_grid(plan, wl):
    """Algorithm 1 as nested loops: per subgrid, per pixel, per sample; then the DFT as a double sum."""
    N, L, S = plan.grid_size, plan.subgrid_size, plan.image_size
    g = np.zeros((4, N, N), np.complex128)
    for p in range(plan.nr_subgrids):
        sub = plan.subgrids[p]
        bl, x0, y0 = sub[F["bl"]], sub[F["x0"]], sub[F["y0"]]
        slot, s1, s2 = sub[F["slot"]], sub[F["st1"]], sub[F["st2"]]
        u0, v0 = (x0 + L / 2 - N / 2) / S, (y0 + L / 2 - N / 2) / S
        img = np.zeros((4, L, L), np.complex128)
        for j in range(L):
            for i in range(L):
                l, m = (i - L / 2) * S / L, (j - L / 2) * S / L
                n = np.sqrt(1.0 - l * l - m * m) - 1.0
                acc = np.zeros((2, 2), np.complex128)
                for t, c in plan.subgrid_samples(p):
                    scale = wl.freqs[c] / C0
                    u, v, w = (wl.uvw[bl, t, q] * scale for q in range(3))
                    phase = 2.0 * np.pi * ((u - u0) * l + (v - v0) * m + w * n)
                    acc += wl.vis[bl, t, c].astype(np.complex128).reshape(2, 2) * np.exp(1j * phase)
                a1 = wl.aterms[slot, s1, j, i].astype(np.complex128).reshape(2, 2)
                a2 = wl.aterms[slot, s2, j, i].astype(np.complex128).reshape(2, 2)
                img[:, j, i] = (float(wl.taper[j, i]) * (a1.conj().T @ acc @ a2)).ravel()
        for b in range(L):
            for a in range(L):
                tot = np.zeros(4, np.complex128)
                for j in range(L):
                    for i in range(L):
                        tot += img[:, j, i] * np.exp(-2j * np.pi * ((a - L / 2) * (i - L / 2)
                                                                    + (b - L / 2) * (j - L / 2)) / L)
                g[:, y0 + b, x0 + a] += tot
    return g


def _brute_degrid(plan, wl, grid_in):
    """Algorithm 2 as nested loops: split, inverse DFT as a double sum, A-terms and taper, per-sample sum."""
    N, L, S = plan.grid_size, plan.subgrid_size, plan.image_size
    out = np.zeros(wl.vis.shape, np.complex128)
    for p in range(plan.nr_subgrids):
        sub = plan.subgrids[p]
        bl, x0, y0 = sub[F["bl"]], sub[F["x0"]], sub[F["y0"]]
        slot, s1, s2 = sub[F["slot"]], sub[F["st1"]], sub[F["st2"]]
        u0, v0 = (x0 + L / 2 - N / 2) / S, (y0 + L / 2 - N / 2) / S
        bimg = np.zeros((L, L, 2, 2), np.complex128)
        for j in range(L):
            for i in range(L):
                tot = np.zeros(4, np.complex128)
                for b in range(L):
                    for a in range(L):
                        tot += grid_in[:, y0 + b, x0 + a] * np.exp(2j * np.pi * ((a - L / 2) * (i - L / 2)
                                                                                 + (b - L / 2) * (j - L / 2)) / L)
                a1 = wl.aterms[slot, s1, j, i].astype(np.complex128).reshape(2, 2)
                a2 = wl.aterms[slot, s2, j, i].astype(np.complex128).reshape(2, 2)
                bimg[j, i] = float(wl.taper[j, i]) * (a1 @ tot.reshape(2, 2) @ a2.conj().T)
        for t, c in plan.subgrid_samples(p):
            scale = wl.freqs[c] / C0
            u, v, w = (wl.uvw[bl, t, q] * scale for q in range(3))
            acc = np.zeros((2, 2), np.complex128)
            for j in range(L):
                for i in range(L):
                    l, m = (i - L / 2) * S / L, (j - L / 2) * S / L
                    n = np.sqrt(1.0 - l * l - m * m) - 1.0
                    acc += bimg[j, i] * np.exp(-2j * np.pi * ((u - u0) * l + (v - v0) * m + w * n))
            out[bl, t, c] = acc.ravel()
    return out


def _tiny_brute_case():
    wl = random_track_workload(seed=17, N=32, L=8, beta=1, nbl=2, nt=6, nch=2, wscale=0.6, random_aterms=True,
                               random_taper=True)
    plan = plan_of(wl)
    assert plan.nr_subgrids >= 2 and plan.nr_dropped == 0
    return wl, plan


def test_brute_force_loops_grid():
    wl, plan = _tiny_brute_case()
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    assert _rel(g, _brute_grid(plan, wl)) < 1e-12


def test_brute_force_loops_degrid():
    wl, plan = _tiny_brute_case()
    rng = np.random.default_rng(23)
    N = plan.grid_size
    x = rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))
    vis = idg.degrid(plan, wl.uvw, wl.freqs, x, wl.aterms, wl.taper)
    assert _rel(vis, _brute_degrid(plan, wl, x)) < 1e-12


def test_linearity_in_the_visibilities():
    wl = random_track_workload(seed=8, random_aterms=True, random_taper=True)
    plan = plan_of(wl)
    rng = np.random.default_rng(29)
    y2 = (rng.standard_normal(wl.vis.shape) + 1j * rng.standard_normal(wl.vis.shape)).astype(np.complex64)
    alpha = 0.75 - 1.25j
    y12 = alpha * wl.vis.astype(np.complex128) + y2
    g1 = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    g2 = idg.grid(plan, wl.uvw, wl.freqs, y2, wl.aterms, wl.taper)
    g12 = idg.grid(plan, wl.uvw, wl.freqs, y12, wl.aterms, wl.taper)
    assert _rel(g12, alpha * g1 + g2) < 1e-12


# ---------------------------------------------------------------------------
# between the lattice points: image-domain gridding approximates the direct image

@pytest.mark.parametrize("L", [24, 32])
def test_image_between_lattice_points_matches_direct_image(L):
    # A point source, w = 0, identity A-terms and the PSWF taper (beta = 7).  The grid's image at
    # every master-grid image pixel, divided by L^2 times the continuous separable taper, must
    # match the direct imaging equation (§2) to the aliasing level of the window (§4): exact
    # only at the subgrid lattice, and growing towards the edge of the field.
    N, beta, S = 128, 7, 1.0
    rng = np.random.default_rng(21)
    nbl, nt = 6, 40
    uvw = np.zeros((nbl, nt, 3))
    t = np.arange(nt)
    for b in range(nbl):
        start = rng.uniform(-N / 4, N / 4, 2)
        vel = rng.uniform(-0.8, 0.8, 2)
        uvw[b, :, 0] = start[0] + vel[0] * t
        uvw[b, :, 1] = start[1] + vel[1] * t
    l0, m0 = 0.11, -0.07
    y = np.exp(-2j * np.pi * (uvw[..., 0] * l0 + uvw[..., 1] * m0))     # measurement equation, 1 Jy
    vis = np.zeros((nbl, nt, 1, 4), np.complex64)
    vis[..., 0, 0] = y
    vis[..., 0, 3] = y
    wl = make_mini(uvw, N=N, L=L, beta=beta, S=S, vis=vis, taper=pswf_taper_2d(L, beta))
    plan = plan_of(wl)
    assert plan.nr_dropped == 0 and plan.nr_subgrids > 4
    g = idg.grid(plan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)[0]
    k = np.arange(N) - N // 2
    lx = k * S / N                                          # image pixel positions of the master grid
    dtft = np.exp(2j * np.pi * np.outer(k, k) / N)          # exp(+2 pi i u_x l) with u_x = (x - N/2) / S
    img = dtft @ g @ dtft.T                                 # rows m, columns l
    alpha = beta * np.pi / 2
    cont = np.array([pro_ang1(0, 0, alpha, 2 * li / S)[0] if abs(2 * li / S) < 1 else np.nan for li in lx])
    cont /= pro_ang1(0, 0, alpha, 0.0)[0]
    u, v = uvw[..., 0].ravel(), uvw[..., 1].ravel()
    direct_img = (np.exp(2j * np.pi * np.outer(lx, v)) * y.ravel()[None, :]) @ np.exp(2j * np.pi * np.outer(u, lx))
    peak = np.abs(direct_img).max()
    for frac, bound in ((0.25, 3e-5), (0.35, 1e-4)):
        keep = np.abs(lx) <= frac * S
        est = img[np.ix_(keep, keep)] / (L * L * np.outer(cont[keep], cont[keep]))
        err = np.abs(est - direct_img[np.ix_(keep, keep)]).max() / peak
        assert err < bound, (L, frac, err)
