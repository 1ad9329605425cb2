"""W-layers on the GPU against the float64 oracle.

* layered gridding and degridding (w offsets per subgrid, one grid per layer),
  plain and persistent forms, on samples whose w no unlayered block can hold;
* the W-stacked image steps (idg_wstack_to_image, idg_image_to_wstack), whole
  transforms at N = 128 with several turns of w-correction;
* the layered major cycle: point-source model image -> W-layer grids -> degrid
  against the oracle's chain and the measurement equation, w-term included.
"""

import numpy as np
import pytest

from oracle import idg as oidg
from oracle import image as oim
from oracle.plan import plan_workload
from synth import C0, pswf_taper_2d
from tests.gpu_common import GRID_RMS_TOL, VIS_RMS_TOL, require_gpu, rms_rel, say, to_dev
from tests.util import make_mini

pytestmark = pytest.mark.gpu

N, L, BETA, S, WSTEP = 128, 32, 7, 1.0, 4.0


def _deep_w(seed, nbl=6, nt=30, nch=4, **kw):
    rng = np.random.default_rng(seed)
    uvw = np.zeros((nbl, nt, 3))
    t = np.arange(nt)
    for b in range(nbl):
        uvw[b, :, 0] = rng.uniform(-N / 5, N / 5) + rng.uniform(-0.5, 0.5) * t
        uvw[b, :, 1] = rng.uniform(-N / 5, N / 5) + rng.uniform(-0.5, 0.5) * t
        uvw[b, :, 2] = rng.choice([-1, 1]) * (rng.uniform(30, 40) + rng.uniform(0.5, 1.5) * t)
    freqs = C0 * (1.0 + 0.01 * np.arange(nch))
    return make_mini(uvw, freqs=freqs, N=N, L=L, beta=BETA, S=S, seed=seed, **kw)


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_layered_grid_and_degrid(form):
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    wl = _deep_w(41, random_aterms=True, random_taper=True)
    oplan = plan_workload(wl, WSTEP)
    plan = idg.Plan.from_workload(wl, w_step=WSTEP)
    plan.set_tuning(form=form)
    assert oplan.nr_dropped == 0 and plan.wlayers() == (oplan.wlayer_min, oplan.nr_wlayers)
    say(f"[wstack grid] form={form} subgrids={oplan.nr_subgrids} layers={oplan.nr_wlayers}")
    d = to_dev(wl)
    grid = torch.zeros(plan.shapes()["grid"], dtype=torch.complex64, device="cuda")
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], grid)
    idg.sync()
    g = grid.cpu().numpy()
    gref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    say(f"    grid rms rel {rms_rel(g, gref):.2e}")
    assert rms_rel(g, gref) < GRID_RMS_TOL
    gin = (np.random.default_rng(5).standard_normal(g.shape) + 1j * np.random.default_rng(6).standard_normal(g.shape))
    gin = gin.astype(np.complex64)
    vis = torch.empty_like(d["vis"])
    idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(gin).cuda(), d["aterms"], d["taper"], vis)
    idg.sync()
    vref = oidg.degrid(oplan, wl.uvw, wl.freqs, gin, wl.aterms, wl.taper)
    say(f"    degrid rms rel {rms_rel(vis.cpu().numpy(), vref):.2e}")
    assert rms_rel(vis.cpu().numpy(), vref) < VIS_RMS_TOL


def test_wstack_image_steps():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    rng = np.random.default_rng(8)
    w0s = [-8.0, 0.0, 12.0]
    g = (rng.standard_normal((3, 4, N, N)) + 1j * rng.standard_normal((3, 4, N, N))).astype(np.complex64)
    cl = (0.5 + rng.random(N)).astype(np.float32)
    cm = (0.5 + rng.random(N)).astype(np.float32)
    tl, tm = torch.from_numpy(cl).cuda(), torch.from_numpy(cm).cuda()
    img = torch.empty((4, N, N), dtype=torch.complex64, device="cuda")
    idg.wstack_to_image(torch.from_numpy(g).cuda(), w0s, S, tl, tm, img)
    idg.sync()
    ref = oim.wstack_to_image(g, w0s, S, cl.astype(np.float64), cm.astype(np.float64))
    say(f"[wstack image] to image rms rel {rms_rel(img.cpu().numpy(), ref):.2e}")
    assert rms_rel(img.cpu().numpy(), ref) < GRID_RMS_TOL
    im = g[0]
    out = torch.empty((3, 4, N, N), dtype=torch.complex64, device="cuda")
    idg.image_to_wstack(torch.from_numpy(im).cuda(), S, tl, tm, w0s, out)
    idg.sync()
    ref = oim.image_to_wstack(im, w0s, S, cl.astype(np.float64), cm.astype(np.float64))
    say(f"    to layers rms rel {rms_rel(out.cpu().numpy(), ref):.2e}")
    assert rms_rel(out.cpu().numpy(), ref) < GRID_RMS_TOL


def test_layered_major_cycle():
    require_gpu()
    import torch
    from scipy.special import pro_ang1
    import paper_1909_07226_amd as idg
    wl = _deep_w(31, nbl=5, nt=30, nch=1, taper=pswf_taper_2d(L, BETA))
    oplan = plan_workload(wl, WSTEP)
    plan = idg.Plan.from_workload(wl, w_step=WSTEP)
    alpha = BETA * np.pi / 2
    lx = (np.arange(N) - N // 2) * S / N
    corr = np.array([pro_ang1(0, 0, alpha, 2 * li / S)[0] if abs(2 * li / S) < 1 else 1.0 for li in lx])
    corr = (L * corr / pro_ang1(0, 0, alpha, 0.0)[0]).astype(np.float32)
    x0, y0 = N // 2 + 36, N // 2 - 28
    model = np.zeros((4, N, N), np.complex64)
    model[0, y0, x0] = model[3, y0, x0] = 1.0
    w0s = plan.w_offsets()
    say(f"[wstack cycle] layers {w0s}")
    tc = torch.from_numpy(corr).cuda()
    grids = torch.empty(plan.shapes()["grid"], dtype=torch.complex64, device="cuda")
    idg.image_to_wstack(torch.from_numpy(model).cuda(), S, tc, tc, w0s, grids)
    d = to_dev(wl)
    vis = torch.empty_like(d["vis"])
    idg.degrid(plan, d["uvw"], d["freqs"], grids, d["aterms"], d["taper"], vis)
    idg.sync()
    v = vis.cpu().numpy()
    c64 = corr.astype(np.float64)
    og = oim.image_to_wstack(model, w0s, S, c64, c64)
    ov = oidg.degrid(oplan, wl.uvw, wl.freqs, og, wl.aterms, wl.taper)
    say(f"    vis rms vs oracle chain {rms_rel(v, ov):.2e}")
    assert rms_rel(v, ov) < VIS_RMS_TOL
    l0, m0 = lx[x0], lx[y0]
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0) - 1.0
    u, vv, w = wl.uvw[..., 0], wl.uvw[..., 1], wl.uvw[..., 2]
    dme = np.exp(-2j * np.pi * (u * l0 + vv * m0 + w * n0))
    err = np.abs(v[..., 0, 0] - dme).max()
    say(f"    vis vs measurement equation max {err:.2e} (w-term up to {np.abs(w * n0).max():.1f} turns)")
    assert err < 1e-4 and np.abs(v[..., 0, 3] - dme).max() < 1e-4


@pytest.mark.parametrize("w0s", [[-40.0, 0.0, 60.0], [-3000.0, 25.0, 4500.0]])
def test_wstack_image_steps_four_step_sampled(w0s):
    # N = 2048 takes the four-step transform with the layer phase fused into its sub-passes; the
    # second set puts up to ~1300 turns of w-term at the field edge (the phase is reduced in float64)
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    n, S2 = 2048, 1.0
    rng = np.random.default_rng(9)
    g = (rng.standard_normal((3, 4, n, n), dtype=np.float32)
         + 1j * rng.standard_normal((3, 4, n, n), dtype=np.float32)).astype(np.complex64)
    cl = (0.5 + rng.random(n)).astype(np.float32)
    cm = (0.5 + rng.random(n)).astype(np.float32)
    xs = np.concatenate([[0, n - 1, n // 2], rng.integers(0, n, 5)])
    ys = np.concatenate([[n - 1, 0, n // 2], rng.integers(0, n, 5)])
    say(f"[wstack four-step] N={n} w0s {w0s} pixels {list(zip(xs.tolist(), ys.tolist()))}")
    tl, tm = torch.from_numpy(cl).cuda(), torch.from_numpy(cm).cuda()
    gd = torch.from_numpy(g).cuda()
    img = torch.empty((4, n, n), dtype=torch.complex64, device="cuda")
    idg.wstack_to_image(gd, w0s, S2, tl, tm, img)
    idg.sync()
    got = img[:, torch.from_numpy(ys).cuda(), torch.from_numpy(xs).cuda()].cpu().numpy()
    ref = oim.wstack_to_image_at(g, w0s, S2, xs, ys, cl.astype(np.float64), cm.astype(np.float64))
    scale = np.sqrt(3 * 2.0) * n / (cl.mean() * cm.mean())
    err = np.abs(got - ref).max() / scale
    say(f"    to image sampled err {err:.2e}")
    assert err < 1e-5          # measured 5-8e-7: a float32 n' at w0 = 4500 (~2.5e-4 rad at the edge) would fail
    im = g[1]
    out = torch.empty((3, 4, n, n), dtype=torch.complex64, device="cuda")
    idg.image_to_wstack(torch.from_numpy(im).cuda(), S2, tl, tm, w0s, out)
    idg.sync()
    got = out[:, :, torch.from_numpy(ys).cuda(), torch.from_numpy(xs).cuda()].cpu().numpy()
    ref = oim.image_to_wstack_at(im, w0s, S2, xs, ys, cl.astype(np.float64), cm.astype(np.float64))
    err = np.abs(got - ref).max() / (np.sqrt(2.0) * n * np.mean(1.0 / cl) * np.mean(1.0 / cm))
    say(f"    to layers sampled err {err:.2e}")
    assert err < 1e-5


def test_layered_adjoint_at_scale():
    # the bench's W-layer configuration: LOFAR-like geometry on a 4x wider field (S = 0.2), 20 layers,
    # 124,673 subgrids, 10.7 GB of layer grids.  <degrid(G), y> = <G, grid(y)> holds at any size.
    require_gpu()
    import dataclasses
    import torch
    import paper_1909_07226_amd as idg
    import synth
    wl = synth.make_workload("lofar")
    wl = dataclasses.replace(wl, image_size=0.2)
    plan = idg.Plan.from_workload(wl, w_step=200.0)
    st = plan.stats()
    say(f"[wstack scale] {st} layers {plan.wlayers()}")
    assert st["nr_dropped"] == 0 and plan.wlayers()[1] > 10
    d = to_dev(wl)
    gen = torch.Generator(device="cuda").manual_seed(5)
    G = torch.randn(plan.shapes()["grid"], dtype=torch.complex64, device="cuda", generator=gen)
    vis = torch.empty_like(d["vis"])
    idg.degrid(plan, d["uvw"], d["freqs"], G, d["aterms"], d["taper"], vis)
    gy = torch.zeros_like(G)
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], gy)
    idg.sync()
    lhs = torch.vdot(vis.flatten().to(torch.complex128), d["vis"].flatten().to(torch.complex128))
    del vis
    rhs = sum(torch.vdot(G[j].flatten().to(torch.complex128), gy[j].flatten().to(torch.complex128))
              for j in range(G.shape[0]))
    rel = float(abs(lhs - rhs) / abs(rhs))
    say(f"    <degrid(G), y> vs <G, grid(y)>: rel {rel:.2e}")
    assert rel < 1e-4


@pytest.mark.parametrize("form,path", [("plain", "auto"), ("persistent", "auto"), ("plain", "direct")])
def test_layered_plan_in_the_separable_form(form, path):
    # a narrow field (S = 0.04) with |w| up to 2e3 wavelengths on W-layers 200 apart: |w - w_0p| <= 100, so
    # the 32 x 32 subgrids take the separable form with w_0p != 0 (first-order cross term around each layer)
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    rng = np.random.default_rng(77)
    nbl, nt, nch = 10, 80, 4
    t = np.arange(nt)
    uvw = np.zeros((nbl, nt, 3))
    for b in range(nbl):
        uvw[b, :, 0] = rng.uniform(-3000, 3000) + rng.uniform(-2, 2) * t
        uvw[b, :, 1] = rng.uniform(-3000, 3000) + rng.uniform(-2, 2) * t
        uvw[b, :, 2] = rng.choice([-1, 1]) * rng.uniform(300, 1900) + rng.uniform(-3, 3) * t
    freqs = C0 * (1.0 + 0.002 * np.arange(nch))
    wl = make_mini(uvw, freqs=freqs, N=512, L=32, beta=BETA, S=0.04, seed=77, random_aterms=True,
                   random_taper=True)
    oplan = plan_workload(wl, 200.0)
    plan = idg.Plan.from_workload(wl, w_step=200.0)
    plan.set_tuning(form=form, sum_path=path)
    paths = plan.sum_paths()
    say(f"[wstack separable] form={form} path={path} subgrids={oplan.nr_subgrids} layers={oplan.nr_wlayers} "
        f"paths={paths}")
    assert oplan.nr_dropped == 0 and oplan.nr_wlayers > 3
    if path == "auto":
        assert paths["direct"][0] == 0 and paths["separable1"][0] > 0
    d = to_dev(wl)
    grid = torch.zeros(plan.shapes()["grid"], dtype=torch.complex64, device="cuda")
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], grid)
    idg.sync()
    g = grid.cpu().numpy()
    gref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    say(f"    grid rms rel {rms_rel(g, gref):.2e}")
    assert rms_rel(g, gref) < GRID_RMS_TOL
    gin = (np.random.default_rng(9).standard_normal(g.shape) + 1j * np.random.default_rng(10).standard_normal(g.shape))
    gin = gin.astype(np.complex64)
    vis = torch.empty_like(d["vis"])
    idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(gin).cuda(), d["aterms"], d["taper"], vis)
    idg.sync()
    vref = oidg.degrid(oplan, wl.uvw, wl.freqs, gin, wl.aterms, wl.taper)
    say(f"    degrid rms rel {rms_rel(vis.cpu().numpy(), vref):.2e}")
    assert rms_rel(vis.cpu().numpy(), vref) < VIS_RMS_TOL
    # at the level of the direct sum on this case (7.5e-7): the first-order term keeps its precision
    assert rms_rel(vis.cpu().numpy(), vref) < 1.5e-6
