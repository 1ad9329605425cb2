"""GPU parity: the HIP path (through the C ABI) against the float64 oracle.

Every comparison uses the same seeded inputs on both sides.  Stage tests
(gridder image, gridder after the transform, batched transform, adder,
splitter) localise a failure; end-to-end tests cover idg_grid / idg_degrid on
the tiny workload, cut-down LOFAR-like and SKA-low-like workloads (several
tiles, ragged time blocks, flags) and every supported subgrid size.  The
full-size workloads, in the schedules the benchmark runs, are covered by
test_gpu_fullsize.py.
"""

import numpy as np
import pytest

import synth
from oracle import idg as oidg
from oracle.plan import F, plan_workload
from tests.gpu_common import (ADJOINT_TOL, GRID_MAX_TOL, GRID_RMS_TOL, VIS_RMS_TOL, max_rel, require_gpu, rms_rel,
                              say, to_dev)
from tests.util import random_track_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    return torch, idg


def _lofar_subset():
    full = synth.make_workload("lofar")
    return synth.subset(full, baselines=np.arange(0, full.nr_baselines, 37), nt=300)


def _skalow_subset():
    full = synth.make_workload("skalow", with_vis=False)
    wl = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 1021))
    rng = np.random.default_rng(99)
    vis = (rng.standard_normal(wl.uvw.shape[:2] + (wl.nr_channels, 4)) * np.sqrt(0.5)
           + 1j * rng.standard_normal(wl.uvw.shape[:2] + (wl.nr_channels, 4)) * np.sqrt(0.5)).astype(np.complex64)
    wl.vis = vis
    return wl


CASES = {
    "tiny": lambda: synth.make_workload("tiny"),
    "lofar-subset": _lofar_subset,
    "skalow-subset-flags": _skalow_subset,
    "tracks-L16-aterms-w": lambda: random_track_workload(seed=5, nbl=6, nt=40, nch=4, random_aterms=True,
                                                         random_taper=True),
}

_cache = {}


def _case(name):
    if name not in _cache:
        wl = CASES[name]()
        _cache[name] = (wl, plan_workload(wl))
    return _cache[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("stage", [0, 1])
@pytest.mark.parametrize("path", ["auto", "direct"])
def test_gridder_subgrids(gpu, name, stage, path):
    torch, idg = gpu
    wl, oplan = _case(name)
    if path == "direct" and wl.subgrid_size != 32:
        pytest.skip("only 32 x 32 subgrids have a second sum path")
    say(f"[gridder stage {stage}] case={name} path={path} subgrids={oplan.nr_subgrids}")
    plan = idg.Plan.from_workload(wl)
    plan.set_tuning(sum_path=path)
    if path == "auto" and wl.subgrid_size == 32:
        sp = plan.sum_paths()
        assert sp["separable0"][0] + sp["separable1"][0] > 0      # the separable form is what is checked here
    d = to_dev(wl)
    L = wl.subgrid_size
    P = plan.nr_subgrids
    ids = np.unique(np.linspace(0, P - 1, min(P, 48)).astype(int))
    first, count = int(ids[0]), int(ids[-1] - ids[0] + 1)
    out = torch.zeros((count, 4, L, L), dtype=torch.complex64, device="cuda")
    idg.grid_subgrids(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], first, count, stage, out)
    idg.sync()
    got = out.cpu().numpy()
    fn = oidg.grid_subgrid_image if stage == 0 else oidg.grid_subgrid
    for p in ids:
        ref = fn(oplan, p, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
        g = got[p - first]
        assert rms_rel(g, ref) < GRID_RMS_TOL, (name, stage, p, rms_rel(g, ref))
        assert max_rel(g, ref) < GRID_MAX_TOL, (name, stage, p, max_rel(g, ref))


@pytest.mark.parametrize("L", [8, 16, 24, 32, 48, 64])
@pytest.mark.parametrize("direction", [-1, 1])
def test_subgrid_transform(gpu, L, direction):
    torch, idg = gpu
    say(f"[subgrid transform] L={L} direction={direction}")
    rng = np.random.default_rng(L + direction)
    x = (rng.standard_normal((7, 4, L, L)) + 1j * rng.standard_normal((7, 4, L, L))).astype(np.complex64)
    t = torch.from_numpy(x).cuda()
    idg.subgrid_fft(t, direction)
    idg.sync()
    fn = oidg.forward_subgrid_dft if direction < 0 else oidg.inverse_subgrid_dft
    for s in range(x.shape[0]):
        ref = fn(x[s].astype(np.complex128))
        assert rms_rel(t[s].cpu().numpy(), ref) < 2e-6


def test_adder_and_splitter(gpu):
    torch, idg = gpu
    wl, oplan = _case("lofar-subset")
    say(f"[adder/splitter] subgrids={oplan.nr_subgrids}")
    plan = idg.Plan.from_workload(wl)
    N, L = wl.grid_size, wl.subgrid_size
    P = oplan.nr_subgrids
    rng = np.random.default_rng(7)
    sub = (rng.standard_normal((P, 4, L, L)) + 1j * rng.standard_normal((P, 4, L, L))).astype(np.complex64)
    base = np.zeros((4, N, N), np.complex64)
    base[:, ::7, ::5] = 1.5 - 0.5j
    g = torch.from_numpy(base).cuda()
    idg.add_subgrids(plan, torch.from_numpy(sub).cuda(), 0, g)
    idg.sync()
    ref = base.astype(np.complex64).copy()
    for p in range(P):                       # same order as the tile owner: plan order, float32
        x0, y0 = oplan.subgrids[p, F["x0"]], oplan.subgrids[p, F["y0"]]
        ref[:, y0:y0 + L, x0:x0 + L] += sub[p]
    assert np.array_equal(g.cpu().numpy(), ref)          # exact: same additions in the same order
    # splitter: exact copy
    out = torch.empty((P, 4, L, L), dtype=torch.complex64, device="cuda")
    idg.split_subgrids(plan, g, 0, out)
    idg.sync()
    gh = g.cpu().numpy()
    oh = out.cpu().numpy()
    for p in range(P):
        x0, y0 = oplan.subgrids[p, F["x0"]], oplan.subgrids[p, F["y0"]]
        assert np.array_equal(oh[p], gh[:, y0:y0 + L, x0:x0 + L])


def _grid_gpu(torch, idg, wl, plan, d, **kw):
    g = torch.zeros((4, wl.grid_size, wl.grid_size), dtype=torch.complex64, device="cuda")
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g, **kw)
    idg.sync()
    return g


@pytest.mark.parametrize("name", list(CASES))
def test_grid_end_to_end(gpu, name):
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[idg_grid] case={name} subgrids={oplan.nr_subgrids} vis={oplan.nr_gridded}")
    plan = idg.Plan.from_workload(wl, scratch_bytes=4 * 32 * 1024 * 8 * 9)   # small batches: several adder passes
    d = to_dev(wl)
    g = _grid_gpu(torch, idg, wl, plan, d).cpu().numpy()
    ref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    say(f"    grid rms rel {rms_rel(g, ref):.2e} max rel {max_rel(g, ref):.2e}")
    assert rms_rel(g, ref) < GRID_RMS_TOL
    assert max_rel(g, ref) < GRID_MAX_TOL
    # untouched pixels stay exactly zero
    assert np.all(g[ref == 0] == 0)


@pytest.mark.parametrize("name", list(CASES))
def test_degrid_end_to_end(gpu, name):
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[idg_degrid] case={name} subgrids={oplan.nr_subgrids}")
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)
    rng = np.random.default_rng(3)
    N = wl.grid_size
    grid_in = np.zeros((4, N, N), np.complex64)
    # random values on the part of the grid the subgrids cover (elsewhere irrelevant)
    for p in range(oplan.nr_subgrids):
        x0, y0, L = oplan.subgrids[p, F["x0"]], oplan.subgrids[p, F["y0"]], wl.subgrid_size
        grid_in[:, y0:y0 + L, x0:x0 + L] = 1.0
    mask = grid_in != 0
    grid_in[mask] = (rng.standard_normal(mask.sum()) + 1j * rng.standard_normal(mask.sum())).astype(np.complex64)
    vis = torch.full(tuple(wl.vis.shape), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")   # garbage to overwrite
    idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(grid_in).cuda(), d["aterms"], d["taper"], vis)
    idg.sync()
    got = vis.cpu().numpy()
    ref = oidg.degrid(oplan, wl.uvw, wl.freqs, grid_in, wl.aterms, wl.taper)
    planned = np.zeros(wl.vis.shape[:3], bool)
    for p in range(oplan.nr_subgrids):
        tc = oplan.subgrid_samples(p)
        planned[oplan.subgrids[p, F["bl"]], tc[:, 0], tc[:, 1]] = True
    say(f"    vis rms rel {rms_rel(got[planned], ref[planned]):.2e}")
    assert rms_rel(got[planned], ref[planned]) < VIS_RMS_TOL
    assert np.all(got[~planned] == 0)      # flagged and dropped samples are written as zero


@pytest.mark.parametrize("name", ["tiny", "skalow-subset-flags", "tracks-L16-aterms-w"])
def test_adjoint_on_gpu(gpu, name):
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[adjoint] case={name}")
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)
    N = wl.grid_size
    rng = np.random.default_rng(21)
    x = (rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))).astype(np.complex64)
    gy = _grid_gpu(torch, idg, wl, plan, d).cpu().numpy()
    vx = torch.empty(tuple(wl.vis.shape), dtype=torch.complex64, device="cuda")
    idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(x).cuda(), d["aterms"], d["taper"], vx)
    idg.sync()
    lhs = np.vdot(vx.cpu().numpy().astype(np.complex128), wl.vis.astype(np.complex128))
    rhs = np.vdot(x.astype(np.complex128), gy.astype(np.complex128))
    say(f"    adjoint rel {abs(lhs - rhs) / abs(rhs):.2e}")
    assert abs(lhs - rhs) / abs(rhs) < ADJOINT_TOL


def test_grid_is_deterministic(gpu):
    torch, idg = gpu
    wl, oplan = _case("lofar-subset")
    say("[determinism]")
    plan = idg.Plan.from_workload(wl, scratch_bytes=4 * 32 * 1024 * 8 * 5)
    d = to_dev(wl)
    a = _grid_gpu(torch, idg, wl, plan, d)
    b = _grid_gpu(torch, idg, wl, plan, d)
    assert torch.equal(a, b)


@pytest.mark.parametrize("L", [8, 16, 24, 32, 48, 64])
def test_every_subgrid_size(gpu, L):
    torch, idg = gpu
    say(f"[subgrid size] L={L}")
    N = max(128, 4 * L)
    wl = random_track_workload(seed=L, N=N, L=L, beta=min(7, L // 2 - 1), nbl=3, nt=30, nch=3,
                               random_aterms=True, random_taper=True)
    oplan = plan_workload(wl)
    assert oplan.nr_subgrids > 0
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)
    g = _grid_gpu(torch, idg, wl, plan, d).cpu().numpy()
    ref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    assert rms_rel(g, ref) < GRID_RMS_TOL
    vref = oidg.degrid(oplan, wl.uvw, wl.freqs, ref.astype(np.complex64), wl.aterms, wl.taper)
    planned = np.abs(vref).sum(-1) > 0
    for shape in ("standard", "wide"):
        plan.set_tuning(degrid_shape=shape)
        vis = torch.empty(tuple(wl.vis.shape), dtype=torch.complex64, device="cuda")
        idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(ref.astype(np.complex64)).cuda(), d["aterms"],
                   d["taper"], vis)
        idg.sync()
        assert rms_rel(vis.cpu().numpy()[planned], vref[planned]) < VIS_RMS_TOL, shape


def test_edge_subgrids_and_single_sample_blocks(gpu):
    torch, idg = gpu
    say("[edges]")
    # tracks that run into the grid edge (x0 = 0 / x0 + L = N blocks, dropped blocks) and 1-sample blocks
    N, L = 64, 16
    uvw = np.zeros((3, 12, 3))
    uvw[0, :, 0] = -N / 2 + L / 2 - 0.4 + 0.05 * np.arange(12)  # x 7.6 .. 8.15: centre 8, corner x0 = 0
    uvw[1, :, 0] = N / 2 - L / 2 + 0.4 - 0.05 * np.arange(12)   # x 56.4 .. 55.85: centre 56, x0 + L = N
    uvw[2, :, 0] = 13.0 * np.arange(12) - 20                   # fast: 1-sample blocks, then off the grid
    uvw[:, :, 1] = np.linspace(-20, 20, 3)[:, None]
    from tests.util import make_mini
    wl = make_mini(uvw, N=N, L=L, beta=3, tmax=64, random_aterms=True, random_taper=True, seed=8)
    oplan = plan_workload(wl)
    assert oplan.subgrids[:, F["x0"]].min() == 0 and (oplan.subgrids[:, F["x0"]] + L).max() == N
    assert oplan.subgrids[:, F["nvis"]].min() == 1 and oplan.nr_dropped > 0
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)
    g = _grid_gpu(torch, idg, wl, plan, d).cpu().numpy()
    ref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    assert rms_rel(g, ref) < GRID_RMS_TOL


def test_empty_plan_degrid_zeroes(gpu):
    torch, idg = gpu
    say("[empty plan]")
    from tests.util import make_mini
    uvw = np.zeros((1, 4, 3))
    uvw[0, :, 2] = 50.0                        # w-support too large: every sample dropped
    wl = make_mini(uvw, N=64, L=16, beta=3)
    plan = idg.Plan.from_workload(wl)
    assert plan.stats()["nr_subgrids"] == 0 and plan.stats()["nr_dropped"] == 4
    d = to_dev(wl)
    g = torch.zeros((4, 64, 64), dtype=torch.complex64, device="cuda")
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
    vis = torch.full((1, 4, 1, 4), 3.0 + 0j, dtype=torch.complex64, device="cuda")
    idg.degrid(plan, d["uvw"], d["freqs"], g, d["aterms"], d["taper"], vis)
    idg.sync()
    assert torch.count_nonzero(g).item() == 0 and torch.count_nonzero(vis).item() == 0


@pytest.mark.parametrize("name", ["tiny", "lofar-subset", "skalow-subset-flags"])
def test_persistent_form_equals_plain(gpu, name):
    # the work-queue form runs the same per-subgrid arithmetic: results are bitwise identical
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[persistent form] case={name}")
    d = to_dev(wl)
    out = {}
    for form in ("plain", "persistent"):
        plan = idg.Plan.from_workload(wl, scratch_bytes=4 * 32 * 1024 * 8 * 7)
        plan.set_tuning(form=form, blocks_per_cu=2 if form == "persistent" else 0)
        g = _grid_gpu(torch, idg, wl, plan, d)
        v = torch.empty(tuple(wl.vis.shape), dtype=torch.complex64, device="cuda")
        idg.degrid(plan, d["uvw"], d["freqs"], g, d["aterms"], d["taper"], v)
        idg.sync()
        out[form] = (g, v)
    assert torch.equal(out["plain"][0], out["persistent"][0])
    assert torch.equal(out["plain"][1], out["persistent"][1])


@pytest.mark.parametrize("name", ["lofar-subset", "skalow-subset-flags", "tracks-L16-aterms-w"])
def test_wide_degridder_shape(gpu, name):
    # the wide shape (8 visibilities per lane, pixel halves added across the wave) against the
    # oracle; its persistent form is bitwise equal to its plain form
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[wide degridder] case={name}")
    assert oplan.subgrids[:, F["nvis"]].max() >= 64        # the wide tasks do occur
    d = to_dev(wl)
    rng = np.random.default_rng(5)
    N = wl.grid_size
    grid_in = np.zeros((4, N, N), np.complex64)
    for p in range(oplan.nr_subgrids):
        x0, y0, L = oplan.subgrids[p, F["x0"]], oplan.subgrids[p, F["y0"]], wl.subgrid_size
        grid_in[:, y0:y0 + L, x0:x0 + L] = 1.0
    mask = grid_in != 0
    grid_in[mask] = (rng.standard_normal(mask.sum()) + 1j * rng.standard_normal(mask.sum())).astype(np.complex64)
    gdev = torch.from_numpy(grid_in).cuda()
    ref = oidg.degrid(oplan, wl.uvw, wl.freqs, grid_in, wl.aterms, wl.taper)
    planned = np.zeros(wl.vis.shape[:3], bool)
    for p in range(oplan.nr_subgrids):
        tc = oplan.subgrid_samples(p)
        planned[oplan.subgrids[p, F["bl"]], tc[:, 0], tc[:, 1]] = True
    out = {}
    for form in ("plain", "persistent"):
        plan = idg.Plan.from_workload(wl)
        plan.set_tuning(form=form, degrid_shape="wide")
        v = torch.full(tuple(wl.vis.shape), 5.0 + 5.0j, dtype=torch.complex64, device="cuda")
        idg.degrid(plan, d["uvw"], d["freqs"], gdev, d["aterms"], d["taper"], v)
        idg.sync()
        out[form] = v
    got = out["plain"].cpu().numpy()
    say(f"    vis rms rel {rms_rel(got[planned], ref[planned]):.2e}")
    assert rms_rel(got[planned], ref[planned]) < VIS_RMS_TOL
    assert np.all(got[~planned] == 0)
    assert torch.equal(out["plain"], out["persistent"])


def test_adder_chunks_split_long_tile_lists(gpu):
    # a tiny chunk length splits every tile list: still deterministic and equal to the oracle
    torch, idg = gpu
    wl, oplan = _case("lofar-subset")
    say("[adder chunks]")
    d = to_dev(wl)
    plan = idg.Plan.from_workload(wl)
    plan.set_tuning(adder_chunk=2)
    a = _grid_gpu(torch, idg, wl, plan, d)
    b = _grid_gpu(torch, idg, wl, plan, d)
    assert torch.equal(a, b)
    ref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    assert rms_rel(a.cpu().numpy(), ref) < GRID_RMS_TOL
    # the standalone adder with split lists against the same float32 additions (tolerance: order differs)
    N, L = wl.grid_size, wl.subgrid_size
    P = oplan.nr_subgrids
    rng = np.random.default_rng(9)
    sub = (rng.standard_normal((P, 4, L, L)) + 1j * rng.standard_normal((P, 4, L, L))).astype(np.complex64)
    g = torch.zeros((4, N, N), dtype=torch.complex64, device="cuda")
    idg.add_subgrids(plan, torch.from_numpy(sub).cuda(), 0, g)
    idg.sync()
    ref = np.zeros((4, N, N), np.complex128)
    for p in range(P):
        x0, y0 = oplan.subgrids[p, F["x0"]], oplan.subgrids[p, F["y0"]]
        ref[:, y0:y0 + L, x0:x0 + L] += sub[p]
    assert max_rel(g.cpu().numpy(), ref) < 1e-6


@pytest.mark.parametrize("name", ["lofar-subset", "skalow-subset-flags"])
@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_separable_form_matches_oracle(gpu, name, form):
    # 32 x 32 subgrids whose w-term allows it run the separable form on the matrix cores (sum_path
    # "auto"); the direct sum ("direct") and the oracle agree with it to float32 level
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[separable form] case={name} form={form}")
    d = to_dev(wl)
    ref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    out = {}
    for path in ("auto", "direct"):
        plan = idg.Plan.from_workload(wl, scratch_bytes=4 * 32 * 1024 * 8 * 9)
        plan.set_tuning(form=form, sum_path=path)
        g = _grid_gpu(torch, idg, wl, plan, d).cpu().numpy()
        out[path] = g
        say(f"    {path}: grid rms rel {rms_rel(g, ref):.2e} max rel {max_rel(g, ref):.2e}")
        assert rms_rel(g, ref) < GRID_RMS_TOL and max_rel(g, ref) < GRID_MAX_TOL, path
        assert np.all(g[ref == 0] == 0)
    assert rms_rel(out["auto"], out["direct"]) < GRID_RMS_TOL


@pytest.mark.parametrize("name", ["lofar-subset", "skalow-subset-flags"])
@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_separable_degridder_matches_oracle(gpu, name, form):
    # the degridder's separable form (sum_path "auto") and its direct sum ("direct") against the oracle
    torch, idg = gpu
    wl, oplan = _case(name)
    say(f"[separable degridder] case={name} form={form}")
    d = to_dev(wl)
    rng = np.random.default_rng(13)
    N, L = wl.grid_size, wl.subgrid_size
    grid_in = np.zeros((4, N, N), np.complex64)
    for p in range(oplan.nr_subgrids):
        x0, y0 = oplan.subgrids[p, F["x0"]], oplan.subgrids[p, F["y0"]]
        grid_in[:, y0:y0 + L, x0:x0 + L] = 1.0
    mask = grid_in != 0
    grid_in[mask] = (rng.standard_normal(mask.sum()) + 1j * rng.standard_normal(mask.sum())).astype(np.complex64)
    gdev = torch.from_numpy(grid_in).cuda()
    ref = oidg.degrid(oplan, wl.uvw, wl.freqs, grid_in, wl.aterms, wl.taper)
    planned = np.zeros(wl.vis.shape[:3], bool)
    for p in range(oplan.nr_subgrids):
        tc = oplan.subgrid_samples(p)
        planned[oplan.subgrids[p, F["bl"]], tc[:, 0], tc[:, 1]] = True
    out, err = {}, {}
    for path in ("auto", "direct"):
        plan = idg.Plan.from_workload(wl)
        plan.set_tuning(form=form, sum_path=path)
        v = torch.full(tuple(wl.vis.shape), 5.0 + 5.0j, dtype=torch.complex64, device="cuda")
        idg.degrid(plan, d["uvw"], d["freqs"], gdev, d["aterms"], d["taper"], v)
        idg.sync()
        got = v.cpu().numpy()
        out[path] = got
        err[path] = rms_rel(got[planned], ref[planned])
        say(f"    {path}: vis rms rel {err[path]:.2e}")
        assert err[path] < VIS_RMS_TOL, path
        assert np.all(got[~planned] == 0)
    assert rms_rel(out["auto"][planned], out["direct"][planned]) < VIS_RMS_TOL
    # the separable form is as accurate as the direct sum: its first-order term must not lose precision (the
    # cross term c ~ 1e-7 underflowed fp16 before it was scaled by 2^-cross_exp, which cost 2-6x here)
    assert err["auto"] < 1.5 * err["direct"] + 2e-7, err


def test_trim_scratch_between_calls(gpu):
    # the library's scratch pool hands its unused memory back; later calls allocate again and agree bitwise
    torch, idg = gpu
    wl, _ = _case("tiny")
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)
    N = wl.grid_size
    g1 = torch.zeros((4, N, N), dtype=torch.complex64, device="cuda")
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g1)
    idg.trim_scratch(0)
    g2 = torch.zeros_like(g1)
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g2)
    idg.trim_scratch(1 << 20)
    idg.sync()
    assert torch.equal(g1, g2)


def test_device_rates_are_plausible(gpu):
    # the microkernels behind the benchmark's measured fractions: positive, below the published peaks, and the
    # fp16 matrix cores far above the unpacked float32 multiply-adds
    torch, idg = gpu
    r = idg.device_rates()
    assert 5.0 < r["fp32_fma_tflops"] <= 157.3 * 1.05
    assert 10.0 < r["sincos_ginstr_per_s"] < 2000.0
    assert 100.0 < r["fp16_mfma_tflops"] <= 2500.0 * 1.05
    assert r["fp16_mfma_tflops"] > 8 * r["fp32_fma_tflops"]
