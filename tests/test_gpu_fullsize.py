"""GPU parity at the full workload sizes, in every schedule the benchmark's autotuner can pick.

The benchmark times idg_grid + idg_degrid on the full SKA-low-like share (one
gridder launch over all 1.97 M subgrids, a 64 GB subgrid scratch, adder tile
lists cut into chunks and combined) and on the full LOFAR-like workload.  The
autotuner chooses, per plan, the gridder and degridder forms (plain, or the
persistent work queue at 0, 1 or 2 workgroups per CU), the degridder shape
(standard or wide) and the adder chunk (32, 64, 256 or 1024).  These tests run
the full plans under those schedules and compare with the float64 oracle on
outputs it can compute one by one, and by identities that hold at any size:

* grid tiles: a 32 x 32 tile of the grid (all four polarisations) against the
  oracle's sum of every subgrid overlapping it (Algorithm 1); tiles whose
  contribution lists are cut into several adder chunks (partial tiles and the
  combine pass) and tiles with short lists, under every adder chunk;
* the gridder forms give bitwise-identical grids (the plain form one
  workgroup per subgrid, the persistent form pulling costliest-first);
* sampled visibilities (Algorithm 2) of the subgrids with the fewest and the
  most samples, of subgrids with flagged samples and of random subgrids, under
  both degridder shapes; the two degridder forms are bitwise identical;
* every flagged sample is written as exactly 0;
* the adjoint identity <degrid(G), y> = <G, grid(y)> over the whole plan.
"""

import numpy as np
import pytest

import synth
from oracle import idg as oidg
from oracle.plan import F
from oracle.plan import Plan as OPlan
from tests.gpu_common import ADJOINT_TOL, GRID_MAX_TOL, GRID_RMS_TOL, VIS_RMS_TOL, max_rel, require_gpu, rms_rel, say

pytestmark = pytest.mark.gpu

TILE = 32
ADDER_CHUNKS = (32, 64, 256, 1024)          # the autotuner's candidates


@pytest.fixture(scope="module")
def gpu():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    return torch, idg


class Full:
    """A full-size workload, its library plan (scratch for the whole plan: one gridder launch, as the
    benchmark runs it), the oracle's view of the same plan and the device inputs."""

    def __init__(self, torch, idg, name):
        say(f"[full {name}] building the workload")
        wl = synth.make_workload(name)
        plan = idg.Plan.from_workload(wl)
        nsub = plan.nr_subgrids
        plan = idg.Plan.from_workload(wl, scratch_bytes=nsub * 4 * wl.subgrid_size ** 2 * 8 + (1 << 20))
        sub, smp = plan.export()
        st = plan.stats()
        self.oplan = OPlan(wl.grid_size, wl.image_size, wl.subgrid_size, wl.kernel_size, wl.max_timesteps,
                           wl.aterm_timesteps, wl.nr_baselines, wl.nr_timesteps, wl.nr_channels, sub,
                           smp.astype(np.int64), st["nr_gridded"], st["nr_dropped"], st["nr_flagged"])
        self.wl, self.plan, self.sub = wl, plan, sub
        dev = "cuda"
        self.d = dict(uvw=torch.from_numpy(wl.uvw).to(dev), freqs=torch.from_numpy(wl.freqs).to(dev),
                      vis=torch.from_numpy(wl.vis).to(dev), aterms=torch.from_numpy(wl.aterms).to(dev),
                      taper=torch.from_numpy(wl.taper).to(dev))
        self.torch, self.idg = torch, idg
        say(f"[full {name}] {nsub} subgrids, {st['nr_gridded']} visibilities")

    def grid(self, **tuning):
        torch, idg, d = self.torch, self.idg, self.d
        self.plan.set_tuning(**tuning)
        N = self.wl.grid_size
        g = torch.zeros((4, N, N), dtype=torch.complex64, device="cuda")
        idg.grid(self.plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
        idg.sync()
        return g

    def degrid(self, grid_d, **tuning):
        torch, idg, d = self.torch, self.idg, self.d
        self.plan.set_tuning(**tuning)
        v = torch.full(tuple(self.wl.vis.shape), 7.0 + 7.0j, dtype=torch.complex64, device="cuda")
        idg.degrid(self.plan, d["uvw"], d["freqs"], grid_d, d["aterms"], d["taper"], v)
        idg.sync()
        return v

    # -- tiles ---------------------------------------------------------------------------------

    def tile_counts(self):
        """{tile id (ty * ntx + tx): number of subgrids overlapping it}."""
        L = self.wl.subgrid_size
        x0, y0 = self.sub[:, F["x0"]], self.sub[:, F["y0"]]
        ntx = -(-self.wl.grid_size // TILE)
        ids = []
        for dy in range(L // TILE + 2):
            for dx in range(L // TILE + 2):
                tx, ty = x0 // TILE + dx, y0 // TILE + dy
                ok = (tx <= (x0 + L - 1) // TILE) & (ty <= (y0 + L - 1) // TILE)
                ids.append((ty * ntx + tx)[ok])
        u, c = np.unique(np.concatenate(ids), return_counts=True)
        return dict(zip(u.tolist(), c.tolist()))

    def oracle_tile(self, tile):
        """[4, TILE, TILE] complex128: the sum of every overlapping subgrid (Algorithm 1) over the tile."""
        wl, L = self.wl, self.wl.subgrid_size
        ntx = -(-wl.grid_size // TILE)
        ty, tx = divmod(tile, ntx)
        xa, ya = tx * TILE, ty * TILE
        x0, y0 = self.sub[:, F["x0"]], self.sub[:, F["y0"]]
        hit = np.flatnonzero((x0 <= xa + TILE - 1) & (x0 + L - 1 >= xa) & (y0 <= ya + TILE - 1) & (y0 + L - 1 >= ya))
        out = np.zeros((4, TILE, TILE), np.complex128)
        for p in hit:
            v = oidg.grid_subgrid(self.oplan, int(p), wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
            sx, sy = int(x0[p]), int(y0[p])
            # overlap of [sx, sx + L) x [sy, sy + L) with the tile
            gx0, gx1 = max(sx, xa), min(sx + L, xa + TILE)
            gy0, gy1 = max(sy, ya), min(sy + L, ya + TILE)
            out[:, gy0 - ya:gy1 - ya, gx0 - xa:gx1 - xa] += v[:, gy0 - sy:gy1 - sy, gx0 - sx:gx1 - sx]
        return out, hit.size

    def pick_tiles(self, rng, n_random=4, ranges=((1024, 2048), (2048, 3072))):
        """Tiles to compare: for each count range, the least-loaded tile in it (a list cut into two
        adder chunks of 1024, then three), and a few random tiles with shorter lists (bounded oracle cost)."""
        counts = self.tile_counts()
        ids = np.array(list(counts.keys()))
        c = np.array(list(counts.values()))
        picks = []
        for lo, hi in ranges:
            sel = np.flatnonzero((c > lo) & (c <= hi))
            if sel.size:
                picks.append(int(ids[sel[np.argmin(c[sel])]]))
        short = np.flatnonzero(c <= 256)
        picks += [int(t) for t in ids[rng.choice(short, min(n_random, short.size), replace=False)]]
        return picks, counts

    def gpu_tile(self, g, tile):
        ntx = -(-self.wl.grid_size // TILE)
        ty, tx = divmod(tile, ntx)
        return g[:, ty * TILE:(ty + 1) * TILE, tx * TILE:(tx + 1) * TILE].cpu().numpy()

    # -- visibilities --------------------------------------------------------------------------

    def pick_subgrids(self, rng, n_random=12):
        nv = self.sub[:, F["nvis"]]
        box = self.sub[:, F["nt"]] * self.sub[:, F["nc"]]
        flagged = np.flatnonzero(nv < box)
        picks = {int(np.argmin(nv)), int(np.argmax(nv))}
        if flagged.size:
            picks |= {int(p) for p in rng.choice(flagged, min(4, flagged.size), replace=False)}
        picks |= {int(p) for p in rng.choice(self.sub.shape[0], n_random, replace=False)}
        return sorted(picks)

    def vis_of(self, v, p):
        tc = self.oplan.subgrid_samples(p)
        return v[int(self.sub[p, F["bl"]])].cpu().numpy()[tc[:, 0], tc[:, 1]]


@pytest.fixture(scope="module")
def skalow_full(gpu):
    torch, idg = gpu
    f = Full(torch, idg, "skalow")
    yield f
    f.d = None
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def lofar_full(gpu):
    torch, idg = gpu
    f = Full(torch, idg, "lofar")
    yield f
    f.d = None
    torch.cuda.empty_cache()


def _tiles_under_every_chunk(f, seed, ranges):
    rng = np.random.default_rng(seed)
    tiles, counts = f.pick_tiles(rng, ranges=ranges)
    refs = {}
    for t in tiles:
        refs[t], n = f.oracle_tile(t)
        say(f"    tile {t}: {n} subgrids")
    for chunk in ADDER_CHUNKS:
        g = f.grid(form="persistent", blocks_per_cu=0, adder_chunk=chunk)
        for t in tiles:
            got, ref = f.gpu_tile(g, t), refs[t]
            e_rms, e_max = rms_rel(got, ref), max_rel(got, ref)
            say(f"    chunk {chunk} tile {t} ({counts[t]} subgrids): rms {e_rms:.2e} max {e_max:.2e}")
            assert e_rms < GRID_RMS_TOL and e_max < GRID_MAX_TOL, (chunk, t, e_rms, e_max)
        del g


def _gridder_forms_bitwise(f, chunk):
    ref = f.grid(form="plain", blocks_per_cu=0, adder_chunk=chunk)
    for bpc in (0, 2):
        g = f.grid(form="persistent", blocks_per_cu=bpc, adder_chunk=chunk)
        assert f.torch.equal(g, ref), bpc
        del g
    return ref


def _sampled_visibilities(f, seed):
    torch = f.torch
    rng = np.random.default_rng(seed)
    N = f.wl.grid_size
    gen = torch.Generator(device="cuda").manual_seed(seed)
    gin = torch.complex(torch.randn((4, N, N), generator=gen, device="cuda"),
                        torch.randn((4, N, N), generator=gen, device="cuda")).to(torch.complex64)
    gh = gin.cpu().numpy()
    picks = f.pick_subgrids(rng)
    refs = {p: oidg.degrid_subgrid(f.oplan, p, f.wl.uvw, f.wl.freqs, gh, f.wl.aterms, f.wl.taper) for p in picks}
    flags = None if f.wl.flags is None else torch.from_numpy(f.wl.flags).cuda() != 0
    for shape in ("standard", "wide"):
        vp = f.degrid(gin, form="plain", blocks_per_cu=0, degrid_shape=shape)
        v = f.degrid(gin, form="persistent", blocks_per_cu=0, degrid_shape=shape)
        assert torch.equal(v, vp), shape                     # the work queue changes no arithmetic
        del vp
        for p in picks:
            got = f.vis_of(v, p)
            e = rms_rel(got, refs[p])
            assert e < VIS_RMS_TOL, (shape, p, int(f.sub[p, F["nvis"]]), e)
        say(f"    degrid {shape}: {len(picks)} subgrids (K_p {int(f.sub[picks, F['nvis']].min())}.."
            f"{int(f.sub[picks, F['nvis']].max())}) within {VIS_RMS_TOL}")
        if flags is not None:
            assert int(torch.count_nonzero(v[flags]).item()) == 0, shape   # flagged samples are exactly 0
        del v
    return gin


def _adjoint(f, gin):
    torch = f.torch
    gy = f.grid(form="persistent", blocks_per_cu=0)
    vx = f.degrid(gin, form="persistent", blocks_per_cu=0)
    lhs = torch.vdot(vx.flatten().to(torch.complex128), f.d["vis"].flatten().to(torch.complex128)).item()
    rhs = torch.vdot(gin.flatten().to(torch.complex128), gy.flatten().to(torch.complex128)).item()
    err = abs(lhs - rhs) / abs(rhs)
    say(f"    adjoint rel {err:.2e}")
    assert err < ADJOINT_TOL


def test_skalow_full_grid_tiles_every_chunk(gpu, skalow_full):
    say("[skalow full] grid tiles vs oracle under every adder chunk (persistent gridder, one launch)")
    _tiles_under_every_chunk(skalow_full, seed=31, ranges=((1024, 2048), (2048, 3072)))


def test_skalow_full_gridder_forms_bitwise(gpu, skalow_full):
    say("[skalow full] plain and persistent gridder forms give the same grid")
    _gridder_forms_bitwise(skalow_full, chunk=1024)


def test_skalow_full_sampled_visibilities_and_adjoint(gpu, skalow_full):
    say("[skalow full] sampled visibilities (both shapes, both forms), flagged zeros, adjoint")
    gin = _sampled_visibilities(skalow_full, seed=41)
    _adjoint(skalow_full, gin)


def test_lofar_full_grid_tiles_every_chunk(gpu, lofar_full):
    say("[lofar full] grid tiles vs oracle under every adder chunk (persistent gridder)")
    # the LOFAR-like subgrids hold ~900 samples each: one long list keeps the oracle's cost bounded
    _tiles_under_every_chunk(lofar_full, seed=32, ranges=((1024, 2048),))


def test_lofar_full_gridder_forms_bitwise_and_sum(gpu, lofar_full):
    # any size: the sum of a subgrid's uv pixels is L^2 times its image at l = m = 0, i.e.
    # L^2 c[L/2, L/2] A_s1^H (sum_k Y_k) A_s2 at the centre pixel; summed over all subgrids
    f = lofar_full
    torch = f.torch
    say("[lofar full] gridder forms bitwise; grid sum property")
    g = _gridder_forms_bitwise(f, chunk=64)
    total = g.to(torch.complex128).sum(dim=(1, 2)).cpu().numpy()
    wl, sub, smp = f.wl, f.sub, f.oplan.samples
    L = wl.subgrid_size
    c = float(wl.taper[L // 2, L // 2])
    ref = np.zeros(4, np.complex128)
    for p in range(sub.shape[0]):
        bl, off, n = sub[p, F["bl"]], sub[p, F["vis_offset"]], sub[p, F["nvis"]]
        tc = smp[off:off + n]
        y = wl.vis[bl, tc[:, 0], tc[:, 1]].astype(np.complex128).sum(0).reshape(2, 2)
        a1 = wl.aterms[sub[p, F["slot"]], sub[p, F["st1"]], L // 2, L // 2].astype(np.complex128).reshape(2, 2)
        a2 = wl.aterms[sub[p, F["slot"]], sub[p, F["st2"]], L // 2, L // 2].astype(np.complex128).reshape(2, 2)
        ref += (np.conj(a1.T) @ y @ a2).reshape(4)
    ref *= L * L * c
    say(f"    sum rel err {np.abs(total - ref).max() / np.abs(ref).max():.2e}")
    assert np.abs(total - ref).max() / np.abs(ref).max() < 1e-5


def test_lofar_full_sampled_subgrids(gpu, lofar_full):
    # the transformed subgrids (stage 1) of the largest subgrid (2048 samples, 8 staging rounds) and random ones
    f = lofar_full
    torch, idg = f.torch, f.idg
    say(f"[lofar full] sampled subgrids of {f.plan.nr_subgrids}")
    rng = np.random.default_rng(5)
    ids = list(rng.choice(f.plan.nr_subgrids, 12, replace=False)) + [int(np.argmax(f.sub[:, F["nvis"]]))]
    L = f.wl.subgrid_size
    out = torch.empty((1, 4, L, L), dtype=torch.complex64, device="cuda")
    d, wl = f.d, f.wl
    for p in ids:
        idg.grid_subgrids(f.plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], int(p), 1, 1, out)
        idg.sync()
        ref = oidg.grid_subgrid(f.oplan, int(p), wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
        assert rms_rel(out[0].cpu().numpy(), ref) < GRID_RMS_TOL, p


def test_lofar_full_sampled_visibilities_and_adjoint(gpu, lofar_full):
    say("[lofar full] sampled visibilities (both shapes, both forms), adjoint")
    gin = _sampled_visibilities(lofar_full, seed=42)
    _adjoint(lofar_full, gin)
