"""GPU parity where subgrids hold many channels: phasor runs over channels.

Both kernels advance the phasor from one channel to the next by one complex
multiplication when the channel frequencies are evenly spaced.  These cases
stress what decides a run: 40 channels in every subgrid (runs are cut every
16 channels), more than 256 samples per subgrid (runs are cut at staging
chunk ends), random flags (runs are cut at gaps, degridder lanes lose their
runs), and unevenly spaced channels (no runs at all).  Every case is compared
with the float64 oracle at the same tolerances as the other parity tests.
"""

import numpy as np
import pytest

from oracle import idg as oidg
from oracle.plan import F, plan_workload
from synth import C0
from tests.gpu_common import GRID_MAX_TOL, GRID_RMS_TOL, VIS_RMS_TOL, max_rel, require_gpu, rms_rel, say, to_dev
from tests.util import make_mini

pytestmark = pytest.mark.gpu

NCH = 40


def _many_channel_workload(seed, flag_fraction=0.0, jitter=0.0):
    """Slow uv tracks: every block of 24 timesteps x 40 channels fits one subgrid (L = 16)."""
    rng = np.random.default_rng(seed)
    nbl, nt = 5, 24
    uvw = np.zeros((nbl, nt, 3))
    t = np.arange(nt)
    for b in range(nbl):
        start = rng.uniform(-8, 8, 2)
        vel = rng.uniform(-0.12, 0.12, 2)
        uvw[b, :, 0] = start[0] + vel[0] * t
        uvw[b, :, 1] = start[1] + vel[1] * t
        uvw[b, :, 2] = rng.uniform(-1.5, 1.5) + 0.02 * t
    freqs = C0 * (1.0 + 0.0015 * np.arange(NCH))
    if jitter:
        freqs = freqs + C0 * jitter * rng.uniform(-1, 1, NCH)
    flags = (rng.random((nbl, nt, NCH)) < flag_fraction).astype(np.uint8) if flag_fraction else None
    return make_mini(uvw, freqs=freqs, N=64, L=16, beta=3, flags=flags, seed=seed, random_aterms=True,
                     random_taper=True)


CASES = {
    "even-40ch": lambda: _many_channel_workload(11),
    "even-40ch-flags": lambda: _many_channel_workload(12, flag_fraction=0.1),
    "uneven-40ch": lambda: _many_channel_workload(13, jitter=2e-4),
}


@pytest.fixture(scope="module")
def gpu():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    return torch, idg


@pytest.mark.parametrize("name", list(CASES))
def test_many_channel_subgrids(gpu, name):
    torch, idg = gpu
    wl = CASES[name]()
    oplan = plan_workload(wl)
    nvis = oplan.subgrids[:, F["nvis"]]
    nc = oplan.subgrids[:, F["nc"]]
    say(f"[channel runs] case={name} subgrids={oplan.nr_subgrids} vis={oplan.nr_gridded} "
        f"max channels/subgrid={nc.max()} max samples/subgrid={nvis.max()}")
    assert nc.max() > 16 and nvis.max() > 256       # the run cuts under test do occur
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)

    g = torch.zeros((4, wl.grid_size, wl.grid_size), dtype=torch.complex64, device="cuda")
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
    idg.sync()
    gref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    g = g.cpu().numpy()
    say(f"    grid rms rel {rms_rel(g, gref):.2e} max rel {max_rel(g, gref):.2e}")
    assert rms_rel(g, gref) < GRID_RMS_TOL
    assert max_rel(g, gref) < GRID_MAX_TOL

    rng = np.random.default_rng(4)
    N = wl.grid_size
    grid_in = (rng.standard_normal((4, N, N)) + 1j * rng.standard_normal((4, N, N))).astype(np.complex64)
    vref = oidg.degrid(oplan, wl.uvw, wl.freqs, grid_in, wl.aterms, wl.taper)
    planned = np.zeros(wl.vis.shape[:3], bool)
    for p in range(oplan.nr_subgrids):
        tc = oplan.subgrid_samples(p)
        planned[oplan.subgrids[p, F["bl"]], tc[:, 0], tc[:, 1]] = True
    for shape in ("standard", "wide"):
        plan.set_tuning(degrid_shape=shape)
        v = torch.full(tuple(wl.vis.shape), 3.0 - 1.0j, dtype=torch.complex64, device="cuda")
        idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(grid_in).cuda(), d["aterms"], d["taper"], v)
        idg.sync()
        got = v.cpu().numpy()
        say(f"    {shape} degridder: vis rms rel {rms_rel(got[planned], vref[planned]):.2e}")
        assert rms_rel(got[planned], vref[planned]) < VIS_RMS_TOL, shape
        assert np.all(got[~planned] == 0)
