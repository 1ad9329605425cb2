"""Autotuner on the GPU: it picks valid settings, caches them, and the tuned plan stays exact."""

import numpy as np
import pytest

from oracle import idg as oidg
from oracle.plan import plan_workload
from tests.gpu_common import GRID_RMS_TOL, VIS_RMS_TOL, require_gpu, rms_rel, say, to_dev
from tests.util import random_track_workload

pytestmark = pytest.mark.gpu


def test_autotune_choice_cache_and_parity(tmp_path, monkeypatch):
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    from paper_1909_07226_amd import autotune as at
    monkeypatch.setenv("IDG_TUNING_CACHE", str(tmp_path / "tuning.json"))
    wl = random_track_workload(seed=41, N=128, L=16, beta=3, nbl=8, nt=60, nch=8, random_aterms=True,
                               random_taper=True)
    oplan = plan_workload(wl)
    plan = idg.Plan.from_workload(wl)
    d = to_dev(wl)
    N = wl.grid_size
    grid = torch.zeros((4, N, N), dtype=torch.complex64, device="cuda")
    say(f"[autotune] subgrids={oplan.nr_subgrids} vis={oplan.nr_gridded}")
    info = at.autotune(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], grid, reps=1)
    t = info["tuning"]
    assert not info["cached"] and info["timings_ms"]
    assert (t["grid_form"], t["grid_blocks_per_cu"]) in at.GRID_CANDIDATES
    assert (t["degrid_form"], t["degrid_blocks_per_cu"]) in at.GRID_CANDIDATES
    assert t["adder_chunk"] in at.CHUNK_CANDIDATES and t["degrid_shape"] in at.DEGRID_SHAPES
    assert plan.get_tuning() == t
    # a second plan of the same shape takes the cached choice
    plan2 = idg.Plan.from_workload(wl)
    info2 = at.autotune(plan2, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], grid, reps=1)
    assert info2["cached"] and plan2.get_tuning() == t
    # the tuned plan grids and degrids within the parity bar
    grid.zero_()
    idg.grid(plan2, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], grid)
    vis = torch.empty_like(d["vis"])
    idg.degrid(plan2, d["uvw"], d["freqs"], grid, d["aterms"], d["taper"], vis)
    idg.sync()
    g = grid.cpu().numpy()
    gref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    vref = oidg.degrid(oplan, wl.uvw, wl.freqs, g, wl.aterms, wl.taper)
    planned = np.abs(vref).sum(-1) > 0
    say(f"    tuning {t}; grid rms rel {rms_rel(g, gref):.2e}")
    assert rms_rel(g, gref) < GRID_RMS_TOL
    assert rms_rel(vis.cpu().numpy()[planned], vref[planned]) < VIS_RMS_TOL
