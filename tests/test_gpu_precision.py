"""Precision study: float64 subgrid offsets vs an all-float32 phase, bright source 5 deg off centre.

Data: the LOFAR-like geometry with a 10 Jy point source at (l, m) = (sin 5 deg, 0),
visibilities from the measurement equation in float64 (cast to complex64), identity
A-terms.  The source lies outside the imaged field, so the per-sample phases u*l
before subtracting the subgrid centre reach hundreds of cycles -- the case where
float32 loses phase.  For both variants the grid, the degridded visibilities (from
the oracle's grid) and the grid -> degrid round trip are compared with the float64
oracle.  The float64-offset path must meet the 1e-5 parity bar; the all-float32
variant is reported (and must be the worse of the two).
"""

import numpy as np
import pytest

import synth
from oracle import idg as oidg
from oracle.plan import plan_workload
from tests.gpu_common import GRID_RMS_TOL, VIS_RMS_TOL, require_gpu, rms_rel, say, to_dev

pytestmark = pytest.mark.gpu


def test_precision_fp64_offsets_vs_fp32_phase():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    full = synth.make_workload("precision")
    wl = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 32), nt=256)
    oplan = plan_workload(wl)
    say(f"[precision] subgrids={oplan.nr_subgrids} vis={oplan.nr_gridded}")
    gref = oidg.grid(oplan, wl.uvw, wl.freqs, wl.vis, wl.aterms, wl.taper)
    g64 = gref.astype(np.complex64)
    vref = oidg.degrid(oplan, wl.uvw, wl.freqs, g64, wl.aterms, wl.taper)
    rt_ref = oidg.degrid(oplan, wl.uvw, wl.freqs, gref, wl.aterms, wl.taper)
    planned = np.abs(vref).sum(-1) > 0
    d = to_dev(wl)
    res = {}
    for name, fp32 in (("fp64_offsets", False), ("fp32_phase", True)):
        plan = idg.Plan.from_workload(wl, phase_fp32=fp32)
        g = torch.zeros((4, wl.grid_size, wl.grid_size), dtype=torch.complex64, device="cuda")
        idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
        v = torch.empty(tuple(wl.vis.shape), dtype=torch.complex64, device="cuda")
        idg.degrid(plan, d["uvw"], d["freqs"], torch.from_numpy(g64).cuda(), d["aterms"], d["taper"], v)
        rt = torch.empty_like(v)
        idg.degrid(plan, d["uvw"], d["freqs"], g, d["aterms"], d["taper"], rt)
        idg.sync()
        res[name] = dict(grid=rms_rel(g.cpu().numpy(), gref),
                         degrid=rms_rel(v.cpu().numpy()[planned], vref[planned]),
                         round_trip=rms_rel(rt.cpu().numpy()[planned], rt_ref[planned]))
        say(f"    {name}: grid rms rel {res[name]['grid']:.2e}, degrid {res[name]['degrid']:.2e}, "
            f"grid->degrid {res[name]['round_trip']:.2e}")
    assert res["fp64_offsets"]["grid"] < GRID_RMS_TOL
    assert res["fp64_offsets"]["degrid"] < VIS_RMS_TOL
    assert res["fp64_offsets"]["round_trip"] < VIS_RMS_TOL
    assert res["fp32_phase"]["grid"] > res["fp64_offsets"]["grid"]
