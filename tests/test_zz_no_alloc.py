"""idg_grid_noalloc (the entry point that allocates no device memory) against idg_grid.

Both run the same kernels over the same batches, so the grids must be bitwise
equal.  Two calls in a row share the library's fixed device scratch; the second
uses a smaller plan (other subgrid size, fewer subgrids), so a stale scratch
from the first call would show.  Also: a plan whose batch does not fit the
fixed scratch is refused with IDG_ERANGE, and a plan with no device copy yet
with IDG_ESTATE, both before anything is launched.
"""

import numpy as np
import pytest

import synth
from tests.gpu_common import require_gpu, say, to_dev

pytestmark = pytest.mark.gpu


def _lofar_subset():
    full = synth.make_workload("lofar")
    return synth.subset(full, baselines=np.arange(0, full.nr_baselines, 37), nt=300)


def _grids(torch, idg, wl, plan, d, form):
    plan.set_tuning(form=form)
    N = wl.grid_size
    gen = torch.Generator(device="cuda").manual_seed(N)
    base = torch.complex(torch.randn((4, N, N), generator=gen, device="cuda"),
                         torch.randn((4, N, N), generator=gen, device="cuda")).to(torch.complex64)
    ref = base.clone()
    idg.grid(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], ref)   # also makes the device copy
    out = base.clone()
    idg.grid_noalloc(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], out)
    idg.sync()
    return ref, out


def test_grid_noalloc_equals_grid_two_calls():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    cases = [("lofar-subset", _lofar_subset(), 32 << 20), ("tiny", synth.make_workload("tiny"), 8 << 20)]
    for form in ("persistent", "plain"):
        for name, wl, scratch in cases:        # the second call has the smaller plan
            plan = idg.Plan.from_workload(wl, scratch_bytes=scratch)
            d = to_dev(wl)
            ref, out = _grids(torch, idg, wl, plan, d, form)
            say(f"[noalloc] {name} form={form} subgrids={plan.nr_subgrids} L={wl.subgrid_size}")
            assert torch.equal(out, ref), (name, form)
            assert torch.count_nonzero(out - ref).item() == 0


def test_grid_noalloc_refuses_what_does_not_fit():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    wl = synth.make_workload("tiny")
    d = to_dev(wl)
    N = wl.grid_size
    g = torch.zeros((4, N, N), dtype=torch.complex64, device="cuda")
    plan = idg.Plan.from_workload(wl, scratch_bytes=8 << 20)
    with pytest.raises(idg.IDGError) as e:             # no device copy of this plan yet
        idg.grid_noalloc(plan, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
    assert e.value.code == -5
    # every 4th LOFAR-like baseline: ~10,000 subgrids of 32 x 32 in one batch need ~320 MB, more than the
    # fixed scratch
    full = synth.make_workload("lofar")
    wl = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 4))
    d = to_dev(wl)
    N = wl.grid_size
    g = torch.zeros((4, N, N), dtype=torch.complex64, device="cuda")
    big = idg.Plan.from_workload(wl)
    assert big.nr_subgrids * 4 * 32 * 32 * 8 > idg.NOALLOC_SCRATCH_BYTES
    idg.grid(big, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
    idg.sync()
    before = g.clone()
    with pytest.raises(idg.IDGError) as e:
        idg.grid_noalloc(big, d["uvw"], d["freqs"], d["vis"], d["aterms"], d["taper"], g)
    assert e.value.code == -4
    idg.sync()
    assert torch.equal(g, before)                      # nothing was launched
