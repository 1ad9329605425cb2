"""Pins of the oracle planner (CPU only).

The paper fixes only the box criterion (§3.2, Fig. 2) and the shift bound of
§4.3 (a sample may sit at most (L - beta + 1)/2 pixels from the subgrid
centre), so the planner is pinned by (a) hand-worked cases whose expected
blocks and corners were computed on paper from the rule, and (b) invariants on
the realistic workloads: every unflagged sample is planned once or counted as
dropped, blocks respect T_max and A-term slots, and every planned sample lies
within the shift bound of its subgrid centre, with its w-support included.
"""

import numpy as np
import pytest

import synth
from oracle.plan import C0, F, plan_workload
from tests.util import make_mini


def _track(nt, x_of_t, y=0.0, w=0.0):
    uvw = np.zeros((1, nt, 3))
    uvw[0, :, 0] = x_of_t(np.arange(nt))
    uvw[0, :, 1] = y
    uvw[0, :, 2] = w
    return uvw


def _cols(plan, *names):
    return [tuple(int(plan.subgrids[p, F[n]]) for n in names) for p in range(plan.nr_subgrids)]


def test_greedy_time_blocks():
    # N = 128, S = 1, f = c0: x = 64 + u.  Track u = 2t, L = 16, beta = 3: a block may span 12 px,
    # i.e. 7 timesteps.  Blocks [0,7) x 64..76 centre 70 -> x0 62; [7,14) 78..90 -> 84 -> 76;
    # [14,20) 92..102 centre floor(97.5) = 97 -> 89.  y = 64 -> y0 = 56.
    wl = make_mini(_track(20, lambda t: 2.0 * t), N=128, L=16, beta=3)
    plan = plan_workload(wl)
    assert _cols(plan, "t0", "nt", "x0", "y0", "nvis") == [(0, 7, 62, 56, 7), (7, 7, 76, 56, 7), (14, 6, 89, 56, 6)]
    assert plan.nr_dropped == 0


def test_tmax_and_aterm_slots_cut_blocks():
    wl = make_mini(_track(20, lambda t: 2.0 * t), N=128, L=16, beta=3, tmax=5)
    assert _cols(plan_workload(wl), "t0", "nt", "x0") == [(0, 5, 60), (5, 5, 70), (10, 5, 80), (15, 5, 90)]
    wl = make_mini(_track(20, lambda t: 2.0 * t), N=128, L=16, beta=3, aslot=4)
    assert _cols(plan_workload(wl), "t0", "nt", "slot") == [(0, 4, 0), (4, 4, 1), (8, 4, 2), (12, 4, 3), (16, 4, 4)]


def test_w_support_shrinks_blocks_and_drops():
    # w = 9 wavelengths at S = 1 -> ceil(9) = 9 px of w-support: span + 3 + 9 <= 15 -> span <= 3 -> 2 timesteps
    wl = make_mini(_track(6, lambda t: 2.0 * t, w=9.0), N=128, L=16, beta=3)
    assert _cols(plan_workload(wl), "t0", "nt") == [(0, 2), (2, 2), (4, 2)]
    # w = 13 -> 3 + 13 > 15 even for one sample: everything is dropped
    wl = make_mini(_track(6, lambda t: 2.0 * t, w=13.0), N=128, L=16, beta=3)
    plan = plan_workload(wl)
    assert plan.nr_subgrids == 0 and plan.nr_dropped == 6


def test_channel_groups_split_in_halves():
    # u = 20 at f = c0 * {1.0, 1.1, 2.0, 2.1}: x = 84, 86, 104, 106 -> split into [0,2) and [2,4)
    wl = make_mini(_track(3, lambda t: 20.0 + 0 * t), freqs=C0 * np.array([1.0, 1.1, 2.0, 2.1]), N=256, L=16, beta=3)
    assert _cols(plan_workload(wl), "c0", "nc", "t0", "nt") == [(0, 2, 0, 3), (2, 2, 0, 3)]
    # three channels {1.0, 1.1, 2.0}: [0,3) fails -> [0,1) + [1,3); [1,3) spans 86..104 -> [1,2) + [2,3)
    wl = make_mini(_track(3, lambda t: 20.0 + 0 * t), freqs=C0 * np.array([1.0, 1.1, 2.0]), N=256, L=16, beta=3)
    assert _cols(plan_workload(wl), "c0", "nc") == [(0, 1), (1, 1), (2, 1)]


def test_grid_edge_drops_block():
    # centre near x = 4 with L = 16 would need x0 < 0: dropped, not wrapped
    wl = make_mini(_track(2, lambda t: -60.0 + 0 * t), N=128, L=16, beta=3)
    plan = plan_workload(wl)
    assert plan.nr_subgrids == 0 and plan.nr_dropped == 2


def test_flags_count_but_do_not_shape():
    flags = np.zeros((1, 20, 1), np.uint8)
    flags[0, 7:14] = 1                         # the whole second block is flagged
    flags[0, 2] = 1
    wl = make_mini(_track(20, lambda t: 2.0 * t), N=128, L=16, beta=3, flags=flags)
    plan = plan_workload(wl)
    assert _cols(plan, "t0", "nt", "x0", "nvis") == [(0, 7, 62, 6), (14, 6, 89, 6)]
    assert plan.nr_flagged == 8 and plan.nr_gridded == 12
    assert [tuple(r) for r in plan.subgrid_samples(0)] == [(t, 0) for t in range(7) if t != 2]


def _check_invariants(wl, plan):
    N, L, S, beta = wl.grid_size, wl.subgrid_size, wl.image_size, wl.kernel_size
    nbl, nt, nch = wl.nr_baselines, wl.nr_timesteps, wl.nr_channels
    total = nbl * nt * nch
    assert plan.nr_gridded + plan.nr_dropped + plan.nr_flagged == total
    assert plan.nr_gridded == plan.samples.shape[0] == int(plan.subgrids[:, F["nvis"]].sum())
    seen = np.zeros((nbl, nt, nch), bool)
    s = wl.freqs / C0
    prev = (-1, -1, -1)
    for p in range(plan.nr_subgrids):
        sub = plan.subgrids[p]
        bl, t0, nts, c0, nc = (int(sub[F[k]]) for k in ("bl", "t0", "nt", "c0", "nc"))
        key = (bl, c0, t0)
        assert key > prev
        prev = key
        assert 1 <= nts <= wl.max_timesteps
        assert t0 // wl.aterm_timesteps == (t0 + nts - 1) // wl.aterm_timesteps == sub[F["slot"]]
        assert tuple(sub[[F["st1"], F["st2"]]]) == tuple(wl.baselines[bl])
        x0, y0 = int(sub[F["x0"]]), int(sub[F["y0"]])
        assert 0 <= x0 and x0 + L <= N and 0 <= y0 and y0 + L <= N
        tc = plan.subgrid_samples(p)
        assert np.all((tc[:, 0] >= t0) & (tc[:, 0] < t0 + nts) & (tc[:, 1] >= c0) & (tc[:, 1] < c0 + nc))
        assert not seen[bl, tc[:, 0], tc[:, 1]].any()
        seen[bl, tc[:, 0], tc[:, 1]] = True
        if wl.flags is not None:
            assert not wl.flags[bl, tc[:, 0], tc[:, 1]].any()
        # shift bound (§4.3) with the block's w-support: |x - centre| <= (L - beta - W) / 2 for every sample
        blk = wl.uvw[bl, t0:t0 + nts]
        u = blk[:, None, :] * s[None, c0:c0 + nc, None]
        x = u[..., 0] * S + N / 2
        y = u[..., 1] * S + N / 2
        wmax = np.ceil(np.abs(u[..., 2]).max() * S * S)
        bound = (L - beta - wmax) / 2 + 1e-9
        assert np.abs(x - (x0 + L / 2)).max() <= bound
        assert np.abs(y - (y0 + L / 2)).max() <= bound
    if wl.flags is not None:
        assert not (seen & (wl.flags != 0)).any()
    assert int(seen.sum()) == plan.nr_gridded


def test_invariants_tiny():
    wl = synth.make_workload("tiny", with_vis=False)
    plan = plan_workload(wl)
    assert plan.nr_subgrids == 56 and plan.nr_gridded == 3584 and plan.nr_dropped == 0
    _check_invariants(wl, plan)


def test_invariants_lofar_subset():
    wl = synth.subset(synth.make_workload("lofar", with_vis=False), baselines=np.arange(0, 1128, 37), nt=300)
    plan = plan_workload(wl)
    assert plan.nr_subgrids > 60
    _check_invariants(wl, plan)


def test_invariants_skalow_subset_with_flags():
    full = synth.make_workload("skalow", with_vis=False)
    wl = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 1021))
    plan = plan_workload(wl)
    assert plan.nr_flagged > 0 and plan.nr_subgrids > 100
    _check_invariants(wl, plan)
