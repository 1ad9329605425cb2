"""Host-side tests of the C ABI (no GPU calls).

* the library loads and exports every function include/idg.h declares;
* the library's C++ planner produces exactly the oracle planner's plan
  (integer-identical subgrid records and sample lists);
* invalid arguments are rejected with the documented error codes.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle.plan import plan_workload
from tests.util import make_mini, random_track_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

idg = pytest.importorskip("paper_1909_07226_amd")
if not os.path.exists(idg.LIB_PATH):
    pytest.skip("libidg.so not built", allow_module_level=True)


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "idg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(idg_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(idg.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(idg._lib.EXPORTED)
    assert idg.version() == 10200


def _compare(wl, w_step=0.0):
    ref = plan_workload(wl, w_step)
    p = idg.Plan.from_workload(wl, w_step=w_step)
    st = p.stats()
    assert st == dict(nr_subgrids=ref.nr_subgrids, nr_gridded=ref.nr_gridded, nr_dropped=ref.nr_dropped,
                      nr_flagged=ref.nr_flagged)
    sub, smp = p.export()
    assert np.array_equal(sub, ref.subgrids)
    assert np.array_equal(smp.astype(np.int64), ref.samples)
    return p, ref


@pytest.mark.parametrize("seed", [3, 4, 5, 7])
def test_plan_parity_random_tracks(seed):
    _compare(random_track_workload(seed=seed, nbl=5, nt=40, nch=4))


def test_plan_parity_hand_cases():
    uvw = np.zeros((1, 20, 3))
    uvw[0, :, 0] = 2.0 * np.arange(20)
    for kw in (dict(), dict(tmax=5), dict(aslot=4)):
        _compare(make_mini(uvw, N=128, L=16, beta=3, **kw))
    uvw[0, :, 2] = 9.0
    _compare(make_mini(uvw, N=128, L=16, beta=3))
    flags = np.zeros((1, 20, 1), np.uint8)
    flags[0, 7:14] = 1
    uvw[0, :, 2] = 0.0
    _compare(make_mini(uvw, N=128, L=16, beta=3, flags=flags))


@pytest.mark.parametrize("w_step", [0.7, 4.0])
def test_plan_parity_w_layers(w_step):
    # deep w (|w| S^2 up to 40 px at L = 32) across channels: layers, per-timestep layers in the
    # channel-group step, the block's own offset in the time scan
    rng = np.random.default_rng(17)
    uvw = np.zeros((6, 30, 3))
    t = np.arange(30)
    for b in range(6):
        uvw[b, :, 0] = rng.uniform(-30, 30) + rng.uniform(-0.6, 0.6) * t
        uvw[b, :, 1] = rng.uniform(-30, 30) + rng.uniform(-0.6, 0.6) * t
        uvw[b, :, 2] = rng.choice([-1, 1]) * (rng.uniform(5, 40) + rng.uniform(0, 0.5) * t)
    wl = make_mini(uvw, freqs=synth.C0 * (1.0 + 0.05 * np.arange(4)), N=128, L=32, beta=7)
    p, ref = _compare(wl, w_step)
    assert p.wlayers() == (ref.wlayer_min, ref.nr_wlayers) and ref.nr_wlayers > 1
    assert p.shapes()["grid"] == (ref.nr_wlayers, 4, 128, 128)


def test_plan_parity_lofar_subset_with_layers():
    # LOFAR-like geometry on a 4x wider field (S = 0.2): |w| S^2 reaches ~80 pixels without layers
    import dataclasses
    wl = synth.make_workload("lofar", with_vis=False)
    wl = dataclasses.replace(wl, image_size=0.2, baselines=wl.baselines[::64], uvw=wl.uvw[::64, :256])
    _, ref0 = _compare(wl)
    _, ref = _compare(wl, 50.0)
    assert ref.nr_gridded > ref0.nr_gridded and ref.nr_wlayers > 1


def test_plan_parity_tiny():
    p, ref = _compare(synth.make_workload("tiny", with_vis=False))
    assert ref.nr_subgrids == 56


def test_plan_parity_skalow_subset_flags():
    full = synth.make_workload("skalow", with_vis=False)
    _compare(synth.subset(full, baselines=np.arange(0, full.nr_baselines, 257)))


@pytest.mark.slow
def test_plan_parity_lofar_full():
    _compare(synth.make_workload("lofar", with_vis=False))


def _mini_params(**over):
    wl = random_track_workload(seed=3)
    args = dict(grid_size=wl.grid_size, image_size=wl.image_size, subgrid_size=wl.subgrid_size,
                kernel_size=wl.kernel_size, max_timesteps=wl.max_timesteps, aterm_timesteps=wl.aterm_timesteps,
                nr_stations=wl.nr_stations, baselines=wl.baselines, uvw=wl.uvw, freqs=wl.freqs)
    args.update(over)
    return args


@pytest.mark.parametrize("over", [dict(subgrid_size=20), dict(grid_size=63), dict(grid_size=8),
                                  dict(kernel_size=16), dict(max_timesteps=0), dict(aterm_timesteps=0),
                                  dict(image_size=0.0), dict(image_size=2.0), dict(nr_stations=1)])
def test_invalid_params_rejected(over):
    with pytest.raises(idg.IDGError) as e:
        idg.Plan(**_mini_params(**over))
    assert e.value.code == -1


def test_invalid_inputs_rejected():
    args = _mini_params()
    uvw = args["uvw"].copy()
    uvw[1, 2, 0] = np.nan
    with pytest.raises(idg.IDGError) as e:
        idg.Plan(**dict(args, uvw=uvw))
    assert e.value.code == -1 and "not finite" in str(e.value)
    bl = args["baselines"].copy()
    bl[0] = (2, 2)
    with pytest.raises(idg.IDGError):
        idg.Plan(**dict(args, baselines=bl))
    bl[0] = (0, 99)
    with pytest.raises(idg.IDGError):
        idg.Plan(**dict(args, baselines=bl))
    with pytest.raises(idg.IDGError):
        idg.Plan(**dict(args, freqs=-args["freqs"]))


def test_strict_reports_dropped_samples():
    uvw = np.zeros((1, 6, 3))
    uvw[0, :, 0] = 2.0 * np.arange(6)
    uvw[0, :, 2] = 13.0                       # w-support too large for L = 16: every sample is dropped
    wl = make_mini(uvw, N=128, L=16, beta=3)
    p = idg.Plan.from_workload(wl)
    assert p.stats()["nr_dropped"] == 6
    with pytest.raises(idg.IDGError) as e:
        idg.Plan.from_workload(wl, strict=True)
    assert e.value.code == -4


def test_empty_plan():
    wl = make_mini(np.zeros((2, 0, 3)), N=64, L=16, beta=3)
    p = idg.Plan.from_workload(wl)
    assert p.stats() == dict(nr_subgrids=0, nr_gridded=0, nr_dropped=0, nr_flagged=0)


def test_tuning_round_trip_and_validation():
    p = idg.Plan(**_mini_params())
    assert p.get_tuning() == dict(grid_form="plain", degrid_form="plain", grid_blocks_per_cu=0,
                                  degrid_blocks_per_cu=0, adder_chunk=0, degrid_shape="standard", sum_path="auto")
    p.set_tuning(form="persistent", blocks_per_cu=3, adder_chunk=17, degrid_shape="wide", sum_path="direct")
    assert p.get_tuning() == dict(grid_form="persistent", degrid_form="persistent", grid_blocks_per_cu=3,
                                  degrid_blocks_per_cu=3, adder_chunk=17, degrid_shape="wide", sum_path="direct")
    p.set_tuning(degrid_form="plain", grid_blocks_per_cu=2)
    t = p.get_tuning()
    assert (t["grid_form"], t["degrid_form"], t["grid_blocks_per_cu"], t["degrid_blocks_per_cu"]) == (
        "persistent", "plain", 2, 3)
    for bad in (dict(form=7), dict(blocks_per_cu=-1), dict(degrid_blocks_per_cu=65), dict(adder_chunk=-2),
                dict(degrid_shape=2), dict(sum_path=5)):
        with pytest.raises(idg.IDGError) as e:
            p.set_tuning(**bad)
        assert e.value.code == -1
    assert p.get_tuning()["adder_chunk"] == 17          # unchanged by the rejected calls
    assert p.get_tuning()["degrid_shape"] == "wide"


def test_image_steps_validate_before_any_device_call():
    # argument checks of idg_grid_to_image / idg_image_to_grid run on the host: fake addresses are
    # never dereferenced when the call is rejected
    L = ctypes.CDLL(idg.LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    for fn in (L.idg_grid_to_image, L.idg_image_to_grid):
        fn.argtypes = [vp, i32, vp, vp, vp, vp]
        fn.restype = ctypes.c_int
        a, b = vp(0x10000000), vp(0x90000000)
        assert fn(a, 100, None, None, b, None) == -1            # not a power of two
        assert fn(a, 32, None, None, b, None) == -1             # below 64
        assert fn(a, 32768, None, None, b, None) == -1          # above 16384
        assert fn(None, 256, None, None, b, None) == -1         # NULL input
        assert fn(a, 256, vp(0x20000000), None, b, None) == -1  # one correction only
        assert fn(a, 256, None, None, vp(0x10000000 + 4096), None) == -1   # overlapping buffers
        L.idg_last_error.restype = ctypes.c_char_p
        assert b"overlap" in L.idg_last_error()


def test_grid_noalloc_validates_before_any_device_call():
    # NULL plan or NULL device pointers are refused on the host; fake addresses are never dereferenced
    L = ctypes.CDLL(idg.LIB_PATH)
    vp = ctypes.c_void_p
    L.idg_grid_noalloc.argtypes = [vp] * 8
    L.idg_grid_noalloc.restype = ctypes.c_int
    f = vp(0x10000000)
    assert L.idg_grid_noalloc(None, f, f, f, f, f, f, None) == -1
    wl = random_track_workload(seed=3, nbl=2, nt=10, nch=2)
    p = idg.Plan.from_workload(wl)
    assert p.nr_subgrids > 0
    assert L.idg_grid_noalloc(p.handle, f, None, f, f, f, f, None) == -1
    L.idg_last_error.restype = ctypes.c_char_p
    assert b"NULL" in L.idg_last_error()
    assert idg.NOALLOC_SCRATCH_BYTES == 128 << 20


def _expected_sum_paths(wl, p, w_step=0.0):
    """Per-subgrid evaluation of the sums, from the plan's samples in float64: order 0 or 1 of the
    separable form where the truncation of exp(2 pi i dw c) stays below 1e-6, else the direct sum."""
    L, S = wl.subgrid_size, wl.image_size
    x = (np.arange(L) - L // 2) * (S / L)
    a = np.sqrt(1.0 - x * x) - 1.0
    n2 = np.sqrt(1.0 - x[None, :] ** 2 - x[:, None] ** 2) - 1.0
    cmax = np.abs(n2 - a[None, :] - a[:, None]).max()
    sub, smp = p.export()
    cols = idg.SUBGRID_FIELDS
    ns, nv = [0, 0, 0], [0, 0, 0]
    for r in sub:
        bl, off, nvis, layer = r[cols.index("bl")], r[cols.index("vis_offset")], r[cols.index("nvis")], \
            r[cols.index("wlayer")]
        t, c = smp[off:off + nvis, 0], smp[off:off + nvis, 1]
        w = wl.uvw[bl, t, 2] * wl.freqs[c] / 299792458.0 - layer * w_step
        theta = 2 * np.pi * np.abs(w).max() * cmax
        k = 0 if theta <= 1e-6 else (1 if theta * theta / 2 <= 1e-6 else 2)
        ns[k] += 1
        nv[k] += int(nvis)
    return {"separable0": (ns[0], nv[0]), "separable1": (ns[1], nv[1]), "direct": (ns[2], nv[2])}


@pytest.mark.parametrize("name", ["lofar", "skalow"])
def test_sum_paths_follow_the_truncation_rule(name):
    full = synth.make_workload(name, with_vis=False)
    wl = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 97 if name == "lofar" else 1031))
    p = idg.Plan.from_workload(wl)
    got = p.sum_paths()
    assert got == _expected_sum_paths(wl, p)
    st = p.stats()
    assert sum(v[0] for v in got.values()) == st["nr_subgrids"]
    assert sum(v[1] for v in got.values()) == st["nr_gridded"]
    assert got["separable0"][0] + got["separable1"][0] > 0
    p.set_tuning(sum_path="direct")
    assert p.sum_paths() == {"separable0": (0, 0), "separable1": (0, 0),
                             "direct": (st["nr_subgrids"], st["nr_gridded"])}


def test_sum_paths_direct_for_other_subgrid_sizes_and_fp32_offsets():
    wl = synth.make_workload("tiny", with_vis=False)      # L = 24
    p = idg.Plan.from_workload(wl)
    st = p.stats()
    assert p.sum_paths()["direct"] == (st["nr_subgrids"], st["nr_gridded"])
    full = synth.make_workload("lofar", with_vis=False)
    wl = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 211))
    p = idg.Plan.from_workload(wl, phase_fp32=True)
    st = p.stats()
    assert p.sum_paths()["direct"] == (st["nr_subgrids"], st["nr_gridded"])
