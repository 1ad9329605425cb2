"""Autotuner for a plan's scheduling knobs (idg_plan_set_tuning).

Candidates are timed on the plan's own data with the library's HIP-event stage
timers (idg_profile): gridder and degridder in the plain form and in the
persistent work-queue form at several workgroups per compute unit, the
degridder in its standard and wide shapes, the adder at several chunk
lengths, and, where the plan has subgrids in the separable form, the direct
sum instead (the two sum paths agree to float32 level).  The fastest setting
of each stage wins; the choice is stored on the plan and cached per (device,
L, N, plan shape) in a JSON file (``$IDG_TUNING_CACHE`` or
``~/.cache/paper_1909_07226_amd/tuning.json``).  Results are identical for the
gridder and degridder forms and equal up to float32 summation order for the
degridder shapes and the adder chunks.
"""

import json
import os

import numpy as np

from . import _lib

GRID_CANDIDATES = (("plain", 0), ("persistent", 0), ("persistent", 1), ("persistent", 2))
DEGRID_SHAPES = ("standard", "wide")
CHUNK_CANDIDATES = (32, 64, 256, 1024)


def _cache_path():
    return os.environ.get("IDG_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1909_07226_amd", "tuning.json"))


def plan_key(plan):
    import torch
    st = plan.stats()
    n = max(1, st["nr_subgrids"])
    mean_k = st["nr_gridded"] / n
    dev = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(dev, "gcnArchName", dev.name)
    return (f"v4|{arch}|L{plan.subgrid_size}|N{plan.grid_size}|P2^{int(np.log2(n))}"
            f"|K2^{int(np.log2(max(1.0, mean_k)))}")


def load_cached(plan):
    try:
        with open(_cache_path()) as f:
            return json.load(f).get(plan_key(plan))
    except (OSError, ValueError):
        return None


def _store(plan, tuning):
    path = _cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            with open(path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
        data[plan_key(plan)] = tuning
        with open(path + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass


def _stage_ms(fn, stage, reps, stream):
    _lib.profile(True)
    _lib.profile_read(reset=True)
    for _ in range(reps):
        fn()
    _lib.sync(stream)
    prof = _lib.profile_read(reset=True)
    _lib.profile(False)
    return prof[stage][0] / reps


def autotune(plan, uvw, freqs, vis, aterms, taper, grid, vis_out=None, reps=2, use_cache=True, log=None):
    """Choose and set the plan's tuning; returns {"tuning": ..., "timings_ms": ...}.

    ``grid`` is scratch output for gridding and input for degridding (its
    contents are overwritten); ``vis_out`` receives degridded visibilities.
    """
    import torch
    if use_cache:
        cached = load_cached(plan)
        if cached:
            plan.set_tuning(**cached)
            return {"tuning": cached, "timings_ms": None, "cached": True}
    stream = torch.cuda.current_stream()
    vis_out = torch.empty_like(vis) if vis_out is None else vis_out
    timings = {}

    def do_grid():
        grid.zero_()
        _lib.grid(plan, uvw, freqs, vis, aterms, taper, grid, stream)

    def do_degrid():
        _lib.degrid(plan, uvw, freqs, grid, aterms, taper, vis_out, stream)

    plan.set_tuning(sum_path="auto")
    # the degridder shape selects among the direct-sum degridders only: with every subgrid in the separable
    # form it changes nothing, and timing it would pick at random between equal times
    shapes = DEGRID_SHAPES if plan.sum_paths()["direct"][0] > 0 else ("standard",)
    best_g = best_d = None
    for form, bpc in GRID_CANDIDATES:
        plan.set_tuning(grid_form=form, degrid_form=form, grid_blocks_per_cu=bpc, degrid_blocks_per_cu=bpc)
        do_grid()
        do_degrid()                     # warm-up (device upload, caches)
        _lib.sync(stream)
        tg = _stage_ms(do_grid, "gridder", reps, stream)
        timings[f"gridder/{form}/{bpc}"] = round(tg, 4)
        if best_g is None or tg < best_g[0]:
            best_g = (tg, form, bpc)
        tds = []
        for shape in shapes:
            plan.set_tuning(degrid_shape=shape)
            do_degrid()
            td = _stage_ms(do_degrid, "degridder", reps, stream)
            timings[f"degridder/{form}/{bpc}/{shape}"] = round(td, 4)
            tds.append(f"{shape} {td:.3f} ms")
            if best_d is None or td < best_d[0]:
                best_d = (td, form, bpc, shape)
        if log:
            log(f"[autotune] {form}/{bpc}: gridder {tg:.3f} ms, degridder " + ", ".join(tds))
    plan.set_tuning(grid_form=best_g[1], grid_blocks_per_cu=best_g[2], degrid_form=best_d[1],
                    degrid_blocks_per_cu=best_d[2], degrid_shape=best_d[3])
    paths = plan.sum_paths()
    if paths["separable0"][0] + paths["separable1"][0] > 0:
        # one knob for both directions: keep the path with the smaller gridder + degridder time
        plan.set_tuning(sum_path="direct")
        do_grid()
        do_degrid()
        _lib.sync(stream)
        tg = _stage_ms(do_grid, "gridder", reps, stream)
        td = _stage_ms(do_degrid, "degridder", reps, stream)
        timings["sum_path/direct"] = round(tg + td, 4)
        timings["sum_path/auto"] = round(best_g[0] + best_d[0], 4)
        if log:
            log(f"[autotune] sum path: auto {best_g[0] + best_d[0]:.3f} ms, direct {tg + td:.3f} ms")
        if tg + td >= best_g[0] + best_d[0]:
            plan.set_tuning(sum_path="auto")
    best_c = None
    for chunk in CHUNK_CANDIDATES:
        plan.set_tuning(adder_chunk=chunk)
        do_grid()
        _lib.sync(stream)
        ta = _stage_ms(do_grid, "adder", reps, stream)
        timings[f"adder/{chunk}"] = round(ta, 4)
        if best_c is None or ta < best_c[0]:
            best_c = (ta, chunk)
        if log:
            log(f"[autotune] adder chunk {chunk}: {ta:.3f} ms")
    plan.set_tuning(adder_chunk=best_c[1])
    tuning = plan.get_tuning()
    if use_cache:
        _store(plan, tuning)
    return {"tuning": tuning, "timings_ms": timings, "cached": False}
