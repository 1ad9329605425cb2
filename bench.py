#!/usr/bin/env python3
"""Throughput of image-domain gridding + degridding on one MI355X.

One step = idg_grid of every planned visibility of the workload into a zeroed
4 x N x N grid, then idg_degrid of every planned visibility from that grid --
the whole hot path (plan reused, as in every major cycle of an imager).
Inputs are resident in HBM before the timed region.  Prints one JSON line:
value = planned visibilities / (wall time of grid + degrid), in MVis/s.

    python bench.py [--steps K] [--warmup W] [--workload lofar|tiny|skalow]

The roofline entry is for the gridder kernel: algorithmic work 34 flop per
(visibility, subgrid pixel) -- one phase multiply-add and 16 multiply-adds of
the 4-polarisation complex accumulate; sin and cos are not counted -- divided
by the gridder's average launch time from HIP events recorded by the library
on the launching stream.  The CPU baseline is the float64 oracle on a bounded
sample, timed on this host.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

FLOP_PER_VIS_PIX = 34
FP32_PEAK_TFLOPS = 157.3           # MI355X FP32 vector peak (256 CU x 4 SIMD x 16 lanes x 2 (packed) x 2 x 2.4 GHz)
WORKLOAD_DESC = {
    "lofar": "lofar-like: 48 stations (1128 baselines), 2048 x 1 s, 16 ch 120-180 MHz, |w| <= 2e3 lambda, "
             "L=32 subgrids of <=128 timesteps, 4096^2 grid at 2.5 arcsec, near-identity A-terms every 256 s",
    "tiny": "tiny: 8 stations (28 baselines), 32 x 10 s, 4 ch 150-151 MHz, w=0, L=24, 512^2 grid at 1 arcmin",
    "skalow": "skalow-like share: 512 stations (130816 baselines), 64 x 1 s, 16 ch 50-350 MHz, L=32, "
              "8192^2 grid at 1 arcsec, A-terms every 32 timesteps, 10% flags",
}


ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(ROOT, "paper_1909_07226_amd", "csrc", "kernels.hip")
HBM_RECORD = os.path.join(ROOT, "profiles", "lofar_hbm_counters.md")


def kernel_source_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def gridder_traffic(workload, form):
    """HBM bytes per gridder launch from the committed counter summary.

    The summary's ``traffic-record:`` line holds FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch) of the gridder and the factors that map each counter onto
    the bytes of a plain elementwise kernel of known size.  Returns None when
    there is no record for this workload and schedule, or when the kernel
    source has changed since the counters were taken.
    """
    try:
        with open(HBM_RECORD) as f:
            m = re.search(r"^traffic-record: (.*)$", f.read(), re.M)
    except OSError:
        return None
    if not m:
        return None
    rec = dict(kv.split("=", 1) for kv in m.group(1).split())
    if rec.get("workload") != workload or rec.get("form") != form or rec.get("kernels_sha256") != kernel_source_hash():
        return None
    return int(round(float(rec["fetch_kib"]) * 1024 * float(rec["fetch_factor"])
                     + float(rec["write_kib"]) * 1024 * float(rec["write_factor"])))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_worker(args):
    # cpu_baseline leg only: the float64 oracle, one subgrid at a time
    from threadpoolctl import threadpool_limits
    import oracle.idg as oidg
    p, direction = args
    with threadpool_limits(1):
        if direction == "grid":
            oidg.grid_subgrid(_G["plan"], p, _G["uvw"], _G["freqs"], _G["vis"], _G["aterms"], _G["taper"])
        else:
            oidg.degrid_subgrid(_G["plan"], p, _G["uvw"], _G["freqs"], _G["grid"], _G["aterms"], _G["taper"])
    return p


_G = {}


def cpu_baseline(wl, budget_s):
    """Time the oracle (as it stands) on every 16th baseline's subgrids, within ~budget_s seconds."""
    import multiprocessing as mp
    import synth
    from oracle.plan import F, plan_workload
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    sub_wl = synth.subset(wl, baselines=np.arange(0, wl.nr_baselines, 16))
    oplan = plan_workload(sub_wl)
    nvis = oplan.subgrids[:, F["nvis"]]
    # calibrate on a few subgrids, then pick a prefix of the subgrid list that fits the budget
    _G.update(plan=oplan, uvw=sub_wl.uvw, freqs=sub_wl.freqs, vis=sub_wl.vis, aterms=sub_wl.aterms,
              taper=sub_wl.taper, grid=np.zeros((4, wl.grid_size, wl.grid_size), np.complex64))
    t = time.perf_counter()
    for p in range(min(4, oplan.nr_subgrids)):
        _oracle_worker((p, "grid"))
        _oracle_worker((p, "degrid"))
    per_vis = (time.perf_counter() - t) / max(1, int(nvis[:4].sum()))
    target = budget_s * cores / per_vis
    n = int(np.searchsorted(np.cumsum(nvis), target)) + 1
    n = max(1, min(n, oplan.nr_subgrids))
    ids = list(range(n))
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_worker, [(p, "grid") for p in ids], chunksize=4)
        t1 = time.perf_counter()
        pool.map(_oracle_worker, [(p, "degrid") for p in ids], chunksize=4)
        t2 = time.perf_counter()
    k = int(nvis[:n].sum())
    return {"value": round(k / (t2 - t0) / 1e6, 6), "unit": "MVis/s", "cores": cores, "kind": "oracle",
            "sample": f"float64 numpy oracle, grid then degrid of the first {n} of {oplan.nr_subgrids} subgrids "
                      f"of every 16th baseline ({k} visibilities), {cores} processes",
            "grid_s": round(t1 - t0, 3), "degrid_s": round(t2 - t1, 3)}


HBM_PEAK_GBS = 8000.0               # MI355X HBM3E


def touched_tile_count(plan, tile=32):
    """Number of distinct tile x tile grid tiles that the plan's subgrids overlap."""
    sub, _ = plan.export()
    from paper_1909_07226_amd._lib import SUBGRID_FIELDS
    F = {n: i for i, n in enumerate(SUBGRID_FIELDS)}
    L = plan.subgrid_size
    x0, y0 = sub[:, F["x0"]], sub[:, F["y0"]]
    ntx = -(-plan.grid_size // tile)
    span = L // tile + 2
    ids = []
    for dy in range(span):
        for dx in range(span):
            tx, ty = x0 // tile + dx, y0 // tile + dy
            ok = (tx <= (x0 + L - 1) // tile) & (ty <= (y0 + L - 1) // tile)
            ids.append((ty * ntx + tx)[ok])
    return int(np.unique(np.concatenate(ids)).size)


def hbm_stages(idg, torch, plan, grid, stream, adder_ms_per_step, log, max_subgrids=65536, reps=5):
    """HBM rates of the memory-bound stages against the 8 TB/s peak.

    splitter (idg_split_subgrids) and the batched subgrid transform
    (idg_subgrid_fft, in place) run standalone here; inside idg_degrid and
    idg_grid they are fused and move no HBM bytes of their own.  Algorithmic
    bytes: the splitter reads and writes 4 L^2 x 8 bytes per subgrid, the
    transform the same; the adder (timed inside idg_grid) reads every subgrid
    once and reads and writes every touched grid tile once.  The master grid
    <-> image steps (idg_grid_to_image, idg_image_to_grid) overwrite `grid`
    with the round trip of its contents.
    """
    L = plan.subgrid_size
    P = plan.stats()["nr_subgrids"]
    n = min(P, max_subgrids)
    sub_bytes = 4 * L * L * 8
    buf = torch.empty((n, 4, L, L), dtype=torch.complex64, device="cuda")

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    t = timed(lambda: idg.split_subgrids(plan, grid, 0, buf, stream))
    out["splitter"] = dict(ms=round(t, 4), bytes=2 * n * sub_bytes, subgrids=n)
    t = timed(lambda: idg.subgrid_fft(buf, -1, stream))
    out["subgrid_fft"] = dict(ms=round(t, 4), bytes=2 * n * sub_bytes, subgrids=n)
    # master grid <-> image (four passes over the [4, N, N] array: rows, transpose, rows, transpose);
    # algorithmic bytes are one read of the input and one write of the output
    N = grid.shape[-1]
    corr = torch.ones(N, dtype=torch.float32, device="cuda")
    img = torch.empty_like(grid)
    arr = 4 * N * N * 8
    t = timed(lambda: idg.grid_to_image(grid, corr, corr, img, stream))
    out["grid_to_image"] = dict(ms=round(t, 4), bytes=2 * arr, grid_size=N, passes=4,
                                pass_gb_s=round(8 * arr / (t * 1e-3) / 1e9, 1))
    t = timed(lambda: idg.image_to_grid(img, corr, corr, grid, stream))
    out["image_to_grid"] = dict(ms=round(t, 4), bytes=2 * arr, grid_size=N, passes=4,
                                pass_gb_s=round(8 * arr / (t * 1e-3) / 1e9, 1))
    del img
    tiles = touched_tile_count(plan)
    out["adder"] = dict(ms=round(adder_ms_per_step, 4), bytes=P * sub_bytes + 2 * tiles * 4 * 32 * 32 * 8,
                        subgrids=P, touched_tiles=tiles)
    for k, v in out.items():
        gbs = v["bytes"] / (v["ms"] * 1e-3) / 1e9
        v["gb_s"] = round(gbs, 1)
        v["frac"] = round(gbs / HBM_PEAK_GBS, 4)
        log(f"[bench] {k}: {v['bytes'] / 1e9:.3f} GB in {v['ms']:.3f} ms = {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.1%})")
    del buf
    return out


def serving_leg(lofar_wl, lofar_dev, n_jobs, log):
    """Replay one request trace twice: continuous batching (4 slots, persistent form) and a FIFO
    (1 slot, plain form).  p50/p99 of completion - arrival."""
    import torch
    import synth
    from paper_1909_07226_amd import serve
    tiny = synth.make_workload("tiny", nt=2048, nch=16)
    dev = "cuda"
    tiny_dev = dict(uvw=torch.from_numpy(tiny.uvw).to(dev), freqs=torch.from_numpy(tiny.freqs).to(dev),
                    vis=torch.from_numpy(tiny.vis).to(dev), aterms=torch.from_numpy(tiny.aterms).to(dev),
                    taper=torch.from_numpy(tiny.taper).to(dev))
    g = torch.Generator(device=dev).manual_seed(11)
    grids = {c: torch.complex(torch.randn((4, n, n), generator=g, device=dev),
                              torch.randn((4, n, n), generator=g, device=dev)).to(torch.complex64)
             for c, n in (("tiny", tiny.grid_size), ("lofar", lofar_wl.grid_size))}
    trace = synth.serving_trace(n_jobs=n_jobs)
    t = time.perf_counter()
    jobs, templates = serve.jobs_from_trace(trace, {"tiny": tiny, "lofar": lofar_wl},
                                            {"tiny": tiny_dev, "lofar": lofar_dev}, grids)
    log(f"[bench] serving: {len(jobs)} jobs, {len(templates)} plans built in {time.perf_counter() - t:.1f} s")
    out = {"trace": f"{n_jobs} jobs, Poisson arrivals at 50 jobs/s, 50% grid / 50% degrid, 50% 8-station "
                    f"(N=512, L=24) / 50% LOFAR-like (N=4096, L=32), nt ~ U{{64..2048}}, nch ~ U{{4..16}}"}
    # warm-up outside the timed trace: every plan uploads its device metadata once
    for cls, tp in ((k[0], v) for k, v in templates.items()):
        for kind in ("grid", "degrid"):
            j = serve.Job(kind, tp["plan"], tp["uvw"], tp["freqs"], tp["aterms"], tp["taper"], vis=tp["vis"],
                          grid=grids[cls])
            j.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    for label, slots, form in (("continuous", 4, "persistent"), ("fifo_plain", 1, "plain")):
        for tp in templates.values():
            tp["plan"].set_tuning(form=form)
        with serve.Server(slots=slots, mem_budget=48 << 30) as srv:
            futs = serve.replay(srv, jobs, trace["arrivals"])
        summ = serve.latency_summary(futs)
        summ.update(slots=slots, form=form, failed=sum(1 for f in futs if f._error is not None))
        out[label] = summ
        log(f"[bench] serving {label}: {summ}")
    return out


def wstack_leg(idg, torch, wl, tuned, log, image_size=0.2, w_step=200.0, steps=3):
    """W-layers at scale: the workload's geometry on a wider field (S = image_size), where |w| S^2
    exceeds what a subgrid can hold.  Plans without and with layers (spacing w_step wavelengths),
    grid + degrid MVis/s of the layered plan, and the W-stacked transform of all layer grids."""
    import dataclasses
    wide = dataclasses.replace(wl, image_size=image_size)
    out = {"image_size": image_size, "w_step": w_step}
    out["unlayered"] = idg.Plan.from_workload(wide).stats()
    plan = idg.Plan.from_workload(wide, w_step=w_step)
    nsub = plan.stats()["nr_subgrids"]
    plan = idg.Plan.from_workload(wide, w_step=w_step,
                                  scratch_bytes=nsub * 4 * wide.subgrid_size ** 2 * 8 + (1 << 20))
    plan.set_tuning(**tuned)
    st = plan.stats()
    lo, nl = plan.wlayers()
    N = wide.grid_size
    dev = "cuda"
    uvw, freqs = torch.from_numpy(wide.uvw).to(dev), torch.from_numpy(wide.freqs).to(dev)
    vis, aterms = torch.from_numpy(wide.vis).to(dev), torch.from_numpy(wide.aterms).to(dev)
    taper = torch.from_numpy(wide.taper).to(dev)
    grids = torch.zeros(plan.shapes()["grid"], dtype=torch.complex64, device=dev)
    vis_out = torch.empty_like(vis)
    stream = torch.cuda.current_stream()

    def step():
        grids.zero_()
        idg.grid(plan, uvw, freqs, vis, aterms, taper, grids, stream)
        idg.degrid(plan, uvw, freqs, grids, aterms, taper, vis_out, stream)

    step()
    idg.sync(stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    img = torch.empty((4, N, N), dtype=torch.complex64, device=dev)
    w0s = plan.w_offsets()
    idg.wstack_to_image(grids, w0s, image_size, None, None, img, stream)
    e0.record(stream)
    idg.wstack_to_image(grids, w0s, image_size, None, None, img, stream)
    e1.record(stream)
    e1.synchronize()
    ti = e0.elapsed_time(e1)
    out.update(layered=st, wlayer_min=lo, nr_wlayers=nl, grid_gb=round(nl * 4 * N * N * 8 / 1e9, 2),
               ms_per_step=round(ms, 3), mvis_s=round(st["nr_gridded"] / (ms * 1e-3) / 1e6, 1),
               wstack_to_image_ms=round(ti, 3), per_layer_ms=round(ti / nl, 3))
    log(f"[bench] W-layers (S = {image_size}, w_step = {w_step}): {nl} layers, gridded {st['nr_gridded']} "
        f"(without layers {out['unlayered']['nr_gridded']}); grid+degrid {ms:.2f} ms = {out['mvis_s']} MVis/s; "
        f"W-stacked image {ti:.2f} ms ({ti / nl:.3f} ms per layer)")
    del grids, img
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lofar", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", default="auto", choices=("auto", "plain", "persistent"),
                    help="gridder/degridder schedule: autotuned (default), one workgroup per subgrid, or a "
                         "persistent work queue")
    ap.add_argument("--blocks-per-cu", type=int, default=0, help="persistent form: workgroups per CU (0 = max)")
    ap.add_argument("--degrid-shape", default="standard", choices=("standard", "wide"),
                    help="degridder task shape when --form is given (autotuned otherwise)")
    ap.add_argument("--adder-chunk", type=int, default=0, help="adder: longest tile-list run per workgroup (0 = 256)")
    ap.add_argument("--serve-jobs", type=int, default=400, help="jobs in the serving trace (0 = skip serving)")
    ap.add_argument("--no-wstack", action="store_true", help="skip the W-layer leg (wider field, layered plan)")
    ap.add_argument("--scratch-gb", type=float, default=0.0,
                    help="subgrid scratch budget in GB (0 = enough for the whole plan: one gridder launch)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="finish with a plain device copy of BYTES (reference for HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1909_07226_amd as idg
    import synth
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a HIP device")
    idg.lib()

    log(f"[bench] building workload {args.workload}")
    wl = synth.make_workload(args.workload)
    t = time.perf_counter()
    plan = idg.Plan.from_workload(wl)
    plan_ms = (time.perf_counter() - t) * 1e3
    nsub = plan.stats()["nr_subgrids"]
    scratch = int(args.scratch_gb * 1e9) if args.scratch_gb > 0 else nsub * 4 * wl.subgrid_size ** 2 * 8 + (1 << 20)
    if scratch != 2 << 30:
        # the scratch budget is a plan parameter: re-plan with it (planning time is the first plan's)
        plan = idg.Plan.from_workload(wl, scratch_bytes=scratch)
    st = plan.stats()
    nvis = st["nr_gridded"]
    L, N = wl.subgrid_size, wl.grid_size
    log(f"[bench] plan: {st} in {plan_ms:.0f} ms")
    dev = "cuda"
    uvw = torch.from_numpy(wl.uvw).to(dev)
    freqs = torch.from_numpy(wl.freqs).to(dev)
    vis = torch.from_numpy(wl.vis).to(dev)
    aterms = torch.from_numpy(wl.aterms).to(dev)
    taper = torch.from_numpy(wl.taper).to(dev)
    grid = torch.zeros((4, N, N), dtype=torch.complex64, device=dev)
    vis_out = torch.empty_like(vis)
    stream = torch.cuda.current_stream()

    def step():
        grid.zero_()
        idg.grid(plan, uvw, freqs, vis, aterms, taper, grid, stream)
        idg.degrid(plan, uvw, freqs, grid, aterms, taper, vis_out, stream)

    def timed(steps, warmup):
        for _ in range(warmup):
            step()
        idg.sync(stream)
        torch.cuda.synchronize()
        idg.profile(True)
        idg.profile_read(reset=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(stream)
        for i in range(steps):
            step()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        idg.sync(stream)
        prof = idg.profile_read(reset=True)
        idg.profile(False)
        per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
        timed.dist = dict(median=round(float(np.median(per_step)), 4),
                          p90=round(float(np.percentile(per_step, 90)), 4),
                          min=round(float(per_step.min()), 4), max=round(float(per_step.max()), 4))
        return (t1 - t0) * 1e3 / steps, prof

    tune_info = None
    if args.form == "auto":
        from paper_1909_07226_amd.autotune import autotune
        log("[bench] autotuning the schedule (outside the timed region)")
        tune_info = autotune(plan, uvw, freqs, vis, aterms, taper, grid, vis_out, use_cache=False, log=log)
    else:
        plan.set_tuning(form=args.form, blocks_per_cu=args.blocks_per_cu, degrid_shape=args.degrid_shape)
    if args.adder_chunk:
        plan.set_tuning(adder_chunk=args.adder_chunk)
    log(f"[bench] tuning {plan.get_tuning()}; warmup {args.warmup}, timing {args.steps} steps")
    ms_step, prof = timed(args.steps, args.warmup)
    step_dist = dict(timed.dist)
    value = nvis / (ms_step * 1e-3) / 1e6
    k = args.steps
    g_ms, g_n = prof["gridder"]
    a_ms, a_n = prof["adder"]
    d_ms, d_n = prof["degridder"]
    z_ms, z_n = prof["zero"]
    grid_ms = (g_ms + a_ms) / k
    degrid_ms = (d_ms + z_ms) / k
    flops_step = FLOP_PER_VIS_PIX * float(nvis) * L * L
    g_launch_ms = g_ms / max(1, g_n)
    d_launch_ms = d_ms / max(1, d_n)
    flops_launch = flops_step / max(1, g_n // k)
    achieved = flops_launch / (g_launch_ms * 1e-3) / 1e12
    d_achieved = (flops_step / max(1, d_n // k)) / (d_launch_ms * 1e-3) / 1e12
    log(f"[bench] {ms_step:.2f} ms/step, {value:.1f} MVis/s; gridder {g_launch_ms:.3f} ms/launch "
        f"({achieved:.2f} TFLOP/s), adder {a_ms / max(1, a_n):.3f} ms, degridder {d_launch_ms:.3f} ms "
        f"({d_achieved:.2f} TFLOP/s)")
    tuned = plan.get_tuning()
    plain_form = None
    if args.form == "auto":
        plan.set_tuning(form="plain", blocks_per_cu=0, adder_chunk=tuned["adder_chunk"], degrid_shape="standard")
        p_ms, _ = timed(args.steps, 1)
        plain_form = {"ms_per_step": round(p_ms, 4), "value": round(nvis / (p_ms * 1e-3) / 1e6, 3),
                      "step_ms": dict(timed.dist)}
        log(f"[bench] plain form: {plain_form}")
        plan.set_tuning(**tuned)

    result = {
        "metric": "MVis/s grid+degrid, % of FP32 VALU peak; p50/p99 job latency vs plain",
        "value": round(value, 3),
        "unit": "MVis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "step_ms": step_dist,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[args.workload], "nr_visibilities": nvis,
                   "nr_subgrids": st["nr_subgrids"], "subgrid_size": L, "grid_size": N,
                   "polarisations": 4, "phase_offsets": "f64", "taper": "PSWF beta=7",
                   "scratch_bytes": scratch,
                   "tuning": tuned},
        "roofline": {"bound": "alu", "kernel": "gridder", "achieved": round(achieved, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": gridder_traffic(args.workload, tuned["grid_form"]), "traffic_unit": "bytes/launch",
                     "kernels_sha256": kernel_source_hash(),
                     "work_per_launch": f"{FLOP_PER_VIS_PIX} flop x {nvis} vis x {L * L} pix",
                     "avg_launch_ms": round(g_launch_ms, 4)},
        "grid_mvis_s": round(nvis / (grid_ms * 1e-3) / 1e6, 3),
        "degrid_mvis_s": round(nvis / (degrid_ms * 1e-3) / 1e6, 3),
        "kernels_ms_per_step": {"gridder": round(g_ms / k, 4), "adder": round(a_ms / k, 4),
                                "degridder": round(d_ms / k, 4), "zero": round(z_ms / k, 4)},
        "degridder_roofline": {"achieved": round(d_achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(d_achieved / FP32_PEAK_TFLOPS, 4)},
        "plan_ms": round(plan_ms, 1),
        "plain_form": plain_form,
        "autotune_ms": tune_info["timings_ms"] if tune_info else None,
        "cpu_baseline": None,
    }
    result["hbm_stages"] = hbm_stages(idg, torch, plan, grid, stream, a_ms / k, log)
    if not args.no_wstack and args.workload == "lofar":
        result["wstack"] = wstack_leg(idg, torch, wl, tuned, log)
    if args.serve_jobs > 0 and args.workload == "lofar":
        result["serving"] = serving_leg(wl, dict(uvw=uvw, freqs=freqs, vis=vis, aterms=aterms, taper=taper),
                                        args.serve_jobs, log)
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, ~{args.cpu_budget:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
        log(f"[bench] cpu baseline {result['cpu_baseline']}")
    if args.copy_calibration > 0:
        # an elementwise kernel that reads BYTES and writes BYTES (torch's copy_ may use the DMA engines)
        src = torch.empty(args.copy_calibration // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {args.copy_calibration} bytes read and written")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
