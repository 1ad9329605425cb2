#!/usr/bin/env python3
"""Throughput of image-domain gridding + degridding on one MI355X.

One step = idg_grid of every planned visibility of the workload into a zeroed
4 x N x N grid, then idg_degrid of every planned visibility from that grid --
the whole hot path (plan reused, as in every major cycle of an imager).
Inputs are resident in HBM before the timed region.  Prints one JSON line:
value = planned visibilities / (wall time of grid + degrid), in MVis/s.

    python bench.py [--steps K] [--warmup W] [--workload skalow|lofar|tiny]

The headline workload is the SKA-low-like single-GPU share (the largest
configuration that fits one GPU); the LOFAR-like workload runs as a second
leg (key "lofar"), with the W-layer and serving legs on its geometry.

Roofline.  The gridder and degridder evaluate each subgrid's sums in one of
two forms (the plan reports which, per subgrid):
- the direct sum (a phasor per visibility and pixel) on the FP32 VALU; its
  work, the method's operation count, is
    34 flop per (visibility, subgrid pixel): one phase multiply-add and 16
       multiply-adds of the 4-polarisation complex accumulate (sin and cos not
       counted);
    136 flop per pixel per subgrid: the two 2 x 2 complex Jones products and
       the taper;
    5 L^2 log2(L^2) flop per polarisation per subgrid: the subgrid transform;
- the separable form (32 x 32 subgrids): per polarisation, complex products
  (32 x K)(K x 32) of row and column phasor factors on the fp16 matrix cores;
  its work is 32 flop per (visibility, pixel) for the order-0 product and
  another 32 for the first-order w cross term.
When the separable form carries most of a kernel's visibilities the kernel is
priced as a matrix-core contraction: "achieved" is the separable form's work
per launch over the launch time, against the dense fp16 peak (the fp16
high/low operand parts that give 22-bit operands execute 3x the order-0
products; "executed" reports that rate).  "direct_equivalent" divides the
method's operation count above by the same time, against the FP32 vector
peak: the rate a direct-sum kernel would need to match it.  "frac_of_measured"
divides by the rate this device sustains for that instruction kind instead
(idg_device_rates microkernels, reported under "device_rates").  Launch times come
from HIP events recorded by the library on the launching stream.  "roofline"
is for the dominant (longer) of the two kernels; both are reported.  The CPU
baseline is the float64 oracle on a bounded sample, timed on this host.
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

FLOP_PER_VIS_PIX = 34
FLOP_PER_PIX_ATERM = 136
# MI355X published FP32 vector peak: 256 CUs x 256 flop per CU-cycle x 2.4 GHz, which counts packed FMAs
# (2 per lane per instruction); the library's kernels issue unpacked FMAs only, which reach half of it
FP32_PEAK_TFLOPS = 157.3
# MI355X dense fp16 matrix-core peak (no structured sparsity)
FP16_MFMA_PEAK_TFLOPS = 2500.0
# separable form: flop per (visibility, pixel) of one complex product over 4 polarisations (8 per pol)
FLOP_PER_VIS_PIX_SEP = 32
HBM_PEAK_GBS = 8000.0               # MI355X HBM3E
WORKLOAD_DESC = {
    "skalow": "skalow-like share: 512 stations (130816 baselines), 64 x 1 s, 16 ch 50-350 MHz, L=32, "
              "8192^2 grid at 1 arcsec, A-terms every 32 timesteps, 10% flags",
    "lofar": "lofar-like: 48 stations (1128 baselines), 2048 x 1 s, 16 ch 120-180 MHz, |w| <= 2e3 lambda, "
             "L=32 subgrids of <=128 timesteps, 4096^2 grid at 2.5 arcsec, near-identity A-terms every 256 s",
    "tiny": "tiny: 8 stations (28 baselines), 32 x 10 s, 4 ch 150-151 MHz, w=0, L=24, 512^2 grid at 1 arcmin",
}
# baseline stride of the oracle's bounded sample (cpu_baseline)
CPU_SAMPLE_STRIDE = {"skalow": 32, "lofar": 16, "tiny": 1}

ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(ROOT, "paper_1909_07226_amd", "csrc", "kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def algorithmic_flops(nvis, nsub, L):
    """Flops of one direction (gridder or degridder) over nvis visibilities in nsub subgrids of L x L."""
    npix = L * L
    return (FLOP_PER_VIS_PIX * float(nvis) * npix + FLOP_PER_PIX_ATERM * float(npix) * nsub
            + 5.0 * npix * math.log2(npix) * 4 * nsub)


def separable_flops(paths, L):
    """Work of the separable form over one direction: (algorithmic, executed) flops.

    paths: plan.sum_paths(); order-0 subgrids take one complex product per
    polarisation, order-1 subgrids two.  Executed counts the three high/low
    products of the order-0 term (the order-1 term takes the high parts only).
    """
    n0, n1 = paths["separable0"][1], paths["separable1"][1]
    npix = L * L
    alg = FLOP_PER_VIS_PIX_SEP * npix * (float(n0) + 2.0 * n1)
    exe = FLOP_PER_VIS_PIX_SEP * npix * (3.0 * n0 + 4.0 * n1)
    return alg, exe


def kernel_roofline(flops_direct, paths, L, launch_ms, launches):
    """The roofline object of one kernel (gridder or degridder) from its average launch time."""
    t = launch_ms * 1e-3
    direct = flops_direct / launches / t / 1e12
    n_sep = paths["separable0"][1] + paths["separable1"][1]
    out = {"direct_equivalent": {"achieved": round(direct, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": round(direct / FP32_PEAK_TFLOPS, 4)},
           "sum_paths": paths}
    if n_sep > paths["direct"][1]:
        alg, exe = separable_flops(paths, L)
        achieved = alg / launches / t / 1e12
        out.update(bound="mfma", achieved=round(achieved, 3), peak=FP16_MFMA_PEAK_TFLOPS, unit="TFLOP/s",
                   frac=round(achieved / FP16_MFMA_PEAK_TFLOPS, 5),
                   executed={"achieved": round(exe / launches / t / 1e12, 3),
                             "frac": round(exe / launches / t / 1e12 / FP16_MFMA_PEAK_TFLOPS, 5)},
                   flop_per_launch=alg / launches,
                   work_per_launch=f"{FLOP_PER_VIS_PIX_SEP} flop x {L * L} pix x ({paths['separable0'][1]} vis "
                                   f"+ 2 x {paths['separable1'][1]} vis)"
                                   + (f", over {launches} launches" if launches > 1 else ""))
    else:
        out.update(bound="alu", achieved=round(direct, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                   frac=round(direct / FP32_PEAK_TFLOPS, 4), flop_per_launch=flops_direct / launches)
    return out


def add_measured_fracs(r, rates):
    """Fractions of the rates this device sustains (idg_device_rates) beside those of its published peaks."""
    if not rates or not r:
        return r
    fp32, mfma = rates["fp32_fma_tflops"], rates["fp16_mfma_tflops"]
    r["frac_of_measured"] = round(r["achieved"] / (mfma if r["bound"] == "mfma" else fp32), 5)
    if "executed" in r:
        r["executed"]["frac_of_measured"] = round(r["executed"]["achieved"] / mfma, 5)
    if "direct_equivalent" in r:
        de = r["direct_equivalent"]
        de["frac_of_measured"] = round(de["achieved"] / fp32, 4)
    return r


def hbm_record_path(workload):
    return os.path.join(PROFILES, f"{workload}_hbm_counters.md")


def kernel_traffic(workload, kernel, schedule, path=None):
    """HBM bytes per launch of `kernel` ("gridder" / "degridder") from the committed counter summary.

    The summary's ``traffic-record:`` lines hold FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch) of one kernel and the factors that map each counter onto the
    bytes of a plain elementwise kernel of known size.  ``schedule`` is the
    tuning string the counters were taken with.  Returns None when there is no
    record for this workload, kernel and schedule, or when the kernel source
    has changed since the counters were taken.
    """
    try:
        with open(path or hbm_record_path(workload)) as f:
            text = f.read()
    except OSError:
        return None
    for m in re.finditer(r"^traffic-record: (.*)$", text, re.M):
        rec = dict(kv.split("=", 1) for kv in m.group(1).split())
        if (rec.get("workload") == workload and rec.get("kernel") == kernel and rec.get("schedule") == schedule
                and rec.get("kernels_sha256") == kernel_source_hash()):
            return int(round(float(rec["fetch_kib"]) * 1024 * float(rec["fetch_factor"])
                             + float(rec["write_kib"]) * 1024 * float(rec["write_factor"])))
    return None


def schedule_string(tuning, kernel):
    """The part of a plan's tuning that selects `kernel`'s launch shape and sum path."""
    path = tuning.get("sum_path", "auto")
    if kernel == "gridder":
        return f"{tuning['grid_form']}/{tuning['grid_blocks_per_cu']}/{path}"
    return f"{tuning['degrid_form']}/{tuning['degrid_blocks_per_cu']}/{tuning['degrid_shape']}/{path}"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU baseline (the float64 oracle on a bounded sample of the same workload)


def host_cores():
    """(cores this process may run on, CPU model, cgroup CPU quota in cores or None)."""
    aff = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, period = f.read().split()[:2]
            if q != "max":
                quota = float(q) / float(period)
    except (OSError, ValueError):
        pass
    return aff, model, quota


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


def cpu_baseline(wl, budget_s, max_procs):
    """Time the oracle (as it stands) on a baseline subset's subgrids, within ~budget_s seconds."""
    import multiprocessing as mp
    import synth
    from oracle.plan import F, plan_workload
    aff, model, quota = host_cores()
    cores = aff if quota is None else max(1, min(aff, int(quota)))
    procs = max(1, min(cores, max_procs))
    stride = CPU_SAMPLE_STRIDE.get(wl.name, 16)
    sub_wl = synth.subset(wl, baselines=np.arange(0, wl.nr_baselines, stride))
    oplan = plan_workload(sub_wl)
    nvis = oplan.subgrids[:, F["nvis"]]
    # calibrate on a few subgrids, then pick a prefix of the subgrid list that fits the budget
    _G.update(plan=oplan, uvw=sub_wl.uvw, freqs=sub_wl.freqs, vis=sub_wl.vis, aterms=sub_wl.aterms,
              taper=sub_wl.taper, grid=np.zeros((4, wl.grid_size, wl.grid_size), np.complex64))
    t = time.perf_counter()
    ncal = min(8, oplan.nr_subgrids)
    for p in range(ncal):
        _oracle_worker((p, "grid"))
        _oracle_worker((p, "degrid"))
    per_vis = (time.perf_counter() - t) / max(1, int(nvis[:ncal].sum()))
    target = budget_s * procs / per_vis
    n = int(np.searchsorted(np.cumsum(nvis), target)) + 1
    n = max(1, min(n, oplan.nr_subgrids))
    ids = list(range(n))
    ctx = mp.get_context("fork")
    with ctx.Pool(procs) as pool:
        t0 = time.perf_counter()
        pool.map(_oracle_worker, [(p, "grid") for p in ids], chunksize=4)
        t1 = time.perf_counter()
        pool.map(_oracle_worker, [(p, "degrid") for p in ids], chunksize=4)
        t2 = time.perf_counter()
    k = int(nvis[:n].sum())
    return {"value": round(k / (t2 - t0) / 1e6, 6), "unit": "MVis/s", "cores": procs, "kind": "oracle",
            "sample": f"float64 numpy oracle, grid then degrid of the first {n} of {oplan.nr_subgrids} subgrids "
                      f"of every {stride}th baseline of the {wl.name} workload ({k} visibilities), "
                      f"{procs} worker processes",
            "cpu_model": model, "affinity_cores": aff, "cgroup_quota_cores": quota,
            "grid_s": round(t1 - t0, 3), "degrid_s": round(t2 - t1, 3)}


# ---------------------------------------------------------------------------
# HBM-bound stages


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


# passes over the [4][N][N] array of the master grid <-> image steps: one row pass, then one column
# pass (N <= 1024) or the two sub-passes of the four-step column transform (N >= 2048)
def image_passes(N):
    return 2 if N <= 1024 else 3


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
    # master grid <-> image; algorithmic bytes are one read of the input and one write of the output,
    # and every pass reads and writes the array once
    N = grid.shape[-1]
    corr = torch.ones(N, dtype=torch.float32, device="cuda")
    img = torch.empty_like(grid)
    arr = 4 * N * N * 8
    npass = image_passes(N)
    t = timed(lambda: idg.grid_to_image(grid, corr, corr, img, stream))
    out["grid_to_image"] = dict(ms=round(t, 4), bytes=2 * arr, grid_size=N, passes=npass,
                                pass_gb_s=round(2 * npass * arr / (t * 1e-3) / 1e9, 1))
    t = timed(lambda: idg.image_to_grid(img, corr, corr, grid, stream))
    out["image_to_grid"] = dict(ms=round(t, 4), bytes=2 * arr, grid_size=N, passes=npass,
                                pass_gb_s=round(2 * npass * arr / (t * 1e-3) / 1e9, 1))
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


# ---------------------------------------------------------------------------
# legs on the LOFAR-like geometry: serving and W-layers


def serving_leg(lofar_wl, lofar_dev, n_jobs, log):
    """Replay one request trace under continuous batching (4 slots; persistent and plain forms) and a
    FIFO (1 slot, plain form), at the trace's rate and saturated.  p50/p99 of completion - arrival."""
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
    # at the trace's rate, and with the arrivals compressed 50x (2500 jobs/s offered: more than the GPU
    # completes, so the queue never drains and the schedule decides the throughput)
    for rate_label, scale in (("", 1.0), ("saturated_", 0.02)):
        for label, slots, form in (("continuous", 4, "persistent"), ("continuous_plain", 4, "plain"),
                                   ("fifo_plain", 1, "plain")):
            for tp in templates.values():
                tp["plan"].set_tuning(form=form)
            with serve.Server(slots=slots, mem_budget=48 << 30, keep_results=False) as srv:
                futs = serve.replay(srv, jobs, trace["arrivals"] * scale)
            summ = serve.latency_summary(futs)
            errors = sorted({f"{type(f._error).__name__}: {f._error}"[:200] for f in futs if f._error is not None})
            summ.update(slots=slots, form=form,
                        offered_jobs_per_s=round(float(len(jobs) / (trace["arrivals"][-1] * scale)), 1),
                        failed=sum(1 for f in futs if f._error is not None), errors=errors[:3])
            out[rate_label + label] = summ
            log(f"[bench] serving {rate_label + label}: {summ}")
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


# ---------------------------------------------------------------------------
# one workload: plan, schedule, timed steps


class Leg:
    """Plan and device inputs of one workload, and the timed grid + degrid step."""

    def __init__(self, idg, torch, name, args, log):
        import synth
        self.idg, self.torch, self.name, self.log = idg, torch, name, log
        log(f"[bench] building workload {name}")
        t = time.perf_counter()
        wl = synth.make_workload(name)
        log(f"[bench] workload built in {time.perf_counter() - t:.1f} s")
        t = time.perf_counter()
        plan = idg.Plan.from_workload(wl)
        self.plan_ms = (time.perf_counter() - t) * 1e3
        nsub = plan.stats()["nr_subgrids"]
        scratch = (int(args.scratch_gb * 1e9) if args.scratch_gb > 0
                   else nsub * 4 * wl.subgrid_size ** 2 * 8 + (1 << 20))
        if scratch != 2 << 30:
            # the scratch budget is a plan parameter: re-plan with it (planning time is the first plan's)
            plan = idg.Plan.from_workload(wl, scratch_bytes=scratch)
        self.wl, self.plan, self.scratch = wl, plan, scratch
        self.st = plan.stats()
        log(f"[bench] plan: {self.st} in {self.plan_ms:.0f} ms")
        dev = "cuda"
        self.uvw = torch.from_numpy(wl.uvw).to(dev)
        self.freqs = torch.from_numpy(wl.freqs).to(dev)
        self.vis = torch.from_numpy(wl.vis).to(dev)
        self.aterms = torch.from_numpy(wl.aterms).to(dev)
        self.taper = torch.from_numpy(wl.taper).to(dev)
        N = wl.grid_size
        self.grid = torch.zeros((4, N, N), dtype=torch.complex64, device=dev)
        self.vis_out = torch.empty_like(self.vis)
        self.stream = torch.cuda.current_stream()

    def dev_inputs(self):
        return dict(uvw=self.uvw, freqs=self.freqs, vis=self.vis, aterms=self.aterms, taper=self.taper)

    def step(self):
        idg = self.idg
        self.grid.zero_()
        idg.grid(self.plan, self.uvw, self.freqs, self.vis, self.aterms, self.taper, self.grid, self.stream)
        idg.degrid(self.plan, self.uvw, self.freqs, self.grid, self.aterms, self.taper, self.vis_out, self.stream)

    def timed(self, steps, warmup):
        """(ms per step from the host clock, stage profile, per-step HIP-event distribution)."""
        idg, torch = self.idg, self.torch
        for _ in range(warmup):
            self.step()
        idg.sync(self.stream)
        torch.cuda.synchronize()
        idg.profile(True)
        idg.profile_read(reset=True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record(self.stream)
        for i in range(steps):
            self.step()
            ev[i + 1].record(self.stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        idg.sync(self.stream)
        prof = idg.profile_read(reset=True)
        idg.profile(False)
        per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
        dist = dict(median=round(float(np.median(per_step)), 4), p90=round(float(np.percentile(per_step, 90)), 4),
                    min=round(float(per_step.min()), 4), max=round(float(per_step.max()), 4))
        return (t1 - t0) * 1e3 / steps, prof, dist

    def schedule(self, args):
        """Set the plan's schedule: autotuned (args.form == "auto") or as given.  Returns autotune info."""
        plan = self.plan
        tune_info = None
        if args.tuning:
            plan.set_tuning(**json.loads(args.tuning))
        elif args.form == "auto":
            from paper_1909_07226_amd.autotune import autotune
            self.log(f"[bench] {self.name}: autotuning the schedule (outside the timed region)")
            tune_info = autotune(plan, self.uvw, self.freqs, self.vis, self.aterms, self.taper, self.grid,
                                 self.vis_out, use_cache=False, log=self.log)
        else:
            plan.set_tuning(form=args.form, blocks_per_cu=args.blocks_per_cu, degrid_shape=args.degrid_shape,
                            sum_path=args.sum_path)
        if args.adder_chunk:
            plan.set_tuning(adder_chunk=args.adder_chunk)
        return tune_info

    def measure(self, args, steps, warmup):
        """Timed steps under the current schedule, with per-kernel rooflines."""
        ms_step, prof, dist = self.timed(steps, warmup)
        nvis, nsub = self.st["nr_gridded"], self.st["nr_subgrids"]
        L = self.wl.subgrid_size
        k = steps
        flops_step = algorithmic_flops(nvis, nsub, L)
        tuned = self.plan.get_tuning()
        kernels = {}
        paths = self.plan.sum_paths()
        for kern in ("gridder", "degridder"):
            ms, n = prof[kern]
            launch_ms = ms / max(1, n)
            per_step_launches = max(1, n // k)
            r = kernel_roofline(flops_step, paths, L, launch_ms, per_step_launches)
            r.setdefault("work_per_launch",
                         f"({FLOP_PER_VIS_PIX} flop x {nvis} vis + {FLOP_PER_PIX_ATERM} flop x {nsub} subgrids) x "
                         f"{L * L} pix + 5 L^2 log2(L^2) x 4 pol x {nsub} subgrids"
                         + (f", over {per_step_launches} launches" if per_step_launches > 1 else ""))
            kernels[kern] = {"bound": r.pop("bound"), "kernel": kern, "achieved": r.pop("achieved"),
                             "peak": r.pop("peak"), "unit": r.pop("unit"), "frac": r.pop("frac"),
                             "traffic": kernel_traffic(self.name, kern, schedule_string(tuned, kern)),
                             "traffic_unit": "bytes/launch", "schedule": schedule_string(tuned, kern),
                             "kernels_sha256": kernel_source_hash(), **r,
                             "avg_launch_ms": round(launch_ms, 4), "launches_per_step": per_step_launches}
        a_ms, _ = prof["adder"]
        z_ms, _ = prof["zero"]
        g_ms = (prof["gridder"][0] + a_ms) / k
        d_ms = (prof["degridder"][0] + z_ms) / k
        dominant = max(("gridder", "degridder"), key=lambda kk: prof[kk][0])
        out = {"value": round(nvis / (ms_step * 1e-3) / 1e6, 3), "ms_per_step": round(ms_step, 4), "step_ms": dist,
               "grid_mvis_s": round(nvis / (g_ms * 1e-3) / 1e6, 3),
               "degrid_mvis_s": round(nvis / (d_ms * 1e-3) / 1e6, 3),
               "kernels_ms_per_step": {kk: round(prof[kk][0] / k, 4) for kk in ("gridder", "adder", "degridder",
                                                                                 "zero")},
               "roofline": kernels[dominant], "gridder_roofline": kernels["gridder"],
               "degridder_roofline": kernels["degridder"], "tuning": tuned}
        self.log(f"[bench] {self.name}: {ms_step:.2f} ms/step, {out['value']:.1f} MVis/s; "
                 f"gridder {kernels['gridder']['avg_launch_ms']:.3f} ms/launch ({kernels['gridder']['frac']:.1%} of "
                 f"{kernels['gridder']['bound']}), "
                 f"adder {a_ms / k:.3f} ms, degridder {kernels['degridder']['avg_launch_ms']:.3f} ms/launch "
                 f"({kernels['degridder']['frac']:.1%} of {kernels['degridder']['bound']})")
        return out

    def config(self):
        wl = self.wl
        return {"workload": WORKLOAD_DESC[self.name], "nr_visibilities": self.st["nr_gridded"],
                "nr_subgrids": self.st["nr_subgrids"], "subgrid_size": wl.subgrid_size, "grid_size": wl.grid_size,
                "polarisations": 4, "phase_offsets": "f64", "taper": "PSWF beta=7", "scratch_bytes": self.scratch,
                "tuning": self.plan.get_tuning()}

    def release(self):
        for k in ("uvw", "freqs", "vis", "aterms", "taper", "grid", "vis_out"):
            setattr(self, k, None)
        self.torch.cuda.empty_cache()


def run_leg(idg, torch, name, args, log, compare_plain=True):
    leg = Leg(idg, torch, name, args, log)
    tune_info = leg.schedule(args)
    log(f"[bench] {name}: tuning {leg.plan.get_tuning()}; warmup {args.warmup}, timing {args.steps} steps")
    res = leg.measure(args, args.steps, args.warmup)
    res["plan_ms"] = round(leg.plan_ms, 1)
    res["autotune_ms"] = tune_info["timings_ms"] if tune_info else None
    res["plain_form"] = None
    if compare_plain and args.form == "auto" and not args.tuning:
        tuned = leg.plan.get_tuning()
        # the plain form with the same degridder shape and adder chunk: only the launch form differs
        leg.plan.set_tuning(form="plain", blocks_per_cu=0, adder_chunk=tuned["adder_chunk"],
                            degrid_shape=tuned["degrid_shape"])
        p_ms, prof, dist = leg.timed(args.steps, 1)
        k = args.steps
        res["plain_form"] = {"ms_per_step": round(p_ms, 4),
                             "value": round(leg.st["nr_gridded"] / (p_ms * 1e-3) / 1e6, 3), "step_ms": dist,
                             "degrid_shape": tuned["degrid_shape"],
                             "kernels_ms_per_step": {kk: round(prof[kk][0] / k, 4) for kk in ("gridder", "adder",
                                                                                              "degridder")}}
        log(f"[bench] {name}: plain form {res['plain_form']}")
        leg.plan.set_tuning(**tuned)
    return leg, res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="skalow", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="most worker processes for the CPU baseline (the host's CPU share of one GPU)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", default="auto", choices=("auto", "plain", "persistent"),
                    help="gridder/degridder schedule: autotuned (default), one workgroup per subgrid, or a "
                         "persistent work queue")
    ap.add_argument("--blocks-per-cu", type=int, default=0, help="persistent form: workgroups per CU (0 = max)")
    ap.add_argument("--degrid-shape", default="standard", choices=("standard", "wide"),
                    help="degridder task shape when --form is given (autotuned otherwise)")
    ap.add_argument("--tuning", default="", metavar="JSON",
                    help="the plan's whole schedule as idg Plan.get_tuning() returns it (overrides --form)")
    ap.add_argument("--sum-path", default="auto", choices=("auto", "direct"),
                    help="with --form plain/persistent: separable form where it applies, or the direct sum")
    ap.add_argument("--adder-chunk", type=int, default=0, help="adder: longest tile-list run per workgroup (0 = 256)")
    ap.add_argument("--no-lofar", action="store_true",
                    help="skip the LOFAR-like leg (and the W-layer and serving legs on its geometry)")
    ap.add_argument("--serve-jobs", type=int, default=400, help="jobs in the serving trace (0 = skip serving)")
    ap.add_argument("--no-wstack", action="store_true", help="skip the W-layer leg (wider field, layered plan)")
    ap.add_argument("--no-device-rates", action="store_true",
                    help="skip the device-rate microbenchmarks (idg_device_rates)")
    ap.add_argument("--no-hbm-stages", action="store_true", help="skip the standalone HBM-bound stage timings")
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
    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a HIP device")
    idg.lib()
    rates = None
    if not args.no_device_rates:
        rates = {k: round(v, 2) for k, v in idg.device_rates().items()}
        log(f"[bench] device rates: {rates}")

    leg, res = run_leg(idg, torch, args.workload, args, log)
    for key in ("roofline", "gridder_roofline", "degridder_roofline"):
        add_measured_fracs(res[key], rates)
    result = {
        "metric": "MVis/s grid+degrid, % of FP32 VALU peak; p50/p99 job latency vs plain",
        "value": res["value"],
        "unit": "MVis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "step_ms": res["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": leg.config(),
        "roofline": res["roofline"],
        "cpu_baseline": None,
        "device_rates": rates,
    }
    for key in ("gridder_roofline", "degridder_roofline", "grid_mvis_s", "degrid_mvis_s", "kernels_ms_per_step",
                "plan_ms", "plain_form", "autotune_ms"):
        result[key] = res[key]
    if not args.no_hbm_stages:
        result["hbm_stages"] = hbm_stages(idg, torch, leg.plan, leg.grid, leg.stream,
                                          res["kernels_ms_per_step"]["adder"], log)
    head_wl = leg.wl
    lleg = None
    if args.workload == "lofar":
        lleg = leg
    else:
        leg.release()
        idg.trim_scratch()
        if not args.no_lofar:
            lleg, lres = run_leg(idg, torch, "lofar", args, log)
            lres["config"] = lleg.config()
            for key in ("roofline", "gridder_roofline", "degridder_roofline"):
                add_measured_fracs(lres[key], rates)
            result["lofar"] = lres
    if lleg is not None:
        if not args.no_wstack:
            result["wstack"] = wstack_leg(idg, torch, lleg.wl, lleg.plan.get_tuning(), log)
        if args.serve_jobs > 0:
            idg.trim_scratch()
            result["serving"] = serving_leg(lleg.wl, lleg.dev_inputs(), args.serve_jobs, log)
        lleg.release()
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, ~{args.cpu_budget:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(head_wl, args.cpu_budget, args.cpu_procs)
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
