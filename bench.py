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
import json
import os
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="lofar", choices=sorted(WORKLOAD_DESC))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)", file=sys.stderr)
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

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    idg.sync(stream)
    torch.cuda.synchronize()
    idg.profile(True)
    idg.profile_read(reset=True)
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    idg.sync(stream)
    prof = idg.profile_read(reset=True)
    idg.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
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

    result = {
        "metric": "MVis/s grid+degrid, % of FP32 VALU peak; p50/p99 job latency vs plain",
        "value": round(value, 3),
        "unit": "MVis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC[args.workload], "nr_visibilities": nvis,
                   "nr_subgrids": st["nr_subgrids"], "subgrid_size": L, "grid_size": N,
                   "polarisations": 4, "phase_offsets": "f64", "taper": "PSWF beta=7"},
        "roofline": {"bound": "alu", "kernel": "gridder", "achieved": round(achieved, 3),
                     "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": None, "work_per_launch": f"{FLOP_PER_VIS_PIX} flop x {nvis} vis x {L * L} pix",
                     "avg_launch_ms": round(g_launch_ms, 4)},
        "grid_mvis_s": round(nvis / (grid_ms * 1e-3) / 1e6, 3),
        "degrid_mvis_s": round(nvis / (degrid_ms * 1e-3) / 1e6, 3),
        "kernels_ms_per_step": {"gridder": round(g_ms / k, 4), "adder": round(a_ms / k, 4),
                                "degridder": round(d_ms / k, 4), "zero": round(z_ms / k, 4)},
        "degridder_roofline": {"achieved": round(d_achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": round(d_achieved / FP32_PEAK_TFLOPS, 4)},
        "plan_ms": round(plan_ms, 1),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline (oracle, ~{args.cpu_budget:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
        log(f"[bench] cpu baseline {result['cpu_baseline']}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
