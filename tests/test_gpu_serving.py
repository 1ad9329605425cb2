"""Serving loop on the GPU: invariance of results in the mix, admission and failure isolation."""

import numpy as np
import pytest

import synth
from tests.gpu_common import require_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    require_gpu()
    import torch
    import paper_1909_07226_amd as idg
    from paper_1909_07226_amd import serve
    tiny = synth.make_workload("tiny", nt=256, nch=16)
    full = synth.make_workload("lofar")
    lofar = synth.subset(full, baselines=np.arange(0, full.nr_baselines, 8), nt=512)
    dev = "cuda"

    def to_dev(wl):
        return dict(uvw=torch.from_numpy(wl.uvw).to(dev), freqs=torch.from_numpy(wl.freqs).to(dev),
                    vis=torch.from_numpy(wl.vis).to(dev), aterms=torch.from_numpy(wl.aterms).to(dev),
                    taper=torch.from_numpy(wl.taper).to(dev))

    g = torch.Generator(device=dev).manual_seed(3)
    grids = {c: torch.complex(torch.randn((4, n, n), generator=g, device=dev),
                              torch.randn((4, n, n), generator=g, device=dev)).to(torch.complex64)
             for c, n in (("tiny", tiny.grid_size), ("lofar", lofar.grid_size))}
    trace = synth.serving_trace(n_jobs=24, rate=400.0, n_windows=4,
                                sizes={"tiny": (256, 16, 256), "lofar": (512, 16, 256)})
    jobs, templates = serve.jobs_from_trace(trace, {"tiny": tiny, "lofar": lofar},
                                            {"tiny": to_dev(tiny), "lofar": to_dev(lofar)}, grids,
                                            scratch_bytes=64 << 20)
    return torch, idg, serve, trace, jobs, templates


def test_results_alone_equal_results_in_the_mix(env):
    torch, idg, serve, trace, jobs, templates = env
    say(f"[serving invariance] {len(jobs)} jobs")
    for tp in templates.values():
        tp["plan"].set_tuning(form="persistent")
    with serve.Server(slots=4, mem_budget=16 << 30) as srv:
        futs = serve.replay(srv, jobs, trace["arrivals"])
    mixed = [f.result() for f in futs]
    assert all(f.latency is not None and f.latency > 0 for f in futs)
    summ = serve.latency_summary(futs)
    assert summ["jobs"] == len(jobs) and summ["p99_ms"] >= summ["p50_ms"] > 0
    for tp in templates.values():
        tp["plan"].set_tuning(form="plain")
    for job, res in zip(jobs, mixed):
        alone = job.launch(torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert torch.equal(alone, res), job.name


def test_admission_refuses_oversized_job_and_isolates_failures(env):
    torch, idg, serve, trace, jobs, templates = env
    say("[serving admission]")
    small = [j for j in jobs if j.plan.grid_size == 512][:3]
    big = next(j for j in jobs if j.plan.grid_size == 4096 and j.kind == "grid")   # 512 MiB grid + scratch
    budget = max(j.mem_bytes for j in small) + 1
    assert big.mem_bytes > budget
    # a job whose visibilities have the wrong dtype fails inside its launch
    j0 = small[0]
    broken = serve.Job("grid", j0.plan, j0.uvw, j0.freqs, j0.aterms, j0.taper,
                       vis=torch.zeros(tuple(j0.plan.shapes()["vis"]), dtype=torch.complex128, device="cuda"))
    with serve.Server(slots=2, mem_budget=budget) as srv:
        futs = [srv.submit(small[0]), srv.submit(big), srv.submit(broken), srv.submit(small[1]),
                srv.submit(small[2])]
        for f in futs:
            f._done.wait(120)
    with pytest.raises(MemoryError):
        futs[1].result()
    with pytest.raises(TypeError):
        futs[2].result()
    for f in (futs[0], futs[3], futs[4]):
        assert f.result() is not None


def _digest(torch, out):
    """Bitwise digest of a complex64 tensor: weighted int64 sums of its 8-byte words (mod 2^64)."""
    x = out.reshape(-1).view(torch.int64)
    n = x.numel()
    m = n - n % 64
    w = torch.tensor([(0x9E3779B97F4A7C15 * (i + 1)) % (1 << 61) + 1 for i in range(64)], dtype=torch.int64,
                     device=x.device)
    a = x[:m].view(-1, 64)
    rows = a.sum(1)
    idx = torch.arange(rows.numel(), dtype=torch.int64, device=x.device) * 2654435761 + 1
    return torch.stack([(a * w).sum(), (rows * idx).sum(), (x[m:] * w[:n - m]).sum()])


class _DigestJob:
    """A serving job whose output is replaced by its digest on the job's own stream."""

    def __init__(self, torch, job):
        self.__dict__.update(job.__dict__)
        self._torch, self._job = torch, job

    def launch(self, stream):
        out = self._job.launch(stream)
        with self._torch.cuda.stream(stream):
            return _digest(self._torch, out)


def test_full_trace_results_alone_equal_results_in_the_mix():
    # the serving benchmark's 400-job trace (8-station and LOFAR-like classes, full datasets), replayed with
    # 4 slots in the persistent form; every job's output must equal, bit for bit, that of the job run alone
    require_gpu()
    import torch
    from paper_1909_07226_amd import serve
    tiny = synth.make_workload("tiny", nt=2048, nch=16)
    lofar = synth.make_workload("lofar")
    dev = "cuda"

    def to_dev(wl):
        return dict(uvw=torch.from_numpy(wl.uvw).to(dev), freqs=torch.from_numpy(wl.freqs).to(dev),
                    vis=torch.from_numpy(wl.vis).to(dev), aterms=torch.from_numpy(wl.aterms).to(dev),
                    taper=torch.from_numpy(wl.taper).to(dev))

    g = torch.Generator(device=dev).manual_seed(11)
    grids = {c: torch.complex(torch.randn((4, n, n), generator=g, device=dev),
                              torch.randn((4, n, n), generator=g, device=dev)).to(torch.complex64)
             for c, n in (("tiny", tiny.grid_size), ("lofar", lofar.grid_size))}
    trace = synth.serving_trace(n_jobs=400)
    jobs, templates = serve.jobs_from_trace(trace, {"tiny": tiny, "lofar": lofar},
                                            {"tiny": to_dev(tiny), "lofar": to_dev(lofar)}, grids)
    say(f"[serving invariance, full trace] {len(jobs)} jobs, {len(templates)} plans")
    djobs = [_DigestJob(torch, j) for j in jobs]
    for tp in templates.values():
        tp["plan"].set_tuning(form="persistent")
    with serve.Server(slots=4, mem_budget=48 << 30) as srv:
        futs = serve.replay(srv, djobs, trace["arrivals"] * 0.05)     # 20x the trace's rate: jobs overlap
    mixed = [f.result().cpu() for f in futs]
    summ = serve.latency_summary(futs)
    say(f"    mix: {summ}")
    assert summ["jobs"] == len(jobs)
    for tp in templates.values():
        tp["plan"].set_tuning(form="plain")
    stream = torch.cuda.current_stream()
    for job, dj, res in zip(jobs, djobs, mixed):
        alone = dj.launch(stream).cpu()
        assert torch.equal(alone, res), job.name
