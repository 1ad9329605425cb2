"""Host-side logic of bench.py (no GPU): the traffic record, the flop count and the touched-tile count."""

import math
import os

import numpy as np

import bench
import paper_1909_07226_amd as idg
from paper_1909_07226_amd._lib import SUBGRID_FIELDS
from tests.util import random_track_workload


def test_touched_tile_count_matches_brute_force():
    wl = random_track_workload(seed=31, N=128, L=16, beta=3, nbl=5, nt=40, nch=3)
    plan = idg.Plan.from_workload(wl)
    sub, _ = plan.export()
    F = {n: i for i, n in enumerate(SUBGRID_FIELDS)}
    L = plan.subgrid_size
    for tile in (8, 16, 32):
        tiles = set()
        for x0, y0 in zip(sub[:, F["x0"]], sub[:, F["y0"]]):
            for y in range(y0, y0 + L):
                for x in range(x0, x0 + L):
                    tiles.add((y // tile, x // tile))
        assert bench.touched_tile_count(plan, tile=tile) == len(tiles)


def test_algorithmic_flops_terms():
    # 34 flop per visibility x pixel, 136 per pixel per subgrid, 5 L^2 log2 L^2 per polarisation per subgrid
    assert bench.algorithmic_flops(10, 0, 32) == 34 * 10 * 1024
    assert bench.algorithmic_flops(0, 3, 32) == 3 * (136 * 1024 + 5 * 1024 * 10 * 4)
    assert math.isclose(bench.algorithmic_flops(0, 1, 24), 136 * 576 + 5 * 576 * math.log2(576) * 4)
    # the SKA-low-like share: 120,570,964 visibilities in 1,965,283 subgrids of 32 x 32
    assert math.isclose(bench.algorithmic_flops(120570964, 1965283, 32), 4.874e12, rel_tol=1e-3)


def test_traffic_record_requires_matching_kernel_source(tmp_path, monkeypatch):
    record = ("traffic-record: workload=skalow kernel=degridder schedule=persistent/0/standard fetch_kib=1000 "
              "write_kib=500 fetch_factor=2.0 write_factor=1.0 kernels_sha256={h}\n")
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    h = bench.kernel_source_hash()
    rec = tmp_path / "record.md"
    rec.write_text("# summary\n\n" + record.format(h=h))
    p = str(rec)
    assert bench.kernel_traffic("skalow", "degridder", "persistent/0/standard", p) == (1000 * 2 + 500) * 1024
    assert bench.kernel_traffic("skalow", "degridder", "plain/0/standard", p) is None    # other schedule
    assert bench.kernel_traffic("skalow", "gridder", "persistent/0/standard", p) is None  # other kernel
    assert bench.kernel_traffic("lofar", "degridder", "persistent/0/standard", p) is None  # other workload
    src.write_text("// kernel source, changed\n")                                       # counters are stale now
    assert bench.kernel_traffic("skalow", "degridder", "persistent/0/standard", p) is None
    os.remove(rec)
    assert bench.kernel_traffic("skalow", "degridder", "persistent/0/standard", p) is None  # no summary at all


def test_schedule_string():
    t = dict(grid_form="persistent", degrid_form="plain", grid_blocks_per_cu=0, degrid_blocks_per_cu=2,
             adder_chunk=64, degrid_shape="wide")
    assert bench.schedule_string(t, "gridder") == "persistent/0/auto"
    assert bench.schedule_string(t, "degridder") == "plain/2/wide/auto"
    t["sum_path"] = "direct"
    assert bench.schedule_string(t, "gridder") == "persistent/0/direct"


def test_kernel_roofline_prices_the_separable_form_on_the_matrix_cores():
    L = 32
    # all visibilities in the separable form, half of them with the first-order term
    paths = {"separable0": (10, 1000), "separable1": (10, 1000), "direct": (0, 0)}
    alg, exe = bench.separable_flops(paths, L)
    assert alg == 32 * 1024 * (1000 + 2 * 1000)
    assert exe == 32 * 1024 * (3 * 1000 + 4 * 1000)
    r = bench.kernel_roofline(1e12, paths, L, launch_ms=2.0, launches=1)
    assert r["bound"] == "mfma" and r["peak"] == bench.FP16_MFMA_PEAK_TFLOPS
    assert abs(r["achieved"] - round(alg / 2e-3 / 1e12, 3)) < 1e-9
    assert r["direct_equivalent"]["achieved"] == 500.0       # 1e12 flop in 2 ms
    assert r["direct_equivalent"]["peak"] == bench.FP32_PEAK_TFLOPS
    # mostly direct sums: the FP32 vector roofline
    paths = {"separable0": (1, 10), "separable1": (0, 0), "direct": (10, 1000)}
    r = bench.kernel_roofline(1e12, paths, L, launch_ms=10.0, launches=2)
    assert r["bound"] == "alu" and r["achieved"] == 50.0 and r["frac"] == round(50.0 / 157.3, 4)


def test_committed_traffic_records_are_parseable():
    # every committed counter summary holds well-formed records (their hashes may or may not match the source)
    for name in sorted(os.listdir(bench.PROFILES)):
        if not name.endswith("_hbm_counters.md"):
            continue
        with open(os.path.join(bench.PROFILES, name)) as f:
            lines = [ln for ln in f if ln.startswith("traffic-record:")]
        for ln in lines:
            fields = dict(kv.split("=", 1) for kv in ln.split()[1:])
            for key in ("workload", "kernel", "schedule", "fetch_kib", "write_kib", "fetch_factor", "write_factor",
                        "kernels_sha256"):
                assert key in fields, (name, key)
            assert np.isfinite(float(fields["fetch_kib"])) and float(fields["fetch_factor"]) > 0


def test_host_cores_reports_affinity_and_model():
    aff, model, quota = bench.host_cores()
    assert aff == len(os.sched_getaffinity(0)) and aff >= 1
    assert isinstance(model, str) and model
    assert quota is None or quota > 0


def test_image_passes():
    assert bench.image_passes(512) == 2 and bench.image_passes(1024) == 2
    assert bench.image_passes(2048) == 3 and bench.image_passes(8192) == 3


def test_measured_fractions():
    rates = {"fp32_fma_tflops": 125.0, "sincos_ginstr_per_s": 280.0, "fp16_mfma_tflops": 2000.0}
    paths = {"separable0": (10, 1000), "separable1": (10, 1000), "direct": (0, 0)}
    r = bench.kernel_roofline(1e12, paths, 32, launch_ms=2.0, launches=1)
    bench.add_measured_fracs(r, rates)
    assert r["frac_of_measured"] == round(r["achieved"] / 2000.0, 5)
    assert r["executed"]["frac_of_measured"] == round(r["executed"]["achieved"] / 2000.0, 5)
    assert r["direct_equivalent"]["frac_of_measured"] == round(500.0 / 125.0, 4)
    assert bench.add_measured_fracs(dict(r), None) == r      # no rates: unchanged
