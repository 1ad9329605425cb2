"""Host-side logic of bench.py (no GPU): the traffic record and the touched-tile count."""

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


def test_traffic_record_requires_matching_kernel_source(tmp_path, monkeypatch):
    record = ("traffic-record: workload=lofar form=persistent kernel=k fetch_kib=1000 write_kib=500 "
              "fetch_factor=2.0 write_factor=1.0 kernels_sha256={h}\n")
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    h = bench.kernel_source_hash()
    rec = tmp_path / "record.md"
    monkeypatch.setattr(bench, "HBM_RECORD", str(rec))
    rec.write_text("# summary\n\n" + record.format(h=h))
    assert bench.gridder_traffic("lofar", "persistent") == (1000 * 2 + 500) * 1024
    assert bench.gridder_traffic("lofar", "plain") is None            # other schedule
    assert bench.gridder_traffic("skalow", "persistent") is None      # other workload
    src.write_text("// kernel source, changed\n")                      # counters are stale now
    assert bench.gridder_traffic("lofar", "persistent") is None
    os.remove(rec)
    assert bench.gridder_traffic("lofar", "persistent") is None      # no summary at all


def test_committed_traffic_record_is_parseable():
    # the committed summary holds one well-formed record (its hash may or may not match the source)
    with open(bench.HBM_RECORD) as f:
        lines = [ln for ln in f if ln.startswith("traffic-record:")]
    assert len(lines) == 1
    fields = dict(kv.split("=", 1) for kv in lines[0].split()[1:])
    for key in ("workload", "form", "fetch_kib", "write_kib", "fetch_factor", "write_factor", "kernels_sha256"):
        assert key in fields
    assert np.isfinite(float(fields["fetch_kib"])) and float(fields["fetch_factor"]) > 0
