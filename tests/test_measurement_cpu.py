"""Host logic of the measurement (no GPU, no profiler): the HBM-traffic
counter scaling against the calibration copy, the guard that drops a
recorded traffic figure once the kernels' sources have changed, and the
benchmark's refusal of more than one GPU."""
import json

import pytest

from paper_1607_05707_amd import profiling


def _rows(counter, copy_kib, kernel_kib):
    rows = [(profiling.COPY_KERNEL, copy_kib / 4.0),    # a small copy
            (profiling.COPY_KERNEL, copy_kib),          # the calibration copy
            ("void irgl::init_kernel(irgl::Params, int)", 99.0)]
    rows += [("void irgl::persistent_kernel<512, irgl::SsspOp>(irgl::Params)", v) for v in kernel_kib]
    rows += [("void irgl::persistent_kernel<1024, irgl::BfsOp>(irgl::Params)", 1.0)]
    return rows


def test_traffic_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    # a 1024 MiB copy that FETCH_SIZE reads as 512 MiB (factor 2) and
    # WRITE_SIZE as 1024 MiB (factor 1)
    tables = {("f.db", "FETCH_SIZE"): _rows("FETCH_SIZE", 512 * 1024.0, [1000.0, 3000.0]),
              ("w.db", "WRITE_SIZE"): _rows("WRITE_SIZE", 1024 * 1024.0, [500.0, 700.0])}
    monkeypatch.setattr(profiling, "counter_rows", lambda db, counter: tables[(db, counter)])
    out = tmp_path / "t.json"
    rc = profiling.main(["traffic", "--fetch-db", "f.db", "--write-db", "w.db", "--calib-mb", "1024",
                         "--kernel", "persistent_kernel<512, irgl::SsspOp>", "--workload", "w",
                         "--command", "c", "--out", str(out)])
    assert rc == 0
    rec = json.loads(out.read_text())
    assert rec["fetch"]["dispatches"] == 2 and rec["fetch"]["factor"] == pytest.approx(2.0)
    assert rec["write"]["factor"] == pytest.approx(1.0)
    assert rec["fetch"]["bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert rec["write"]["bytes_per_launch"] == pytest.approx(600.0 * 1024)
    assert rec["traffic_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0 + 600.0 * 1024)
    assert rec["source_digest"] == profiling.source_digest()
    # the record is current, so the bench may use it
    assert profiling.load_traffic(str(out))["kernel"] == "persistent_kernel<512, irgl::SsspOp>"


def test_stale_or_missing_records_are_dropped(tmp_path):
    assert profiling.load_traffic(str(tmp_path / "missing.json")) is None
    bad = tmp_path / "bad.json"
    bad.write_text("{not json")
    assert profiling.load_traffic(str(bad)) is None
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"kernel": "k", "traffic_bytes_per_launch": 1, "source_digest": "0" * 64}))
    assert profiling.load_traffic(str(stale)) is None


def test_digest_covers_every_kernel_source():
    names = {p.rsplit("/", 1)[-1] for p in profiling.digest_files()}
    assert "irgl.hip" in names
    for h in ("irgl_device.h", "irgl_ops.h", "irgl_expand.h", "irgl_query.h", "irgl_batch.h", "irgl_topo.h"):
        assert h in names


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: the refusal comes before anything touches a device
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
