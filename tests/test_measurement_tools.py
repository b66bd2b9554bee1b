"""CPU checks of the measurement tooling: the rocprofv3 summaries (on a small synthetic
results database with the tables rocprofv3 writes) and the benchmark's use of the
committed HBM-traffic record."""
import json
import sqlite3

import pytest

import bench
from paper_1410_3677_amd import rocprof_summary as rs


def _db(path, kernels, counters):
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, start integer, duration integer)")
    c.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
              "value real)")
    c.executemany("insert into kernels values (?, ?, ?)", kernels)
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", counters)
    c.commit()
    c.close()
    return str(path)


def test_trace_statistics_and_last_dispatches(tmp_path):
    ka = "void fstat::(anonymous namespace)::k_tmpl_a_pair<float, 512, 3>(fstat::TmplArgs)"
    kb = "void fstat::k_tmpl_b_stream<float, 512, 0, true>(fstat::TmplArgs)"
    db = _db(tmp_path / "t.db", [(ka, 0, 1000), (kb, 10, 3000), (ka, 20, 2000), (ka, 30, 3000)], [])
    out = rs.trace(db)
    assert "| `k_tmpl_a_pair<float, 512, 3>` | 3 | 6.0 | 2.00 | 1.00 | 3.00 |" in out
    assert "| `k_tmpl_b_stream<float, 512, 0, true>` | 1 | 3.0 | 3.00 | 3.00 | 3.00 |" in out
    last = rs.trace(db, match="k_tmpl_a", last=2)
    assert "| `k_tmpl_a_pair<float, 512, 3>` | 2 | 5.0 | 2.50 | 2.00 | 3.00 |" in last
    assert "k_tmpl_b" not in last


def test_traffic_scaling_by_the_copy_kernel(tmp_path):
    copy = "void at::native::MulFunctor<float>(...)"
    ka = "void fstat::k_tmpl_a_pair<float, 512, 3>(fstat::TmplArgs)"
    # the copy moves 1 MiB each way; FETCH_SIZE reads half of it (per instance sums)
    f = _db(tmp_path / "f.db", [], [(1, copy, "FETCH_SIZE", 256.0), (1, copy, "FETCH_SIZE", 256.0),
                                    (2, ka, "FETCH_SIZE", 10.0), (3, ka, "FETCH_SIZE", 30.0)])
    w = _db(tmp_path / "w.db", [], [(1, copy, "WRITE_SIZE", 1024.0), (2, ka, "WRITE_SIZE", 2048.0),
                                    (3, ka, "WRITE_SIZE", 2048.0)])
    res = rs.traffic(f, w, 1 << 20, "MulFunctor", 512)
    assert res["fetch_scale"] == pytest.approx(2.0) and res["write_scale"] == pytest.approx(1.0)
    k = res["kernels"]["template_a"]
    assert k["fetch_kib_raw"] == pytest.approx(20.0) and k["write_kib_raw"] == pytest.approx(2048.0)
    assert k["bytes_per_launch"] == pytest.approx(20.0 * 1024 * 2 + 2048.0 * 1024)
    assert k["templates_per_launch"] == 512


def test_counter_table(tmp_path):
    ka = "void fstat::k_tmpl_a_pair<float, 512, 3>(fstat::TmplArgs)"
    db = _db(tmp_path / "c.db", [], [(1, ka, "SQ_INSTS_VALU_FMA_F32", 3.0), (1, ka, "SQ_INSTS_VALU_FMA_F32", 5.0),
                                     (2, ka, "SQ_INSTS_VALU_FMA_F32", 4.0), (1, ka, "SQ_INSTS_VALU_ADD_F32", 1.0),
                                     (2, ka, "SQ_INSTS_VALU_ADD_F32", 3.0)])
    out = rs.counters(db)
    assert "| kernel | dispatches | SQ_INSTS_VALU_ADD_F32 | SQ_INSTS_VALU_FMA_F32 |" in out
    assert "| `k_tmpl_a_pair<float, 512, 3>` | 2 | 2 | 6 |" in out


def test_traffic_record_is_used_only_for_the_current_sources():
    with open(bench.os.path.join(bench.ROOT, "profiles", "template_kernels_traffic.txt")) as fh:
        rec = json.load(fh)
    if rec["source_sha256"] != bench.source_digest():
        assert bench.measured_traffic("template_a", 512, rec["variants"]) is None
        pytest.skip("kernel sources changed since the counters were taken: the bench reports traffic null")
    v = rec["variants"]
    got = bench.measured_traffic("template_a", 512, v)
    assert got == rec["kernels"]["template_a"]["bytes_per_launch"]
    # within 1% of the algorithmic bytes: 512 templates x 2 x 2^18 x 8 B + the resampled series
    algo = 512 * 2 * (1 << 18) * 8 + 2 * 86164 * 8
    assert abs(got - algo) / algo < 0.01
    assert bench.measured_traffic("template_a", 256, v) is None
    assert bench.measured_traffic("template_a", 512, v ^ 1) is None
    assert bench.measured_traffic("no_such_kernel", 512, v) is None
