"""The benchmark's measurement arithmetic (CPU): the algorithmic-byte and
touched-byte counts, the counter summaries' parsing and their gating on the
query kernel's source hash, and the committed summaries' fields."""
from __future__ import annotations

import os

import bench


def test_b_alg_counts_each_term():
    # q and answer 32, 16 per candidate, list range 8, 4 per entry, 36 per
    # tested edge, 52 per tested face
    assert bench.b_alg(0, 0, 0, 0) == 12 + 20 + 8
    assert bench.b_alg(1, 0, 0, 0) - bench.b_alg(0, 0, 0, 0) == 16
    assert bench.b_alg(0, 1, 0, 0) - bench.b_alg(0, 0, 0, 0) == 4
    assert bench.b_alg(0, 0, 1, 0) - bench.b_alg(0, 0, 0, 0) == 36
    assert bench.b_alg(0, 0, 0, 1) - bench.b_alg(0, 0, 0, 0) == 52
    # the headline workload's per-query counts
    # 40 + 16 * 26.02 + 4 * 42.84 + 36 * 5.17 + 52 * 5.15
    assert abs(bench.b_alg(26.02, 42.84, 5.17, 5.15) - 1081.60) < 0.01


def test_touched_bytes_exceed_algorithmic():
    # the layout reads more than the method's minimum: entry boxes, forms, list head
    for args in ((26.0, 1.55, 42.8, 5.2, 5.2), (16.6, 1.07, 37.1, 4.5, 4.5)):
        v, st, e, fe, ff = args
        assert bench.touched_bytes(v, st, e, fe, ff) > bench.b_alg(v, e, fe, ff)


def test_summary_gated_on_source_hash(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text("# comment: ignored\n"
                    f"kernel_source_hash: {bench.kernel_source_hash()}\nqueries: 10000000\nl2_hit_rate: 0.5\n")
    vals = bench._summary(str(good), 10_000_000)
    assert vals is not None and float(vals["l2_hit_rate"]) == 0.5
    assert bench._summary(str(good), 1_000_000) is None            # another batch size
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_source_hash: 0000000000000000\nqueries: 10000000\n")
    assert bench._summary(str(stale), 10_000_000) is None           # another kernel source
    assert bench._summary(str(tmp_path / "missing.txt"), 10_000_000) is None


def test_committed_summaries_hold_the_fields_the_bench_reads():
    for path, keys in ((bench.TRAFFIC_FILE, ("hbm_bytes_per_launch", "hbm_read_bytes_per_launch",
                                             "hbm_write_bytes_per_launch", "l2_hit_rate")),
                       (bench.SQ_FILE, ("valu_issue_frac", "lanes_active_frac", "valu_insts_per_wave"))):
        assert os.path.exists(path), path
        vals = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        assert len(vals["kernel_source_hash"]) == 16 and int(vals["queries"]) == 10_000_000
        for k in keys:
            float(vals[k])
