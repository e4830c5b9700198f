"""Host-side measurement tools (no GPU): the kernel-busy fraction and the
counter table read rocprofv3 databases; synthetic databases with known
dispatch intervals and counter values check their arithmetic."""
from __future__ import annotations

import sqlite3
import sys

import pytest

from paper_2607_20650_amd import counter_table, profile_summary


def _db(path, kernels=(), counters=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    con.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    con.executemany("insert into kernels values (?, ?, ?)", kernels)
    con.executemany("insert into counters_collection values (?, ?, ?)", counters)
    con.commit()
    con.close()
    return str(path)


def test_busy_fraction_is_the_union_of_intervals_over_the_span(tmp_path):
    db = _db(tmp_path / "t.db", kernels=[
        ("void k_batched<0, float>", 0, 10), ("void k_batched<0, float>", 2, 5),
        ("other", 10, 20), ("void k_batched<0, float>", 20, 30)])
    frac, span_s, n = profile_summary.busy_fraction(db, "k_batched")
    assert frac == pytest.approx(20 / 30) and span_s == pytest.approx(30e-9) and n == 3


def test_busy_fraction_span_ends_at_the_latest_end(tmp_path):
    # the last dispatch to start ends first: the span still runs to 100
    db = _db(tmp_path / "t.db", kernels=[("k_batched", 0, 100), ("k_batched", 10, 20)])
    frac, span_s, n = profile_summary.busy_fraction(db, "k_batched")
    assert frac == 1.0 and span_s == pytest.approx(100e-9) and n == 2


def _counters(name, waves, per_dispatch, hit, miss):
    rows = []
    for d in range(3):  # three dispatches; the middle value is the median
        scale = (0.9, 1.0, 1.2)[d]
        rows += [(name, "SQ_WAVES", waves), (name, "TCC_HIT_sum", hit * scale), (name, "TCC_MISS_sum", miss * scale)]
        rows += [(name, c, v * scale) for c, v in per_dispatch.items()]
    return rows


def test_counter_table_per_64_nodes_and_two_kernel_mean(tmp_path, monkeypatch):
    nodes = 4096 * 64
    ins = {"SQ_INSTS_VALU": 150 * 4096, "SQ_INSTS_SALU": 50 * 4096, "SQ_INSTS_LDS": 0.0,
           "SQ_INSTS_VMEM_RD": 10 * 4096, "SQ_INSTS_VMEM_WR": 9 * 4096}
    odd = dict(ins, SQ_INSTS_VALU=250 * 4096)
    # a kernel whose wavefront updates 16 x 64 nodes: 256 wavefronts for the same nodes
    marched = {k: 2 * v for k, v in ins.items()}
    db = _db(tmp_path / "c.db", counters=_counters("void k_aa_even<0, float>", 4096, ins, 3e6, 1e6)
             + _counters("void k_aa_odd<0, float>", 4096, odd, 3e6, 1e6)
             + _counters("void k3_pull_aos_z<float>", 256, marched, 1e6, 1e6))
    out = tmp_path / "table.md"
    monkeypatch.setattr(sys, "argv", ["counter_table", "--out", str(out),
                                      "--entry", f"AA|{db}|k_aa_even+k_aa_odd|{nodes}",
                                      "--entry", f"march|{db}|k3_pull_aos_z|{nodes}"])
    counter_table.main()
    rows = {l.split("|")[1].strip(): [c.strip() for c in l.split("|")[2:-1]]
            for l in out.read_text().splitlines() if l.startswith("| AA") or l.startswith("| march")}
    # hit 75%, 4096 waves of 64 nodes; VALU the mean of 150 and 250 per 64 nodes
    assert rows["AA"] == ["75.0%", "4096", "64", "200", "50", "0.0", "10.0", "9.0"]
    # 256 waves of 1024 nodes; counts per 64 nodes, not per wavefront
    assert rows["march"] == ["50.0%", "256", "1024", "300", "100", "0.0", "20.0", "18.0"]
