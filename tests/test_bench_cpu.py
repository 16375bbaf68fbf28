"""CPU checks of bench.py's host-side pieces: the oracle baseline's two modes
(all threads over a few systems with the recycle space carried, one thread on
the first system) on a small sequence, and the source digest that gates the
profile-derived constants.  No GPU call is made."""
import hashlib
import os

import pytest

import bench
from paper_1010_0762_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_baseline_reports_both_modes():
    seq = wl.cfg1_sequence(3)
    out = bench.cpu_baseline(seq, nsys=2)
    assert out["kind"] == "oracle" and out["unit"] == "dual-system solves/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "systems 0-1" in out["sample"]
    one = out["single_thread"]
    assert one["cores"] == 1 and one["value"] > 0 and "system 0" in one["sample"]


def test_profile_constants_follow_the_sources():
    """The traffic and trace constants apply only to the sources they were
    measured on: the digest bench.py compares is the sha256 prefix of the
    kernel and runtime sources, in that order."""
    h = hashlib.sha256()
    for f in bench.TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1010_0762_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    dig = h.hexdigest()[:16]
    assert bench.sources_digest() == dig
    for rec in (bench.TRAFFIC_K_IT1, bench.TRAFFIC_K_IT1_MIXED, bench.TRACE_K_IT1):
        assert set(rec) >= {"sources_sha256_16"}
    stale = {"sources_sha256_16": "0" * 16, "avg_us": 1.0}
    assert bench._if_current(stale, "avg_us") is None
    current = {"sources_sha256_16": dig, "avg_us": 1.0}
    assert bench._if_current(current, "avg_us") == 1.0
