"""Consistency of the committed profile behind the bench's roofline traffic:
the HBM traffic in profiles/forward_control_traffic.json was measured on the
kernel sources it names (their hash), equals its calibrated FETCH_SIZE and
WRITE_SIZE readings, and its launch average is the one in the rocprofv3
summary it cites."""
from __future__ import annotations

import hashlib
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _profile():
    with open(os.path.join(ROOT, "profiles", "forward_control_traffic.json")) as f:
        return json.load(f)


def test_traffic_profile_was_taken_on_the_current_kernel_sources():
    prof = _profile()
    h = hashlib.sha256()
    for f in prof["sources"]:
        with open(os.path.join(ROOT, f), "rb") as src:
            h.update(src.read())
    assert h.hexdigest()[:16] == prof["source_hash"], \
        "the calculation kernel's sources changed since its HBM counters were taken"


def test_traffic_is_the_calibrated_counter_sum():
    prof = _profile()
    kib = prof["fetch_kib_raw"] / prof["fetch_scale"] + prof["write_kib_raw"] / prof["write_scale"]
    t = kib * 1024.0
    assert abs(t - prof["traffic_bytes_per_launch"]) <= 1e-6 * t + 1024


def test_launch_average_matches_the_cited_trace():
    prof = _profile()
    with open(os.path.join(ROOT, prof["rocprof_trace"])) as f:
        rows = [l for l in f.read().splitlines() if l.startswith("| " + prof["kernel"] + " |")]
    assert len(rows) == 1
    assert float(rows[0].split("|")[3]) == prof["rocprof_avg_launch_us"]
