"""CPU: the served path's continuous-batching scheduler (csrc/scheduler.h,
free of HIP calls) driven by a fake executor from several submitter
threads, built twice with g++: plain, and with ThreadSanitizer.  The fake
executor checks at every launch that the slot is idle, that at most
max_inflight batches run, that the footprint (resident populations plus
running requests) stays under the cap and that each submitter's requests
are admitted in submission order; the test program checks tickets, results,
statistics, rejection by footprint, launch errors, continuous batching
(several requests per batch under load) and shutdown with queued
requests; each with and without admission by the submitting thread, plus
a light load where every request finds the scheduler idle."""
from __future__ import annotations

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_fake_executor.cpp")
INC = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2404_01817_amd", "csrc")]


def _build_and_run(tmp_path, name, flags, env=None):
    exe = str(tmp_path / name)
    r = subprocess.run(["g++", "-std=c++17", "-g", "-pthread", *flags, *INC, SRC, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, **(env or {})))
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "scheduler checks passed" in r.stdout
    return r


def test_scheduler_with_fake_executor(tmp_path):
    _build_and_run(tmp_path, "sched_plain", ["-O2", "-Wall", "-Werror"])


def test_scheduler_under_thread_sanitizer(tmp_path):
    r = _build_and_run(tmp_path, "sched_tsan", ["-O1", "-fsanitize=thread"],
                       env={"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"})
    assert "ThreadSanitizer" not in r.stderr, r.stderr
