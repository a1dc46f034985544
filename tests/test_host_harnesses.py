"""Host logic under AddressSanitizer and UndefinedBehaviorSanitizer, no GPU.

Three C++ harnesses, built here with g++ (-fsanitize=address,undefined) against
the library's HIP-free headers and run as child processes:

* serve_sched_harness.cpp drives the batching server's scheduling
  (serve_sched.h: arena ranges, request life cycle, start policy) with a fake
  executor: random submissions, cancellations and steps, steps completing in
  order after random delays (up to three in flight), random LM stops.  It checks
  after every operation that live and free ranges tile the arena, that requests
  start in admission order within the fill budget (graph requests with pending
  lists are skipped, never started), that no slot is released while a step in
  flight may use it, and at the end that every request not cancelled retired
  exactly once with all its iterations (or an LM stop) and the arena is free.
  RangeAlloc is also checked against a byte map.
* graph_lists_harness.cpp rebuilds every graph list by brute force (the CSR in
  edge-list order, the split form's halo staging and slots, the fused form's one-
  and two-ring rows and slots, or a passed cap when they are refused) for random,
  hub, grid, loop and repeated-edge graphs and for Morton-ordered icospheres
  written here from the workload generator, and checks that an edge naming a
  missing vertex is refused.
* angle_trig_harness.cpp checks the branch-free FP32 sine and cosine that the
  FP32 warp energy forms from its stored angles (angle_trig.h) against the C
  library's double sin and cos on a dense grid of angles, at and beside every
  quadrant boundary and at tiny angles: within 2^-23 absolute (one FP32 ulp of 1)
  over [-3000, 3000] radians.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_06525_amd", "csrc")
HERE = os.path.dirname(os.path.abspath(__file__))
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-fno-omit-frame-pointer", "-I", CSRC]


def _build(src, out):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    r = subprocess.run([gxx, *FLAGS, os.path.join(HERE, src), "-o", str(out)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return str(out)


def _run(args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run(args, capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]
    return r.stdout


def test_server_scheduling_with_a_fake_executor(tmp_path):
    exe = _build("serve_sched_harness.cpp", tmp_path / "sched")
    for seed in range(1, 7):
        _run([exe, str(seed), "20000"])


def test_graph_lists_against_brute_force(tmp_path):
    exe = _build("graph_lists_harness.cpp", tmp_path / "lists")
    files = []
    for level in (3, 5):
        d = w.arap_mesh(level, seed=3)
        e = np.asarray(d["edges"], np.int32)
        f = tmp_path / f"ico{level}.bin"
        with open(f, "wb") as fh:
            np.array([d["V"], e.shape[0]], np.int32).tofile(fh)
            e.tofile(fh)
        files.append(str(f))
    out = _run([exe, "1", *files])
    assert "with fused rows" in out
    for seed in (2, 3):
        _run([exe, str(seed)])


def test_angle_sine_and_cosine(tmp_path):
    exe = _build("angle_trig_harness.cpp", tmp_path / "trig")
    for lim in ("1", "100", "3000"):
        out = _run([exe, lim, "2.0"])
        assert float(out.split()[1]) <= 2.0
