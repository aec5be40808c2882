"""The HIP-graph cache's host logic (csrc/graph_cache.h) under sanitizers.

A captured graph bakes in device addresses, so the cache keys entries on
object identities that are never reused, drops every entry that depends on a
destroyed object, re-captures instead of replaying after any scratch region
was freed or moved, and stays bounded.  The header has no HIP dependency; a
small C++ program checks those rules built with g++ under AddressSanitizer +
UndefinedBehaviorSanitizer, and its concurrent part under ThreadSanitizer.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "graph_cache_test.cpp")
INC = os.path.join(ROOT, "paper_2412_13269_amd", "csrc")


def _build_and_run(tmp_path, flags, name):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / name)
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I", INC, SRC, "-o", exe, "-pthread", *flags]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "graph cache ok" in r.stdout


def test_graph_cache_rules_under_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"], "gc_asan")


def test_graph_cache_concurrent_use_under_tsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread", "-DPFX_THREADS"], "gc_tsan")
