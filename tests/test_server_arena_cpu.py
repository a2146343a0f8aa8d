"""Request-loop arena bookkeeping on the CPU (paper_2309_04841_amd/csrc/arena.hpp).

Reproduces the fragmentation that could stall the queue: a cost vector placed
first fit in the middle of the arena leaves enough free bytes for a request but
no contiguous block, and with nothing in flight no finishing request would ever
free one.  Cost vectors placed from the top keep the request space contiguous,
and a blocked head request with nothing in flight is rejected, not waited on.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2309_04841_amd", "csrc")


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    exe = tmp_path_factory.mktemp("arena") / "arena_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", f"-I{CSRC}",
                           os.path.join(HERE, "arena_check.cpp"), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    vals = {}
    for line in out.splitlines():
        parts = line.split()
        for i in range(0, len(parts), 2):
            vals[parts[i]] = int(parts[i + 1])
    return vals


def test_first_fit_cost_vector_fragments(report):
    assert report["firstfit_cost_at"] == 4
    assert report["firstfit_free_total"] == 8 and report["firstfit_largest"] == 4
    assert report["firstfit_six_fits"] == 0
    # a blocked head request is rejected when nothing is in flight, waits otherwise
    assert report["head_blocked_idle_rejects"] == 1 and report["head_blocked_busy_waits"] == 1


def test_cost_vector_from_the_top_keeps_requests_contiguous(report):
    assert report["top_cost_at"] == 8
    assert report["top_largest"] == 8 and report["top_six_fits"] == 1


def test_exact_bookkeeping(report):
    assert report["size_granules"] == 1000
    assert (report["x"], report["y"], report["z"]) == (0, 998, 1)
    assert report["full_low_fails"] == 1 and report["full_high_fails"] == 1
    assert report["used_granules"] == 1000
    assert report["after_release_ranges"] == 1 and report["after_release_largest"] == 998
    assert report["all_free_ranges"] == 1 and report["all_free_largest"] == 1000 and report["used"] == 0 and report["peak"] == 1000
