"""Host logic of the CG chunk sizing (chunk_planner.h), compiled with g++ and
driven on synthetic snapshots; no GPU.

The expected sizes follow from the rule: without a decay, chunks start at 4
(or check_every if smaller) and double up to check_every; with one, a chunk
takes half the iterations left to the trigger, ln(trigger / rr) / rate with
rate = ln(rr1 / rr0) / (it1 - it0), minus the chunk still in flight, clamped
to [4, check_every]; the soonest active right-hand side decides.

Each check runs on a plain build and on one under the host address and
undefined-behaviour sanitizers (any report aborts the driver).
"""
import math
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_07884_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "chunk_planner.h"
using rbf::ChunkPlanner;
static void seen1(ChunkPlanner& p, long it, double rr, double trig) {
  p.seen(it, 1, &rr, &trig, nullptr);
}
int main() {
  {  // no decay yet: 4, 8, 16, 32, 32
    ChunkPlanner p(32);
    for (int k = 0; k < 5; ++k) printf("%ld ", (long)p.next(0));
    printf("\n");
  }
  {  // decay 1 -> 0.5 over 32 iterations, trigger 0.1, 32 in flight
    ChunkPlanner p(32);
    seen1(p, 0, 1.0, 0.1);
    seen1(p, 32, 0.5, 0.1);
    const long a = (long)p.next(32), b = (long)p.next(0);
    printf("%ld %ld\n", a, b);
  }
  {  // slow decay: far from the trigger, capped at check_every
    ChunkPlanner p(32);
    seen1(p, 0, 1.0, 1e-6);
    seen1(p, 32, 0.99, 1e-6);
    printf("%ld\n", (long)p.next(8));
  }
  {  // below the trigger already, and a growing residual
    ChunkPlanner p(32);
    seen1(p, 0, 1.0, 0.5);
    seen1(p, 8, 0.4, 0.5);
    const long a = (long)p.next(0);
    seen1(p, 16, 0.45, 0.5);
    const long b = (long)p.next(0), c = (long)p.next(0);
    printf("%ld %ld %ld\n", a, b, c);
  }
  {  // restart after a refresh, and a check_every below 4
    ChunkPlanner p(32);
    seen1(p, 0, 1.0, 0.1);
    seen1(p, 32, 0.5, 0.1);
    p.restart();
    ChunkPlanner q(3);
    const long a = (long)p.next(0), b = (long)q.next(0), c = (long)q.next(0);
    printf("%ld %ld %ld\n", a, b, c);
  }
  {  // several right-hand sides: the soonest active one decides
    ChunkPlanner p(64);
    double r0[3] = {1.0, 1.0, 1.0}, r1[3] = {0.5, 0.9, 0.01}, t[3] = {1e-4, 0.5, 1e-9};
    int act[3] = {1, 1, 0};
    p.seen(0, 3, r0, t, act);
    p.seen(16, 3, r1, t, act);
    printf("%ld\n", (long)p.next(0));
  }
  return 0;
}
"""


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def lines(tmp_path_factory, request):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("planner")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    extra = SANITIZE if request.param == "sanitized" else []
    subprocess.run([gxx, "-std=c++17", "-O1", *extra, "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return [[int(v) for v in line.split()] for line in out.strip().splitlines()]


def want(rr0, rr1, it0, it1, trig, inflight, cmax):
    rate = math.log(rr1 / rr0) / (it1 - it0)
    left = math.log(trig / rr1) / rate if rr1 > trig else 0.0
    w = 0.5 * left - inflight
    return 4 if w <= 4 else (cmax if w >= cmax else int(w))


def test_ramp_without_decay(lines):
    assert lines[0] == [4, 8, 16, 32, 32]


def test_decay_estimate(lines):
    assert lines[1] == [want(1.0, 0.5, 0, 32, 0.1, 32, 32), want(1.0, 0.5, 0, 32, 0.1, 0, 32)]
    assert lines[1] == [5, 32]
    assert lines[2] == [32]


def test_trigger_passed_and_growth(lines):
    # at or below the trigger: the smallest chunk; ||r|| grew: no estimate,
    # doubling from the last chunk
    assert lines[3] == [4, 4, 8]


def test_restart_and_small_check_every(lines):
    assert lines[4] == [4, 3, 3]


def test_soonest_active_rhs_decides(lines):
    # rhs 1 reaches its trigger first; rhs 2 (inactive) would be sooner still
    r1 = want(1.0, 0.9, 0, 16, 0.5, 0, 64)
    r0 = want(1.0, 0.5, 0, 16, 1e-4, 0, 64)
    assert lines[5] == [min(r0, r1)]
