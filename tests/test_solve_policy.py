"""Host decisions of the mixed-precision solve (solve_policy.h), compiled with
g++ and driven on synthetic inputs; no GPU.

* stall rule: a reliable update whose float64 ||r||^2 is above a quarter of the
  previous update's counts as a stall, `limit` in a row end the float32
  solve, progress resets the count, the first update never counts;
* fallback: only a stall or a breakdown of a float32 solve with iterations
  left goes on in float64 -- by re-assembly when the plan holds its points,
  from the float64 accumulators when it was made from point chunks; the
  iteration cap and every other status return as they are.

Each check runs on a plain build and on one under the host address and
undefined-behaviour sanitizers (any report aborts the driver).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_07884_amd", "csrc")

OK, MAXITER, FALLBACK, INVALID, BREAKDOWN, HIP = 0, 1, 2, -1, -4, -5

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <initializer_list>
#include "solve_policy.h"
using namespace rbf;
int main() {
  // stall watch: limit, then a sequence of rr values; prints 0/1 per update
  {
    StallWatch w(2);
    const double rr[] = {1.0, 0.5, 0.3, 0.2, 0.01, 0.009, 0.0089, 0.00001};
    for (double v : rr) printf("%d ", (int)w.update(v));
    printf("\n");
    StallWatch one(1);
    const double r2[] = {1.0, 0.81, 0.1, 0.02};
    for (double v : r2) printf("%d ", (int)one.update(v));
    printf("\n");
    StallWatch zero(0);  // limit 0: every update "ends" (the caller ignores it)
    printf("%d %d\n", (int)zero.update(1.0), (int)zero.update(0.1));
    printf("%d\n", kDefaultStallLimit);
  }
  // fallback table: status x mixed x has_points x left
  const int st[] = {0, 1, 2, -1, -4, -5};
  for (int a : st)
    for (int mixed = 0; mixed < 2; ++mixed)
      for (int pts = 0; pts < 2; ++pts)
        for (long left : {0L, 1L, 1000L})
          printf("%d %d %d %ld %d\n", a, mixed, pts, left,
                 (int)fallback_action(a, 2, -4, mixed != 0, pts != 0, left));
  return 0;
}
"""


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def out(tmp_path_factory, request):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("policy")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    extra = SANITIZE if request.param == "sanitized" else []
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", *extra, "-I", CSRC, str(src),
                    "-o", str(exe)], check=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines()


def test_stall_watch(out):
    # limit 2: 1 -> .5 (ratio .5 > .25: stall 1), .3 (.6: stall 2 -> end),
    # .2 (.67: 3), .01 (.05: progress, reset), .009 (.9: 1), .0089 (2), 1e-5 (reset)
    assert out[0].split() == ["0", "0", "1", "1", "0", "0", "1", "0"]
    # limit 1: the second update at 0.81 of the first already ends the solve;
    # 0.1 and 0.02 (ratio 0.2) are progress
    assert out[1].split() == ["0", "1", "0", "0"]
    assert out[2].split() == ["1", "1"]
    assert out[3] == "8"


def test_fallback_table(out):
    none, reasm, accum = 0, 1, 2
    rows = [list(map(int, line.split())) for line in out[4:]]
    assert len(rows) == 6 * 2 * 2 * 3
    for status, mixed, pts, left, act in rows:
        if mixed and left > 0 and status in (FALLBACK, BREAKDOWN):
            assert act == (reasm if pts else accum), (status, mixed, pts, left, act)
        else:
            assert act == none, (status, mixed, pts, left, act)
    # the iteration cap never triggers an assembly
    assert all(act == none for status, *_, act in rows if status == MAXITER)
