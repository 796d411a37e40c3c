"""The committed profile summaries: each names the command that made it (a
rocprofv3 run of committed files), and the counted HBM traffic of the CG
iteration agrees with the algorithmic and layout bytes of its workload."""
import glob
import json
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")


def test_every_summary_names_its_command():
    files = sorted(glob.glob(os.path.join(PROFILES, "*.md")))
    assert files
    for f in files:
        text = open(f).read()
        cmds = [l for l in text.splitlines() if "rocprofv3 " in l]
        assert cmds, f
        for c in cmds:
            # the program follows "--" directly and is a committed file
            assert " -- python3 /root/repo/bench.py" in c, (f, c)
            assert "_work" not in c, (f, c)


def test_traffic_files_are_consistent():
    files = sorted(glob.glob(os.path.join(PROFILES, "cg_iter_fp32_*_traffic.json")))
    assert len(files) == 3
    for f in files:
        t = json.load(open(f))
        assert re.fullmatch(r"[0-9a-f]{16}", t["kernel_digest"]), f
        cal = t["calibration"]
        # FETCH_SIZE counts half the bytes a plain copy reads, WRITE_SIZE all
        assert abs(cal["fetch_factor"] - cal["copy_bytes"] / 1024 / cal["fetch_kib"]) < 1e-3
        assert abs(cal["write_factor"] - cal["copy_bytes"] / 1024 / cal["write_kib"]) < 1e-3
        b = (t["fetch_kib_per_dispatch"] * cal["fetch_factor"]
             + t["write_kib_per_dispatch"] * cal["write_factor"]) * 1024
        assert abs(b - t["bytes_per_launch"]) <= 1e-3 * t["bytes_per_launch"] + 2048, f
        # the counted bytes cover what the layout must move and stay within
        # 1.5 times it (padding and records fetched by more than one XCD)
        ratio = t["bytes_per_launch"] / t["layout_bytes_per_launch"]
        assert 1.0 <= ratio <= 1.5, (f, ratio)
        assert len(t["commands"]) == 4 and all("rocprofv3 --pmc" in c for c in t["commands"])


def test_digest_covers_the_iteration_kernel():
    # the digest is taken over the iteration kernel's source and layouts:
    # 16 hex digits, stable between calls
    d = bench.kernel_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", d) and d == bench.kernel_digest()
