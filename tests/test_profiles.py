"""The committed rocprofv3 summaries belong to the committed kernels: the HBM
byte counts that bench.py reports as roofline.traffic, and every summary that
names a kernel source hash, carry the hash of the current kernel sources; the
counted bytes are plausible against the algorithmic bytes (no GPU)."""
import json
import os
import re

import bench

PROFILES = os.path.join(bench.ROOT, "profiles")


def test_traffic_record_matches_the_kernel_sources():
    with open(os.path.join(PROFILES, "traffic.json")) as f:
        rec = json.load(f)
    h = bench.kernel_source_hash()
    for key in ("laplace3d_7pt_128", "zipf2_1e6"):
        r = rec[key]
        assert r["kernel_source_sha"] == h, f"{key}: counters taken on other kernel sources; retake them"
        # bytes = FETCH_SIZE * (copy scale, about 2) + WRITE_SIZE (KiB), per launch
        est = (r["fetch_kib"] * 1.9999 + r["write_kib"]) * 1024
        assert abs(r["bytes_per_launch"] - est) <= 1e-4 * est
        assert 0.5 <= r["bytes_per_launch"] / r["alg_bytes_per_launch"] <= 10
        assert bench.traffic_record(key) == r["bytes_per_launch"]
    # the Zipf SpMV is two kernels (the column tiles, then the SpMV kernel)
    assert len(rec["zipf2_1e6"]["kernel"]) == 2


def test_summaries_name_the_current_kernel_sources():
    h = bench.kernel_source_hash()
    named = 0
    for name in sorted(os.listdir(PROFILES)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(PROFILES, name)) as f:
            text = f.read()
        for m in re.finditer(r"[Kk]ernel source hash[^`]*`([0-9a-f]{16})`", text):
            assert m.group(1) == h, f"{name} names kernel sources {m.group(1)}, current {h}"
            named += 1
    assert named >= 3
