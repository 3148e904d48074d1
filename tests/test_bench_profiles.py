"""The benchmark's readers of the committed counter summaries (CPU only): the
HBM traffic and the measured bound of the blocked annealer are taken from
profiles/ only while the summaries name the current annealer sources, and
then parse to the figures the summaries print."""
import hashlib
import os
import re

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _profile(name):
    with open(os.path.join(ROOT, "profiles", name)) as f:
        return f.read()


def test_annealer_digest_covers_kernel_layout_and_schedule():
    h = hashlib.sha256()
    for name in ("anneal_block.hip", "pack.cpp", "schedule.cpp"):
        with open(os.path.join(ROOT, "paper_2407_19987_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    assert bench.annealer_digest() == h.hexdigest()


def test_summaries_name_the_current_sources():
    digest = bench.annealer_digest()
    for name in ("anneal_block_cu_path_order3_n128_fp16x2.md", "anneal_block_traffic_order3_n128_b4096_fp16x2.md",
                 "anneal_block_order3_n128_b4096_fp16x2.md"):
        assert digest in _profile(name), f"{name} was measured on other annealer sources"


def test_traffic_and_bound_parse():
    traffic = bench.read_traffic("fp16x2", bench.REPLICAS, bench.SWEEPS, 4)
    txt = _profile("anneal_block_traffic_order3_n128_b4096_fp16x2.md")
    row = re.search(r"`anneal_block_kernel<5, 16>` \| \d+ \| ([0-9.]+) \| ([0-9.]+) \|", txt)
    fs = float(re.search(r"FETCH x ([0-9.]+)", txt).group(1))
    ws = float(re.search(r"WRITE x ([0-9.]+)", txt).group(1))
    assert traffic == (float(row.group(1)) * fs + float(row.group(2)) * ws) * 1024.0
    mb = bench.read_cu_path("fp16x2", bench.REPLICAS, bench.SWEEPS, 4, 53.8)
    assert mb is not None and 0.3 < mb["frac"] < 1.0 and 0.5 < mb["data_return_busy"] <= 1.0
    # other workloads are not what the summaries measured
    assert bench.read_traffic("fp16x2", 2 * bench.REPLICAS, bench.SWEEPS, 4) is None
    assert bench.read_cu_path("bf16x2", bench.REPLICAS, bench.SWEEPS, 4, 53.8) is None
