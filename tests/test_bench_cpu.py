"""Host-side pieces of bench.py that need no GPU: the percentile rule, the
exact tables it reads, the scaled weights of its L = 128 profile pass, the
refusal of more than one GPU, and the committed counter summaries it reads
(used only while they were taken on the current kernel sources)."""
import math
import os
import subprocess
import sys

import numpy as np

import bench
import oracle

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))


def test_nearest_rank_percentiles():
    v = list(range(1, 101))
    assert bench.nearest_rank(v, 50) == 50 and bench.nearest_rank(v, 99) == 99
    assert bench.nearest_rank(v, 100) == 100 and bench.nearest_rank(v, 0) == 1
    assert bench.nearest_rank([3.0], 99) == 3.0 and bench.nearest_rank([], 50) is None
    assert bench.nearest_rank([5, 1, 4, 2, 3], 50) == 3


def test_exact_tables_have_two_ground_states():
    for L in (4, 8, 16, 32, 64):
        lg = bench.exact_ln_g(L)
        assert lg.size == L * L + 1
        assert abs(lg[0] - math.log(2.0)) < 1e-9
        assert not np.isfinite(lg[1]) and not np.isfinite(lg[L * L - 1])
    assert bench.exact_ln_g(128) is None


def test_scaled_weights_keep_the_fast_tables():
    # the L = 128 profile pass must run the kernels with 32-bit thresholds:
    # no move a configuration can propose may have T = 0
    L = 128
    N = L * L
    om = bench.scaled_log_weights(L)
    assert om.shape == (N + 1,) and np.all(np.isfinite(om))
    t = oracle.thresholds(N, om)
    for k in range(N + 1):
        if k in (1, N - 1):
            continue
        for d in range(5):
            kp = k + d - 2
            if 0 <= kp <= N and kp not in (1, N - 1):
                assert t[k, d] > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_summaries_match_the_current_kernel_sources():
    # the traffic and the chain instruction count in the benchmark line come
    # from profiles taken on the sources in the tree
    bytes_, note = bench.traffic_per_launch()
    assert bytes_ is not None and bytes_ > 0, note + " -- re-take the counter profiles on the current sources"
    roof, note = bench.chain_roof(4.0e11, 16384)
    assert roof is not None, note + " -- re-count the chain instructions on the current sources"
    assert roof["chain_waves"] == 256
    # 256 waves x 64 lanes x 2.4 GHz / (4 clocks x instructions per attempt)
    assert math.isclose(roof["peak"], 256 * 64 * 2.4e9 / (4 * roof["chain_instructions_per_attempt"]))


def test_summaries_of_other_kernel_sources_are_not_used(tmp_path, monkeypatch):
    stale_traffic = tmp_path / "traffic.txt"
    stale_traffic.write_text("kernel_source_sha256_16 = 0000000000000000\nhbm_bytes_per_launch = 123\n")
    stale_chain = tmp_path / "chain.md"
    stale_chain.write_text("kernel_source_sha256_16 = 0000000000000000\nchain_instructions_per_attempt = 18\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale_traffic))
    monkeypatch.setattr(bench, "CHAIN_FILE", str(stale_chain))
    bytes_, note = bench.traffic_per_launch()
    assert bytes_ is None and "not used" in note
    roof, note = bench.chain_roof(4.0e11, 16384)
    assert roof is None and "not used" in note
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    bytes_, note = bench.traffic_per_launch()
    assert bytes_ is None and "missing" in note

