"""Host-side checks of bench.py (no GPU): it runs on one GPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""   # no JSON line


def test_committed_profiles_match_the_kernel_sources():
    """The counter and trace summaries under profiles/ were taken on the
    current sources of the kernels bench.py reports (their sha256 prefixes
    match), so the bench line's traffic and in-filter figures are not null."""
    sys.path.insert(0, ROOT)
    import bench
    fed = "fed_stream2_kernel<4>"
    traffic = bench.counter_traffic(fed)
    assert traffic is not None and 335e6 <= traffic <= 2 * 335.5e6   # at least the algorithmic bytes
    assert bench.selection_traffic() is not None
    assert bench.counter_traffic("sweep_fused_kernel<8>", "sweep_fused_kernel<8> [select]") is not None
    t_filter = bench.trace_mean_us(fed, fed + " [filter]")
    t_loop = bench.trace_mean_us(fed, fed + " [roofline loop]")
    assert t_filter is not None and t_loop is not None and 0 < t_loop <= t_filter
    # the volume substep's counters: at least its 32 algorithmic bytes per voxel
    vol = bench.counter_traffic("fed3_kernel", summary="volume256_hbm_counters.txt")
    assert vol is not None and 32 * 256 ** 3 <= vol <= 2 * 32 * 256 ** 3
    assert "fed3_kernel sources sha256 prefix: " + bench.source_digest("fed3_kernel") in open(
        os.path.join(ROOT, "profiles", "volume256_kernel_trace.txt")).read()


def test_bench_centreline_segments_match_the_oracle():
    """The matching leg builds its ground-truth segments itself (the bench may
    not call the oracle outside its CPU baseline): the same segments and
    types as the oracle's construction, on the creases workload's centrelines
    (at 512^2)."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle
    from paper_1611_06906_amd import synth
    w = synth.creases4096(H=512, W=512)
    _, _, lines = w.ground_truth()
    segs, types = bench._centreline_segments(lines)
    ref, ref_types = oracle.gt_segments(lines)
    assert segs.shape == ref.shape and len(segs) > 1000
    assert np.array_equal(types, ref_types)
    assert np.array_equal(segs, ref.astype(np.float32))
