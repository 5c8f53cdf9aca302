"""Host-only checks of the benchmark script: the one-GPU rule and the counter summaries
its roofline reads."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summaries_match_the_kernel_source():
    """The HBM byte counts the roofline reports were taken on the current stepping
    source, for every batch width the tuner times and every distinct launch variant
    (re-take them with rocprofv3 after a change)."""
    import bench
    for name, batches, variants in (("step_fp32_c2_counters.md", (16, 32, 64), range(16)),
                                    ("step_fp64_c2_counters.md", (8, 16, 32, 64), range(16)),
                                    ("step_fp32_c4_counters.md", (8, 16, 32), range(8))):
        text = open(os.path.join(ROOT, "profiles", name)).read()
        assert re.search(r"kernel_source_hash:\s*(\w+)", text).group(1) == bench.kernel_source_hash()
        for b in batches:
            algo = float(re.search(rf"algorithmic_bytes_per_launch_b{b}:\s*(\d+)", text).group(1))
            for v in variants:
                if v >= 8 and v & 12 != 12:
                    continue               # bit 3 only with bit 2
                t = bench.traffic_from_profile(name, b, v)
                # measured traffic is at least the algorithmic bytes; XCD-contiguous tiles
                # re-read within 1.25x, linear ones (neighbour rows fetched again by other
                # XCDs' L2s, up to 1.7x on the Morton-ordered 3D mesh at B = 8) within 1.8x
                bound = 1.25 if v & 2 else 1.8
                assert t is not None and algo <= t <= bound * algo, (name, b, v, t, algo)
        assert "rocprofv3 --pmc FETCH_SIZE" in text and "rocprofv3 --pmc WRITE_SIZE" in text
