"""CPU checks of the benchmark script: it refuses runs over several GPUs
before touching a device, and the committed rocprofv3 summaries describe the
current kernel sources (so the bench line's roofline.traffic is reported,
not null)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_several_gpus_are_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one MI355X" in r.stderr
    assert r.stdout == ""


def test_committed_profiles_match_the_kernel_sources():
    h = bench.kernel_hash()
    assert bench.measured_traffic() is not None
    for name in ("kernel_trace_step_d3q18_f32_aa_cavity128.txt",
                 "pmc_step_d3q18_f32_aa_cavity128.txt",
                 "pmc_step_d3q18_storages_cavity128.txt",
                 "kernel_trace_batch256_cavities.txt",
                 "pmc_batch256_cavities.txt",
                 "pmc_step_d3q18_f32_aa_cavity256.txt"):
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        m = re.search(r"kernel_source_hash:\s*(\w+)", txt)
        assert m and m.group(1) == h, name
        assert "rocprofv3" in txt and "bench.py" in txt, name


def test_traffic_is_close_to_the_algorithmic_bytes():
    # 144 B per node of the 128^3 headline lattice per launch
    alg = 144 * 128 ** 3
    assert 1.0 <= bench.measured_traffic() / alg < 1.02
