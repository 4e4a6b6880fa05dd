"""Host-side contract of bench.py (no GPU): the one-GPU guard, the source hash the profile
counters are keyed to, and the counter file it reads."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, cwd=ROOT, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_source_hash_is_a_sha256_of_the_kernel_sources():
    r = _run("--source-hash")
    assert r.returncode == 0
    assert re.fullmatch(r"[0-9a-f]{64}", r.stdout.strip())


def test_counter_file_is_parsed_and_keyed_to_the_sources():
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic()
    path = bench.COUNTERS_FILE
    text = open(path).read()
    key = re.search(r"^source_sha256 = ([0-9a-f]{64})$", text, re.M).group(1)
    if key == bench.source_hash():
        # calibrated bytes per launch: more than the 268 MB of dL/dy the kernel writes
        assert t is not None and 2.68e8 < t < 1e9
    else:
        assert t is None
