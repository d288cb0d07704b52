"""Host-side checks of bench.py (no GPU): the one-GPU contract and the
counter summaries the roofline line reads."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr


def test_print_hash_is_the_digest_of_the_kernel_sources():
    for kind in bench.KERNELS:
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--print-hash", kind],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0
        assert re.fullmatch(r"[0-9a-f]{64}", r.stdout.strip()), r.stdout
        assert r.stdout.strip() == bench.source_hash(kind)


def test_committed_counter_summaries_match_the_current_kernels():
    """The HBM traffic the bench line reports comes from profiles/ only while
    the summary's recorded source hash equals the kernel sources' hash."""
    for kind, (_, fname, _) in bench.KERNELS.items():
        text = open(os.path.join(ROOT, "profiles", fname)).read()
        assert "@source_sha256: " + bench.source_hash(kind) in text, fname
        t = bench.measured_traffic(kind)
        assert t is not None and t > 0, kind


def test_cpu_model_is_a_string():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()
