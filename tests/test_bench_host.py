"""Host-side logic of bench.py, on the CPU: the one-GPU refusal, and the
lookup of committed counter summaries that fills the roofline's traffic."""

import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_traffic_is_read_only_from_a_summary_of_the_current_source(tmp_path):
    b = _bench()
    h = b.kernel_source_hash()
    assert len(h) == 16 and h == b.kernel_source_hash()
    # the committed summaries carry the hash of the source they were taken on
    # (the CG passes evaluate q again at both sizes: k_cg_rq)
    for kernel, n in (("k_cg_rq", 256), ("k_cg_rq", 500)):
        path = os.path.join(ROOT, "profiles", f"{kernel}_blobs{n}_pmc.txt")
        txt = open(path).read()
        stated = [ln.split(":", 1)[1].strip() for ln in txt.splitlines() if ln.startswith("source_sha256:")]
        hbm = [float(ln.split(":", 1)[1]) for ln in txt.splitlines() if ln.startswith("hbm_bytes_per_launch:")]
        assert len(stated) == 1 and len(hbm) == 1
        got = b.traffic_from_profile(kernel, n, stated[0])
        assert got == hbm[0]
        # any other source: no traffic figure
        assert b.traffic_from_profile(kernel, n, "0" * 16) is None
    assert b.traffic_from_profile("k_cg_step", 123, h) is None
