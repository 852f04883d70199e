"""Host-side behaviour of bench.py that needs no GPU: the refusal of more than
one GPU, and the all-core CPU baseline's child protocol (ready, go, rate) on a
tiny workload."""
import argparse
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout


def test_all_core_baseline_children():
    a = argparse.Namespace(nx=32, nv=32, ppc=2, cpu_steps=2)
    rate, secs = bench.cpu_baseline_all_cores(a, 2)
    assert rate > 0 and secs > 0


def test_traffic_summaries_belong_to_current_sources():
    """The PMC traffic the bench line reports comes from the committed
    summaries, each tied by a digest to the reconstruction sources it was
    measured on; after a change to those sources the counters are to be taken
    again (until then the bench reports the traffic as unknown)."""
    for workload, tags in (("bump_on_tail", ("recon_fp32", "recon_fp32_kahan", "recon_fp64")),
                           ("two_stream_3v", ("recon3_fp32", "recon3_fp64"))):
        for tag in tags:
            t = bench.measured_traffic(workload, tag)
            assert t is not None and t > 0, (workload, tag)
