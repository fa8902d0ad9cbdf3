"""Host-side parts of the measurement in bench.py: the CPU-baseline leg and
the HBM-traffic record of the forward-NN kernel.  No GPU is needed."""
import hashlib
import os
import subprocess
import sys

import oracle
from paper_2412_08346_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_cpu_baseline_fields_and_bounded_sample():
    pb, st = synth.workload_small(k_max=6)
    cb = bench.cpu_baseline(pb, st, seconds=0.0)  # one whole iteration
    assert set(cb) == {"value", "unit", "cores", "kind", "sample", "one_core"}
    assert cb["kind"] == "oracle" and cb["unit"] == "particle-iters/s"
    assert cb["cores"] == oracle.threads() and cb["value"] > 0
    one = cb["one_core"]
    assert one["cores"] == 1 and one["value"] > 0 and one["unit"] == "particle-iters/s"
    assert one["sample"].startswith(f"1 iteration of the {pb.K} particles of one")
    assert cb["sample"].startswith(f"1 iteration(s) of all {pb.k_tot} particles")
    cb = bench.cpu_baseline(pb, st, seconds=1e9)  # capped by k_max
    assert cb["sample"].startswith(f"{st.k_max} iteration(s)")


def test_traffic_record_follows_the_kernel_source():
    h = hashlib.sha256()
    for f in bench.NN_SOURCES:
        with open(os.path.join(ROOT, "paper_2412_08346_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    # the record is reported only for the kernel source it was measured on;
    # after a change to that source the traffic is null until re-measured
    same = h.hexdigest() == bench.NN_TRAFFIC["sha256"]
    import paper_2412_08346_amd as A
    for v in range(A.ASICP_LAUNCH_CHOICES):
        ch = A.launch_choice(v)
        key = f"{ch['xcd_map']},{ch['fine']},{ch['query_blocks']},{ch['chunk_points']}"
        b = bench.nn_traffic("paper", ch, False)
        assert b == (bench.NN_TRAFFIC["bytes"].get(key) if same else None)
        # other workloads and the full scan were not measured: null
        assert bench.nn_traffic("batched", ch, False) is None
        assert bench.nn_traffic("paper", ch, True) is None


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0 and "one GPU" in p.stderr
