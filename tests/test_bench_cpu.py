"""Host-side pieces of the benchmark (CPU only): the one-GPU guard, the
counter-summary lookup behind roofline.traffic, and the algorithmic byte
model of a CG operator application."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_lookup_follows_the_source_hash(tmp_path):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "summary.md"
    prof.write_text("# summary\n\nsome text: not a key\nsource_sha256: %s\norder_class: 2\n"
                    "traffic_bytes_per_dispatch: 12345\n" % sha)
    assert bench.traffic_from_profile(str(prof), str(src), order_class=2) == 12345.0
    assert bench.traffic_from_profile(str(prof), str(src), order_class=1) is None   # other class
    src.write_text("// kernel v2\n")                                                # source changed
    assert bench.traffic_from_profile(str(prof), str(src), order_class=2) is None
    assert bench.traffic_from_profile(str(tmp_path / "missing.md"), str(src)) is None


def test_committed_summaries_name_their_kernel_sources():
    # every counter summary that bench.py reads carries a hash and a figure
    for prof in (bench.EIG_PROFILE, bench.PCG_PROFILE):
        text = open(prof).read()
        assert "source_sha256:" in text and "traffic_bytes_per_dispatch:" in text


def test_cg_byte_model_counts_each_operand_once():
    # A: 3 x 4 with 5 nonzeros, P: 4 x 4 diagonal (4 nonzeros); float32:
    # A and A' values + int32 columns once each, P once, 6 n + 2 m vector elements
    A = sp.csr_matrix(np.array([[1.0, 0, 2, 0], [0, 3, 0, 0], [4, 0, 0, 5]]))
    P = sp.csr_matrix(np.diag([1.0, 2, 3, 4]))
    inst = synth.ConicInstance(P=P, q=np.zeros(4), A=A, b=np.zeros(3), cones=[synth.Cone("nonneg", 3)])
    assert bench.pcg_bytes_per_iteration(inst, 4) == 2 * 5 * 8 + 4 * 8 + 4 * (6 * 4 + 2 * 3)
    assert bench.pcg_bytes_per_iteration(inst, 8) == 2 * 5 * 12 + 4 * 12 + 8 * (6 * 4 + 2 * 3)
