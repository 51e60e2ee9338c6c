"""Host-only checks of bench.py's command-line contract (no GPU needed)."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_summary_keys_match_the_kernel_names():
    """The pass -> kernel-instance names bench.py looks up in the committed
    counter summary follow the kernels' template parameters."""
    sys.path.insert(0, ROOT)
    import bench
    t = dict(row_points=16, row_points_inv=8, col_points=16, col_width=8, col_shared=1, stencil_rows=8,
             fused_points=16)
    assert bench._pass_instance(0, t) == "fw::c64::(anonymous namespace)::k_srows<256, 16, 0, 256>"
    assert bench._pass_instance(2, t) == "fw::c64::k_cols<256, 16, 0, true, 512>"
    assert bench._pass_instance(2, dict(t, col_shared=2)) == "fw::c64::k_cols_split<256, 16>"
    assert bench._pass_instance(3, t) == "fw::c64::k_rows<256, 8, true, 1>"
    name = ("void fw::c64::k_rows<256, 8, true, 1>(HIP_vector_type<float, 2u> const*, int)")
    assert bench._instance_name(name) == "fw::c64::k_rows<256, 8, true, 1>"
    assert bench.PASS_MATCH[3](name) and not bench.PASS_MATCH[1](name)
