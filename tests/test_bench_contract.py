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
    assert (bench._pass_instance(0, dict(t, fused_points=12), n=384) ==
            "fw::c64::(anonymous namespace)::k_srows<384, 12, 0, 512>")
    assert bench._pass_instance(2, t) == "fw::c64::k_cols<256, 16, 0, true, 512>"
    assert bench._pass_instance(2, dict(t, col_shared=2)) == "fw::c64::k_cols_split<256, 16>"
    assert bench._pass_instance(2, dict(t, col_points=4, col_shared=4)) == "fw::c64::k_cols_tw<256, 4, 8>"
    assert bench._pass_instance(3, t) == "fw::c64::k_rows<256, 8, true, 1>"
    name = ("void fw::c64::k_rows<256, 8, true, 1>(HIP_vector_type<float, 2u> const*, int)")
    assert bench._instance_name(name) == "fw::c64::k_rows<256, 8, true, 1>"
    assert bench.PASS_MATCH[3](name) and not bench.PASS_MATCH[1](name)
    tw = "void fw::c64::k_cols_tw<256, 4, 8>(HIP_vector_type<float, 2u>*, fw::c64::ProbDev)"
    assert bench.PASS_MATCH[2](tw) and bench._instance_name(tw) == "fw::c64::k_cols_tw<256, 4, 8>"
    # the direction-update mode of the fused kernel (the roofline kernel)
    px = bench._pass_instance(bench.PX_PASS, t)
    assert px == "fw::c64::(anonymous namespace)::k_srows<256, 16, 3, 512>"
    assert bench._pass_instance(bench.PX_PASS, dict(t, fused_points=8)).endswith("k_srows<256, 8, 3, 512>")
    full = "void " + px + "(HIP_vector_type<float, 2u> const*, int)"
    assert bench.PASS_MATCH[bench.PX_PASS](full) and not bench.PASS_MATCH[0](full)
    assert bench._instance_name(full) == px


def test_counter_summary_keeps_full_direction_update_launches(tmp_path):
    """The summary scales both counters by the 1 GiB copy and, for the
    direction-update pass, keeps only launches in which every system worked."""
    sys.path.insert(0, ROOT)
    import bench
    px = "void fw::c64::(anonymous namespace)::k_srows<256, 16, 3, 512>(int)"
    mv = "void fw::c64::k_rows<256, 8, true, 1>(int)"
    cp = "__amd_rocclr_copyBuffer"
    rows = {"FETCH_SIZE": [(cp, 524288.0), (px, 100.0), (px, 100.0), (px, 2.0), (mv, 10.0), (mv, 30.0)],
            "WRITE_SIZE": [(cp, 1048576.0), (px, 50.0), (px, 50.0), (px, 1.0), (mv, 5.0), (mv, 5.0)]}
    paths = []
    for counter, recs in rows.items():
        path = tmp_path / f"{counter}.csv"
        lines = ["Kernel_Name,Counter_Name,Counter_Value"] + [f'"{n}",{counter},{v}' for n, v in recs]
        path.write_text("\n".join(lines) + "\n")
        paths.append(str(path))
    out = tmp_path / "summary.json"
    bench.summarize_counters(paths[0], paths[1], "test", str(out))
    import json
    d = json.loads(out.read_text())
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    e = d["passes"][str(bench.PX_PASS)]["instances"]["fw::c64::(anonymous namespace)::k_srows<256, 16, 3, 512>"]
    assert e["launches"] == 2 and e["hbm_bytes_per_launch"] == (100.0 * 2.0 + 50.0) * 1024.0
    m = d["passes"]["3"]["instances"]["fw::c64::k_rows<256, 8, true, 1>"]
    assert m["launches"] == 2 and m["hbm_bytes_per_launch"] == (20.0 * 2.0 + 5.0) * 1024.0


def test_multigrid_counter_summary_attributes_dispatches_by_order(tmp_path):
    """Arnoldi-kernel counters are attributed to (step j, grid) by dispatch
    order, counting back from the end (the solve before the timed launches
    runs the same kernels), and compared with the algorithmic bytes."""
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    probs = W.four_grids()
    reps, m = 2, 32
    steps = [0, 16, 31]
    upd = "fw::c64::k_gm_update(fw::c64::GmArgs, int, int, int)"
    dots = "fw::c64::k_gm_dots(fw::c64::GmArgs, int)"
    proj = ["void fw::c64::k_rows<%d, 12, true, 5>(int)" % p["nx"] for p in probs]
    cp = "__amd_rocclr_copyBuffer"
    disp = []   # (name, fetch KiB, write KiB)
    disp += [(upd, 1e9, 1e9)] * 7          # the solve's launches: excluded
    for j in steps:
        for kind in ("update", "dots", "projections"):
            for _ in range(reps + 1):
                for ip, p in enumerate(probs):
                    cs = p["nsys"] * p["nx"] * p["nz"]
                    # counter bytes = 1.25 x the algorithmic bytes (fetch scaled x2 by the copy)
                    alg = bench.GM_BYTES[kind](j) * cs
                    name = upd if kind == "update" else dots if kind == "dots" else proj[ip]
                    disp.append((name, 0.5 * 1.25 * alg / 2.0 / 1024.0, 0.5 * 1.25 * alg / 1024.0))
    disp.append((cp, 524288.0, 1048576.0))
    paths = []
    for k, counter in ((1, "FETCH_SIZE"), (2, "WRITE_SIZE")):
        path = tmp_path / f"{counter}.csv"
        lines = ["Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
        lines += [f'{i},"{d[0]}",{counter},{d[k]}' for i, d in enumerate(disp)]
        path.write_text("\n".join(lines) + "\n")
        paths.append(str(path))
    out = tmp_path / "mg.json"
    bench.summarize_multigrid_counters(paths[0], paths[1], "test", m, reps, str(out))
    import json
    d = json.loads(out.read_text())
    got = {(e["kernel"], e["j"], e["grid"]): e for e in d["gmres"]}
    assert len(got) == 3 * 3 * len(probs)
    for e in got.values():
        assert abs(e["ratio"] - 1.25) < 1e-9 and e["launches"] == reps + 1
