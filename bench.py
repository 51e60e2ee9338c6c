#!/usr/bin/env python
"""Benchmark of the elastic Lippmann-Schwinger hot path on one MI355X.

Workload: 256 x 256 VTI grid (dx 8 m; Vp0 2500, Vs0 1200, eps 0.15,
delta 0.05, rho 2200), random-layered contrast (seed 1), 16 surface point
forces, 5 Hz, 2 % damping, complex64 fields with FP64 Krylov scalars.

One step = the whole hot path over this batch: incident fields u0 = G0 conv s
for the 16 sources, the batched BiCGSTAB solve of A u^b = u0 to 1e-6, one
Frechet application J dm (virtual source, one solve per system, receiver
gather) and one adjoint application J* r (receiver scatter, one solve per
system, correlation summed over sources), each solve graph-captured and run
to 1e-6.  `value` is the sustained LS matvec rate of the step:
    sum over the three solves and all systems of (2 iters + 1) * nx * nz
divided by the step's wall time (G cell-systems per second).

Also reported: the isolated batched matvec rate, time-to-1e-6 of the batched
solve against the plain per-source solve (same kernels, nsys = 1, host check
every iteration), the per-pass kernel times, the roofline of the dominant
kernel (the BiCGSTAB direction-update mode of the fused stencil + row FFT,
timed with every system running) and the CPU oracle timed on a bounded sample
of the same step.
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time
from types import SimpleNamespace

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LS matvec GPoints/s + time-to-1e-6 residual, batched c64 vs plain, % HBM peak"
HBM_PEAK_GBS = 8000.0
RTOL = 1e-6
NREC = 128
PASS_NAMES = ["k_body_force (contrast stencil)", "k_rows<256,fwd> (row FFT)",
              "k_cols<256,GREEN> (column FFT + G_hat + inverse column FFT)",
              "k_rows<256,inv,APPLY> (inverse row FFT + LS epilogue)"]
# algorithmic HBM bytes per cell-system for each pass (complex64 = 8 B per
# component, 2 components): read + write of the field, plus the epilogue's
# read of u; pass 0 also reads the 5 fp32 maps once per cell (20 B per cell,
# shared by the nsys systems).
PASS_BYTES = [32.0, 32.0, 32.0, 48.0]
# the stencil fused with the forward rows moves what the stencil alone moves:
# u in, the row-transformed b out (plus the maps)
FUSED_NAME = "k_srows (contrast stencil fused with the forward row FFT)"
MAP_BYTES_PER_CELL = 20.0
# algorithmic HBM bytes per cell-system of one batched BiCGSTAB iteration:
# direction-update stencil (reads s, t, p_old, v, x; writes p, r, x and the
# row-transformed b: 144 B), s-update stencil (reads r, v; writes s, b: 64 B),
# two column passes (2 x 32 B), two inverse row passes with the v / t
# epilogues (read the spectrum, the field and r^; write v or t: 2 x 64 B);
# 64 B more when the stencils and the forward rows are separate kernels
ITER_BYTES_FUSED, ITER_BYTES_SPLIT = 400.0, 464.0
# the direction-update mode of the fused kernel alone (the largest kernel of a
# BiCGSTAB iteration): 144 B per cell-system plus the maps
PX_BYTES = 144.0
PX_NAME = ("k_srows, direction-update mode (previous iteration's r / x updates and p = r + beta (p - omega v) "
           "fused into the contrast stencil and the forward row FFT)")
PX_PASS = 4   # its entry in the counter summary


CSRC = os.path.join(ROOT, "paper_2402_02116_amd", "csrc")
COUNTERS = os.path.join(ROOT, "profiles", "counters_vti256x16.json")


def _kernel_source_hash():
    """Hash of every kernel source: counter summaries taken on other sources are stale."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


# kernel-name test of each pass (template arguments vary with the tuned variant)
# (the complex64 build's kernels live in namespace fw::c64)
PASS_MATCH = [lambda n: ((n.startswith("void fw::c64::k_body_force<") or n.startswith("void fw::c64::k_body_force_z<"))
                         and ", 0>(" in n)
              or re.search(r"c64::\(anonymous namespace\)::k_srows<\d+, \d+, 0, \d+>\(", n) is not None,
              lambda n: n.startswith("void fw::c64::k_rows<") and ", false, 0>" in n,
              lambda n: (n.startswith("void fw::c64::k_cols<") and ", 0, " in n)
              or n.startswith("void fw::c64::k_cols_split<") or n.startswith("void fw::c64::k_cols_tw<"),
              lambda n: n.startswith("void fw::c64::k_rows<") and ", true, 1>" in n,
              lambda n: re.search(r"c64::\(anonymous namespace\)::k_srows<\d+, \d+, 3, \d+>\(", n) is not None]


def _instance_name(kernel):
    """'fw::c64::k_rows<256, 16, false, 0>' from the demangled name with its
    parameter list (the namespace part may itself contain parentheses)."""
    import re
    m = re.match(r"(?:void )?(.*?>)\(", kernel)
    return m.group(1) if m else kernel


def summarize_counters(fetch_csv, write_csv, cmd, out_path=None):
    """profiles/counters_vti256x16.json from two rocprofv3 --pmc runs of
    `bench.py --passes-only` (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch).
    Each counter is scaled by what it reads for the 1 GiB device copy that the
    same run ends with (2 x 512 MiB moved: read 1 GiB, write 1 GiB)."""
    import csv
    import statistics

    def per_kernel(path, counter):
        out = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return out

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    gib_kib = 1024.0 * 1024.0
    # the largest copy dispatch is the 1 GiB device-to-device copy
    copy_f = max((max(v) for n, v in fetch.items() if "copy" in n.lower()), default=None)
    copy_w = max((max(v) for n, v in write.items() if "copy" in n.lower()), default=None)
    sf, sw = gib_kib / copy_f, gib_kib / copy_w
    passes = {}
    for k, match in enumerate(PASS_MATCH):
        inst = {}
        for n in fetch:
            if not match(n) or n not in write:
                continue
            fv, wv = fetch[n], write[n]
            if k == PX_PASS:
                # the timed launches run every system; a solve's launches after
                # its systems stopped exit early and are left out
                fv = [x for x in fv if x >= 0.5 * max(fv)]
                wv = [x for x in wv if x >= 0.5 * max(wv)]
            f, w = statistics.median(fv), statistics.median(wv)
            inst[_instance_name(n)] = dict(
                fetch_kib=f, write_kib=w, launches=len(fv), hbm_bytes_per_launch=(f * sf + w * sw) * 1024.0)
        if inst:
            passes[str(k)] = dict(kernel=PX_NAME if k == PX_PASS else PASS_NAMES[k], instances=inst)
    out = dict(source_hash=_kernel_source_hash(), command=cmd, fetch_scale=sf, write_scale=sw,
               copy_fetch_kib=copy_f, copy_write_kib=copy_w, passes=passes)
    with open(out_path or COUNTERS, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))
    return 0


def summarize_multigrid_counters(fetch_csv, write_csv, cmd, restart, reps, out_path):
    """profiles/counters_multigrid.json from two rocprofv3 --pmc runs of
    `bench.py --workload multigrid --passes-only` (FETCH_SIZE, then WRITE_SIZE).
    Per problem (grid): the four matvec passes; per Arnoldi-step kernel and
    step j: counter bytes per launch against the algorithmic bytes.  The run
    launches, in this order: the passes of every problem (pass k of all
    problems, reps + 1 times), then for j = 0, m/2, m - 1 the update, dots and
    projection kernels of every problem (reps + 1 times each, problems in plan
    order); dispatches are attributed by that order, counting from the end
    (the solve before them launches the same kernels)."""
    import csv
    import statistics
    import workloads as W

    probs = W.four_grids()

    def rows(path, counter):
        out = []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter:
                out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"])))
        out.sort()
        return out

    fetch, write = rows(fetch_csv, "FETCH_SIZE"), rows(write_csv, "WRITE_SIZE")
    gib_kib = 1024.0 * 1024.0
    copy_f = max(v for _, n, v in fetch if "copy" in n.lower())
    copy_w = max(v for _, n, v in write if "copy" in n.lower())
    sf, sw = gib_kib / copy_f, gib_kib / copy_w

    def by_name(rs):
        d = {}
        for _, n, v in rs:
            d.setdefault(n, []).append(v)
        return d

    fn, wn = by_name(fetch), by_name(write)
    cells = [p["nx"] * p["nz"] for p in probs]
    nsys = [p["nsys"] for p in probs]
    steps = sorted({0, restart // 2, restart - 1})
    out = dict(source_hash=_kernel_source_hash(), command=cmd, fetch_scale=sf, write_scale=sw,
               copy_fetch_kib=copy_f, copy_write_kib=copy_w, grids=[p["nx"] for p in probs], restart=restart,
               gmres=[], passes=[])

    def entry(fv, wv, alg):
        f, w = statistics.median(fv), statistics.median(wv)
        b = (f * sf + w * sw) * 1024.0
        return dict(fetch_kib=f, write_kib=w, launches=len(fv), counter_bytes_per_launch=b,
                    algorithmic_bytes_per_launch=alg, ratio=round(b / alg, 4))

    # Arnoldi kernels: the update and dots kernels share one name over the
    # problems (problem = dispatch index mod the problem count); the projection
    # epilogue is the inverse row kernel with EPI 5 (one name per grid)
    np_ = len(probs)
    for kind, pat in (("update", "k_gm_update("), ("dots", "k_gm_dots(")):
        name = next((n for n in fn if pat in n and n in wn), None)
        if name is None:
            continue
        per = (reps + 1) * np_
        fv, wv = fn[name][-per * len(steps):], wn[name][-per * len(steps):]
        for gi, j in enumerate(steps):
            for ip in range(np_):
                sel = [i for i in range(gi * per, (gi + 1) * per) if i % np_ == ip]
                alg = GM_BYTES[kind](j) * nsys[ip] * cells[ip]
                out["gmres"].append(dict(kernel=kind, j=j, grid=probs[ip]["nx"],
                                         **entry([fv[i] for i in sel], [wv[i] for i in sel], alg)))
    for ip, p in enumerate(probs):
        name = next((n for n in fn if re.search(rf"k_rows<{p['nx']}, \d+, true, 5>", n) and n in wn), None)
        if name is None:
            continue
        per = reps + 1
        fv, wv = fn[name][-per * len(steps):], wn[name][-per * len(steps):]
        for gi, j in enumerate(steps):
            alg = GM_BYTES["projections"](j) * nsys[ip] * cells[ip]
            out["gmres"].append(dict(kernel="projections", j=j, grid=p["nx"],
                                     **entry(fv[gi * per:(gi + 1) * per], wv[gi * per:(gi + 1) * per], alg)))
    # matvec passes: the kernel instances of each grid (template N = the grid)
    for k, match in enumerate(PASS_MATCH[:4]):
        for ip, p in enumerate(probs):
            for n in fn:
                if not match(n) or n not in wn:
                    continue
                nm = _instance_name(n)
                if k == 0 and "k_body_force" in nm:
                    continue   # the fused stencil + rows serves every grid here
                if f"<{p['nx']}," not in nm:
                    continue
                alg = PASS_BYTES[k] * nsys[ip] * cells[ip] + (MAP_BYTES_PER_CELL * cells[ip] if k == 0 else 0.0)
                # launches with every system running (a solve's launches for
                # stopped systems exit early)
                fv = [x for x in fn[n] if x >= 0.5 * max(fn[n])]
                wv = [x for x in wn[n] if x >= 0.5 * max(wn[n])]
                out["passes"].append(dict(pass_=k, grid=p["nx"], instance=nm, **entry(fv, wv, alg)))
    out["passes"] = [{("pass" if kk == "pass_" else kk): v for kk, v in d.items()} for d in out["passes"]]
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    for d in out["gmres"]:
        print(f"{d['kernel']:12s} j={d['j']:2d} grid={d['grid']:4d} ratio {d['ratio']:.3f}")
    for d in out["passes"]:
        print(f"pass {d['pass']} grid={d['grid']:4d} {d['instance']:50s} ratio {d['ratio']:.3f}")
    return 0


def _pass_instance(k, tuning, n=256):
    """Kernel instance of pass k on an n^2 grid under the plan's variants."""
    if k == PX_PASS:
        # 512 threads while a thread's row segment is at most 32 points long
        p = tuning["fused_points"]
        return f"fw::c64::(anonymous namespace)::k_srows<{n}, {p}, 3, {512 if n >= 256 and n // p <= 32 else 256}>"
    if k == 0:
        if tuning.get("fused_points"):
            # the plain mode runs 512-thread blocks on rows of 384 points or more (short row segments)
            p = tuning["fused_points"]
            return f"fw::c64::(anonymous namespace)::k_srows<{n}, {p}, 0, {512 if n >= 384 and n // p <= 32 else 256}>"
        if tuning.get("stencil_sys") == -1:   # the z-marching stencil
            return f"fw::c64::k_body_force_z<64, {tuning['stencil_rows']}, 0>"
        return f"fw::c64::k_body_force<64, {tuning['stencil_rows']}, 0>"
    if k == 1:
        return f"fw::c64::k_rows<{n}, {tuning['row_points']}, false, 0>"
    if k == 2:
        if tuning["col_shared"] == 2:
            return f"fw::c64::k_cols_split<{n}, {tuning['col_points']}>"
        if tuning["col_shared"] == 4:   # twiddles in LDS, compile-time tile width
            return f"fw::c64::k_cols_tw<{n}, {tuning['col_points']}, {tuning['col_width']}>"
        seq = "true" if tuning["col_shared"] else "false"
        nt = 1024 if tuning["col_shared"] == 3 else 512
        return f"fw::c64::k_cols<{n}, {tuning['col_points']}, 0, {seq}, {nt}>"
    return f"fw::c64::k_rows<{n}, {tuning.get('row_points_inv') or tuning['row_points']}, true, 1>"


def _traffic_from_profiles(kernel_pass, tuning):
    """HBM bytes per launch from the committed counter summary, or None when the
    kernels (sources or the chosen variant) differ from those the counters saw."""
    path = COUNTERS
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        c = json.load(fh)
    if c.get("source_hash") != _kernel_source_hash():
        return None
    ent = c.get("passes", {}).get(str(kernel_pass), {}).get("instances", {}).get(_pass_instance(kernel_pass, tuning))
    return None if not ent else float(ent["hbm_bytes_per_launch"])


def build_workload():
    import numpy as np
    import workloads as W
    c = W.vti256_layered()
    rec = W.surface_receivers(c["nx"], NREC)
    m0 = W.model_scales(c["c0"], c["rho0"])
    dm = W.round_f32(m0 * W.smooth_maps(4, c["nz"], c["nx"], 10, 0.01)).astype(np.float32)
    r = W.round_f32(W.complex_normal(5, (c["nsys"], NREC, 2))).astype(np.complex64)
    return c, rec, dm, r


def multigrid(a):
    """Batching workload: 128^2 / 192^2 / 256^2 / 384^2 grids at 4 / 6 / 8 / 12 Hz over
    one 4800 m square, 64 surface forces each, in ONE plan (one graph per chunk).
    One step = incident fields + batched solve to 1e-6 of all 256 systems."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2402_02116_amd.plan import Plan
    probs = W.four_grids()
    plan = Plan([dict(nx=p["nx"], nz=p["nz"], dx=p["dx"], c0=p["c0"], rho0=p["rho0"],
                      freq_hz=p["freq_hz"], eta=p["eta"], nsys=p["nsys"]) for p in probs], device="cuda:0")
    for i, p in enumerate(probs):
        plan.set_contrast(i, p["maps"])
    if a.krylov == "gmres":
        plan.set_krylov("gmres", restart=a.restart, cgs2=not a.cgs1)
    src = sum((p["src_ixz"] for p in probs), [])
    frc = sum((p["src_f"] for p in probs), [])
    cells = np.array(sum(([p["nx"] * p["nz"]] * p["nsys"] for p in probs), []))

    def step():
        u0 = plan.incident(src, frc)
        res = plan.solve(u0, rtol=RTOL, maxit=1000)
        per = 1 if a.krylov == "gmres" else 2   # matvecs per iteration
        return int(np.sum((per * res.iters + 1) * cells)), res

    def solve_ms():
        u0 = plan.incident(src, frc)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plan.solve(u0, rtol=RTOL, maxit=1000)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3

    if a.passes_only:
        # counter runs: the tuned variants (same choices as a timed run), one
        # solve so that the GMRES state exists, the passes of every problem
        # and the Arnoldi-step kernels at steps 0, m/2 and m - 1, then the
        # 1 GiB device copy the counters are scaled by
        if not (a.no_autotune or a.tuning):
            plan.autotune(reps=10)
        _fixed_tuning(plan, a)
        step()
        rl = _pass_rooflines(plan, reps=a.reps)
        gl = _gmres_rooflines(plan, probs, a.restart, reps=a.reps) if a.krylov == "gmres" else None
        src_t = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        for _ in range(3):
            dst_t.copy_(src_t)
        torch.cuda.synchronize()
        print(json.dumps(dict(passes_only=True, pass_rooflines=rl, gmres_rooflines=gl,
                              tuning=[plan.tuning(i) for i in range(len(probs))])), flush=True)
        return 0

    tuning = None
    if not a.no_autotune:
        step()
        t_default = min(solve_ms() for _ in range(2))
        t0 = time.perf_counter()
        tuned = plan.autotune(reps=10)
        t_tune = time.perf_counter() - t0
        step()
        t_tuned = min(solve_ms() for _ in range(2))
        tuning = dict(tune_s=round(t_tune, 2), solve_ms_default=round(t_default, 3),
                      solve_ms_tuned=round(t_tuned, 3),
                      choices={str(p["nx"]): t for p, t in zip(probs, tuned)})
        print(f"[bench] autotune {t_tune:.2f} s: solve {t_default:.1f} ms (default variants) -> "
              f"{t_tuned:.1f} ms (tuned)", file=sys.stderr, flush=True)
        for p, t in zip(probs, tuned):
            print(f"[bench]   {p['nx']}^2: {t}", file=sys.stderr, flush=True)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pts = 0
    for _ in range(a.steps):
        n, res = step()
        pts += n
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    u0 = plan.incident(src, frc)
    t = time.perf_counter()
    res = plan.solve(u0, rtol=RTOL, maxit=1000)
    t_solve = (time.perf_counter() - t) * 1e3
    out = dict(metric=METRIC, value=round(pts / dt / 1e9, 3), unit="GPoints/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=round(dt / a.steps * 1e3, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="c64", data="synthetic",
               config=dict(workload="4 grids 128^2..384^2 (4, 6, 8, 12 Hz), 64 forces each, one plan: "
                                    "incident + batched solve to 1e-6",
                           grids=[p["nx"] for p in probs], nsys=int(len(src)), rtol=RTOL,
                           cells_per_matvec=int(cells.sum())),
               time_to_1e6_ms=round(t_solve, 3), iters=[int(res.iters.min()), int(res.iters.max())],
               max_true_relres=float(res.relres.max()), autotune=tuning,
               krylov=a.krylov if a.krylov == "bicgstab" else f"gmres({a.restart}, {'cgs1' if a.cgs1 else 'cgs2'})",
               pass_rooflines=_pass_rooflines(plan))
    if a.krylov == "gmres":
        out["gmres_rooflines"] = _gmres_rooflines(plan, probs, a.restart)
    if not a.no_cpu_baseline:
        per = 1 if a.krylov == "gmres" else 2
        mvs, k = [], 0
        for p in probs:
            mvs.append((p, int(np.sum(per * res.iters[k:k + p["nsys"]] + 1))))
            k += p["nsys"]
        out["cpu_baseline"] = cpu_extrapolated(mvs, "GPoints/s",
                                               lambda sec: sum(q["nx"] * q["nz"] * m for q, m in mvs) / sec / 1e9)
    print(json.dumps(out), flush=True)
    return 0


# algorithmic bytes per cell-system of the GMRES Arnoldi-step kernels at step
# j (complex64 2-D fields, 16 B per field per cell-system): the basis update
# reads w and the j + 1 basis vectors and writes w; the re-orthogonalisation
# projections read w and the j + 1 basis vectors; the inverse row transform
# with the projection epilogue reads the spectrum, w_j and the j + 1 basis
# vectors and writes w
GM_BYTES = {"update": lambda j: (j + 3) * 16.0, "dots": lambda j: (j + 2) * 16.0,
            "projections": lambda j: (j + 4) * 16.0}


def _gmres_rooflines(plan, probs, m, reps=10):
    """Time and algorithmic HBM rate of the Arnoldi-step kernels at the first,
    middle and last step of a cycle, every system running."""
    cs = sum(p["nsys"] * p["nx"] * p["nz"] for p in probs)
    out = []
    for j in sorted({0, m // 2, m - 1}):
        for kind, fb in GM_BYTES.items():
            us = plan.time_gmres_pass(kind, j, reps)
            nbytes = fb(j) * cs
            gbs = nbytes / (us * 1e-6) / 1e9
            out.append(dict(kernel=kind, j=j, us=round(us, 1), bytes=nbytes, gbs=round(gbs, 1),
                            frac=round(gbs / HBM_PEAK_GBS, 3)))
            print(f"[bench] GMRES {kind} at step {j}: {us:.1f} us, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f})",
                  file=sys.stderr, flush=True)
    return out


def _pass_rooflines(plan, reps=5):
    """Per-pass kernel time (HIP events around back-to-back launches on the
    plan's stream, all problems of the plan) and algorithmic HBM rate of one
    matvec, as fractions of the 8 TB/s peak."""
    import torch
    u = torch.randn(plan.field_elems, dtype=plan.cdtype, device=plan.device)
    Au = plan.new_field()
    out = []
    for k in range(4):
        nbytes = 0.0
        for i, p in enumerate(plan.problems):
            cells, ns = p["nx"] * p["nz"], p["nsys"]
            fused = plan.tuning(i)["fused_points"] != 0
            if k == 1 and fused:
                continue   # part of pass 0
            nbytes += PASS_BYTES[k] * ns * cells + (MAP_BYTES_PER_CELL * cells if k == 0 else 0.0)
        if nbytes == 0.0:
            continue
        for j in range(k):
            plan.apply_pass(j, u, Au)
        us = plan.time_pass(k, u, Au, reps)
        gbs = nbytes / (us * 1e-6) / 1e9
        out.append(dict(pass_=k, us=round(us, 1), gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 3)))
        print(f"[bench] pass {k}: {us:.1f} us, {gbs:.0f} GB/s algorithmic ({gbs / HBM_PEAK_GBS:.2f} of peak)",
              file=sys.stderr, flush=True)
    del u, Au
    return [{("pass" if k == "pass_" else k): v for k, v in d.items()} for d in out]


def _fixed_tuning(plan, a):
    """Apply --tuning (a JSON object for every problem, or a list with one
    object per problem); returns the plan's variants, or None without it."""
    if not a.tuning:
        return None
    fixed = json.loads(a.tuning)
    n = len(plan.problems)
    per = fixed if isinstance(fixed, list) else [fixed] * n
    if len(per) != n:
        raise SystemExit(f"--tuning: {len(per)} entries for {n} problems")
    for i, t in enumerate(per):
        plan.set_tuning(i, **{k: v for k, v in t.items() if k != "time_us"})
    return [plan.tuning(i) for i in range(n)]


def _tik_plan(probs, rec, krylov, a, precision="c64"):
    from paper_2402_02116_amd.plan import Plan
    plan = Plan([dict(nx=p["nx"], nz=p["nz"], dx=p["dx"], c0=p["c0"], rho0=p["rho0"], freq_hz=p["freq_hz"],
                      eta=p["eta"], nsys=p["nsys"]) for p in probs], device="cuda:0", precision=precision)
    for i, p in enumerate(probs):
        plan.set_contrast(i, p["maps"])
        plan.set_receivers(i, rec)
    if krylov == "gmres":
        plan.set_krylov("gmres", restart=a.restart, cgs2=not a.cgs1)
    tuned = None if (a.no_autotune or a.tuning) else plan.autotune(reps=5)
    return plan, _fixed_tuning(plan, a) or tuned


def jacobian(a):
    """Differentiation workload: 512^2 VTI at 5 m, 32 surface forces x (5, 8) Hz =
    64 systems, 101 receivers.  Times one J (m0 q), one J* r and one
    Tikhonov loss + gradient (J and J* together, Laplacian regulariser)."""
    import numpy as np
    import torch
    import workloads as W
    w = W.vti512_jacobian()
    probs, rec = w["problems"], w["rec_ixz"]
    plan, tuned = _tik_plan(probs, rec, a.krylov, a)
    src = sum((p["src_ixz"] for p in probs), [])
    frc = sum((p["src_f"] for p in probs), [])
    ub = plan.solve(plan.incident(src, frc), rtol=RTOL, maxit=2000).x
    m0v = w["m0"].ravel()
    q = torch.as_tensor(w["dq"], dtype=torch.float32).cuda()
    r = torch.as_tensor(np.concatenate([x.ravel() for x in w["r"]]).astype(np.complex64)).cuda()
    cells = np.array(sum(([p["nx"] * p["nz"]] * p["nsys"] for p in probs), []))
    per = 1 if a.krylov == "gmres" else 2

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3, int(np.sum((per * plan.solve_stats()[0] + 1) * cells))

    for _ in range(a.warmup):
        plan.tikhonov_grad(ub, r, m0v, q, lam=w["lam"], reg=w["reg"], rtol=RTOL)
    tj, pj = zip(*[timed(lambda: plan.frechet_rel(ub, q, m0v, rtol=RTOL)) for _ in range(a.steps)])
    ta, pa = zip(*[timed(lambda: plan.adjoint_rel(ub, r, m0v, rtol=RTOL)) for _ in range(a.steps)])
    tg = [timed(lambda: plan.tikhonov_grad(ub, r, m0v, q, lam=w["lam"], reg=w["reg"], rtol=RTOL))[0]
          for _ in range(a.steps)]
    ms = float(np.median(tg))
    pts = (np.median(pj) + np.median(pa)) / ms * 1e3 / 1e9
    out = dict(metric=METRIC, value=round(float(pts), 3), unit="GPoints/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=round(ms, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="c64", data="synthetic",
               config=dict(workload="512x512 VTI (dx 5 m), 32 surface forces x (5, 8) Hz, 101 receivers: "
                                    "Tikhonov loss + gradient (J and J*, Laplacian, lambda 1e-3) to 1e-6",
                           nsys=int(len(src)), rtol=RTOL),
               ms_per_J=round(float(np.median(tj)), 3), ms_per_Jstar=round(float(np.median(ta)), 3),
               ms_per_gradient=round(ms, 3), krylov=a.krylov, autotune=tuned)
    if not a.no_cpu_baseline:
        cell = probs[0]["nx"] * probs[0]["nz"]
        mv = int((np.median(pj) + np.median(pa)) / cell)
        out["cpu_baseline"] = cpu_extrapolated([(probs[0], mv)], "GPoints/s", lambda sec: mv * cell / sec / 1e9)
    print(json.dumps(out), flush=True)
    return 0


def _normal_run(w, a, precision, rtol, niter=20, chunk=5):
    """The linear DBI step of the 1024^2 workload on one plan of the given
    precision: background solve u^b, the perturbed model's solve u* (contrast
    q^b + dq*), data r = R u* - R u^b, then `niter` CG iterations on the
    Tikhonov normal equation from q = 0 in resumable chunks (fwils_normal_cg_steps).
    Returns a dict of timings, the residual history and every iterate (float64, host)."""
    import numpy as np
    import torch
    import workloads as W
    probs, rec = w["problems"], w["rec_ixz"]
    plan, tuned = _tik_plan(probs, rec, a.krylov, a, precision)
    src = sum((p["src_ixz"] for p in probs), [])
    frc = sum((p["src_f"] for p in probs), [])
    u0 = plan.incident(src, frc)
    t0 = time.perf_counter()
    bg = plan.solve(u0, rtol=rtol, maxit=3000, strict=True)
    ub = bg.x
    torch.cuda.synchronize()
    t_ub = time.perf_counter() - t0
    print(f"[bench] {precision} background solve of {len(src)} systems: {t_ub:.2f} s", file=sys.stderr, flush=True)
    m0 = w["m0"]
    maps_true = W.round_f32(probs[0]["maps"] + m0 * w["dq_true"])
    for i in range(len(probs)):
        plan.set_contrast(i, maps_true)
    ut = plan.solve(u0, rtol=rtol, maxit=3000, strict=True).x
    for i, p in enumerate(probs):
        plan.set_contrast(i, p["maps"])
    r = plan.receiver_data(ut) - plan.receiver_data(ub)
    del ut, u0
    torch.cuda.empty_cache()
    print(f"[bench] {precision} data r = R u(q^b + dq*) - R u^b from two forward solves", file=sys.stderr, flush=True)
    m0v = m0.ravel()
    hist = []
    iters = []
    times = []
    done = 0
    while done < niter:
        n = 1 if done == 0 else min(chunk, niter - done)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, h, qi = plan.normal_cg_steps(ub, r, m0v, done, n, lam=w["lam"], reg=w["reg"], rtol=rtol)
        torch.cuda.synchronize()
        times.append((n, time.perf_counter() - t))
        hist.extend(h.tolist() if done == 0 else h[1:].tolist())
        iters.append(qi.double().cpu().numpy())
        done += n
        print(f"[bench] {precision} normal CG: {done}/{niter} iterations, {times[-1][1]:.2f} s for the last {n}"
              f"{' (with the right-hand side J* r)' if n == 1 and done == 1 else ''}, residual {hist[-1]:.4e}",
              file=sys.stderr, flush=True)
    del ub, r
    rl = _pass_rooflines(plan) if precision == "c64" else None
    del plan
    torch.cuda.empty_cache()
    later = [(n, dt) for n, dt in times[1:]]
    per_iter = sum(dt for _, dt in later) / max(1, sum(n for n, _ in later))
    return dict(t_ub=t_ub, t_first=times[0][1], per_iter=per_iter, hist=np.array(hist),
                iterates=np.concatenate(iters), tuned=tuned, nsys=len(src), rooflines=rl, bg_iters=bg.iters)


def normal_cg(a):
    """Full linear DBI step: 1024^2 VTI at 5 m, 128 surface forces x (4, 7, 10) Hz =
    384 systems, 201 receivers; data r = R u(q^b + dq*) - R u^b from two forward
    solves about the smooth background; 20 CG iterations on the Tikhonov normal
    equation (L = I, lambda 1e-3) with FP64 CG scalars.  value = CG iterations per
    second over iterations 2..20.  With --fp64-reference the same step is run
    again in complex128 on the GPU, and the complex64 iterates and residual
    history are compared with it at every iteration."""
    import numpy as np
    import workloads as W
    w = W.vti1024_normal()
    if a.passes_only:
        # counter runs: the tuned passes of every problem, then the 1 GiB
        # device copy the counters are scaled by
        import torch
        plan, tuned = _tik_plan(w["problems"], w["rec_ixz"], a.krylov, a, "c64")
        rl = _pass_rooflines(plan, reps=a.reps)
        src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps(dict(passes_only=True, pass_rooflines=rl, tuning=tuned)), flush=True)
        return 0
    niter = w["cg_iters"] if a.cg_iters <= 0 else a.cg_iters
    r64 = _normal_run(w, a, "c64", RTOL, niter)
    ref = None
    if a.fp64_reference:
        r128 = _normal_run(w, a, "c128", 1e-10, niter)
        q64, q128 = r64["iterates"], r128["iterates"]
        e_q = [float(np.linalg.norm(q64[k] - q128[k]) / np.linalg.norm(q128[k])) for k in range(niter)]
        e_h = [float(abs(x - y) / abs(y)) for x, y in zip(r64["hist"], r128["hist"])]
        ref = dict(cg_iters=niter, rel_error_q_per_iteration=[float(f"{e:.3e}") for e in e_q],
                   rel_error_residual_per_iteration=[float(f"{e:.3e}") for e in e_h],
                   s_background_solve_c128=round(r128["t_ub"], 2), s_per_cg_iteration_c128=round(r128["per_iter"], 2),
                   rtol_c128=1e-10, residual_history_c128=[float(f"{h:.6e}") for h in r128["hist"]])
        print(f"[bench] complex64 vs complex128 GPU run, per iteration: q {ref['rel_error_q_per_iteration']}, "
              f"residual {ref['rel_error_residual_per_iteration']}", file=sys.stderr, flush=True)
    it = r64["per_iter"]
    out = dict(metric=METRIC, value=round(1.0 / it, 4), unit="CG iterations/s", n_gpus=1, steps=niter, warmup=0,
               ms_per_step=round(it * 1e3, 1), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="c64", data="synthetic",
               config=dict(workload="1024x1024 VTI (dx 5 m), 128 surface forces x (4, 7, 10) Hz, 201 receivers: "
                                    "20 CG iterations of the Tikhonov normal equation (L = I, lambda 1e-3), "
                                    "data R u(q^b + dq*) - R u^b",
                           nsys=int(r64["nsys"]), rtol=RTOL, cg_iters=niter),
               s_background_solve=round(r64["t_ub"], 2), s_first_cg_iteration_with_rhs=round(r64["t_first"], 2),
               residual_history=[float(f"{h:.6e}") for h in r64["hist"]],
               krylov=a.krylov, autotune=r64["tuned"], fp64_gpu_reference=ref, pass_rooflines=r64["rooflines"])
    if not a.no_cpu_baseline:
        # one CG iteration is two solves per system (J and J*), each taken to
        # cost the background solve's matvecs
        per = 1 if a.krylov == "gmres" else 2
        mvs, k = [], 0
        for p in w["problems"]:
            mvs.append((p, 2 * int(np.sum(per * r64["bg_iters"][k:k + p["nsys"]] + 1))))
            k += p["nsys"]
        out["cpu_baseline"] = cpu_extrapolated(mvs, "CG iterations/s", lambda sec: 1.0 / sec)
    print(json.dumps(out), flush=True)
    return 0


# algorithmic bytes per cell-system of the 3-D passes (complex64, three
# components: 24 B per field): stencil u -> b; x transforms; the y forward, z
# forward-Green-inverse and y inverse transforms (three kernels); inverse x
# transforms reading the spectrum and u and writing A u
PASS3_BYTES = (48.0, 48.0, 3 * 48.0, 72.0)
PASS3_NAMES = ("k_stencil3 (contrast stencil, six strains)", "k_rows (x transforms)",
               "k_axis y / z with 3x3 G_hat / y (three kernels)", "k_rows (inverse x transforms + LS epilogue)")


def hess3d(a):
    """3-D workload: the 80 x 40 x 32 grid of 25 m cells of the paper's modified
    3-D VTI Hess example (a layered stand-in model), 100 vertical surface forces
    at 7 Hz, 400 surface receivers.  Step = incident fields + batched solve to
    1e-6 + J dm (six VTI maps) + J* r (FP64 maps); value = sustained LS-matvec
    rate (cell-systems per second)."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2402_02116_amd.plan import Plan3
    torch.cuda.set_device(0)
    w = W.hess3d_vti()
    nx, ny, nz, ns = w["nx"], w["ny"], w["nz"], w["nsys"]
    cells = nx * ny * nz
    plan = Plan3([dict(nx=nx, ny=ny, nz=nz, dx=w["dx"], c0=w["c0"], rho0=w["rho0"], freq_hz=w["freq_hz"],
                       eta=w["eta"], nsys=ns, params="vti")], device="cuda:0")
    plan.set_contrast(0, w["maps"])
    plan.set_receivers(0, w["rec_ixyz"])
    if a.krylov == "gmres":
        plan.set_krylov("gmres", restart=a.restart, cgs2=not a.cgs1)
    per = 1 if a.krylov == "gmres" else 2
    dm = torch.as_tensor(W.round_f32(W.contrast3(13, nz, ny, nx, w["scales"], ell=3.0, std=0.01)),
                         dtype=torch.float32).cuda()
    r = torch.as_tensor(W.round_f32(W.complex_normal(14, (ns, len(w["rec_ixyz"]), 3))).astype(np.complex64)
                        .ravel()).cuda()

    def step():
        u0 = plan.incident(w["src_ixyz"], w["src_f"])
        res = plan.solve(u0, rtol=RTOL, maxit=1500)
        n1 = int(np.sum(per * res.iters + 1))
        plan.frechet(res.x, [dm], rtol=RTOL)
        n2 = int(np.sum(per * plan.solve_stats()[0] + 1))
        plan.adjoint(res.x, r, rtol=RTOL)
        n3 = int(np.sum(per * plan.solve_stats()[0] + 1))
        return n1 + n2 + n3, res

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv = 0
    for _ in range(a.steps):
        n, res = step()
        mv += n
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = mv * cells / dt / 1e9
    print(f"[bench] hess3d {a.steps} steps: {dt / a.steps * 1e3:.2f} ms/step, {mv / a.steps:.0f} matvecs/step, "
          f"{value:.3f} GPoints/s, iterations {res.iters.min()}-{res.iters.max()}", file=sys.stderr, flush=True)
    u = res.x
    Au = plan.new_field()
    passes = []
    for k in range(4):
        for j in range(k):
            plan.apply_pass(j, u, Au)
        us = plan.time_pass(k, u, Au, a.reps)
        nbytes = PASS3_BYTES[k] * ns * cells + (24.0 * cells if k == 0 else 0.0)
        gbs = nbytes / (us * 1e-6) / 1e9
        passes.append(dict(pass_=k, kernel=PASS3_NAMES[k], us=round(us, 2), bytes=nbytes, gbs=round(gbs, 1),
                           frac=round(gbs / HBM_PEAK_GBS, 3)))
        print(f"[bench] hess3d pass {k} {PASS3_NAMES[k]}: {us:.1f} us, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.2f})",
              file=sys.stderr, flush=True)
    single = [p for p in passes if p["pass_"] != 2]
    dom = max(single, key=lambda p: p["us"])
    out = dict(metric=METRIC, value=round(value, 3), unit="GPoints/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=round(dt / a.steps * 1e3, 3), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="c64", data="synthetic",
               config=dict(workload="80x40x32 VTI (dx 25 m), layered stand-in for the modified 3-D Hess model, "
                                    "100 surface forces, 7 Hz, 400 receivers: incident + solve + J + J* to 1e-6",
                           grid=[nx, ny, nz], nsys=ns, nrec=len(w["rec_ixyz"]), rtol=RTOL),
               roofline=dict(bound="hbm", kernel=dom["kernel"], achieved=dom["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(dom["gbs"] / HBM_PEAK_GBS, 4), traffic=None,
                             bytes_per_launch=dom["bytes"], avg_launch_us=dom["us"]),
               pass_rooflines=[{("pass" if k == "pass_" else k): v for k, v in p.items()} for p in passes],
               krylov=a.krylov)
    if not a.no_cpu_baseline:
        from oracle import elastic3d as E3, operators
        P = E3.LSProblem3D(nx, ny, nz, w["dx"], w["c0"], w["rho0"], w["freq_hz"], w["eta"], maps=w["maps"],
                           params="vti")
        u1 = np.ones((1, 3, nz, ny, nx), dtype=complex)
        P.apply(u1)
        t = time.perf_counter()
        for _ in range(2):
            P.apply(u1)
        t_mv = (time.perf_counter() - t) / 2
        mvs = mv // a.steps
        out["cpu_baseline"] = dict(value=cells / t_mv / 1e9, unit="GPoints/s", cores=operators._WORKERS,
                                   kind="oracle, extrapolated", cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
                                   seconds=round(mvs * t_mv, 1),
                                   sample=f"one measured 3-D oracle matvec (complex128, one system) "
                                          f"{t_mv * 1e3:.1f} ms, times the {mvs} matvecs of one GPU step")
    print(json.dumps(out), flush=True)
    return 0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_step(c, rec, dm, r, nsample):
    """The oracle through one step (incident, solve, J, J*) on the first
    nsample systems: (matvecs, seconds)."""
    import numpy as np
    from oracle import LSProblem, operators
    P = LSProblem(c["nx"], c["nz"], c["dx"], c["c0"], c["rho0"], c["freq_hz"], c["eta"], c["maps"])
    src, f = c["src_ixz"][:nsample], c["src_f"][:nsample]
    t = time.perf_counter()
    u0 = P.incident(src, f)
    ub, i1 = P.solve(u0, tol=RTOL)
    w, i2 = P.solve(P.convolve(P.virtual_source(ub, dm.astype(np.float64))), tol=RTOL)
    operators.sample(w, rec)
    fa = operators.sample_transpose(np.conj(r[:nsample].astype(np.complex128)), rec, c["nx"], c["nz"])
    ua, i3 = P.solve(P.convolve(fa), tol=RTOL)
    P.correlate(ua, ub)
    dt = time.perf_counter() - t
    return sum(2 * i.iters + 1 for i in i1 + i2 + i3), dt


def cpu_baseline(c, rec, dm, r, nsample):
    """The oracle on the host cores, on `nsample` of the systems of one step,
    with its scipy.fft workers (at most 16, one GPU's share of the box), and
    again on two systems with one thread (scipy.fft workers and BLAS)."""
    from threadpoolctl import threadpool_limits
    from oracle import operators
    mv, dt = _oracle_step(c, rec, dm, r, nsample)
    saved = operators._WORKERS
    try:
        operators._WORKERS = 1
        with threadpool_limits(limits=1):
            mv1, dt1 = _oracle_step(c, rec, dm, r, 2)
    finally:
        operators._WORKERS = saved
    cells = c["nx"] * c["nz"]
    return dict(value=mv * cells / dt / 1e9, unit="GPoints/s", cores=saved, kind="oracle",
                cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
                sample=f"{nsample} of the {c['nsys']} systems through the whole step (incident, solve, "
                       f"J, J*), complex128 numpy/scipy, {mv} matvecs in {dt:.1f} s",
                one_core=dict(value=mv1 * cells / dt1 / 1e9, unit="GPoints/s", cores=1,
                              sample=f"2 systems through the whole step, one thread, {mv1} matvecs in {dt1:.1f} s"))


def oracle_matvec_seconds(nx, nz, dx, c0, rho0, freq_hz, maps, reps=2):
    """Seconds of one oracle LS matvec (complex128, one system) on the host."""
    import numpy as np
    from oracle import LSProblem
    P = LSProblem(nx, nz, dx, c0, rho0, freq_hz, 0.02, maps)
    u = np.ones((1, 2, nz, nx), dtype=complex)
    P.apply(u)
    t = time.perf_counter()
    for _ in range(reps):
        P.apply(u)
    return (time.perf_counter() - t) / reps


def cpu_extrapolated(grids_matvecs, unit, value_fn):
    """The oracle's time for the matvecs a GPU run made, extrapolated from one
    measured oracle matvec per grid: grids_matvecs = [(problem dict, matvecs)].
    value_fn(seconds) gives the value in the bench line's unit."""
    from oracle import operators
    secs = 0.0
    parts = []
    for p, mv in grids_matvecs:
        t = oracle_matvec_seconds(p["nx"], p["nz"], p["dx"], p["c0"], p["rho0"], p["freq_hz"], p["maps"])
        secs += mv * t
        parts.append(f"{p['nx']}x{p['nz']}: {t * 1e3:.1f} ms x {mv}")
    return dict(value=value_fn(secs), unit=unit, cores=operators._WORKERS, kind="oracle, extrapolated",
                cpu_model=_cpu_model(), host_cpus=os.cpu_count(), seconds=round(secs, 1),
                sample="one measured oracle matvec (complex128, one system) per grid times the matvecs of this "
                       "GPU run: " + "; ".join(parts))


def _dbi_run(a, w, precision):
    """The sequential inversion of workload w in one precision: (final contrast
    as float64 numpy, per-stage records, seconds of the timed inversion,
    autotune choice).  Observed data come from forward solves in the true
    model in complex64 (both precisions invert the same data values)."""
    import numpy as np
    import torch
    from paper_2402_02116_amd.dbi import invert_sequential
    from paper_2402_02116_amd.plan import Plan
    nsrc = len(w["src_ixz"])
    plans, d_obs, tuned = [], [], None
    for f in w["freqs"]:
        mk = lambda prec: Plan([dict(nx=w["nx"], nz=w["nz"], dx=w["dx"], c0=w["c0"], rho0=w["rho0"],
                                     freq_hz=f, eta=w["eta"], nsys=nsrc)], device="cuda:0", precision=prec)
        plan = mk(precision)
        plan.set_receivers(0, w["rec"])
        if a.krylov == "gmres":
            plan.set_krylov("gmres", restart=a.restart, cgs2=not a.cgs1)
        if not a.no_autotune:   # one grid: the first plan's choice serves every frequency
            if tuned is None:
                tuned = plan.autotune(reps=5)
            else:
                plan.set_tuning(0, **{k: v for k, v in tuned[0].items() if k != "time_us"})
        fwd = plan if precision == "c64" else mk("c64")
        if fwd is not plan:
            fwd.set_receivers(0, w["rec"])
        fwd.set_contrast(0, w["c_true"])
        u = fwd.solve(fwd.incident(w["src_ixz"], w["src_f"]), rtol=1e-7, maxit=5000).x
        d_obs.append(fwd.receiver_data(u).to(plan.cdtype))
        del u, fwd
        plans.append(plan)
    torch.cuda.synchronize()
    print(f"[bench] dbi ({precision}): observed data at {len(plans)} frequencies", file=sys.stderr, flush=True)
    t = time.perf_counter()
    c, stages = invert_sequential(plans, w["src_ixz"], w["src_f"], d_obs, w["c_start"], w["m0"],
                                  lam0=a.dbi_lambda, niter=a.dbi_cg, tol=1e-3, max_outer=10,
                                  rtol=RTOL if precision == "c64" else 1e-10, maxit=5000)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t
    for st in stages:
        print(f"[bench] dbi {precision} {st['freq_hz']:4.1f} Hz: {st['updates']} updates, eps_d {st['eps'][0]:.4f} -> "
              f"{st['eps'][-1]:.4f}", file=sys.stderr, flush=True)
    c = c.double().cpu().numpy()
    del plans, d_obs
    torch.cuda.empty_cache()
    return c, stages, secs, tuned


def dbi_inversion(a):
    """Distorted-Born inversion shaped like the paper's 2-D VTI reservoir
    example: 192 x 48 cells of 20 m, 48 surface forces, 96 receivers, nine
    frequencies 3..19 Hz inverted one after the other, each stage stopping at
    eps_d < 1e-3 or after 10 updates, --dbi-cg CG iterations per update
    (lambda0 --dbi-lambda, self-adaptive cooling).  Observed data come from
    forward solves in the true model (before the timed region); the timed
    region is the whole sequential inversion from the smoothed model.  With
    --fp64-reference the inversion is repeated in complex128 and the
    complex64 model's error against it reported."""
    import numpy as np
    import workloads as W
    w = W.reservoir_dbi()
    nsrc = len(w["src_ixz"])
    c, stages, secs, tuned = _dbi_run(a, w, "c64")
    m0 = w["m0"].reshape(5, 1, 1)
    m_true, m_start, m_end = m0 + w["c_true"], m0 + w["c_start"], m0 + c
    eps_m = [float(np.linalg.norm(m[p] - m_true[p]) / np.linalg.norm(m_true[p])) for m in (m_start, m_end)
             for p in range(5)]
    updates = sum(st["updates"] for st in stages)
    ref = None
    if a.fp64_reference:
        c128, st128, secs128, _ = _dbi_run(a, w, "c128")
        ref = dict(s_total_c128=round(secs128, 2), updates_c128=sum(st["updates"] for st in st128),
                   rel_error_model=[round(float(np.linalg.norm(c[p] - c128[p]) / np.linalg.norm(m0[p] + c128[p])), 9)
                                    for p in range(5)],
                   rel_error_contrast=float(np.linalg.norm(c - c128) / np.linalg.norm(c128)),
                   eps_last_c128=[round(st["eps"][-1], 6) for st in st128], rtol_c128=1e-10)
        print(f"[bench] dbi complex64 vs complex128: {ref}", file=sys.stderr, flush=True)
    out = dict(metric=METRIC, value=round(updates / secs, 3), unit="DBI updates/s", n_gpus=1, steps=1, warmup=0,
               ms_per_step=round(secs * 1e3, 1), higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype="c64", data="synthetic",
               config=dict(workload="192x48 VTI (dx 20 m), random-layered true model, smoothed start, "
                                    "48 surface forces, 96 receivers, 3..19 Hz sequential DBI "
                                    "(eps_d < 1e-3 or 10 updates per frequency)",
                           nsys=nsrc, cg_iters=a.dbi_cg, lambda0=a.dbi_lambda, rtol=RTOL),
               updates=updates, s_total=round(secs, 2), ms_per_update=round(secs * 1e3 / max(updates, 1), 1),
               stages=[dict(freq_hz=st["freq_hz"], updates=st["updates"], eps_first=round(st["eps"][0], 5),
                            eps_last=round(st["eps"][-1], 5)) for st in stages],
               eps_m_start=[round(x, 5) for x in eps_m[:5]], eps_m_end=[round(x, 5) for x in eps_m[5:]],
               krylov=a.krylov, autotune=tuned, fp64_gpu_reference=ref)
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=50, help="launches per kernel timing")
    ap.add_argument("--cpu-sample", type=int, default=12, help="systems in the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in kernel variants")
    ap.add_argument("--tuning", default="", help="kernel variants as JSON (fwils_tuning fields): one object for "
                                                 "every problem or a list with one per problem; replaces the "
                                                 "autotuner's choice (default, normal, multigrid --passes-only)")
    ap.add_argument("--krylov", choices=["auto", "bicgstab", "gmres"], default="auto",
                    help="auto: GMRES(32) with one Gram-Schmidt pass for the four-grid workload (hard "
                         "12 Hz systems), BiCGSTAB for the others (1.7x faster than GMRES on the dbi "
                         "workload, whose small systems make the Arnoldi projections dominate)")
    ap.add_argument("--restart", type=int, default=0,
                    help="GMRES restart length (<= 32); default 16 for the four-grid workload (the fastest of "
                         "8..32 there), 32 otherwise")
    ap.add_argument("--cgs1", action="store_true", help="GMRES without the re-orthogonalisation pass")
    ap.add_argument("--cgs2", action="store_true", help="GMRES with the re-orthogonalisation pass")
    ap.add_argument("--workload", choices=["vti256x16", "multigrid", "jacobian", "normal", "dbi", "hess3d"],
                    default="vti256x16")
    ap.add_argument("--dbi-cg", type=int, default=10, help="dbi workload: CG iterations per model update")
    ap.add_argument("--dbi-lambda", type=float, default=1e-2, help="dbi workload: initial lambda")
    ap.add_argument("--fp64-reference", action="store_true",
                    help="normal / dbi workloads: rerun in complex128 on the GPU and report the complex64 error")
    ap.add_argument("--cg-iters", type=int, default=0,
                    help="normal workload: CG iterations (default: the workload's 20)")
    ap.add_argument("--passes-only", action="store_true",
                    help="only the per-pass kernel launches and the 1 GiB copy (for counter runs)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/counters_vti256x16.json from two rocprofv3 --pmc runs")
    ap.add_argument("--counter-command", default="", help="the rocprofv3 command, recorded in the summary")
    ap.add_argument("--counters-out", default=None, help="summary file (default profiles/counters_vti256x16.json)")
    a = ap.parse_args(argv)
    if a.restart <= 0:
        a.restart = 16 if a.workload == "multigrid" else 32
    if a.summarize_counters and a.workload == "multigrid":
        return summarize_multigrid_counters(a.summarize_counters[0], a.summarize_counters[1], a.counter_command,
                                            a.restart, a.reps, a.counters_out or os.path.join(ROOT, "profiles",
                                                                                     "counters_multigrid.json"))
    if a.summarize_counters:
        return summarize_counters(a.summarize_counters[0], a.summarize_counters[1], a.counter_command,
                                  a.counters_out)
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (the path shards "
              f"independent (source, frequency) systems across GPUs, one process per GPU)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2402_02116_amd.plan import Plan

    torch.cuda.set_device(0)
    if a.krylov == "auto":
        a.krylov = "gmres" if a.workload == "multigrid" else "bicgstab"
        a.cgs1 = a.cgs1 or not a.cgs2
    elif a.cgs2:
        a.cgs1 = False
    if a.workload == "multigrid":
        return multigrid(a)
    if a.workload == "jacobian":
        return jacobian(a)
    if a.workload == "normal":
        return normal_cg(a)
    if a.workload == "dbi":
        return dbi_inversion(a)
    if a.workload == "hess3d":
        return hess3d(a)
    c, rec, dm_np, r_np = build_workload()
    nx, nz, ns = c["nx"], c["nz"], c["nsys"]
    cells = nx * nz
    plan = Plan([dict(nx=nx, nz=nz, dx=c["dx"], c0=c["c0"], rho0=c["rho0"], freq_hz=c["freq_hz"],
                      eta=c["eta"], nsys=ns)], device="cuda:0")
    plan.set_contrast(0, c["maps"])
    plan.set_receivers(0, rec)
    if a.krylov == "gmres":
        plan.set_krylov("gmres", restart=a.restart, cgs2=not a.cgs1)
    mv_per_iter = 1 if a.krylov == "gmres" else 2
    tuning = None
    if not a.no_autotune:
        t0 = time.perf_counter()
        tuning = dict(choice=plan.autotune(reps=20)[0])
        tuning["tune_s"] = round(time.perf_counter() - t0, 2)
        print(f"[bench] autotune: {tuning}", file=sys.stderr, flush=True)
    if a.tuning:
        # fixed kernel variants (a profiled run repeats a timed run's choice:
        # a profiler's overhead can change what the autotuner picks)
        tuning = dict(choice=_fixed_tuning(plan, a)[0], fixed=True)
        print(f"[bench] fixed variants: {tuning}", file=sys.stderr, flush=True)
    dm = torch.as_tensor(dm_np).cuda()
    r = torch.as_tensor(r_np.ravel()).cuda()

    if a.passes_only:
        tbr = SimpleNamespace(x=plan.incident(c["src_ixz"], c["src_f"]))
    else:
        def step():
            u0 = plan.incident(c["src_ixz"], c["src_f"])
            res = plan.solve(u0, rtol=RTOL, maxit=1000)
            n1 = int(np.sum(mv_per_iter * res.iters + 1))
            plan.frechet(res.x, [dm], rtol=RTOL)
            n2 = int(np.sum(mv_per_iter * plan.solve_stats()[0] + 1))
            plan.adjoint(res.x, r, rtol=RTOL)
            n3 = int(np.sum(mv_per_iter * plan.solve_stats()[0] + 1))
            return n1 + n2 + n3

        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mv = 0
        for _ in range(a.steps):
            mv += step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms_step = dt / a.steps * 1e3
        value = mv * cells / dt / 1e9
        print(f"[bench] {a.steps} steps: {ms_step:.3f} ms/step, {mv / a.steps:.0f} matvecs/step, "
              f"{value:.2f} GPoints/s sustained", file=sys.stderr, flush=True)

        # time-to-1e-6: batched graph solve vs plain per-source solve
        u0 = plan.incident(c["src_ixz"], c["src_f"])
        def timed_solve(**kw):
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = plan.solve(u0, rtol=RTOL, maxit=1000, **kw)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3, res
        plain_krylov = a.krylov
        for _ in range(2):
            timed_solve()
        tb = sorted(timed_solve()[0] for _ in range(5))
        tbr = timed_solve()[1]
        if a.krylov == "gmres":   # the per-source plain loop is BiCGSTAB's
            plan.set_krylov("bicgstab")
            plain_krylov = "bicgstab"
        for _ in range(2):
            timed_solve(plain=True)
        tp = sorted(timed_solve(plain=True)[0] for _ in range(3))
        tpr = timed_solve(plain=True)[1]
        same = bool(torch.equal(tbr.x, tpr.x))
        print(f"[bench] time to 1e-6: batched {tb[len(tb) // 2]:.3f} ms, plain {tp[len(tp) // 2]:.3f} ms, "
              f"iters {tbr.iters.min()}-{tbr.iters.max()}, max true relres {tbr.relres.max():.2e}, "
              f"identical results {same}", file=sys.stderr, flush=True)
        # the batching gain alone: the same solves one source at a time through
        # the graph-chunked path of a one-system plan with the same variants
        # (no per-iteration host round trip, unlike the plain loop)
        plan1 = Plan([dict(nx=nx, nz=nz, dx=c["dx"], c0=c["c0"], rho0=c["rho0"], freq_hz=c["freq_hz"],
                           eta=c["eta"], nsys=1)], device="cuda:0")
        plan1.set_contrast(0, c["maps"])
        plan1.set_tuning(0, **{k: v for k, v in plan.tuning(0).items() if k != "time_us"})
        if a.krylov == "gmres":
            plan1.set_krylov("gmres", restart=a.restart, cgs2=not a.cgs1)
        u0s = [plan1.incident([c["src_ixz"][k]], [c["src_f"][k]]) for k in range(ns)]
        def per_source_graph():
            torch.cuda.synchronize()
            t = time.perf_counter()
            its = [int(plan1.solve(u, rtol=RTOL, maxit=1000).iters[0]) for u in u0s]
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3, its
        per_source_graph()
        tg = sorted(per_source_graph()[0] for _ in range(3))
        del plan1, u0s
        print(f"[bench] time to 1e-6, one source at a time through the graph path: {tg[1]:.3f} ms",
              file=sys.stderr, flush=True)

    # isolated batched matvec and its four kernels, HIP events on the plan's stream
    u = tbr.x
    Au = plan.new_field()
    stream = torch.cuda.current_stream()
    def event_time(fn, reps):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    t_apply = event_time(lambda: plan.apply(u, out=Au), a.reps)
    # the kernels of one matvec under the chosen variants: with the stencil
    # fused into the forward rows, pass 1 launches nothing
    fused = plan.tuning(0)["fused_points"] != 0
    passes = [0, 2, 3] if fused else [0, 1, 2, 3]
    names = [FUSED_NAME if (fused and k == 0) else PASS_NAMES[k] for k in passes]
    t_pass = []
    for k in passes:
        for j in range(k):
            plan.apply_pass(j, u, Au)
        t_pass.append(plan.time_pass(k, u, Au, a.reps) * 1e-3)   # ms per launch
    matvec_gps = ns * cells / (t_apply * 1e-3) / 1e9
    bytes_per_launch = [PASS_BYTES[k] * ns * cells + (MAP_BYTES_PER_CELL * cells if k == 0 else 0.0)
                        for k in passes]
    gbs = [bytes_per_launch[i] / (t_pass[i] * 1e-3) / 1e9 for i in range(len(passes))]
    # the direction-update mode of the fused kernel, the largest kernel of a
    # BiCGSTAB iteration and of the step: every system running, continuing
    # from the state of a solve stopped after a few iterations
    t_px = px_bytes = None
    if fused and a.krylov == "bicgstab":
        plan.solve(plan.incident(c["src_ixz"], c["src_f"]), rtol=1e-12, maxit=8)
        t_px = plan.time_krylov_pass(a.reps) * 1e-3   # ms per launch
        px_bytes = PX_BYTES * ns * cells + MAP_BYTES_PER_CELL * cells
        print(f"[bench] direction-update pass {PX_NAME.split(',')[0]}: {t_px * 1e3:.2f} us/launch, "
              f"{px_bytes / (t_px * 1e-3) / 1e9:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    # the roofline is stated for that kernel (for the matvec's stencil pass
    # when the stencil and the rows run apart, or under GMRES)
    if t_px is not None:
        roof_name, roof_bytes, roof_ms = PX_NAME, px_bytes, t_px
        traffic = _traffic_from_profiles(PX_PASS, plan.tuning(0))
    else:
        roof_name, roof_bytes, roof_ms = names[0], bytes_per_launch[0], t_pass[0]
        traffic = _traffic_from_profiles(passes[0], plan.tuning(0))
    roof_gbs = roof_bytes / (roof_ms * 1e-3) / 1e9
    for i, k in enumerate(passes):
        print(f"[bench] pass {k} {names[i]}: {t_pass[i] * 1e3:.2f} us/launch, "
              f"{gbs[i]:.0f} GB/s algorithmic", file=sys.stderr, flush=True)
    mv_bytes = sum(bytes_per_launch)
    print(f"[bench] batched matvec: {t_apply * 1e3:.2f} us, {matvec_gps:.2f} GPoints/s, "
          f"{mv_bytes / (t_apply * 1e-3) / 1e9:.0f} GB/s over its {len(passes)} kernels", file=sys.stderr,
          flush=True)

    # attainable device bandwidth: a plain 1 GiB device-to-device copy (also the
    # reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)
    src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t_copy = event_time(lambda: dst.copy_(src), 10)
    copy_gbs = 2 * src.numel() * 4 / (t_copy * 1e-3) / 1e9
    del src, dst
    print(f"[bench] device copy 1 GiB: {t_copy * 1e3:.1f} us, {copy_gbs:.0f} GB/s (read + write)",
          file=sys.stderr, flush=True)

    if a.passes_only:
        # every candidate variant of every pass, so that the counter summary
        # covers whichever variant the autotuner picks in a timed run
        chosen = plan.tuning(0)
        for k, kind in ((0, "stencil"), (0, "fuse"), (1, "rows"), (2, "cols"), (3, "rows")):
            for cand in plan.tuning_candidates(0, kind):
                if kind != "fuse":
                    cand = dict(cand, fused_points=0)   # the separate stencil and row kernels
                plan.set_tuning(0, **cand)
                for j in range(k):
                    plan.apply_pass(j, u, Au)
                for _ in range(a.reps):
                    plan.apply_pass(k, u, Au)
                if kind == "fuse" and a.krylov == "bicgstab":
                    # the direction-update mode of this fused variant
                    plan.solve(plan.incident(c["src_ixz"], c["src_f"]), rtol=1e-12, maxit=8)
                    plan.time_krylov_pass(a.reps)
        plan.set_tuning(0, **{f: chosen[f] for f in chosen if f != "time_us"})
        torch.cuda.synchronize()
        print(json.dumps(dict(passes_only=True, pass_us=[round(t * 1e3, 3) for t in t_pass],
                              pass_gbs=[round(g, 1) for g in gbs], copy_gbs=round(copy_gbs, 1),
                              tuning=plan.tuning(0))), flush=True)
        return 0
    # the batched solve as a whole: algorithmic bytes of its BiCGSTAB iterations
    # (every system's own count) over its wall time, set-up and checks included
    solve_bw = None
    if a.krylov == "bicgstab":
        per = ITER_BYTES_FUSED if plan.tuning(0)["fused_points"] else ITER_BYTES_SPLIT
        sbytes = float(np.sum(tbr.iters)) * per * cells
        sgbs = sbytes / (tb[len(tb) // 2] * 1e-3) / 1e9
        solve_bw = dict(bytes=sbytes, ms=round(tb[len(tb) // 2], 3), gbs=round(sgbs, 1),
                        frac=round(sgbs / HBM_PEAK_GBS, 4), bytes_per_iteration_per_cell=per)
    # the 256^2 working set (about 170 MB) fits the 256 MB Infinity Cache: the
    # counter traffic is L2 <-> memory-side traffic, an upper bound on the HBM
    # bytes, and the fraction is stated against the measured copy rate as well
    roof = dict(bound="hbm", kernel=roof_name, achieved=round(roof_gbs, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(roof_gbs / HBM_PEAK_GBS, 4),
                traffic=None if traffic is None else round(traffic, 1),
                bytes_per_launch=roof_bytes, avg_launch_us=round(roof_ms * 1e3, 3),
                frac_of_copy=round(roof_gbs / copy_gbs, 4),
                note="traffic = L2-miss bytes (FETCH_SIZE + WRITE_SIZE), an upper bound on HBM bytes: "
                     "the working set fits the Infinity Cache")
    out = dict(metric=METRIC, value=round(value, 3), unit="GPoints/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=round(ms_step, 4), higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="c64", data="synthetic",
               config=dict(workload="256x256 VTI (dx 8 m), random-layered contrast, 16 surface forces, "
                                    "5 Hz, 128 receivers: incident + solve + J + J* to 1e-6",
                           grid=[nz, nx], nsys=ns, freq_hz=c["freq_hz"], rtol=RTOL, nrec=NREC),
               roofline=roof,
               krylov=a.krylov if a.krylov == "bicgstab" else f"gmres({a.restart}, {'cgs1' if a.cgs1 else 'cgs2'})",
               time_to_1e6_ms=dict(batched=round(tb[len(tb) // 2], 3), plain=round(tp[len(tp) // 2], 3),
                                   plain_krylov=plain_krylov,
                                   speedup=round(tp[len(tp) // 2] / tb[len(tb) // 2], 2),
                                   per_source_graph=round(tg[1], 3),
                                   speedup_vs_per_source_graph=round(tg[1] / tb[len(tb) // 2], 2),
                                   iters=[int(tbr.iters.min()), int(tbr.iters.max())],
                                   max_true_relres=float(tbr.relres.max()), identical=same,
                                   criterion="recursive residual <= 1e-6 and true residual <= 2e-6"),
               solve_bandwidth=solve_bw,
               copy_gbs=round(copy_gbs, 1), autotune=tuning,
               matvec=dict(gpoints_s=round(matvec_gps, 3), us=round(t_apply * 1e3, 3),
                           kernels=names, pass_us=[round(t * 1e3, 3) for t in t_pass],
                           pass_gbs=[round(g, 1) for g in gbs]))
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, rec, dm_np, r_np, a.cpu_sample)
        print(f"[bench] cpu oracle: {out['cpu_baseline']}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
