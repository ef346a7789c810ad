#!/usr/bin/env python3
"""Benchmark of the separable Helmholtz solver on one MI355X.

Workload (one step = one full solve of the decomposed grid):
  uniform core 256 x 256 (h = 1) + 16 PML cells per side (steps 1.2^k (1+0.5i)),
  287 x 287 interior nodes, nz = 200 in 20 layers, 4 x 4 blocks (separators at
  15, 143, 271 on x and y) solved by the two-level interface reduction;
  unit point source at the grid centre; complex128.  Inputs are resident in
  HBM before the timed region.

Prints one JSON line: unknowns*RHS/s of the complex128 solve, the mixed
complex64 + FP64-refinement solve beside it, the roofline of the dominant
kernel from hipEvents recorded on the solve's stream, and the FP64 CPU oracle
timed on the host.  The same line carries two more workloads, each in
complex128 and in mixed precision: 64 independent blocks of uneven sizes with
8 right-hand sides each as one captured graph per solve ("batched_c3"), and
the large 575 x 575 x 256 grid with 16 point sources at 4 frequencies
("large_c5"); and the time of one adjoint gradient with respect to the layer
values of k^2 on the 128 x 128 x 160 grid ("adjoint_c4").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12            # B/s
PEAK_F64 = 78.6e12           # flop/s, FP64 vector = FP64 MFMA on MI355X
PEAK_F32 = 157.3e12          # flop/s, FP32


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(os.path.join(ROOT, "paper_1909_01299_amd", "csrc"))):
        with open(os.path.join(ROOT, "paper_1909_01299_amd", "csrc", name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def time_solves(plan, f, u, steps, warmup, profile=True):
    """Wall time of `steps` solves.  With profile: an untimed run of as many
    solves with hipEvents around every stage (on the solve's stream) gives the
    stage table and the dominant stage; in the timed run only that stage is
    bracketed by events (two per solve), so its kernel time is measured over
    the timed region itself.  Returns (seconds, stage table, dominant stage
    record from the timed region)."""
    import torch
    for _ in range(warmup):
        plan.solve(f, out=u)
    torch.cuda.synchronize()
    stages, dom = [], None
    if profile:
        plan.profile(True)
        plan.profile_read()          # reset accumulators
        for _ in range(steps):
            plan.solve(f, out=u)
        torch.cuda.synchronize()
        stages = plan.profile_read()
        top = max(stages, key=lambda s: s["ms"])["name"]
        plan.profile(True, only=top)
        plan.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(f, out=u)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if profile:
        rec = [s for s in plan.profile_read() if s["launches"] > 0]
        dom = rec[0] if rec else None
        plan.profile(False)
    return dt, stages, dom


def roofline(top, prec):
    """Roofline of the dominant stage (its events from the timed region):
    bound from its algorithmic bytes/flops per launch."""
    if not top:
        return None
    avg_s = top["ms"] / top["launches"] / 1e3
    peak_flops = PEAK_F64 if prec == "c128" else PEAK_F32
    t_mem = top["bytes_per_launch"] / PEAK_HBM
    t_alu = top["flops_per_launch"] / peak_flops
    name = top["name"]
    if t_mem >= t_alu:
        bound, achieved, peak, unit = "hbm", top["bytes_per_launch"] / avg_s / 1e9, PEAK_HBM / 1e9, "GB/s"
    else:
        bound = "mfma" if name.startswith("xform") or "xform" in name else "alu"
        achieved, peak, unit = top["flops_per_launch"] / avg_s / 1e12, peak_flops / 1e12, "TFLOP/s"
    return {"kernel": name, "bound": bound, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4), "avg_launch_us": round(avg_s * 1e6, 2),
            "bytes_per_launch": top["bytes_per_launch"], "flops_per_launch": top["flops_per_launch"]}


# ---------------------------------------------------------------- counter runs
# HBM traffic of the stage kernels comes from two rocprofv3 --pmc runs of
# `bench.py --counters` (FETCH_SIZE, then WRITE_SIZE) and two of
# `bench.py --copy` (a plain 1 GiB copy: the same counters' reading for known
# bytes gives the scale factors); `bench.py --traffic-summary F W CF CW` turns
# the four output folders into profiles/pmc_traffic.json.
COPY_BYTES = 1 << 30


def copy_run():
    import torch
    torch.cuda.set_device(0)
    a = torch.ones(COPY_BYTES // 16, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}), flush=True)


def counters_run(args):
    """Three solves of the decomposed workload (complex128, default tiling);
    per solve the stage kernels are dispatched in a fixed order."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    torch.cuda.set_device(0)
    p, f_np = W.c2_decomposed(core_cells=args.core, pml_cells=args.pml, nz=args.nz, nlayers=args.layers)
    f = hs.to_device(f_np)
    u = torch.empty_like(f)
    plan = hs.Plan(p, "c128", max_rhs=1)
    for _ in range(3):
        plan.solve(f, out=u)
    torch.cuda.synchronize()
    info = plan.info()
    print(json.dumps({"solves": 3, "z_chunks": info["z_chunks"]}), flush=True)


def _counter_rows(folder, counter):
    import csv
    import glob
    out = []
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]),
                                float(r["Counter_Value"])))
    out.sort()
    return out


SWEEP_ORDER = ("zsweep_blocks_v", "zsweep_global", "zsweep_blocks_u")


def _stage_labels(rows):
    """Label the dispatches of complex128 decomposed solves: per solve the z
    sweeps run in the order block sweep v, global sweep, block sweep u;
    contractions: faces, then Σ."""
    labels = []
    nsw = ncon = 0
    for _, name, grid, _ in rows:
        if "k_psweep" in name:
            labels.append(SWEEP_ORDER[nsw % 3])
            nsw += 1
        elif "k_contract<" in name:
            labels.append("face_contract" if ncon % 2 == 0 else "sigma_contract")
            ncon += 1
        else:
            labels.append(None)
    return labels


def traffic_summary(fdir, wdir, cfdir, cwdir):
    scale = {}
    for key, folder, counter in (("fetch", cfdir, "FETCH_SIZE"), ("write", cwdir, "WRITE_SIZE")):
        rows = [r for r in _counter_rows(folder, counter) if "copy" in r[1].lower() or "elementwise" in r[1]]
        kib = max(r[3] for r in rows)
        scale[key] = COPY_BYTES / (kib * 1024.0)
    stages = {}
    for key, folder, counter in (("fetch", fdir, "FETCH_SIZE"), ("write", wdir, "WRITE_SIZE")):
        rows = [r for r in _counter_rows(folder, counter) if "hs::" in r[1]]
        for lab, r in zip(_stage_labels(rows), rows):
            if lab is None:
                continue
            rec = stages.setdefault(lab, {"fetch_kib": [], "write_kib": []})
            rec[key + "_kib"].append(r[3])
    run = "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc {c} --output-format csv -d {d} -o run -- python3 $R/bench.py {a}"
    out = {"source_hash": kernel_source_hash(),
           "commands (R = repository root)": [
               run.format(c="FETCH_SIZE", d=fdir, a="--counters"), run.format(c="WRITE_SIZE", d=wdir, a="--counters"),
               run.format(c="FETCH_SIZE", d=cfdir, a="--copy"), run.format(c="WRITE_SIZE", d=cwdir, a="--copy"),
               f"python3 $R/bench.py --traffic-summary {fdir} {wdir} {cfdir} {cwdir}"],
           "copy_scale": scale, "stages": {}}
    for lab, rec in stages.items():
        fk = float(np.mean(rec["fetch_kib"])) if rec["fetch_kib"] else 0.0
        wk = float(np.mean(rec["write_kib"])) if rec["write_kib"] else 0.0
        out["stages"][lab] = {"fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk,
                              "bytes_per_launch": fk * 1024 * scale["fetch"] + wk * 1024 * scale["write"],
                              "dispatches": len(rec["fetch_kib"])}
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def stats_summary(trace_csv: str, title: str, command: str, stage_labels: bool = False):
    """Text summary of a rocprofv3 kernel trace: per kernel and grid, the
    number of dispatches, the average duration and the share of the total.
    stage_labels (complex128 decomposed solves): the z sweeps of a solve run
    in the order block sweep v, global sweep, block sweep u, and are listed
    apart."""
    import csv
    import re
    agg = {}
    nsw = 0
    with open(trace_csv) as fh:
        rows = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
        for r in rows:
            name = r["Kernel_Name"].replace("hs::(anonymous namespace)::", "")
            name = re.sub(r"HIP_vector_type<(\w+), 2u>", r"\g<1>2", name)
            name = re.sub(r"\(hs::.*|\(.*", "", name).replace("void ", "")
            grid = "x".join(r["Grid_Size_" + a] for a in "XYZ")
            if stage_labels and name.startswith("k_psweep"):
                name += f" [{SWEEP_ORDER[nsw % 3]}]"
                nsw += 1
            key = (name, grid)
            a = agg.setdefault(key, [0, 0.0])
            a[0] += 1
            a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    tot = sum(v[1] for v in agg.values())
    print(f"# rocprofv3 kernel statistics: {title}")
    print(f"# command (R = repository root): {command}")
    print("# columns: dispatches, average us, share of kernel time %, kernel, grid (work-items x*y*z)")
    for (name, grid), (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"{n:6d} {t / n:10.1f} {100 * t / tot:7.2f}  {name}  grid={grid}")


def traffic_for(kernel_stage: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, only while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            d = json.load(fh)
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    rec = d.get("stages", {}).get(kernel_stage)
    return None if rec is None else rec.get("bytes_per_launch")


def cpu_baseline(problem, f, repeat_budget_s=20.0):
    """The FP64 oracle (undecomposed generalized-eigen separable solve) on the
    host: plan (eigendecomposition) excluded, solve timed."""
    from oracle import separable
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    solver = separable.SeparableSolver(problem)
    t_plan = time.perf_counter() - t0
    times = []
    u = None
    while True:
        t0 = time.perf_counter()
        u = solver.solve(f)
        times.append(time.perf_counter() - t0)
        if sum(times) > repeat_budget_s / 2 or len(times) >= 3:
            break
    t = float(np.median(times))
    return u, {"value": problem.unknowns * f.shape[0] / t, "unit": "unknowns*RHS/s", "cores": cores,
               "kind": "oracle", "sample": f"full workload, {f.shape[0]} RHS, median of {len(times)} solves "
                                         f"({t:.2f} s each; eigen tables {t_plan:.2f} s excluded)"}


def bench_c3(steps, warmup, with_oracle, sample_blocks=(0, 5, 40, 63), precs=("c128", "mixed"), refine_steps=1):
    """Batched workload: 64 independent blocks of uneven sizes (half uniform,
    half with stretched complex ends), 8 right-hand sides each, every stage one
    batched launch in a captured graph; complex128 batch vs complex64 +
    FP64-refinement batch on the same inputs."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    blocks = W.c3_blocks()
    nrhs = 8
    unknowns = sum(b.problem.unknowns for b in blocks)
    fs = [hs.to_device(W.c3_rhs(i, b.problem, nrhs)) for i, b in enumerate(blocks)]
    us = [torch.empty_like(f) for f in fs]
    out = {"workload": f"c3_batched 64 blocks (32 uniform, 32 stretched ends), n_x,n_y in [32,256], "
                       f"n_z in [64,256], {nrhs} RHS each",
           "unknowns": unknowns, "nrhs": nrhs}
    for prec in precs:
        t0 = time.perf_counter()
        plans = [hs.Plan(b.problem, prec, max_rhs=1, refine_steps=refine_steps if prec == "mixed" else 0)
                 for b in blocks]
        batch = hs.Batch(plans, [nrhs] * len(plans))
        t_plan = time.perf_counter() - t0
        for _ in range(warmup):
            batch.solve(fs, us)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.solve(fs, us)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rec = {"value": unknowns * nrhs / dt, "unit": "unknowns*RHS/s", "ms_per_step": dt * 1e3,
               "plan_seconds": t_plan}
        if prec == "mixed":
            rec["refine_steps"] = plans[0].info()["refine_steps"]
        if with_oracle:
            from oracle import separable
            errs = []
            for i in sample_blocks:
                pb = blocks[i].problem
                f1 = W.c3_rhs(i, pb, nrhs)[:1]
                ref = separable.solve(pb, f1)
                got = us[i][:1].cpu().numpy()
                errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
            rec["rel_err_vs_oracle_max"] = max(errs)
            rec["oracle_sample"] = f"blocks {list(sample_blocks)}, RHS 0"
        out[prec] = rec
        del batch, plans
        torch.cuda.empty_cache()
    if "mixed" in out and "c128" in out:
        out["mixed_speedup_vs_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    return out


def bench_c4(steps, with_oracle):
    """Adjoint workload: gradient of 0.5 |P u - d|^2 with respect to the 40
    layer values of k^2 on the 128 x 128 x 160 grid (P samples the z-index-9
    plane, d comes from a perturbed k^2).  One gradient = forward solve,
    adjoint source, adjoint solve, layer sums; timed through the autograd
    wrapper (as a training loop calls it) and as the bare sequence of C-ABI
    calls; the gradient is compared with the oracle's."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    p, f, k2_true, plane = W.c4_adjoint()
    plan = hs.Plan(p, "c128")
    fd = hs.to_device(f)
    plan.set_k2(k2_true)
    d = plan.solve(fd)[0, plane].clone()
    plan.set_k2(p.k2)
    k2 = torch.tensor(p.k2, dtype=torch.complex128, requires_grad=True)

    def autograd_step():
        u = hs.helmholtz_solve(k2, fd, plan)
        J = 0.5 * (u[0, plane] - d).abs().pow(2).sum()
        k2.grad = None
        J.backward()
        return J

    def abi_step():
        u = plan.solve(fd)
        g = torch.zeros_like(u)
        g[0, plane] = u[0, plane] - d
        a = plan.solve_adjoint(g)
        return plan.grad_k2(u, a)

    out = {"workload": f"c4_adjoint {p.nx}x{p.ny}x{p.nz}, {p.nlayers} layers, gradient of a plane misfit "
                       f"w.r.t. layer k^2, complex128", "unknowns": p.unknowns}
    for name, fn in (("autograd", autograd_step), ("abi", abi_step)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        out[f"ms_per_gradient_{name}"] = (time.perf_counter() - t0) / steps * 1e3
    if with_oracle:
        from oracle import adjoint
        J = autograd_step()
        _, g_ref, _, _ = adjoint.plane_misfit_grad(p, f[0], plane, d.cpu().numpy())
        g = k2.grad.detach().numpy()
        out["grad_rel_err_vs_oracle"] = float(np.abs(g - g_ref).max() / np.abs(g_ref).max())
        out["misfit"] = float(J.detach())
    return out


def bench_c5(steps, refine_steps=1):
    """Large decomposed grid: core 512 + 32 PML cells per side (575 x 575
    interior nodes), n_z = 256 in 60 layers, 16 point sources off the
    separators, k^2 scaled by omega^2 for omega in (1, 1.5, 2, 3).  One plan
    per precision; each frequency is one k^2 update (hs_set_k2, not timed)
    followed by solves of all 16 right-hand sides at once.  The relative
    residual |f - A u| / |f| of the last solve (FP64 stencil on the GPU) is
    reported per frequency; parity with the oracle at this size is a test."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    p, srcs, omegas = W.c5_multi_rhs()
    nrhs = len(srcs)
    f = torch.zeros((nrhs,) + p.shape, dtype=torch.complex128, device="cuda")
    for r, (x, y, z) in enumerate(srcs):
        f[r, z, y, x] = 1.0
    u = torch.empty_like(f)
    out = {"workload": f"c5_large {p.nx}x{p.ny}x{p.nz}, 4x4 blocks + interface reduction, PML 32/side, "
                       f"60 layers, {nrhs} point sources x {len(omegas)} frequencies",
           "unknowns": p.unknowns, "nrhs": nrhs, "omegas": list(omegas)}
    fnorm = float(torch.linalg.vector_norm(f[0]))
    for prec in ("c128", "mixed"):
        t0 = time.perf_counter()
        plan = hs.Plan(p, prec, max_rhs=nrhs, refine_steps=refine_steps if prec == "mixed" else 0)
        t_plan = time.perf_counter() - t0
        total = 0.0
        resid = []
        for om in omegas:
            plan.set_k2(p.k2 * om ** 2)
            plan.solve(f, out=u)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.solve(f, out=u)
            torch.cuda.synchronize()
            total += (time.perf_counter() - t0) / steps
            r = plan.residual(f[:1], u[:1])
            resid.append(float(torch.linalg.vector_norm(r)) / fnorm)
            del r
        rec = {"value": p.unknowns * nrhs * len(omegas) / total, "unit": "unknowns*RHS/s",
               "ms_per_frequency": total / len(omegas) * 1e3, "plan_seconds": t_plan,
               "rel_residual_rhs0_per_omega": resid}
        if prec == "mixed":
            rec["refine_steps"] = plan.info()["refine_steps"]
        out[prec] = rec
        del plan
        torch.cuda.empty_cache()
    out["mixed_speedup_vs_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-only", action="store_true", help="time only the mixed-precision solve (profiling)")
    ap.add_argument("--core", type=int, default=256, help="uniform core cells per axis")
    ap.add_argument("--pml", type=int, default=16)
    ap.add_argument("--nz", type=int, default=200)
    ap.add_argument("--layers", type=int, default=20)
    ap.add_argument("--no-c3", action="store_true", help="skip the batched 64-block measurement")
    ap.add_argument("--no-c5", action="store_true", help="skip the large 575x575x256 measurement")
    ap.add_argument("--no-c4", action="store_true", help="skip the adjoint-gradient measurement")
    ap.add_argument("--c3-steps", type=int, default=5)
    ap.add_argument("--refine-steps", type=int, default=1,
                    help="FP64-residual refinement steps of the mixed-precision solves (-1: none)")
    ap.add_argument("--copy", action="store_true", help="counter calibration: a plain 1 GiB copy")
    ap.add_argument("--counters", action="store_true", help="three complex128 solves for counter runs")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH", "WRITE", "CFETCH", "CWRITE"),
                    help="write profiles/pmc_traffic.json from four rocprofv3 --pmc output folders")
    ap.add_argument("--c3-only", choices=["c128", "mixed", "both"], help="time only the 64-block batch")
    ap.add_argument("--c4-only", action="store_true", help="time only the adjoint gradient (128x128x160)")
    ap.add_argument("--c5-only", action="store_true",
                    help="time only the large 575x575x256 grid, 16 sources x 4 frequencies (c128 vs mixed)")
    ap.add_argument("--stats-summary", nargs=3, metavar=("TRACE_CSV", "TITLE", "COMMAND"),
                    help="print a text summary of a rocprofv3 kernel trace")
    ap.add_argument("--stage-labels", action="store_true",
                    help="with --stats-summary: list the z sweeps of decomposed solves by stage")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.stats_summary:
        stats_summary(*args.stats_summary, stage_labels=args.stage_labels)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(right-hand sides and frequencies shard across GPUs with a replicated plan "
              "and no communication; blocks of one decomposed grid would exchange only the "
              "separator lines around the global interface solve).", file=sys.stderr)
        sys.exit(2)

    if args.copy:
        copy_run()
        return
    if args.c3_only:
        precs = ("c128", "mixed") if args.c3_only == "both" else (args.c3_only,)
        print(json.dumps(bench_c3(args.c3_steps, 1, False, precs=precs, refine_steps=args.refine_steps)), flush=True)
        return
    if args.counters:
        counters_run(args)
        return
    if args.c4_only:
        print(json.dumps(bench_c4(max(1, args.steps), True)), flush=True)
        return
    if args.c5_only:
        print(json.dumps(bench_c5(max(1, min(args.steps, 3)), refine_steps=args.refine_steps)), flush=True)
        return

    import torch
    import paper_1909_01299_amd as hs
    import workloads as W

    torch.cuda.set_device(0)
    p, f_np = W.c2_decomposed(core_cells=args.core, pml_cells=args.pml, nz=args.nz, nlayers=args.layers)
    nrhs = f_np.shape[0]
    f = hs.to_device(f_np)
    u = torch.empty_like(f)

    if args.mixed_only:
        plan_m = hs.Plan(p, "mixed", max_rhs=nrhs, refine_steps=args.refine_steps)
        um = torch.empty_like(f)
        dtm, _, _ = time_solves(plan_m, f, um, args.steps, args.warmup, profile=False)
        print(json.dumps({"mixed_ms_per_step": dtm / args.steps * 1e3}), flush=True)
        return
    plan = hs.Plan(p, "c128", max_rhs=nrhs)
    tuned = plan.tune(nrhs)
    info = plan.info()
    dt, stages, dom = time_solves(plan, f, u, args.steps, args.warmup)
    ms = dt / args.steps * 1e3
    value = p.unknowns * nrhs / (dt / args.steps)
    u_gpu = u.cpu().numpy()

    mixed = None
    if not args.no_mixed:
        plan_m = hs.Plan(p, "mixed", max_rhs=nrhs, refine_steps=args.refine_steps)
        plan_m.tune(nrhs)
        um = torch.empty_like(f)
        dtm, stages_m, dom_m = time_solves(plan_m, f, um, args.steps, args.warmup)
        mixed = {"value": p.unknowns * nrhs / (dtm / args.steps), "ms_per_step": dtm / args.steps * 1e3,
                 "refine_steps": plan_m.info()["refine_steps"], "u": um.cpu().numpy(),
                 "roofline": roofline(dom_m, "c64"),
                 "stages": {s["name"]: round(s["ms"] / args.steps, 4) for s in stages_m}}
        del plan_m

    cpu = None
    rel_err = rel_err_mixed = None
    if not args.no_cpu_baseline:
        u_ref, cpu = cpu_baseline(p, f_np)
        rel_err = float(np.linalg.norm(u_gpu - u_ref) / np.linalg.norm(u_ref))
        if mixed is not None:
            rel_err_mixed = float(np.linalg.norm(mixed["u"] - u_ref) / np.linalg.norm(u_ref))

    c3 = None
    if not args.no_c3:
        del plan
        torch.cuda.empty_cache()
        c3 = bench_c3(args.c3_steps, 1, not args.no_cpu_baseline, refine_steps=args.refine_steps)
    c4 = None
    if not args.no_c4:
        c4 = bench_c4(10, not args.no_cpu_baseline)
    c5 = None
    if not args.no_c5:
        torch.cuda.empty_cache()
        c5 = bench_c5(2, refine_steps=args.refine_steps)

    rf = roofline(dom, "c128")
    if rf is not None:
        rf["traffic"] = traffic_for(rf["kernel"])
    line = {
        "metric": "unknowns*RHS/s (decomposed 3D Helmholtz solve, complex128)",
        "value": value,
        "unit": "unknowns*RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"c2_decomposed {p.nx}x{p.ny}x{p.nz}, 4x4 blocks + interface reduction, "
                               f"PML {args.pml}/side, {args.layers} layers, centre point source",
                   "unknowns": p.unknowns, "nrhs": nrhs, "blocks": info["nblocks"]},
        "rel_err_vs_oracle": rel_err,
        "roofline": rf,
        "cpu_baseline": cpu,
        "mixed_c64_refine": None if mixed is None else {
            "value": mixed["value"], "ms_per_step": mixed["ms_per_step"],
            "refine_steps": mixed["refine_steps"], "rel_err_vs_oracle": rel_err_mixed,
            "speedup_vs_c128": mixed["value"] / value, "roofline": mixed["roofline"],
            "stages_ms_per_step": mixed["stages"]},
        "batched_c3": c3,
        "adjoint_c4": c4,
        "large_c5": c5,
        "stages_ms_per_step": {s["name"]: round(s["ms"] / args.steps, 4) for s in stages},
        "plan_seconds": info["plan_seconds"],
        "tuned": tuned,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
