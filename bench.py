#!/usr/bin/env python3
"""Benchmark of the separable Helmholtz solver on one MI355X.

Headline workload (one step = every frequency's solve of every source):
  uniform core 512 x 512 (h = 1) + 32 PML cells per side (steps
  1.2^k (1+0.5i)), 575 x 575 interior nodes, n_z = 256 in 60 layers, 4 x 4
  blocks (separators at 31, 287, 543 on x and y) solved by the two-level
  interface reduction; 16 unit point sources off the separators; k^2 scaled
  by omega^2 for omega in (1, 1.5, 2, 3).  One plan per frequency (the plans
  share one workspace); a step solves the 16 right-hand sides at once with
  each plan in turn.  complex128.  Inputs are resident in HBM before the
  timed region.

Prints one JSON line: unknowns*RHS/s of the complex128 solves, the mixed
complex64 + FP64-refinement solves of the same workload beside them, the
roofline of the dominant kernel from hipEvents recorded on the solve's
stream inside the timed region, oracle errors on sampled sources, and the
FP64 CPU oracle timed on the host on one source.  The same line carries three
more workloads: the 287 x 287 x 200 decomposed grid with one centre point
source ("decomposed_c2"), 64 independent blocks of uneven sizes with 8
right-hand sides each as one captured graph per solve ("batched_c3"), and the
time of one adjoint gradient with respect to the layer values of k^2 on the
128 x 128 x 160 grid ("adjoint_c4").
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
    """Complex128 solves for the counter runs, per solve the stage kernels
    dispatched in a fixed order: the headline workload (575 x 575 x 256, 16
    sources, omega = 1; two solves) or, with --counters-workload c2, the
    287 x 287 x 200 grid (three solves)."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    torch.cuda.set_device(0)
    if args.counters_workload == "c2":
        p, f_np = W.c2_decomposed(core_cells=args.core, pml_cells=args.pml, nz=args.nz, nlayers=args.layers)
        f = hs.to_device(f_np)
        solves = 3
    else:
        p, srcs, _ = W.c5_multi_rhs()
        f = point_sources_device(p, srcs)
        solves = 2
    u = torch.empty_like(f)
    plan = hs.Plan(p, "c128", max_rhs=f.shape[0])
    if TUNE_CACHE:
        plan.tune(f.shape[0], cache=TUNE_CACHE)
    for _ in range(solves):
        plan.solve(f, out=u)
    torch.cuda.synchronize()
    info = plan.info()
    print(json.dumps({"workload": args.counters_workload, "solves": solves, "z_chunks": info["z_chunks"]}),
          flush=True)


def point_sources_device(p, srcs):
    import torch
    f = torch.zeros((len(srcs),) + p.shape, dtype=torch.complex128, device="cuda")
    for r, (x, y, z) in enumerate(srcs):
        f[r, z, y, x] = 1.0
    return f


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
    rel = lambda d: d if os.path.isabs(d) else "$R/" + d   # noqa: E731
    ctr = "--counters" + (f" --tune-cache {rel(TUNE_CACHE)}" if TUNE_CACHE else "")
    out = {"source_hash": kernel_source_hash(),
           "commands (R = repository root)": [
               run.format(c="FETCH_SIZE", d=rel(fdir), a=ctr), run.format(c="WRITE_SIZE", d=rel(wdir), a=ctr),
               run.format(c="FETCH_SIZE", d=rel(cfdir), a="--copy"), run.format(c="WRITE_SIZE", d=rel(cwdir), a="--copy"),
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


SQ_SETS = ("SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS "
           "SQ_INSTS_VMEM_RD SQ_LDS_BANK_CONFLICT",
           "SQ_INST_LEVEL_VMEM SQ_ACTIVE_INST_VMEM SQ_INSTS_LDS SQ_WAIT_ANY SQ_LEVEL_WAVES SQ_INSTS_VALU "
           "SQ_INSTS_VMEM_WR SQ_BUSY_CU_CYCLES")


def sq_summary(dir1, dir2):
    """Per-kernel summary of two rocprofv3 --pmc runs over `bench.py
    --counters` (the two counter sets of SQ_SETS): fractions of wave cycles
    spent waiting (any) and issuing VALU / LDS instructions, vector-memory
    instructions in flight per busy cycle, LDS bank-conflict cycles per LDS
    instruction."""
    import csv
    import re
    import collections

    def load(folder):
        agg = collections.OrderedDict()
        with open(os.path.join(folder, "run_counter_collection.csv")) as fh:
            for r in csv.DictReader(fh):
                m = re.search(r"(k_[a-z0-9_]+<[^(]*>)", r["Kernel_Name"])
                name = (m.group(1) if m else r["Kernel_Name"][:30]) + "  grid=" + r["Grid_Size"]
                a = agg.setdefault(name, collections.Counter())
                a[r["Counter_Name"]] += float(r["Counter_Value"])
        return agg
    a1, a2 = load(dir1), load(dir2)
    run = ("cd /tmp && export TMPDIR=/tmp && timeout -s KILL 180 rocprofv3 --pmc {c} --output-format csv "
           "-d {d} -o run -- python3 $R/bench.py --counters" + (f" --tune-cache {TUNE_CACHE}" if TUNE_CACHE else ""))
    print("# rocprofv3 SQ counters per kernel: complex128 solves of the 575x575x256 grid (16 sources, omega = 1)")
    for c, d in zip(SQ_SETS, (dir1, dir2)):
        print("# command (R = repository root): " + run.format(c=c, d=d))
    print(f"# summary: python3 $R/bench.py --sq-summary {dir1} {dir2}")
    print("# columns: waves per dispatch, wait (any) / VALU busy / LDS busy as fractions of wave cycles, "
          "VMEM instructions in flight per busy cycle, LDS bank-conflict cycles per LDS instruction, kernel")
    for name, d in a1.items():
        d = collections.Counter(d)
        d.update(a2.get(name, {}))
        if d.get("SQ_WAVES", 0) < 1000:
            continue
        wc = d.get("SQ_WAVE_CYCLES", 0) or 1
        bc = d.get("SQ_BUSY_CYCLES", 0) or 1
        print(f"{d['SQ_WAVES']:11.0f}  {d['SQ_WAIT_ANY'] / wc:5.2f}  {d['SQ_ACTIVE_INST_VALU'] / wc:5.2f}  "
              f"{d['SQ_ACTIVE_INST_LDS'] / wc:5.2f}  {d['SQ_INST_LEVEL_VMEM'] / bc:5.1f}  "
              f"{d['SQ_LDS_BANK_CONFLICT'] / max(d['SQ_INSTS_LDS'], 1):5.2f}  {name}")


def short_mangled(name):
    """Kernel name and template arguments read from a mangled name that
    c++filt leaves as it is (kernels over _Float16 vectors)."""
    import re
    m = re.search(r"\d+(k_[a-z0-9_]+)I(.*?)EEvP", name)
    if not m:
        return name
    args = []
    for t in re.finditer(r"Lb([01])E|Li(\d+)E|(?:\d+HIP_vector_type|S\d*_)I([fd])Lj2EE|S\d*_", m.group(2)):
        if t.group(1) is not None:
            args.append("true" if t.group(1) == "1" else "false")
        elif t.group(2) is not None:
            args.append(t.group(2))
        elif t.group(3) is not None:
            args.append("float2" if t.group(3) == "f" else "double2")
        else:
            args.append("same type")
    return f"{m.group(1)}<{', '.join(args)}>"


MFMA_COUNTERS = "SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_F16 SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE"


def mfma_summary(triples):
    """Issued matrix-core rate of the dense transform kernels of the 64-block
    batch: per precision P, a rocprofv3 --pmc run of MFMA_COUNTERS and a
    kernel trace of the same command; per kernel and grid, 512 x the MFMA
    MOPS count (FP64 for complex128, F16 for the split-fp16 mixed solves)
    over the kernel-trace time, against the dense peak of that type."""
    import csv
    import re
    import subprocess
    import collections

    def norm(name):
        if name.startswith("_Z"):
            try:
                dem = subprocess.run(["c++filt", name], capture_output=True, text=True).stdout.strip()
            except OSError:
                dem = ""
            name = dem if dem and not dem.startswith("_Z") else short_mangled(name)
        name = name.replace("hs::(anonymous namespace)::", "").replace("void ", "")
        name = re.sub(r"HIP_vector_type<(\w+), 2u>", r"\g<1>2", name)
        return re.sub(r"\(.*", "", name)

    tc = f" --tune-cache {TUNE_CACHE}" if TUNE_CACHE else ""
    print("# rocprofv3 MFMA counters: batched 64 blocks x 8 RHS (one warm-up + one timed solve), dense transform kernels")
    print("# commands (R = repository root), per precision:")
    for i in range(0, len(triples), 3):
        prec, pmc, kt = triples[i:i + 3]
        print(f"#   cd /tmp && export TMPDIR=/tmp && timeout -s KILL 180 rocprofv3 --pmc {MFMA_COUNTERS} --output-format csv "
              f"-d $R/{pmc} -o run -- python3 $R/bench.py --c3-only {prec} --c3-steps 1{tc}")
        print(f"#   cd /tmp && export TMPDIR=/tmp && rocprofv3 --kernel-trace --output-format csv -d $R/{kt} "
              f"-o run -- python3 $R/bench.py --c3-only {prec} --c3-steps 1{tc}")
    print("# summary: python3 $R/bench.py" + tc + " --mfma-summary " + " ".join(triples))
    print("# issued matrix flop/s = 512 * SQ_INSTS_VALU_MFMA_MOPS_<type> / (kernel-trace duration); "
          "peaks (dense): FP64 78.6, fp16 2500 TFLOP/s")
    print("# split-fp16 kernels issue three fp16 products per FP32-class product")
    print("# columns: precision, dispatches, total ms, issued TFLOP/s, fraction of the type's peak, kernel")
    for i in range(0, len(triples), 3):
        prec, pmc, kt = triples[i:i + 3]
        ctr = "SQ_INSTS_VALU_MFMA_MOPS_F64" if prec == "c128" else "SQ_INSTS_VALU_MFMA_MOPS_F16"
        peak = PEAK_F64 if prec == "c128" else 2.5e15
        mops = collections.Counter()
        for _, name, grid, v in _counter_rows(pmc, ctr):
            mops[(norm(name), grid)] += v
        dur = collections.Counter()
        cnt = collections.Counter()
        for path in glob_csv(kt, "*kernel_trace.csv"):
            with open(path) as fh:
                for r in csv.DictReader(fh):
                    g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                    key = (norm(r["Kernel_Name"]), g)
                    dur[key] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
                    cnt[key] += 1
        tot_f = tot_t = 0.0
        for key, m in sorted(mops.items(), key=lambda kv: -dur.get(kv[0], 0)):
            if m <= 0 or dur.get(key, 0) <= 0:
                continue
            fl = 512.0 * m
            tot_f += fl
            tot_t += dur[key]
            print(f"{prec:6s} {cnt[key]:4d} {dur[key] * 1e3:9.2f} {fl / dur[key] / 1e12:8.1f} {fl / dur[key] / peak:6.3f}  "
                  f"{key[0]}  grid={key[1]}")
        if tot_t > 0:
            kind = "F64" if prec == "c128" else "F16"
            print(f"{prec:6s}  all {tot_t * 1e3:9.2f} {tot_f / tot_t / 1e12:8.1f} {tot_f / tot_t / peak:6.3f}  "
                  f"(all {kind} matrix kernels)")


def glob_csv(folder, pattern):
    import glob
    return glob.glob(os.path.join(folder, "**", pattern), recursive=True)


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
            name = r["Kernel_Name"]
            if name.startswith("_Z"):
                name = short_mangled(name)
            name = name.replace("hs::(anonymous namespace)::", "")
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


def host_description():
    """CPU model, thread count and numerical library versions of the host."""
    import platform
    import scipy
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            blas.append(f"{i.get('internal_api')} {i.get('version')} ({i.get('num_threads')} threads)")
    except Exception:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "numpy": np.__version__,
            "scipy": scipy.__version__, "blas": blas}


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        return os.cpu_count()


def cpu_baseline(problem, f, unknowns_per_rhs, repeat_budget_s=20.0, sample=""):
    """The FP64 oracle (undecomposed generalized-eigen separable solve) on the
    host: plan (eigendecomposition) excluded, solves of f timed (median of at
    most 3, within the budget).  Returns (oracle solution, baseline record)."""
    from oracle import separable
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
    nrhs = 1 if f.ndim == 3 else f.shape[0]
    return u, {"value": unknowns_per_rhs * nrhs / t, "unit": "unknowns*RHS/s", "cores": oracle_threads(),
               "kind": "oracle",
               "sample": f"{sample}: {nrhs} RHS, median of {len(times)} solves ({t:.2f} s each; eigen tables "
                         f"{t_plan:.2f} s excluded)",
               "host": host_description()}


def errors_vs(u, ref, problem=None):
    """Relative 2-norm error, largest pointwise error over the largest
    reference value, and (decomposed grids) the error on the separator planes
    as an RMS per node over the RMS of the whole field, and relative to the
    separator field itself."""
    d = u - ref
    out = {"rel2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
           "relmax": float(np.abs(d).max() / np.abs(ref).max())}
    if problem is not None and (len(problem.sep_x) or len(problem.sep_y)):
        m = np.zeros(problem.shape[1:], dtype=bool)
        m[:, problem.sep_x] = True
        m[problem.sep_y, :] = True
        ds, rs = d[:, m], ref[:, m]
        out["rms_sigma"] = float(np.linalg.norm(ds) / np.sqrt(ds.size) / (np.linalg.norm(ref) / np.sqrt(ref.size)))
        out["rel2_sigma"] = float(np.linalg.norm(ds) / np.linalg.norm(rs))
    return out


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
        t0 = time.perf_counter()
        batch.tune(fs, us, cache=TUNE_CACHE)
        t_tune = time.perf_counter() - t0
        for _ in range(warmup):
            batch.solve(fs, us)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            batch.solve(fs, us)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        rec = {"value": unknowns * nrhs / dt, "unit": "unknowns*RHS/s", "ms_per_step": dt * 1e3,
               "plan_seconds": t_plan, "tune_seconds": t_tune}
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
                errs.append(errors_vs(got, ref))
            rec["rel_err_vs_oracle_max"] = max(e["rel2"] for e in errs)
            rec["relmax_err_vs_oracle_max"] = max(e["relmax"] for e in errs)
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


TUNE_CACHE = None   # JSON-lines file of tuned launch shapes (--tune-cache)


def merge_stage_tables(tables):
    """Sum the per-stage records of several plans (same stage names)."""
    out = {}
    for tab in tables:
        for rec in tab:
            m = out.setdefault(rec["name"], dict(rec, ms=0.0, launches=0))
            m["ms"] += rec["ms"]
            m["launches"] += rec["launches"]
    return list(out.values())


def time_plans(plans, f, u, steps, warmup):
    """Wall time of `steps` steps, a step being one solve of f with every plan
    in turn.  An untimed step with hipEvents around every stage gives the
    stage table and the dominant stage; in the timed steps only that stage is
    bracketed by events (two per solve, on the solve's stream), so its kernel
    time comes from the timed region itself.  Returns (seconds, stage table
    per step, dominant stage record from the timed region)."""
    import torch

    def step():
        for pl in plans:
            pl.solve(f, out=u)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    for pl in plans:
        pl.profile(True)
        pl.profile_read()
    step()
    torch.cuda.synchronize()
    stages = merge_stage_tables([pl.profile_read() for pl in plans])
    top = max(stages, key=lambda r: r["ms"])["name"]
    for pl in plans:
        pl.profile(True, only=top)
        pl.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec = [r for r in merge_stage_tables([pl.profile_read() for pl in plans]) if r["launches"] > 0]
    for pl in plans:
        pl.profile(False)
    return dt, stages, (rec[0] if rec else None)


def bench_c5(steps, warmup, refine_steps=1, with_oracle=True, precs=("c128", "mixed"), profile_only=False):
    """Headline workload: 575 x 575 x 256, 4 x 4 blocks + interface reduction,
    16 point sources x 4 frequencies.  Returns the record of each precision
    (throughput, roofline of the dominant stage, stage table) and, with the
    oracle, errors on sampled sources and the oracle's own throughput."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    torch.cuda.set_device(0)
    p, srcs, omegas = W.c5_multi_rhs()
    nrhs = len(srcs)
    f = point_sources_device(p, srcs)
    u = torch.empty_like(f)
    per_step = p.unknowns * nrhs * len(omegas)
    out = {"workload": f"c5_large {p.nx}x{p.ny}x{p.nz}, 4x4 blocks + interface reduction, PML 32/side, "
                       f"60 layers, {nrhs} point sources x {len(omegas)} frequencies (omega in {list(omegas)})",
           "unknowns": p.unknowns, "nrhs": nrhs, "omegas": list(omegas), "unknowns_rhs_per_step": per_step}
    # oracle samples: (frequency index, source index)
    samples = ((0, 0), (3, 1))
    for prec in precs:
        t0 = time.perf_counter()
        plans, ws = [], None
        for om in omegas:
            pl = hs.Plan(p.with_k2(p.k2 * om ** 2), prec, max_rhs=nrhs,
                         refine_steps=refine_steps if prec == "mixed" else 0, workspace=ws)
            ws = pl.workspace
            plans.append(pl)
        t_plan = time.perf_counter() - t0
        # launch shapes tuned once on the first frequency (same shapes for all);
        # a cache file (--tune-cache) lets a profiled run reuse them untuned
        t0 = time.perf_counter()
        tuned = plans[0].tune(nrhs, cache=TUNE_CACHE)
        for pl in plans[1:]:
            pl.set_launch(tuned)
        t_tune = time.perf_counter() - t0
        dt, stages, dom = time_plans(plans, f, u, steps, warmup)
        rec = {"value": per_step * steps / dt, "unit": "unknowns*RHS/s", "ms_per_step": dt / steps * 1e3,
               "ms_per_frequency": dt / steps / len(omegas) * 1e3, "plan_seconds_4_plans": t_plan,
               "tune_seconds": t_tune, "tuned": tuned,
               "roofline": roofline(dom, prec),
               "stages_ms_per_step": {r["name"]: round(r["ms"], 3) for r in stages}}
        if prec == "mixed":
            rec["refine_steps"] = plans[0].info()["refine_steps"]
        if not profile_only:
            # sampled results for the oracle, and the FP64 residual of each
            # frequency's first source (GPU stencil), outside the timed region
            rec["sampled"] = {}
            resid = []
            fnorm = float(torch.linalg.vector_norm(f[0]))
            for k, pl in enumerate(plans):
                pl.solve(f, out=u)
                r = pl.residual(f[:1], u[:1])
                resid.append(float(torch.linalg.vector_norm(r)) / fnorm)
                del r
                for (kk, src) in samples:
                    if kk == k:
                        rec["sampled"][(kk, src)] = u[src].cpu().numpy()
            rec["rel_residual_rhs0_per_omega"] = resid
        out[prec] = rec
        del plans, ws
        torch.cuda.empty_cache()
    if "mixed" in out and "c128" in out:
        out["mixed_speedup_vs_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    if with_oracle and not profile_only:
        from oracle import separable
        fs0 = W.point_source_batch(p, srcs[:1])[0]
        u_ref0, cpu = cpu_baseline(p.with_k2(p.k2 * omegas[0] ** 2), fs0, p.unknowns,
                                   sample=f"the headline grid at omega = {omegas[0]}, source 0 (of 16)")
        out["cpu_baseline"] = cpu
        refs = {samples[0]: u_ref0}
        for (kk, src) in samples[1:]:
            fs = W.point_source_batch(p, [srcs[src]])[0]
            refs[(kk, src)] = separable.solve(p.with_k2(p.k2 * omegas[kk] ** 2), fs)
        for prec in precs:
            errs = {f"omega={omegas[kk]} source {src}": errors_vs(out[prec]["sampled"][(kk, src)], refs[(kk, src)], p)
                    for (kk, src) in samples}
            out[prec]["rel_err_vs_oracle"] = errs
            out[prec]["rel_err_vs_oracle_max"] = max(e["rel2"] for e in errs.values())
            out[prec]["relmax_err_vs_oracle_max"] = max(e["relmax"] for e in errs.values())
    for prec in precs:
        out[prec].pop("sampled", None)
    return out


def bench_c5_streams(steps, warmup):
    """The headline workload (complex128) as two independent halves: the 16
    sources split 8 + 8, each half with its own four plans and workspace on
    its own stream, so the kernels of one half overlap those of the other
    (the z solves are latency-bound and leave HBM bandwidth idle).  Same
    memory as one 16-source plan set.  Timed like the headline (a step is
    every frequency of both halves; synchronised on both sides of the timed
    steps), against one stream of 16-source solves; the results of the two
    schedules must agree bit for bit."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    torch.cuda.set_device(0)
    p, srcs, omegas = W.c5_multi_rhs()
    nrhs = len(srcs)
    f = point_sources_device(p, srcs)
    u = torch.empty_like(f)
    per_step = p.unknowns * nrhs * len(omegas)

    def plan_set(n):
        plans, ws = [], None
        for om in omegas:
            pl = hs.Plan(p.with_k2(p.k2 * om ** 2), "c128", max_rhs=n, workspace=ws)
            ws = pl.workspace
            plans.append(pl)
        return plans

    def timed(step):
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    one = plan_set(nrhs)
    tuned = one[0].tune(nrhs, cache=TUNE_CACHE)
    for pl in one[1:]:
        pl.set_launch(tuned)
    t_one = timed(lambda: [pl.solve(f, out=u) for pl in one])
    ref = u.clone()
    del one
    torch.cuda.empty_cache()
    h = nrhs // 2
    halves = [plan_set(h), plan_set(nrhs - h)]
    for ps in halves:
        for pl in ps:
            pl.set_launch(tuned)
    fs, us = [f[:h], f[h:]], [u[:h], u[h:]]
    main = torch.cuda.current_stream()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def two():
        for s in streams:
            s.wait_stream(main)
        for k in range(len(omegas)):
            for i in range(2):
                halves[i][k].solve(fs[i], out=us[i], stream=streams[i])
        for s in streams:
            main.wait_stream(s)

    t_two = timed(two)
    same = bool(torch.equal(u, ref))
    return {"workload": f"c5_large {p.nx}x{p.ny}x{p.nz}, {nrhs} point sources x {len(omegas)} frequencies, c128",
            "tuned": tuned,
            "one_stream": {"value": per_step / t_one, "ms_per_step": t_one * 1e3},
            "two_streams_8_plus_8": {"value": per_step / t_two, "ms_per_step": t_two * 1e3},
            "speedup": t_one / t_two, "bitwise_equal": same}


def bench_c2(steps, warmup, args, with_oracle, precs=("c128", "mixed")):
    """The 287 x 287 x 200 decomposed grid (one centre point source): tuned
    complex128 and mixed plans, stage tables, oracle errors."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    p, f_np = W.c2_decomposed(core_cells=args.core, pml_cells=args.pml, nz=args.nz, nlayers=args.layers)
    nrhs = f_np.shape[0]
    f = hs.to_device(f_np)
    out = {"workload": f"c2_decomposed {p.nx}x{p.ny}x{p.nz}, 4x4 blocks + interface reduction, "
                       f"PML {args.pml}/side, {args.layers} layers, centre point source",
           "unknowns": p.unknowns, "nrhs": nrhs}
    us = {}
    for prec in precs:
        plan = hs.Plan(p, prec, max_rhs=nrhs, refine_steps=args.refine_steps if prec == "mixed" else 0)
        tuned = plan.tune(nrhs, cache=TUNE_CACHE)
        u = torch.empty_like(f)
        dt, stages, dom = time_plans([plan], f, u, steps, warmup)
        us[prec] = u.cpu().numpy()
        out[prec] = {"value": p.unknowns * nrhs * steps / dt, "ms_per_step": dt / steps * 1e3, "tuned": tuned,
                     "roofline": roofline(dom, prec),
                     "stages_ms_per_step": {r["name"]: round(r["ms"], 4) for r in stages}}
        del plan
    if "mixed" in out and "c128" in out:
        out["mixed_speedup_vs_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    if with_oracle:
        from oracle import separable
        ref = separable.solve(p, f_np)
        for prec in precs:
            out[prec]["rel_err_vs_oracle"] = errors_vs(us[prec][0], ref[0], p)
    return out


def bench_gridding_b(steps, warmup, with_oracle, refine_steps=1):
    """The second gridding of Sec. 2 at the large grid's size: 575 x 575 x 256
    on graded non-uniform x and y steps, 24 x 24 blocks of 23 nodes (dense
    eigenvector transforms everywhere, 23 separators per axis, dense global
    right-hand side), 4 point sources: tuned complex128 and mixed plans, stage
    tables, the dominant stage's roofline, oracle error on the first source;
    and the same grid with nested partitions (complex128): the interface
    problem of the 24 x 24 blocks solved by the cyclic reduction of the 5 x 5
    partition of every fifth separator."""
    import torch
    import paper_1909_01299_amd as hs
    import workloads as W
    p, srcs = W.gridding_b_large()
    nrhs = len(srcs)
    f = point_sources_device(p, srcs)
    out = {"workload": f"gridding_b {p.nx}x{p.ny}x{p.nz}, graded non-uniform x/y steps, "
                       f"{len(p.sep_x) + 1}x{len(p.sep_y) + 1} blocks, {nrhs} point sources",
           "unknowns": p.unknowns, "nrhs": nrhs, "separators_per_axis": [len(p.sep_x), len(p.sep_y)]}
    us = {}
    for prec in ("c128", "mixed"):
        t0 = time.perf_counter()
        plan = hs.Plan(p, prec, max_rhs=nrhs, refine_steps=refine_steps if prec == "mixed" else 0)
        t_plan = time.perf_counter() - t0
        tuned = plan.tune(nrhs, cache=TUNE_CACHE)
        u = torch.empty_like(f)
        dt, stages, dom = time_plans([plan], f, u, steps, warmup)
        us[prec] = u[0].cpu().numpy()
        out[prec] = {"value": p.unknowns * nrhs * steps / dt, "unit": "unknowns*RHS/s",
                     "ms_per_step": dt / steps * 1e3, "plan_seconds": t_plan, "tuned": tuned,
                     "roofline": roofline(dom, prec),
                     "stages_ms_per_step": {r["name"]: round(r["ms"], 3) for r in stages}}
        del plan, u
        torch.cuda.empty_cache()
    out["mixed_speedup_vs_c128"] = out["mixed"]["value"] / out["c128"]["value"]
    # nested partitions: the 24 x 24 blocks' interface problem solved by the
    # cyclic reduction of the 5 x 5 partition made of every fifth separator
    from dataclasses import replace
    coarse_p = replace(p, sep_x=p.sep_x[4::5].copy(), sep_y=p.sep_y[4::5].copy())
    fine = hs.Plan(p, "c128", max_rhs=nrhs)
    coarse = hs.Plan(coarse_p, "c128", max_rhs=nrhs)
    coarse.tune(nrhs, cache=TUNE_CACHE)
    fine.set_coarse(coarse)
    tuned = fine.tune(nrhs, cache=TUNE_CACHE)
    u = torch.empty_like(f)
    dt, stages, dom = time_plans([fine], f, u, steps, warmup)
    us["nested"] = u[0].cpu().numpy()
    out["nested_c128"] = {"value": p.unknowns * nrhs * steps / dt, "unit": "unknowns*RHS/s",
                          "ms_per_step": dt / steps * 1e3, "tuned": tuned,
                          "coarse_separators_per_axis": [len(coarse_p.sep_x), len(coarse_p.sep_y)],
                          "stages_ms_per_step": {r["name"]: round(r["ms"], 3) for r in stages}}
    del fine, coarse, u
    torch.cuda.empty_cache()
    if with_oracle:
        from oracle import separable
        ref = separable.solve(p, W.point_source_batch(p, srcs[:1]))[0]
        for prec in ("c128", "mixed", "nested"):
            key = "nested_c128" if prec == "nested" else prec
            out[key]["rel_err_vs_oracle_src0"] = errors_vs(us[prec], ref, p)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (baseline and errors)")
    ap.add_argument("--core", type=int, default=256, help="decomposed_c2: uniform core cells per axis")
    ap.add_argument("--pml", type=int, default=16)
    ap.add_argument("--nz", type=int, default=200)
    ap.add_argument("--layers", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true", help="headline only (no c2, c3, c4 workloads)")
    ap.add_argument("--no-streams", action="store_true",
                    help="skip the extra record of the headline workload as two halves on two streams")
    ap.add_argument("--c3-steps", type=int, default=5)
    ap.add_argument("--refine-steps", type=int, default=1,
                    help="FP64-residual refinement steps of the mixed-precision solves (-1: none)")
    ap.add_argument("--copy", action="store_true", help="counter calibration: a plain 1 GiB copy")
    ap.add_argument("--counters", action="store_true", help="complex128 solves for counter runs")
    ap.add_argument("--counters-workload", choices=["c5", "c2"], default="c5")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH", "WRITE", "CFETCH", "CWRITE"),
                    help="write profiles/pmc_traffic.json from four rocprofv3 --pmc output folders")
    ap.add_argument("--c2-only", choices=["c128", "mixed", "both"],
                    help="time only the 287x287x200 decomposed grid (no oracle): for kernel traces")
    ap.add_argument("--c3-only", choices=["c128", "mixed", "both"], help="time only the 64-block batch")
    ap.add_argument("--c4-only", action="store_true", help="time only the adjoint gradient (128x128x160)")
    ap.add_argument("--gridding-b-only", action="store_true",
                    help="time only the 575x575x256 grid split 24x24 on graded steps")
    ap.add_argument("--c5-only", choices=["c128", "mixed", "both"],
                    help="time only the headline workload (no oracle): for kernel traces")
    ap.add_argument("--c5-streams", action="store_true",
                    help="the headline workload (complex128) as two 8-source halves on two streams")
    ap.add_argument("--tune-cache", help="JSON-lines cache of tuned launch shapes (read, else written)")
    ap.add_argument("--stats-summary", nargs=3, metavar=("TRACE_CSV", "TITLE", "COMMAND"),
                    help="print a text summary of a rocprofv3 kernel trace")
    ap.add_argument("--sq-summary", nargs=2, metavar=("SQ1", "SQ2"),
                    help="print a per-kernel summary of two rocprofv3 --pmc runs of the SQ counter sets")
    ap.add_argument("--mfma-summary", nargs="+", metavar="P PMC TRACE",
                    help="print the issued matrix-core rate per kernel from (precision, --pmc folder, "
                         "kernel-trace folder) triples")
    ap.add_argument("--stage-labels", action="store_true",
                    help="with --stats-summary: list the z sweeps of decomposed solves by stage")
    args = ap.parse_args()
    global TUNE_CACHE
    TUNE_CACHE = args.tune_cache
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    if args.stats_summary:
        stats_summary(*args.stats_summary, stage_labels=args.stage_labels)
        return
    if args.sq_summary:
        sq_summary(*args.sq_summary)
        return
    if args.mfma_summary:
        mfma_summary(args.mfma_summary)
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
    if args.counters:
        counters_run(args)
        return
    if args.c2_only:
        precs = ("c128", "mixed") if args.c2_only == "both" else (args.c2_only,)
        print(json.dumps(bench_c2(max(1, args.steps), args.warmup, args, False, precs=precs)), flush=True)
        return
    if args.c3_only:
        precs = ("c128", "mixed") if args.c3_only == "both" else (args.c3_only,)
        print(json.dumps(bench_c3(args.c3_steps, 1, False, precs=precs, refine_steps=args.refine_steps)), flush=True)
        return
    if args.c4_only:
        print(json.dumps(bench_c4(max(1, args.steps), True)), flush=True)
        return
    if args.gridding_b_only:
        print(json.dumps(bench_gridding_b(max(1, args.steps), args.warmup, not args.no_cpu_baseline,
                                          refine_steps=args.refine_steps)), flush=True)
        return
    if args.c5_streams:
        print(json.dumps(bench_c5_streams(max(1, args.steps), args.warmup)), flush=True)
        return
    if args.c5_only:
        precs = ("c128", "mixed") if args.c5_only == "both" else (args.c5_only,)
        print(json.dumps(bench_c5(args.steps, args.warmup, args.refine_steps, with_oracle=False, precs=precs,
                                  profile_only=True)), flush=True)
        return

    import torch
    torch.cuda.set_device(0)
    with_oracle = not args.no_cpu_baseline
    c5 = bench_c5(args.steps, args.warmup, args.refine_steps, with_oracle=with_oracle)
    print(json.dumps({"progress": "headline done", "c128_ms_per_step": c5["c128"]["ms_per_step"]}),
          file=sys.stderr, flush=True)
    extras = {}
    if not args.no_extras:
        torch.cuda.empty_cache()
        extras["decomposed_c2"] = bench_c2(20, 3, args, with_oracle)
        print(json.dumps({"progress": "c2 done"}), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["batched_c3"] = bench_c3(args.c3_steps, 1, with_oracle, refine_steps=args.refine_steps)
        print(json.dumps({"progress": "c3 done"}), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["adjoint_c4"] = bench_c4(10, with_oracle)
        print(json.dumps({"progress": "c4 done"}), file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        extras["gridding_b"] = bench_gridding_b(3, 1, with_oracle, refine_steps=args.refine_steps)
        print(json.dumps({"progress": "gridding B done"}), file=sys.stderr, flush=True)
    if not args.no_extras and not args.no_streams:
        torch.cuda.empty_cache()
        extras["c5_two_streams"] = bench_c5_streams(3, 1)

    c128 = c5["c128"]
    rf = c128["roofline"]
    if rf is not None:
        rf["traffic"] = traffic_for(rf["kernel"])
    mixed = c5.get("mixed")
    line = {
        "metric": "unknowns*RHS/s (decomposed 3D Helmholtz solve, complex128)",
        "value": c128["value"],
        "unit": "unknowns*RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": c128["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": c5["workload"], "unknowns": c5["unknowns"], "nrhs": c5["nrhs"],
                   "omegas": c5["omegas"], "unknowns_rhs_per_step": c5["unknowns_rhs_per_step"],
                   "blocks": 16},
        "rel_err_vs_oracle": c128.get("rel_err_vs_oracle"),
        "roofline": rf,
        "cpu_baseline": c5.get("cpu_baseline"),
        "stages_ms_per_step": c128["stages_ms_per_step"],
        "rel_residual_rhs0_per_omega": c128.get("rel_residual_rhs0_per_omega"),
        "plan_seconds_4_plans": c128["plan_seconds_4_plans"],
        "mixed_c64_refine": mixed and {
            "value": mixed["value"], "ms_per_step": mixed["ms_per_step"],
            "refine_steps": mixed.get("refine_steps"), "speedup_vs_c128": c5.get("mixed_speedup_vs_c128"),
            "rel_err_vs_oracle": mixed.get("rel_err_vs_oracle"), "roofline": mixed["roofline"],
            "stages_ms_per_step": mixed["stages_ms_per_step"],
            "rel_residual_rhs0_per_omega": mixed.get("rel_residual_rhs0_per_omega")},
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
