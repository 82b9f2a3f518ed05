#!/usr/bin/env python3
"""Throughput of the SARABANDE hot path on one MI355X.

Default workload: the full 3PCF of two 256^3 float32 lognormal fields (sigma 0.5
and 1.5, P(k) ~ k^-11/3), 10 linear bins over (0, 32] cells, l_max = 6.  One step =
one forward pass over that batch: density FFT, correlation of all 280 binned Y_lm
kernels by FFT, 3PCF contraction and the float64 grid sum.  The kernel spectra are
generated once (the cold set-up, reported separately) and stay resident in HBM.

Prints one JSON line (metric, value in fields/s, roofline of the dominant kernel,
the CPU oracle's throughput on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3PCF/4PCF fields/sec at 256^3 & 128^3 vs plain FP32 GPU at stated err; %HBM/MFMA peak"
HBM_PEAK_GBS = 8000.0


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key, src_files):
    """HBM bytes per launch measured with rocprofv3 counters (committed under profiles/),
    or None when the kernel source changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel_key)
    if not e or e.get("source_hash") != source_hash(src_files):
        return None
    return e.get("bytes_per_launch")


TRAFFIC_SRCS = {0: ["paper_2210_10206_amd/csrc/fft.hip", "paper_2210_10206_amd/csrc/fft_core.h"],
                1: ["paper_2210_10206_amd/csrc/fft.hip", "paper_2210_10206_amd/csrc/fft_core.h"],
                2: ["paper_2210_10206_amd/csrc/fft_last.h", "paper_2210_10206_amd/csrc/fft_core.h"],
                3: ["paper_2210_10206_amd/csrc/contract.hip"]}


def write_traffic(counter_dir, n=256, copy_mib=1024, min_gib=1.0):
    """Turn two rocprofv3 counter runs of `bench.py --steps 1 --copy-probe-mib <copy_mib>`
    (counter_dir/FETCH_SIZE and counter_dir/WRITE_SIZE, csv output) into
    profiles/traffic.json.  Each counter is scaled by bytes / counter of the plain
    copy_mib MiB device copy in the same run (the __amd_rocclr_copyBuffer dispatches of that
    size); the passes over all kernel arrays are the dispatches of each kernel family with at
    least min_gib GiB of either counter, and of the axis-0 and middle passes only the variant
    of the run's last dispatch (the one the autotuner picked and the timed step used).  The
    last pass is two launches per field (packed m = 0 pairs, other groups): their bytes are
    summed."""
    import csv
    import re
    reg = {256: 16}.get(n)   # lengths with the register-resident forms (n = r * r)
    fams = {0: re.compile(rf"fft_pass(_pf)?_kernel<{n}, \d+, \d+, 1,|mid_reg_kernel<{reg}, {n // reg}, \d+, 1>"
                          if reg else rf"fft_pass(_pf)?_kernel<{n}, \d+, \d+, 1,"),
            1: re.compile(rf"axis0_kernel<{n},|axis0_reg_kernel<{reg}, " if reg else rf"axis0_kernel<{n},"),
            2: re.compile(rf"last_contract_kernel<{n},|last_reg_kernel<{reg}, " if reg else
                          rf"last_contract_kernel<{n},")}
    raw = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        path = os.path.join(counter_dir, ctr, "run_counter_collection.csv")
        with open(path) as f:
            raw[ctr] = {int(r["Dispatch_Id"]): (r["Kernel_Name"], float(r["Counter_Value"]))
                        for r in csv.DictReader(f) if r["Counter_Name"] == ctr}
    copy_bytes = copy_mib * 2 ** 20
    scale = {}
    for ctr, want in (("FETCH_SIZE", copy_bytes), ("WRITE_SIZE", copy_bytes)):
        vals = sorted(v for name, v in raw[ctr].values() if "copyBuffer" in name)
        big = [v for v in vals if v * 1024 > 0.25 * want]          # KiB -> bytes
        if not big:
            raise SystemExit(f"no {copy_mib} MiB copy dispatch in the {ctr} run")
        scale[ctr] = want / (sum(big) / len(big) * 1024)
    out = {"_note": f"HBM bytes per dispatch from rocprofv3 FETCH_SIZE / WRITE_SIZE (KiB), each scaled by "
                    f"bytes / counter of a plain {copy_mib} MiB device copy in the same run",
           "_scale": {k: round(v, 4) for k, v in scale.items()}}
    for k, rx in fams.items():
        per_name = {}
        last_name = None
        for did in sorted(raw["FETCH_SIZE"]):
            name, fv = raw["FETCH_SIZE"][did]
            if not rx.search(name) or did not in raw["WRITE_SIZE"]:
                continue
            wv = raw["WRITE_SIZE"][did][1]
            if max(fv, wv) * 1024 < min_gib * 2 ** 30:
                continue
            per_name.setdefault(name, []).append((fv, wv))
            last_name = name
        if not per_name:
            continue
        # one pass over a field's arrays: for the axis-0 and middle passes the variant of the
        # last dispatch (the timed step runs last, with the variant the autotuner chose), for
        # the last pass every dispatch name launched as often as the most frequent one (the
        # packed m = 0 pairs and the other groups are two launches per field), summed
        if k != 2:
            names = [last_name]
            nmax = len(per_name[last_name])
        else:
            nmax = max(len(v) for v in per_name.values())
            names = [q for q in per_name if len(per_name[q]) == nmax]
        fetch = sum(sum(x[0] for x in per_name[q]) / nmax for q in names) * 1024 * scale["FETCH_SIZE"]
        write = sum(sum(x[1] for x in per_name[q]) / nmax for q in names) * 1024 * scale["WRITE_SIZE"]
        out[f"kernel{k}_n{n}"] = {"kernel": " + ".join(names), "dispatches": nmax, "fetch_bytes": round(fetch),
                                  "write_bytes": round(write), "bytes_per_launch": round(fetch + write),
                                  "source_hash": source_hash(TRAFFIC_SRCS[k])}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def block_errors(z, ref):
    """Whole-result error, per-block errors along the leading axis (each relative to that block's
    max |ref|) and the worst entry relative to its own block: the parity measure of the tests."""
    import numpy as np
    z, ref = np.asarray(z), np.asarray(ref)
    per = [float(np.max(np.abs(z[i] - ref[i])) / np.max(np.abs(ref[i]))) for i in range(ref.shape[0])]
    return {"max_rel_err": float(np.max(np.abs(z - ref)) / np.max(np.abs(ref))), "worst_block": max(per),
            "per_block": [round(e, 10) for e in per]}


def counters_for(kernel_key, src_files):
    """MFMA / VALU figures of a contraction kernel from rocprofv3 counter runs (committed under
    profiles/), or None when the kernel source changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", "mfma_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel_key)
    if not e or e.get("source_hash") != source_hash(src_files):
        return None
    return {k: v for k, v in e.items() if k != "source_hash"}


FIELDS_PER_LAUNCH = {"quad": 16, "proj4": 1}   # fields of one timed launch in the c4 / c4var and proj lines
COUNTER_SRCS = {"quad_mfma": ["paper_2210_10206_amd/csrc/quad_mfma.h"],
                "proj4_mfma": ["paper_2210_10206_amd/csrc/proj4_mfma.hip"]}


def write_counters(counter_csv):
    """Turn a rocprofv3 counter run of `bench.py --lines c4,c4var,proj --c4-steps 1 --proj-steps 1`
    (--pmc MfmaUtil VALUBusy MfmaFlopsF32 MfmaFlopsBF16 SQ_INSTS_VALU SQ_INSTS_MFMA, csv output)
    into profiles/mfma_counters.json: per contraction family (4PCF matrix-core kernels by
    precision and parity, projected-4PCF kernels by precision), the duration-weighted MfmaUtil and
    VALUBusy over its dispatches and the issued MFMA flops and instructions of one field: the sum
    over the family's kernels of the counts of each kernel's last dispatch (a timed step's batch
    launch) divided by the fields of that launch, FIELDS_PER_LAUNCH of the family (the 4PCF lines
    run 16-field batches in one launch per Lambda; the autotuner's earlier single-field
    candidates are left out of the counts)."""
    import csv
    import re
    rows = {}
    with open(counter_csv) as f:
        for r in csv.DictReader(f):
            d = rows.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})
            d[r["Counter_Name"]] = float(r["Counter_Value"])
            if r.get("Start_Timestamp") and r.get("End_Timestamp"):
                d["ns"] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])

    def family(name):
        m = re.search(r"quad_mfma_kernel<(\d+), (\d+), (\d+), (\d+)>", name)
        if m:
            la, lb, lc, prec = (int(x) for x in m.groups())
            return f"quad_mfma_prec{prec}_{'odd' if (la + lb + lc) % 2 else 'even'}", (la, lb, lc)
        m = re.search(r"proj4_(mfma|split)_kernel<(\d+)>", name)
        if m:
            return f"proj4_prec{1 if m.group(1) == 'split' else 0}", (int(m.group(2)),)
        return None, None

    fams = {}
    for _, d in sorted(rows.items()):   # dispatch order: each kernel's list ends with its last dispatch
        fam, key = family(d["name"])
        if fam is None:
            continue
        fams.setdefault(fam, {}).setdefault(key, []).append(d)
    out = {"_note": "rocprofv3 counters per contraction family: MfmaUtil = sum SQ_VALU_MFMA_BUSY_CYCLES / "
                    "(GRBM_GUI_ACTIVE x SIMDs), VALUBusy = sum SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE (both "
                    "percent, weighted by dispatch duration); issued MFMA flops (MOPS x 512) and instruction "
                    "counts per field"}
    for fam, kernels in fams.items():
        w = sum(d.get("ns", 1.0) for ds in kernels.values() for d in ds)
        util = sum(d.get("MfmaUtil", 0.0) * d.get("ns", 1.0) for ds in kernels.values() for d in ds) / w
        valu = sum(d.get("VALUBusy", 0.0) * d.get("ns", 1.0) for ds in kernels.values() for d in ds) / w
        per_field = {}
        nf = FIELDS_PER_LAUNCH["quad" if fam.startswith("quad") else "proj4"]
        for c in ("MfmaFlopsF32", "MfmaFlopsBF16", "SQ_INSTS_VALU", "SQ_INSTS_MFMA"):
            per_field[c] = sum(ds[-1].get(c, 0.0) / nf for ds in kernels.values())
        out[fam] = {"kernels": len(kernels), "dispatches": sum(len(ds) for ds in kernels.values()),
                    "mfma_util_pct": round(util, 2), "valu_busy_pct": round(valu, 2),
                    "mfma_flops_f32_per_field": per_field["MfmaFlopsF32"],
                    "mfma_flops_bf16_per_field": per_field["MfmaFlopsBF16"],
                    "valu_insts_per_field": per_field["SQ_INSTS_VALU"],
                    "mfma_insts_per_field": per_field["SQ_INSTS_MFMA"],
                    "source_hash": source_hash(COUNTER_SRCS["quad_mfma" if fam.startswith("quad") else "proj4_mfma"])}
    with open(os.path.join(ROOT, "profiles", "mfma_counters.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def cpu_baseline(field, edges, lmax, target_s=10.0):
    """Oracle throughput on a bounded sample of cells of field 0: two probe sizes give the
    per-cell rate without the oracle's one-off table set-up, then a sample sized for about
    target_s seconds is timed as a whole."""
    import numpy as np
    import oracle
    d = field.astype(np.float64)
    ng = d.size

    def run(n):
        t0 = time.perf_counter()
        oracle.zeta3_full(d, edges, lmax, cells=np.arange(n))
        return time.perf_counter() - t0

    t1, t2 = run(512), run(2560)
    per_cell = max((t2 - t1) / 2048.0, 1e-9)
    n = int(min(ng, max(2560, target_s / per_cell)))
    n = (n // 256) * 256
    dt = run(n)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": (n / ng) / dt, "unit": "fields/s", "cores": int(oracle.max_threads()), "kind": "oracle",
            "cpu_model": model,
            "sample": f"full-3PCF oracle (direct FP64 correlation + contraction) over the first {n} of the "
                      f"{ng} cells of field 0, {dt:.1f} s wall including its table set-up; value scaled to whole "
                      f"fields"}


def run_4pcf_batch(api, steps, warmup, count=16, precision="fp32", mfma=True, parity="even"):
    """Full 4PCF of the 16-field 128^3 batch (sigma_i ~ U[0.5, 2]), 8 bins to 24, even
    Lambda with l <= 4, one plan and one forward per step; the fields/s of the batch and the
    live rate of its dominant kernel (the 3j-coupled contraction: on the matrix cores in
    float32 or split-BF16, or the plain float32 vector-ALU kernel with mfma=False)."""
    import torch
    from fieldgen import c4_batch, linear_edges
    fields, _ = c4_batch(128, count)
    dev = [torch.from_numpy(f).cuda() for f in fields]
    stream = torch.cuda.Stream()
    plan = api.Plan([f.shape for f in fields], linear_edges(24, 8), 4, npcf=4, prepare=False,
                    precision=precision, mfma=mfma, parity=parity)
    with torch.cuda.stream(stream):
        plan.prepare(stream)
    plan.autotune(stream)
    out = torch.empty((len(dev), plan.zeta_doubles), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.forward_raw(dev, out=out, stream=stream)
    stream.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.forward_raw(dev, out=out, stream=stream)
    stream.synchronize()
    el = time.perf_counter() - t0
    recs = plan.launch_records()
    plan.profile(False)
    # the same steps replayed from the HIP graph of the whole batch forward
    with torch.cuda.stream(stream):
        plan.forward_raw(dev, out=out, stream=stream, graph=True)   # capture
    stream.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.forward_raw(dev, out=out, stream=stream, graph=True)
    stream.synchronize()
    el_graph = time.perf_counter() - t0
    q = [r for r in recs if r["kernel"] in (4, 7)]
    ms = sum(r["ms"] for r in q)
    fl = sum(r["flops"] for r in q)
    if mfma:
        kname = ("quad_mfma_kernel<la,lb,lc," + ("1> (split-BF16 MFMA" if precision == "split_bf16" else "0> (float32 MFMA")
                 + ", one launch per canonical Lambda)")
    else:
        kname = "quad_kernel (3j-coupled contraction, float32 VALU)"
    res = {"workload": f"full 4PCF, {count} lognormal 128^3 float32 fields (sigma ~ U[0.5,2]), 8 bins over (0,24], "
                       f"{parity} Lambda with l <= 4 ({'42' if parity == 'even' else '23'})",
           "precision": precision, "matrix_cores": bool(mfma), "contract_tile": plan.contract_tile()[0],
           "fields_per_launch": plan.field_batch, "pass_launches_per_batch": round(len(recs) / steps, 1),
           "value": round(count * steps / el, 3), "unit": "fields/s", "ms_per_step": round(el / steps * 1e3, 2),
           "graph_replay": {"value": round(count * steps / el_graph, 3), "ms_per_step": round(el_graph / steps * 1e3, 2)},
           "contraction": {"kernel": kname,
                           "flops_note": "executed floating-point work of the kernel on real bins (its symmetric pair "
                                         "tiles and paired +-m at m_c = 0 counted as computed; padding excluded), "
                                         "VALU coupling and MFMA contraction together, against the float32 peak",
                           "achieved_tflops": round(fl / (ms * 1e-3) / 1e12, 2) if ms else None,
                           "peak_tflops": 157.3, "frac": round(fl / (ms * 1e-3) / 1e12 / 157.3, 4) if ms else None,
                           "ms_per_field": round(ms / (count * steps), 3),
                           "counters": counters_for(f"quad_mfma_prec{1 if precision == 'split_bf16' else 0}_{parity}",
                                                    COUNTER_SRCS["quad_mfma"]) if mfma else None},
           "stage_ms_per_field": {}}
    if parity == "even":
        import numpy as np
        z = out.cpu().numpy()
        errs = {}
        for i in (0, 1):
            g = os.path.join(ROOT, "tests", "golden", f"c4_full4_128_field{i}.npz")
            if os.path.exists(g):
                ref = np.load(g)["zeta4"].real
                e = block_errors(z[i].reshape(ref.shape), ref)
                errs[f"field{i}"] = {"max_rel_err": e["max_rel_err"], "worst_lambda_block": e["worst_block"]}
        res["err_vs_oracle"] = errs or None
    for r in recs:
        k = {0: "fft", 1: "fft", 4: "contract", 7: "contract"}.get(r["kernel"], "other")
        res["stage_ms_per_field"][k] = res["stage_ms_per_field"].get(k, 0.0) + r["ms"] / (count * steps)
    res["stage_ms_per_field"] = {k: round(v, 3) for k, v in res["stage_ms_per_field"].items()}
    plan.close()
    return res


def run_c5(api, steps, warmup, synth_steps=200):
    """Forward + adjoint of the uneven 48-field batch (edges drawn from 64/96/128/160/192,
    sigma 1 lognormal), 8 bins to 16, lmax 4, one plan, then on a plan that keeps the forward's arrays for
    the adjoint; then the synthesis demo (a keeping plan): 200 Adam
    steps at 128^3 from a Gaussian field towards the sums of the seed-100 lognormal field."""
    import numpy as np
    import torch
    from fieldgen import c5_batch, gaussian_field, lognormal_field, linear_edges
    from paper_2210_10206_amd.synthesis import synthesize
    fields, edges_list = c5_batch()
    dev = [torch.from_numpy(f).cuda() for f in fields]
    edges = linear_edges(16, 8)
    plan = api.Plan([f.shape for f in fields], edges, 4, npcf=3)
    plan.autotune(torch.cuda.current_stream())
    G = torch.from_numpy(np.random.Generator(np.random.PCG64(5)).standard_normal((len(dev), 5, 8, 8))).cuda()
    for _ in range(warmup):
        plan.forward(dev)
        plan.backward(dev, G)
    torch.cuda.synchronize()
    plan.profile(True)
    plan.forward_raw(dev)
    torch.cuda.synchronize()
    fwd_launches = len(plan.launch_records())
    plan.profile(False)
    # the same forward replayed from a HIP graph of the whole batch
    gs = torch.cuda.Stream()
    gout = torch.empty((len(dev), plan.zeta_doubles), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(gs):
        plan.forward_raw(dev, out=gout, stream=gs, graph=True)
    gs.synchronize()
    tg = time.perf_counter()
    with torch.cuda.stream(gs):
        for _ in range(steps):
            plan.forward_raw(dev, out=gout, stream=gs, graph=True)
    gs.synchronize()
    graph_fps = len(fields) * steps / (time.perf_counter() - tg)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forward_raw(dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        plan.backward(dev, G)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ncell = sum(int(np.prod(f.shape)) for f in fields)
    # parity of the same plan against the stored oracle values (outside the timed region): the
    # sums of every stored field, and the gradient at the stored cells for the stored weights
    fwd_err, grad_err = {}, {}
    z = plan.forward_raw(dev).cpu().numpy()
    Gg = np.zeros((len(dev), 5, 8, 8))
    gold_g = {}
    for i, n in enumerate(edges_list):
        fz = os.path.join(ROOT, "tests", "golden", f"c5_full3_{n}_field{i}.npz")
        if os.path.exists(fz):
            ref = np.load(fz)["zeta3"].real
            e = block_errors(z[i].reshape(ref.shape), ref)
            fwd_err[f"{n}^3 field {i}"] = {"max_rel_err": e["max_rel_err"], "worst_l_block": e["worst_block"]}
        fg = os.path.join(ROOT, "tests", "golden", f"c5_grad3_{n}_field{i}.npz")
        if os.path.exists(fg):
            gold_g[i] = np.load(fg)
            Gg[i] = gold_g[i]["G"]
    if gold_g:
        grads = plan.backward(dev, torch.from_numpy(Gg).cuda())
        for i, g in gold_g.items():
            got = grads[i].reshape(-1)[torch.from_numpy(g["cells"]).cuda()].double().cpu().numpy()
            grad_err[f"{edges_list[i]}^3 field {i}"] = float(np.max(np.abs(got - g["grad"])) / np.max(np.abs(g["grad"])))
    plan_fb = plan.field_batch
    plan.close()
    del plan
    torch.cuda.empty_cache()
    # the same batch with the coefficient arrays kept from each forward for the adjoint
    # (SB_FLAG_KEEP_FOR_ADJOINT): every field's arrays at once in scratch
    kp = api.Plan([f.shape for f in fields], edges, 4, npcf=3, keep_for_adjoint=True)
    kp.autotune(torch.cuda.current_stream())
    for _ in range(warmup):
        kp.forward_raw(dev)
        kp.backward(dev, G)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    tk0 = time.perf_counter()
    for i in range(steps):
        kp.forward_raw(dev)
        ev[2 * i].record()
        kp.backward(dev, G)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    tk1 = time.perf_counter()
    kept_adj_ms = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(steps))
    kept_grad_err = {}
    if gold_g:
        kp.forward_raw(dev)
        grads = kp.backward(dev, torch.from_numpy(Gg).cuda())
        for i, g in gold_g.items():
            got = grads[i].reshape(-1)[torch.from_numpy(g["cells"]).cuda()].double().cpu().numpy()
            kept_grad_err[f"{edges_list[i]}^3 field {i}"] = float(np.max(np.abs(got - g["grad"]))
                                                                 / np.max(np.abs(g["grad"])))
    kept_scratch_gb = kp._scratch.numel() / 1e9
    kp.close()
    del kp
    torch.cuda.empty_cache()
    del dev
    res = {"workload": f"uneven batch of {len(fields)} sigma-1 lognormal float32 cubes, edges from "
                       f"64/96/128/160/192 ({ncell / len(fields) / 1e6:.2f} M cells on average), 8 bins over "
                       "(0,16], lmax 4, one plan",
           "fields_per_launch": plan_fb, "pass_launches_per_forward": fwd_launches,
           "forward_fields_per_s": round(len(fields) * steps / (t1 - t0), 2),
           "forward_graph_replay_fields_per_s": round(graph_fps, 2),
           "adjoint_fields_per_s": round(len(fields) * steps / (t2 - t1), 2),
           "forward_plus_adjoint_fields_per_s": round(len(fields) * steps / (t2 - t0), 2),
           "kept_for_adjoint": {"scratch_gb": round(kept_scratch_gb, 1),
                                "adjoint_fields_per_s": round(len(fields) * steps / (kept_adj_ms / 1e3), 2),
                                "forward_plus_adjoint_fields_per_s": round(len(fields) * steps / (tk1 - tk0), 2),
                                "gradient_err_vs_oracle_at_stored_cells": kept_grad_err or None},
           "forward_err_vs_oracle": fwd_err or None,
           "gradient_err_vs_oracle_at_stored_cells": grad_err or None, "synthesis": None}
    if synth_steps <= 0:
        return res
    n = 128
    sp = api.Plan([(n, n, n)], edges, 4, npcf=3, keep_for_adjoint=True)   # each step's backward reads the forward's arrays
    sp.autotune(torch.cuda.current_stream())
    target = sp.forward([torch.from_numpy(lognormal_field((n,) * 3, seed=100, sigma=1.0)).cuda()])[0]
    init = torch.from_numpy(gaussian_field((n,) * 3, seed=101)).cuda()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    _, losses = synthesize(sp, target, init, steps=synth_steps, lr=0.05, history_every=max(1, synth_steps // 10))
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    sp.close()
    res["synthesis"] = {"grid": n, "steps": synth_steps, "seconds": round(t4 - t3, 3),
                        "ms_per_step": round((t4 - t3) / synth_steps * 1e3, 3),
                        "loss_start": losses[0], "loss_end": losses[-1], "kept_for_adjoint": True}
    return res


def run_512(api, steps, warmup):
    """Full 3PCF of one 512^3 field (the 2x2x2 tiling of the sigma 0.5 seed 0 256^3 field: the
    generator's 512^3 FFT would dominate the run), 10 bins to 32, lmax 6: cold set-up and
    warm fields/s with the kernel arrays in chunks of (l, m) groups."""
    import torch
    from fieldgen import lognormal_field, linear_edges
    d = torch.from_numpy(lognormal_field((256,) * 3, seed=0, sigma=0.5)).cuda().repeat(2, 2, 2).contiguous()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = api.Plan([tuple(d.shape)], linear_edges(32, 10), 6, npcf=3, prepare=False)
    with torch.cuda.stream(stream):
        plan.prepare(stream)
    stream.synchronize()
    cold = time.perf_counter() - t0
    plan.autotune(stream)
    out = torch.empty((1, plan.zeta_doubles), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.forward_raw([d], out=out, stream=stream)
    stream.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.forward_raw([d], out=out, stream=stream)
    stream.synchronize()
    el = time.perf_counter() - t0
    recs = plan.launch_records()
    plan.profile(False)
    kinds = {0: "fft_passes", 1: "axis0_correlation", 2: "fused_last_pass", 3: "pair_contraction"}
    per = {}
    for r in recs:
        k = kinds.get(r["kernel"], "other")
        per[k] = per.get(k, 0.0) + r["ms"] / steps
    res = {"workload": "full 3PCF of one 512^3 float32 field (2x2x2 tiling of the 256^3 sigma 0.5 field), "
                       "10 bins over (0,32], lmax 6",
           "value": round(steps / el, 3), "unit": "fields/s", "ms_per_field": round(el / steps * 1e3, 2),
           "cold_setup_ms": round(cold * 1e3, 1),
           "persistent_GiB": round(plan.persistent_bytes / 2 ** 30, 2),
           "scratch_GiB": round(plan.scratch_bytes / 2 ** 30, 2),
           "stage_ms_per_field": {k: round(v, 1) for k, v in per.items()},
           "tuned_launch_shapes": plan.choices()}
    plan.close()
    return res


def run_1024(api, steps, warmup):
    """Full 3PCF of one 1024^3 field (the 4x4x4 tiling of the sigma 0.5 seed 0 256^3 field), 10
    bins to 32, lmax 6: no kernel cache (it would take about 169 GB); each chunk of (l, m) groups
    regenerates its kernel planes, and the 1024-point last pass is fused with the pair sums.
    Fields/s and the per-stage times."""
    import torch
    from fieldgen import lognormal_field, linear_edges
    d = torch.from_numpy(lognormal_field((256,) * 3, seed=0, sigma=0.5)).cuda().repeat(4, 4, 4).contiguous()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = api.Plan([tuple(d.shape)], linear_edges(32, 10), 6, npcf=3, prepare=False)
    with torch.cuda.stream(stream):
        plan.prepare(stream)
    stream.synchronize()
    cold = time.perf_counter() - t0
    out = torch.empty((1, plan.zeta_doubles), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.forward_raw([d], out=out, stream=stream)
    stream.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.forward_raw([d], out=out, stream=stream)
    stream.synchronize()
    el = time.perf_counter() - t0
    recs = plan.launch_records()
    plan.profile(False)
    kinds = {0: "fft_passes", 1: "axis0_correlation", 2: "fused_last_pass", 3: "pair_contraction"}
    per = {}
    for r in recs:
        k = kinds.get(r["kernel"], "other")
        per[k] = per.get(k, 0.0) + r["ms"] / steps
    res = {"workload": "full 3PCF of one 1024^3 float32 field (4x4x4 tiling of the 256^3 sigma 0.5 field), "
                       "10 bins over (0,32], lmax 6, kernel spectra regenerated per chunk of (l, m) groups",
           "value": round(steps / el, 4), "unit": "fields/s", "ms_per_field": round(el / steps * 1e3, 1),
           "setup_ms": round(cold * 1e3, 1),
           "persistent_GiB": round(plan.persistent_bytes / 2 ** 30, 4),
           "scratch_GiB": round(plan.scratch_bytes / 2 ** 30, 2),
           "stage_ms_per_field": {k: round(v, 1) for k, v in per.items()}}
    plan.close()
    del d, out
    torch.cuda.empty_cache()
    return res


def run_proj(api, steps, warmup):
    """Projected 3PCF and 4PCF (Alg. 7, 8) of the 512^2 sigma 1 lognormal field (seed 0), 10
    bins over (0,40], m up to 10, with float32 and split-BF16 contractions: fields/s of each, the
    per-stage times, the live rate of the projected 4PCF contraction, and the error against the
    stored oracle sums (whole result and worst m / (m1, m2) block)."""
    import numpy as np
    import torch
    from fieldgen import lognormal_field, linear_edges
    d = lognormal_field((512, 512), seed=0, sigma=1.0)
    dev = [torch.from_numpy(d).cuda()]
    gpath = os.path.join(ROOT, "tests", "golden", "c2_proj_512.npz")
    gold = np.load(gpath) if os.path.exists(gpath) else None
    stream = torch.cuda.Stream()
    res = {"workload": "projected 3PCF and 4PCF of one 512^2 float32 lognormal field (sigma 1), 10 bins over (0,40], "
                       "m up to 10 (331 (m1, m2) pairs)"}
    for precision in ("fp32", "split_bf16"):
        for npcf in (3, 4):
            plan = api.Plan([d.shape], linear_edges(40, 10), 10, npcf=npcf, prepare=False, precision=precision)
            with torch.cuda.stream(stream):
                plan.prepare(stream)
            plan.autotune(stream)
            out = torch.empty((1, plan.zeta_doubles), dtype=torch.float64, device="cuda")
            with torch.cuda.stream(stream):
                for _ in range(warmup):
                    plan.forward_raw(dev, out=out, stream=stream)
            stream.synchronize()
            plan.profile(True)
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                for _ in range(steps):
                    plan.forward_raw(dev, out=out, stream=stream)
            stream.synchronize()
            el = time.perf_counter() - t0
            recs = plan.launch_records()
            plan.profile(False)
            r = {"value": round(steps / el, 2), "unit": "fields/s", "ms_per_field": round(el / steps * 1e3, 3),
                 "fft_ms_per_field": round(sum(x["ms"] for x in recs if x["stage"] == 0) / steps, 3),
                 "contract_ms_per_field": round(sum(x["ms"] for x in recs if x["stage"] == 1) / steps, 3)}
            if npcf == 4:
                q = [x for x in recs if x["kernel"] == 5]
                ms, fl = sum(x["ms"] for x in q), sum(x["flops"] for x in q)
                if ms:
                    kn = ("proj4_split_kernel<10> (split-BF16 bf16 16x16x32 MFMA" if precision == "split_bf16"
                          else "proj4_mfma_kernel<10> (float32 16x16x4 MFMA")
                    r["contraction"] = {
                        "kernel": kn + ", one launch over the (cell block, canonical m triple) items, "
                                       "XCD-aware order)",
                        "flops_note": "complex-arithmetic work: per cell and canonical triple NB^2 (8 + 8 NB) flops "
                                      "(w c_m1 c_m2 per pair, a complex multiply-add per (pair, b3)), against the "
                                      "float32 peak; the float32 kernel issues the multiply-adds as three real "
                                      "products (Gauss), 3/4 of these flops on MFMA",
                        "achieved_tflops": round(fl / (ms * 1e-3) / 1e12, 2), "peak_tflops": 157.3,
                        "frac": round(fl / (ms * 1e-3) / 1e12 / 157.3, 4),
                        "counters": counters_for(f"proj4_prec{1 if precision == 'split_bf16' else 0}",
                                                 COUNTER_SRCS["proj4_mfma"])}
            if gold is not None:
                z = out.cpu().numpy()[0].view(np.complex128)
                ref = gold["zeta3" if npcf == 3 else "zeta4"]
                e = block_errors(z.reshape(ref.shape), ref)
                r["max_rel_err_vs_oracle"] = e["max_rel_err"]
                r["worst_block_err_vs_oracle"] = e["worst_block"]
            res[f"proj{npcf}pcf_{precision}"] = r
            plan.close()
    return res


def run_256_leg(api, fields, dev, edges, lmax, steps, warmup, precision, fused=True, autotune=True):
    """Full 3PCF of the two 256^3 fields with one plan: fields/s over `steps` forward passes,
    the fused last pass's time per field and the error against the stored oracle sums (whole
    result, per l block, and per zeta_l^{b1 b2} entry relative to its own magnitude)."""
    import numpy as np
    import torch
    n = fields[0].shape[0]
    nbins = len(edges) - 1
    stream = torch.cuda.Stream()
    plan = api.Plan([f.shape for f in fields], edges, lmax, npcf=3, prepare=False, fused=fused, precision=precision,
                    field_batch=None if fused else 1)
    with torch.cuda.stream(stream):
        plan.prepare(stream)
    if autotune:
        plan.autotune(stream)
    out = torch.empty((len(dev), plan.zeta_doubles), dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.forward_raw(dev, out=out, stream=stream)
    stream.synchronize()
    plan.profile(True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            plan.forward_raw(dev, out=out, stream=stream)
    stream.synchronize()
    el = time.perf_counter() - t0
    recs = plan.launch_records()
    plan.profile(False)
    plan.close()
    z = out.cpu().numpy().reshape(len(dev), lmax + 1, nbins, nbins)
    res = {"precision": precision, "fused": fused, "value": round(len(dev) * steps / el, 4), "unit": "fields/s",
           "ms_per_field": round(el / (steps * len(dev)) * 1e3, 3),
           "fused_last_pass_ms_per_field": round(sum(r["ms"] for r in recs if r["kernel"] == 2) / (steps * len(dev)), 3)
           if fused else None,
           "contraction_ms_per_field": round(sum(r["ms"] for r in recs if r["kernel"] == 3) / (steps * len(dev)), 3)
           if not fused else None}
    errs = []
    for i in range(len(dev)):
        g = os.path.join(ROOT, "tests", "golden", f"c3_full3_256_seed{i}.npz")
        if n == 256 and os.path.exists(g):
            ref = np.load(g)["zeta3"].real
            e = block_errors(z[i], ref)
            rel_entry = np.abs(z[i] - ref) / np.abs(ref)
            errs.append({"max_rel_err": e["max_rel_err"], "per_l": e["per_block"],
                         "worst_entry_rel_to_itself": float(np.max(rel_entry)),
                         "median_entry_rel_to_itself": float(np.median(rel_entry))})
    res["err_vs_oracle"] = errs or None
    return res, z


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip sb_autotune (the plain-pass variant choice) before the warmup")
    ap.add_argument("--graph", action="store_true", help="replay the forward from a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unfused", action="store_true", help="plain path: write the coefficients, then contract")
    ap.add_argument("--lines", default="main,split,plain,c4,c4var,big,huge,proj,c5,cpu",
                    help="comma list of the lines to run: main (the metric line), split (its split-BF16 leg), plain "
                         "(the unfused float32 path), c4 (128^3 4PCF batch), c4var (its other contraction paths), "
                         "big (512^3), huge (1024^3), proj (512^2 projected), c5 (uneven batch + adjoint + "
                         "synthesis), cpu (oracle)")
    ap.add_argument("--c4-steps", type=int, default=1, help="steps of the 128^3 4PCF batch (0 skips it)")
    ap.add_argument("--synth-steps", type=int, default=200,
                    help="Adam steps of the synthesis demo after the uneven batch (0 skips it)")
    ap.add_argument("--c5-steps", type=int, default=1,
                    help="steps of the uneven-batch forward + adjoint and the synthesis demo (0 skips them)")
    ap.add_argument("--big-steps", type=int, default=1, help="steps of the 512^3 3PCF line (0 skips it)")
    ap.add_argument("--proj-steps", type=int, default=3, help="steps of the 512^2 projected line (0 skips it)")
    ap.add_argument("--step-samples", type=int, default=10,
                    help="per-step HIP-event samples (eager and graph replay) after the timed steps")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="steps of the plain unfused float32 path on the same fields (0 skips it)")
    ap.add_argument("--split-steps", type=int, default=3,
                    help="steps of the split-BF16 leg of the metric workload (0 skips it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB three times (the reference "
                         "dispatch that scales the HBM byte counters of a counter run)")
    ap.add_argument("--write-traffic", metavar="COUNTER_DIR",
                    help="no GPU work: write profiles/traffic.json from two counter runs and exit")
    ap.add_argument("--write-counters", metavar="COUNTER_CSV",
                    help="no GPU work: write profiles/mfma_counters.json from a counter run and exit")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic, n=args.grid, copy_mib=1024)
        return
    if args.write_counters:
        write_counters(args.write_counters)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the library has no multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    lines = set(x.strip() for x in args.lines.split(",") if x.strip())

    import numpy as np
    import torch
    from fieldgen import lognormal_field, linear_edges
    from paper_2210_10206_amd import api

    n = args.grid
    nbins, rmax, lmax = 10, 32.0, 6
    edges = linear_edges(rmax, nbins)
    fields = dev = None
    if lines & {"main", "split", "plain", "cpu"}:
        print(f"bench: generating 2 lognormal {n}^3 fields", file=sys.stderr, flush=True)
        fields = [lognormal_field((n, n, n), seed=0, sigma=0.5), lognormal_field((n, n, n), seed=1, sigma=1.5)]
        dev = [torch.from_numpy(f).cuda() for f in fields]
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    value = elapsed = None
    roof = None
    per_kernel, stages, step_ms = {}, {}, {}
    tuned = None
    errs, errs_l = [], []
    cold_ms = None
    z = None
    if "main" in lines:
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        plan = api.Plan([f.shape for f in fields], edges, lmax, npcf=3, prepare=False, fused=not args.unfused)
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            plan.prepare(stream)
        stream.synchronize()
        cold_ms = (time.perf_counter() - t0) * 1e3
        if not args.no_autotune:
            plan.autotune(stream)
        out = torch.empty((len(dev), plan.zeta_doubles), dtype=torch.float64, device="cuda")
        print("bench: warmup", file=sys.stderr, flush=True)
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                plan.forward_raw(dev, out=out, stream=stream, graph=args.graph)
        stream.synchronize()
        torch.cuda.synchronize()
        print("bench: timed steps", file=sys.stderr, flush=True)
        if not args.graph:
            plan.profile(True)
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(args.steps):
                plan.forward_raw(dev, out=out, stream=stream, graph=args.graph)
        stream.synchronize()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        recs = plan.launch_records() if not args.graph else []
        plan.profile(False)
        tuned = plan.choices()
        value = len(dev) * args.steps / elapsed

        # parity of this very run against the stored oracle values (when present)
        z = out.cpu().numpy().reshape(len(dev), lmax + 1, nbins, nbins)
        for i in range(len(dev)):
            g = os.path.join(ROOT, "tests", "golden", f"c3_full3_256_seed{i}.npz")
            if n == 256 and os.path.exists(g):
                ref = np.load(g)["zeta3"].real
                e = block_errors(z[i], ref)
                errs.append(e["max_rel_err"])
                # per multipole: max over (b1, b2) of |Z - Z_oracle| / max |Z_oracle| of that l
                errs_l.append(e["per_block"])

        # roofline of the dominant kernel (largest share of the timed region among the passes
        # over all kernel arrays), from the live per-launch HIP-event records
        # arrays per field: one per (l, m) and bin, less the packed m = 0 pairs of the fused path
        narr = ((lmax + 1) * (lmax + 2) // 2 - (lmax + 1) // 2) * nbins
        names = {0: f"middle inverse pass over all {narr} arrays (fft_pass_kernel, fft_pass_pf_kernel or "
                    f"mid_reg_kernel<...,+1>: the variant sb_autotune chose)",
                 1: (f"axis0_reg_kernel<16,16,...>" if n == 256 else f"axis0_kernel<{n},...>")
                    + " (axis-0 pass: kernel-spectrum regeneration + product + inverse transform)",
                 2: (f"last_reg_kernel<16,16,{(nbins + 3) // 4 * 4},PS_PACKED+PS_REAL,0>" if n == 256
                     else f"last_contract_kernel<{n},...>")
                    + " (last inverse pass fused with the MFMA pair sums; two launches per field: the packed "
                      "m = 0 pairs, then the rest)",
                 3: "pair_kernel (unfused 3PCF contraction)"}
        srcs = TRAFFIC_SRCS
        per = {}
        for r in recs:
            # the passes over all arrays of a field: one launch each for the axis-0 and middle
            # passes, two for the last pass (counted as one pass over narr arrays)
            if r["kernel"] not in names or (r["kernel"] in (0, 1, 3) and r["batch"] != narr):
                continue
            e = per.setdefault(r["kernel"], {"ms": 0.0, "bytes": 0.0, "arrays": 0})
            e["ms"] += r["ms"]
            e["bytes"] += r["bytes"]
            e["arrays"] += r["batch"]
        for e in per.values():
            e["n"] = e["arrays"] / narr
        for k, e in per.items():
            per_kernel[names[k]] = {"passes": round(e["n"]), "avg_pass_ms": round(e["ms"] / e["n"], 4),
                                    "achieved_GBs": round(e["bytes"] / (e["ms"] * 1e-3) / 1e9, 1)}
        if per:
            k = max(per, key=lambda q: per[q]["ms"])
            e = per[k]
            achieved = e["bytes"] / (e["ms"] * 1e-3) / 1e9
            traffic = traffic_for(f"kernel{k}_n{n}", srcs[k])
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": names[k],
                    "launches": round(e["n"]), "avg_launch_ms": round(e["ms"] / e["n"], 4),
                    "algorithmic_bytes_per_launch": e["bytes"] / e["n"]}
        for r in recs:
            k = {0: "fft", 1: "contract", 2: "other"}[r["stage"]]
            stages.setdefault(k, [0.0, 0])
            stages[k][0] += r["ms"]
            stages[k][1] += 1
        # per-step HIP-event times (median), eager and replayed from a HIP graph
        if args.step_samples > 0:
            for mode in ("eager", "graph"):
                ms = []
                with torch.cuda.stream(stream):
                    plan.forward_raw(dev, out=out, stream=stream, graph=mode == "graph")   # capture / warm
                    for _ in range(args.step_samples):
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record(stream)
                        plan.forward_raw(dev, out=out, stream=stream, graph=mode == "graph")
                        e1.record(stream)
                        e1.synchronize()
                        ms.append(e0.elapsed_time(e1))
                ms.sort()
                step_ms[mode] = {"median_ms": round(ms[len(ms) // 2], 3), "min_ms": round(ms[0], 3),
                                 "samples": len(ms),
                                 "fields_per_s_at_median": round(len(dev) / (ms[len(ms) // 2] * 1e-3), 3)}
        plan.close()
        del plan, out
        torch.cuda.empty_cache()
    # the split-BF16 leg of the same workload (fused pair sums on bf16 MFMA with hi + lo splits)
    # and the plain float32 path (every coefficient array written by the three passes, then the
    # separate pair contraction; no fusion, no autotuning, no graph), each with its own error
    split = plain = None
    if "split" in lines and args.split_steps > 0:
        print("bench: split-BF16 leg", file=sys.stderr, flush=True)
        split, _ = run_256_leg(api, fields, dev, edges, lmax, args.split_steps, 1, "split_bf16")
        if value:
            split["speedup_vs_plain_fp32"] = None
        torch.cuda.empty_cache()
    if "plain" in lines and args.plain_steps > 0:
        print("bench: plain unfused path", file=sys.stderr, flush=True)
        plain, pz = run_256_leg(api, fields, dev, edges, lmax, args.plain_steps, 1, "fp32", fused=False,
                                autotune=False)
        if value:
            plain["speedup_of_default_path"] = round(value / plain["value"], 3)
            plain["max_abs_diff_vs_default_rel"] = float(np.max(np.abs(pz - z)) / np.max(np.abs(z)))
        if split:
            split["speedup_vs_plain_fp32"] = round(split["value"] / plain["value"], 3)
        torch.cuda.empty_cache()
    c4 = None
    if "c4" in lines and args.c4_steps > 0:
        print("bench: 128^3 4PCF batch", file=sys.stderr, flush=True)
        c4 = run_4pcf_batch(api, args.c4_steps, 1)
        if "c4var" in lines:
            variants = {}
            for prec, mf, par in (("split_bf16", True, "even"), ("fp32", False, "even"), ("fp32", True, "odd")):
                r = run_4pcf_batch(api, args.c4_steps, 1, precision=prec, mfma=mf, parity=par)
                key = f"{prec}_{'mfma' if mf else 'valu'}" + ("_odd_parity_23_lambda" if par == "odd" else "")
                variants[key] = {
                    "value": r["value"], "contraction_ms_per_field": r["contraction"]["ms_per_field"],
                    "achieved_tflops": r["contraction"]["achieved_tflops"], "kernel": r["contraction"]["kernel"],
                    "counters": r["contraction"]["counters"], "err_vs_oracle": r.get("err_vs_oracle")}
            c4["other_contraction_paths"] = variants
    big = None
    if "big" in lines and args.big_steps > 0:
        print("bench: 512^3 3PCF", file=sys.stderr, flush=True)
        big = run_512(api, args.big_steps, 1)
        torch.cuda.empty_cache()
    huge = None
    if "huge" in lines and args.big_steps > 0:
        print("bench: 1024^3 3PCF", file=sys.stderr, flush=True)
        huge = run_1024(api, args.big_steps, 1)
    proj = None
    if "proj" in lines and args.proj_steps > 0:
        print("bench: 512^2 projected 3PCF and 4PCF", file=sys.stderr, flush=True)
        proj = run_proj(api, args.proj_steps, 1)
    c5 = None
    if "c5" in lines and args.c5_steps > 0:
        print("bench: uneven batch forward + adjoint, synthesis demo", file=sys.stderr, flush=True)
        c5 = run_c5(api, args.c5_steps, 1, synth_steps=args.synth_steps)
    cpu = None
    if "cpu" in lines and not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(fields[0], edges, lmax)
    line = {
        "metric": METRIC, "value": round(value, 4) if value else None, "unit": "fields/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3) if elapsed else None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"full 3PCF, 2 lognormal {n}^3 float32 fields (sigma 0.5, 1.5), 10 bins over (0,32], "
                               f"lmax 6, kernel spectra resident, float32 fused pair sums", "grid": n, "nbins": nbins,
                   "lmax": lmax, "batch": 2, "graph": bool(args.graph), "fused": not args.unfused,
                   "autotuned": not args.no_autotune},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cold_setup_ms": round(cold_ms, 1) if cold_ms else None,
        "step_times": step_ms or None,
        "split_bf16_leg": split,
        "plain_fp32_unfused": plain,
        "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items()},
        "per_kernel": per_kernel,
        "tuned_launch_shapes": tuned,
        "max_rel_err_vs_oracle": errs or None,
        "max_rel_err_vs_oracle_per_l": errs_l or None,
        "secondary_4pcf_128": c4,
        "secondary_uneven_adjoint": c5,
        "secondary_3pcf_512": big,
        "secondary_3pcf_1024": huge,
        "secondary_projected_512": proj,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
