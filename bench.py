"""Benchmark: 3D sixth-order infinite-domain Poisson solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 257]

Workload: rho = sum of 5 seeded compact bumps A_i (1 - |x - c_i|^2/w_i^2)^10
(seed 2) on the 257^3 grid of [-1, 1]^3, order 6.  One step is one whole
solve rho -> phi with rho and phi resident in HBM.  Every precision mode is
timed.  The FP64 oracle then solves the same workload on the host (its
boundary sums in the slice-convolution form), which gives the CPU baseline
and every mode's error against the oracle, max |phi - phi_oracle| / max
|phi_oracle| over all nodes; the headline value is the fastest mode within
1e-6 of the oracle (without the oracle run: within 1e-6 of the FP64 GPU path).

Prints ONE JSON line.  Besides the contract fields it carries
  stage_roofline  every volume stage against the HBM roof, the sixth-order
                shell stage against the FP64 roof;
  roofline      HBM roofline of the dominant kernel (per-launch algorithmic
                bytes / its average duration from HIP events on the library's
                stream) and, when counters for the current sources exist
                under profiles/, the HBM traffic they measured; beside the
                8 TB/s peak, the rate a plain 1 GiB device copy attains;
  cpu_baseline  the FP64 oracle on the host cores: the same 257^3 solve with
                per-stage times, plus one-thread times of the 2D 65^2 and the
                3D 129^3 configurations;
  modes         per-precision throughput (mean over the timed steps and the
                median of per-step HIP events), error vs the oracle and vs
                FP64, and stage times;
  adjoint       time of one adjoint solve on the same grid, FP64 and the
                headline mixed mode;
  batched       64 uneven boxes per batch: graph replays of the plain batch and of
                the batch on 5-smooth extensions, eager launches for comparison;
  extended      the same solve through an extended plan (8 nodes added on every
                side, then 5-smooth panel counts), caller nodes per second;
  screening     the screening-charge boundary values against the volume sums
                (FP64, 65^3 to 257^3): time and error against the closed form.

Profiling helpers (same file, so that every profile is taken on committed code):
  --copy-calibration MIB   after the timed work, one plain device copy of MIB MiB
                           (the reference dispatch that scales HBM counters);
  --ingest KIND CSV ...    turn rocprofv3 output into the text summaries kept
                           under profiles/ (KIND = stats | traffic).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "3D 6th-order solve Mpoints/s: mixed-prec vs FP64 at rel err<=1e-6; % HBM BW"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
MODES = ["fp64", "mixed_fp32", "mixed_fp32_slices"]
# kernel (function) that implements each timed stage, as rocprofv3 names it
STAGE_KERNEL = {
    "rho_z": "k_pass",
    "conv_x": "k_cc (B output)",
    "conv_y": "k_cc",
    "rho_y": "k_pass",
    "conv_z": "k_cc",
    "final": "k_final",
    "inv_y": "k_pass",
    "inv_z": "k_pass",
}


def log(msg: str):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of every kernel and plan source (counters taken on other sources are stale)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2108_11871_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def attainable_hbm(torch, mib: int = 1024, reps: int = 10) -> float:
    """GB/s of a plain device-to-device copy of `mib` MiB (bytes read plus
    bytes written over the mean time of `reps` copies, HIP events on the
    stream the copies run on)."""
    x = torch.ones(mib * 131072, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    return 2.0 * mib * 1048576 / (ms * 1e-3) / 1e9


def stage_bytes(n: int, mode: str, nch: dict) -> dict:
    """Algorithmic HBM bytes of one launch of each volume stage (3D cube n^3)."""
    M = n - 1
    I = M - 1
    N = 2 * M
    vol = I ** 3
    wa = 4 if mode == "mixed_fp32_slices" else 8  # slot data of rho
    wb = 4 if mode != "fp64" else 8  # sine-space volume
    kt = I * (M + 1) ** 2 * 8  # FP64 kernel spectra of one face family (every mode)
    A = I * I * N * wa
    part = 2 * N * N * 8  # FP64 chunk partials of both faces (every mode)
    return {
        "rho_z": vol * 8 + A,
        "conv_x": A + kt + vol * wb + nch.get("x", 1) * part,
        "conv_y": A + kt + nch.get("y", 1) * part,
        "rho_y": vol * 8 + A,
        "conv_z": A + kt + nch.get("z", 1) * part,
        # chunk partials of the three families read, face spectra written
        "faces": (nch.get("x", 1) + nch.get("y", 1) + nch.get("z", 1)) * part + 3 * part,
        "final": 2 * vol * wb,
        "inv_y": 2 * vol * wb,
        "inv_z": vol * wb + vol * 8,
    }


def nchunks(n: int, mode: str) -> dict:
    """Chunk counts of the column-contraction kernels (mirrors the plan's choice)."""
    M = n - 1
    I, N = M - 1, 2 * M
    work = int(os.environ.get("IPS_TILE_WORK", "2048"))
    if work not in (1024, 2048, 4096):
        work = 2048

    def tw(NN, ncols):
        nseq = 1
        while 2 * nseq * NN <= work:
            nseq *= 2
        need = 2
        while need < ncols:
            need *= 2
        return min(2 * nseq, need)

    out = {}
    for key in ("x", "y", "z"):
        # a tile holds W/2 first-half columns and their mirrors
        W = tw(N, I)
        hc, Wh = (I + 1) // 2, W // 2
        ncb = (hc + Wh - 1) // Wh
        target = int(os.environ.get("IPS_CC_BLOCKS", "6144"))
        target = target if 256 <= target <= 65536 else 6144
        nch = max(1, min(ncb, (target + N - 1) // N))
        per = (ncb + nch - 1) // nch
        out[key] = (hc + per * Wh - 1) // (per * Wh)
    return out


def time_mode(api, torch, rho_d, h, mode, steps, warmup, ref=None):
    """Whole-job timing of one precision mode on a plain plan (no per-stage
    events inside the timed region), then per-stage means from a separate
    plan that records HIP events around every stage."""
    t0 = time.perf_counter()
    plan = api.Plan(rho_d.shape, h, order=6, precision=mode)
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) * 1e3
    phi = torch.empty_like(rho_d)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan(rho_d, phi)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan(rho_d, phi)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    # per-step times (separate events around every solve): median
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in evs:
        a.record(stream)
        plan(rho_d, phi)
        b.record(stream)
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in evs)
    median = per[len(per) // 2] if len(per) % 2 else 0.5 * (per[len(per) // 2 - 1] + per[len(per) // 2])
    ws = plan.workspace_bytes
    tb = plan.table_bytes
    plan.close()
    # stage means (events on the library's stream around each stage)
    tplan = api.Plan(rho_d.shape, h, order=6, precision=mode, timing=True)
    scratch = torch.empty_like(rho_d)
    for _ in range(max(warmup, 1)):
        tplan(rho_d, scratch)
    torch.cuda.synchronize()
    tplan.reset_stage_times()
    for _ in range(steps):
        tplan(rho_d, scratch)
    torch.cuda.synchronize()
    st = tplan.stage_times()
    tplan.close()
    del scratch
    err = None
    if ref is not None:
        err = float(((phi - ref).abs().max() / ref.abs().max()).item())
    return dict(ms=ms, median_ms=median, cold_ms=cold_ms, stages=st, phi=phi, err=err, workspace=ws, tables=tb)


def cpu_baseline(n: int, seed: int):
    """FP64 oracle on the host cores: one full solve of the benchmark workload
    (n^3, seed, order 6) with its boundary sums in the slice-convolution form,
    stage by stage (phi_star, boundary values, harmonic part).  Returns the
    record and the oracle's phi (for the error of every GPU mode)."""
    from oracle import poisson as P
    from paper_2108_11871_amd import inputs

    rho, h, _ = inputs.workload_bumps_3d(n, seed=seed)
    t0 = time.perf_counter()
    ps = P.phi_star(rho, h)
    t1 = time.perf_counter()
    g = P.boundary_values_fft(rho, h)
    t2 = time.perf_counter()
    ph = P.harmonic(g, h, 6)
    t3 = time.perf_counter()
    phi = ps + ph  # as oracle.solve: phi_star is 0 on the boundary, the harmonic part is g there
    dt = t3 - t0
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info

        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        pass
    rec = {
        "value": n ** 3 / dt / 1e6,
        "unit": "Mpoints/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "one full FP64 oracle solve of the benchmark workload itself (%d^3, 5 bumps, seed %d, "
                  "order 6): dense-matrix sine transforms (BLAS on %d threads), boundary sums in the "
                  "slice-convolution form (numpy FFT, one thread), finite-difference harmonic part; %.1f s"
                  % (n, seed, threads, dt),
        "stage_s": {"phi_star": t1 - t0, "boundary_values": t2 - t1, "harmonic": t3 - t2},
        "host_cpus": os.cpu_count(),
    }
    return rec, phi


def oracle_one_thread():
    """One-thread oracle times of the small configurations: 2D 65^2 order 4
    (direct boundary sums) and 3D 129^3 order 6, seed 1 (slice-convolution
    sums).  Runs in a child process whose BLAS and OpenMP pools have one thread."""
    import subprocess

    code = r"""
import json, sys, time
sys.path.insert(0, %r)
from oracle import poisson as P
from paper_2108_11871_amd import inputs
out = {}
rho, h, _ = inputs.workload_2d_single(65)
P.build_quad(); P.solve(rho[:9, :9], h, 4)
t = time.perf_counter(); P.solve(rho, h, 4); out["2d_65_order4_direct_s"] = time.perf_counter() - t
rho, h, _ = inputs.workload_bumps_3d(129, seed=1)
t = time.perf_counter(); P.solve(rho, h, 6, boundary="fft"); out["3d_129_order6_fft_s"] = time.perf_counter() - t
print(json.dumps(out))
""" % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


# stage -> (kernel-name substring, occurrence within one solve) in dispatch order
STAGE_DISPATCH = {
    "final": ("k_final<", 0),
    "conv_x": ("k_cc", 0),
    "conv_y": ("k_cc", 1),
    "conv_z": ("k_cc", 2),
    # the two forward slot passes of rho (FP64 in, FP32 slots: the mixed-slices mode)
    "rho_z": ("k_pass<float, double, float", 0),
    "rho_y": ("k_pass<float, double, float", 1),
}


def _read_counters(path):
    import csv

    disp = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            e = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"], "v": 0.0})
            e["v"] += float(r["Counter_Value"])
    return [disp[k] for k in sorted(disp)]


def ingest_traffic(fetch_csv, write_csv, n, mode, mib, cmd):
    """Per-launch HBM bytes of the volume stages from two counter passes.

    Each pass holds one solve of `mode` followed by one device copy of `mib`
    MiB.  FETCH_SIZE and WRITE_SIZE are KiB per dispatch; the copy's readings
    give the factor (true bytes / counted bytes) applied to every stage."""
    out = {"source_hash": source_hash(), "command": cmd, "per_launch_bytes": {}, "calibration": {}}
    per = {}
    for cname, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = _read_counters(path)
        copies = [e for e in d if "copy" in e["name"].lower()]
        if not copies:
            raise SystemExit("no copy dispatch in %s" % path)
        counted = copies[-1]["v"] * 1024.0
        factor = mib * 1048576.0 / counted
        out["calibration"][cname] = {"copy_bytes": mib * 1048576, "counted_bytes": counted, "factor": factor}
        for stage, (sub, occ) in STAGE_DISPATCH.items():
            hits = [e for e in d if sub in e["name"]]
            if len(hits) > occ:
                per.setdefault(stage, {})[cname] = hits[occ]["v"] * 1024.0 * factor
        # the whole last solve: from the forward pass of rho before its first
        # contraction to the two inverse passes after its final pass
        last = max(i for i, e in enumerate(d) if "k_final<" in e["name"])
        first = last
        while first > 0 and "k_cc" not in d[first]["name"]:
            first -= 1
        while first > 0 and ("k_cc" in d[first - 1]["name"] or "k_pass" in d[first - 1]["name"]):
            first -= 1
        while first < last and not ("k_pass" in d[first]["name"] and "k_cc" in d[first + 1]["name"]):
            first += 1
        per.setdefault("whole_solve", {})[cname] = sum(e["v"] for e in d[first:last + 3]) * 1024.0 * factor
    for stage, v in per.items():
        if "FETCH_SIZE" in v and "WRITE_SIZE" in v:
            out["per_launch_bytes"]["%s/%d/%s" % (stage, n, mode)] = {
                "fetch": v["FETCH_SIZE"], "write": v["WRITE_SIZE"], "total": v["FETCH_SIZE"] + v["WRITE_SIZE"]}
    path = os.path.join(ROOT, "profiles", "traffic.json")
    old = {}
    if os.path.exists(path):
        with open(path) as fh:
            old = json.load(fh)
        if old.get("source_hash") == out["source_hash"]:
            old["per_launch_bytes"].update(out["per_launch_bytes"])
            out["per_launch_bytes"] = old["per_launch_bytes"]
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


def ingest_counters(csv_a, csv_b, title, cmd, out_name, cu=256, xcd=8):
    """Per-kernel SQ counter summary of the last solve in two rocprofv3 --pmc
    passes (same program, same dispatch order).  GRBM_GUI_ACTIVE is reported
    once per XCD and summed here, so the per-XCD cycle count is the sum / xcd.
      occupancy  = SQ_WAVE_CYCLES * 4 / cycles / CUs / 32   (fraction of the 32 wave slots of a CU)
      VALU busy  = SQ_ACTIVE_INST_VALU / cycles / CUs
      LDS bank   = SQ_LDS_BANK_CONFLICT / cycles / CUs       (cycles stalled by bank conflicts)
      LDS wait   = SQ_WAIT_INST_LDS / SQ_WAVE_CYCLES         (wave time waiting for LDS results)
      any wait   = SQ_WAIT_ANY / SQ_WAVE_CYCLES              (wave time in s_waitcnt)
    and instructions per wave of VALU, LDS and vector-memory reads."""
    import csv

    def load(path):
        disp = {}
        for r in csv.DictReader(open(path)):
            e = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                                                        "wg": int(r["Workgroup_Size"]), "c": {}})
            e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        return [disp[k] for k in sorted(disp)]

    a, b = load(csv_a), load(csv_b)
    # the last solve: from the last rho_z-style forward pass of k_pass before the final k_final
    last_final = max(i for i, e in enumerate(a) if "k_final<" in e["name"])
    first = last_final
    while first > 0 and "k_cc" not in a[first]["name"]:
        first -= 1
    while first > 0 and ("k_cc" in a[first - 1]["name"] or "k_pass" in a[first - 1]["name"]):
        first -= 1
    # the run of passes reaches back into the previous solve's inverse passes:
    # the solve starts at the forward pass of rho that the first contraction follows
    while first < last_final and not ("k_pass" in a[first]["name"] and "k_cc" in a[first + 1]["name"]):
        first += 1
    lines = ["# %s" % title, "", "Command (run from the repository root, one pass per counter set):", "",
             "```", cmd, "```", "", ingest_counters.__doc__.strip().replace("\n    ", "\n"), "",
             "| kernel | waves | occupancy | VALU busy | LDS bank | LDS wait | any wait | VALU/wave | LDS/wave | VMEM rd/wave |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for ea, eb in zip(a[first:last_final + 3], b[first:last_final + 3]):
        c, c2 = ea["c"], eb["c"]
        cyc = c.get("GRBM_GUI_ACTIVE", 0.0) / xcd
        if cyc <= 0:
            continue
        waves = c.get("SQ_WAVES", 0.0)
        wc = max(c.get("SQ_WAVE_CYCLES", 1.0), 1.0)
        nm = ea["name"].replace("void ", "").replace("ips::", "")
        nm = nm.split("(")[0]
        lines.append("| `%s` | %d | %.0f%% | %.0f%% | %.0f%% | %.2f | %.2f | %.0f | %.0f | %.0f |" % (
            nm, waves, 100 * 4 * wc / cyc / cu / 32, 100 * c.get("SQ_ACTIVE_INST_VALU", 0) / cyc / cu,
            100 * c.get("SQ_LDS_BANK_CONFLICT", 0) / cyc / cu, c.get("SQ_WAIT_INST_LDS", 0) / wc,
            c2.get("SQ_WAIT_ANY", 0) / wc, c.get("SQ_INSTS_VALU", 0) / max(waves, 1),
            c.get("SQ_INSTS_LDS", 0) / max(waves, 1), c2.get("SQ_INSTS_VMEM_RD", 0) / max(waves, 1)))
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def ingest_stats(stats_csv, bench_json, title, cmd, out_name, top=20):
    """Kernel table (rocprofv3 --stats) plus the bench line's stage means."""
    import csv

    with open(stats_csv) as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# %s" % title, "", "Command (run from the repository root):", "", "```", cmd, "```", "",
             "| kernel | calls | avg us | min us | max us | % time |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f |" % (
            r["Name"].replace("void ", "").replace("ips::", ""), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    # per-stage means of the individual dispatches, when the kernel trace of the
    # same run sits beside the stats (one name can serve several stages)
    trace = os.path.join(os.path.dirname(stats_csv), os.path.basename(stats_csv).replace("kernel_stats",
                                                                                         "kernel_trace"))
    if trace != stats_csv and os.path.exists(trace):
        with open(trace) as fh:
            disp = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
        per = {}
        for stage, (sub, occ) in STAGE_DISPATCH.items():
            nper = 1 + max(o for s2, o in STAGE_DISPATCH.values() if s2 == sub)
            durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in disp if sub in r["Kernel_Name"]]
            if durs and len(durs) % nper == 0:
                mine = durs[occ::nper]
                per[stage] = (sum(mine) / len(mine), len(mine))
        if per:
            lines += ["", "Per-stage means of the individual dispatches (kernel trace of the same run; a kernel "
                      "name that serves several stages is split by its order within each solve):", ""]
            lines.append(", ".join("%s %.1f us (%d)" % (k, v[0], v[1]) for k, v in per.items()))
    if bench_json:
        with open(bench_json) as fh:
            b = json.loads(fh.read().strip().splitlines()[-1])
        lines += ["", "Bench line of the same run: %.1f Mpoints/s (%s), %.4f ms per solve." % (
            b["value"], b["config"]["precision"], b["ms_per_step"]),
            "Roofline stage `%s`: %.1f us per launch from HIP events on the library stream, %.0f GB/s "
            "algorithmic (%.3f of 8 TB/s)." % (b["roofline"]["stage"], b["roofline"]["avg_launch_ms"] * 1e3,
                                                b["roofline"]["achieved"], b["roofline"]["frac"]),
            "", "Stage means from HIP events (us):", ""]
        for m, v in b["modes"].items():
            lines.append("- %s: %s" % (m, ", ".join("%s %.1f" % (k, t * 1e3) for k, t in v["stage_ms"].items())))
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def time_batched(api, torch, steps, warmup, modes=("fp64", "mixed_fp32_slices")):
    """64 independent boxes of uneven size (seed 3), order 6, whole-batch
    nodes per second: graph replays of the plain batch (every box at its own
    size) and of the smooth batch (every box solved on its 5-smooth
    extension, caller nodes counted), eager launches of the plain FP64 batch
    for comparison."""
    from paper_2108_11871_amd import inputs

    probs = inputs.batched_problems(seed=3, count=64)
    rhos = [torch.from_numpy(p[0]).to("cuda:0") for p in probs]
    shapes = [tuple(r.shape) for r in rhos]
    hs = [p[1] for p in probs]
    nodes = sum(r.numel() for r in rhos)
    ext_nodes = 0
    for s_ in shapes:
        ne, _ = api.extension(s_, 0)
        c = 1
        for v in ne:
            c *= v
        ext_nodes += c
    stream = torch.cuda.current_stream()
    out = {"workload": "64 boxes, n per axis log-uniform in [33, 193], box [-s, s] with s ~ U(0.5, 2) "
                       "per axis, 5-bump sums, order 6, seed 3",
           "nodes": nodes, "smooth_extension_nodes": ext_nodes, "modes": {}}
    runs = [(m, kind) for m in modes for kind in ("graph", "smooth_graph")] + [("fp64", "eager")]
    for mode, kind in runs:
        b = api.Batch(shapes, hs, order=6, precision=mode, eager=(kind == "eager"),
                      smooth=(kind == "smooth_graph"))
        outs = [torch.empty_like(r) for r in rhos]
        for _ in range(max(warmup, 1) + 1):
            b(rhos, outs)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            b(rhos, outs)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out["modes"].setdefault(mode, {})[kind] = {"ms_per_batch": ms, "mpoints_per_s": nodes / (ms * 1e-3) / 1e6}
        b.close()
    return out


def time_adjoint(api, torch, rho_d, h, steps, warmup):
    """One adjoint rho_bar = A^T phi_bar per step on the same grid, in FP64
    and in the headline mixed mode (FP32 transform tiles, FP64 in memory),
    with the mixed result's max-norm difference from the FP64 one."""
    res = {}
    ref = None
    for prec in ("fp64", "mixed_fp32_slices"):
        plan = api.Plan(tuple(rho_d.shape), h, order=6, precision=prec, adjoint=True)
        out = torch.empty_like(rho_d)
        for _ in range(max(warmup, 1)):
            plan.adjoint(rho_d, out)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            plan.adjoint(rho_d, out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        plan.close()
        r = {"ms_per_step": ms, "mpoints_per_s": rho_d.numel() / (ms * 1e-3) / 1e6}
        if ref is None:
            ref = out
        else:
            r["rel_diff_vs_fp64"] = float((out - ref).abs().max() / ref.abs().max())
        res[prec] = r
    return res


def time_extended(api, torch, rho_d, h, mode, margin, steps, warmup):
    """The same workload through an extended plan (margin nodes on every side,
    then 5-smooth panel counts): caller nodes per second."""
    plan = api.Plan(tuple(rho_d.shape), h, order=6, precision=mode, margin=margin)
    ne, _ = api.extension(tuple(rho_d.shape), margin)
    out = torch.empty_like(rho_d)
    for _ in range(max(warmup, 1)):
        plan(rho_d, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        plan(rho_d, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    plan.close()
    return {"margin": margin, "grid_ext": list(ne), "precision": mode, "ms_per_step": ms,
            "mpoints_per_s": rho_d.numel() / (ms * 1e-3) / 1e6}


def time_screening(api, torch, sizes=(65, 129, 257), steps=3):
    """Boundary values by the screening charge (IPS_FLAG_SCREENING; surface sums
    by transforms, and by direct summation) against the volume sums, FP64, on
    the bump-sum workload (seed 2): time per solve, plan table bytes and the
    error against the closed-form potential on every boundary node and on
    sampled interior nodes (max error / max |phi|)."""
    import numpy as np

    from oracle import closed_forms as CF
    from oracle import poisson as P
    from paper_2108_11871_amd import inputs

    out = {}
    stream = torch.cuda.current_stream()
    for n in sizes:
        rho, h, meta = inputs.workload_bumps_3d(n, seed=2)
        rho_d = torch.from_numpy(rho).to("cuda:0")
        mask = P.boundary_mask(rho.shape)
        bidx = np.argwhere(mask)
        rng = np.random.default_rng(n)
        iidx = rng.integers(1, n - 1, (20000, 3))
        idx = np.concatenate([bidx, iidx])
        ex = CF.bump_sum_potential(-1.0 + idx * h[0], meta["centers"], meta["widths"], meta["amps"], meta["p"])
        rec = {}
        for name, screening, direct in (("volume", False, False), ("screening", True, False),
                                        ("screening_direct", True, True)):
            plan = api.Plan(rho.shape, h, order=6, screening=screening, screen_direct=direct)
            phi = plan(rho_d)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(steps):
                plan(rho_d, phi)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            got = phi.cpu().numpy()[idx[:, 0], idx[:, 1], idx[:, 2]]
            nb = len(bidx)
            sc = np.abs(ex).max()
            rec[name] = {"ms_per_step": ms, "table_bytes": plan.table_bytes,
                         "rel_err_boundary": float(np.abs(got[:nb] - ex[:nb]).max() / sc),
                         "rel_err_sampled": float(np.abs(got - ex).max() / sc)}
            plan.close()
        out["%d^3" % n] = rec
        log("screening %d^3: %s" % (n, rec))
    return out


def load_traffic(kernel_stage: str, n: int, mode: str):
    """HBM bytes per launch measured by rocprofv3 counters, if taken on these sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != source_hash():
        return None
    key = "%s/%d/%s" % (kernel_stage, n, mode)
    ent = rec.get("per_launch_bytes", {}).get(key)
    return ent


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=257)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--modes", default=",".join(MODES))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and adjoint timings")
    ap.add_argument("--batched-only", action="store_true", help="only the batched leg (profiling)")
    ap.add_argument("--screening-only", action="store_true", help="only the screening leg (profiling)")
    ap.add_argument("--adjoint-only", action="store_true", help="only the adjoint leg (profiling)")
    ap.add_argument("--ingest", nargs="+", metavar="ARG")
    args = ap.parse_args()

    if args.ingest:
        kind, rest = args.ingest[0], args.ingest[1:]
        if kind == "traffic":  # FETCH_CSV WRITE_CSV MODE MIB COMMAND
            ingest_traffic(rest[0], rest[1], args.n, rest[2], int(rest[3]), rest[4])
        elif kind == "stats":  # STATS_CSV BENCH_JSON OUT_NAME TITLE COMMAND
            ingest_stats(rest[0], rest[1], rest[3], rest[4], rest[2])
        elif kind == "counters":  # CSV_A CSV_B OUT_NAME TITLE COMMAND
            ingest_counters(rest[0], rest[1], rest[3], rest[4], rest[2])
        else:
            raise SystemExit("unknown --ingest kind %r" % kind)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (the solve is not sharded across "
              "GPUs); got --gpus %d, WORLD_SIZE %d" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_11871_amd import api, inputs

    if args.batched_only:
        print(json.dumps(time_batched(api, torch, args.steps, args.warmup)), flush=True)
        return
    if args.screening_only:
        print(json.dumps(time_screening(api, torch, sizes=(args.n,), steps=args.steps)), flush=True)
        return
    if args.adjoint_only:
        rho, h, _ = inputs.workload_bumps_3d(args.n, seed=args.seed)
        rho_d = torch.from_numpy(rho).to("cuda:0")
        print(json.dumps(time_adjoint(api, torch, rho_d, h, args.steps, args.warmup)), flush=True)
        return

    n = args.n
    rho, h, _ = inputs.workload_bumps_3d(n, seed=args.seed)
    rho_d = torch.from_numpy(rho).to("cuda:0")
    npts = n ** 3
    modes = [m for m in args.modes.split(",") if m]

    res = {}
    ref = None
    for mode in modes:
        r = time_mode(api, torch, rho_d, h, mode, args.steps, args.warmup, ref)
        log("%s: %.4f ms per solve (median %.4f)" % (mode, r["ms"], r["median_ms"]))
        if mode == "fp64":
            ref = r["phi"]
        res[mode] = r
    if ref is not None:
        for mode in modes:
            if mode != "fp64" and res[mode]["err"] is None:
                res[mode]["err"] = float(((res[mode]["phi"] - ref).abs().max() / ref.abs().max()).item())

    attain = attainable_hbm(torch)
    log("attainable HBM (device copy of 1 GiB): %.0f GB/s" % attain)

    if args.copy_calibration > 0:
        x = torch.ones(args.copy_calibration * 131072, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    extras = {}
    if not args.no_extras:
        extras["adjoint"] = time_adjoint(api, torch, rho_d, h, max(args.steps // 2, 1), args.warmup)
        log("adjoint: fp64 %.4f ms, mixed_fp32_slices %.4f ms" % (
            extras["adjoint"]["fp64"]["ms_per_step"], extras["adjoint"]["mixed_fp32_slices"]["ms_per_step"]))
        extras["batched"] = time_batched(api, torch, max(args.steps // 2, 1), args.warmup)
        log("batched done")
    # the oracle on the host: CPU baseline and every mode's error against it
    cpu = None
    oerr = {m: None for m in modes}
    if not args.no_cpu_baseline:
        log("oracle solve of the same workload on the host ...")
        cpu, phi_o = cpu_baseline(n, args.seed)
        log("oracle: %.1f s" % (n ** 3 / cpu["value"] / 1e6))
        scale = float(np.abs(phi_o).max())
        for m in modes:
            oerr[m] = float(np.abs(res[m]["phi"].cpu().numpy() - phi_o).max()) / scale
        del phi_o
        log("one-thread oracle runs ...")
        cpu["one_thread_s"] = oracle_one_thread()

    # headline: fastest mode within 1e-6 of the oracle (or of the FP64 GPU path without it)
    if cpu is not None:
        ok = [m for m in modes if oerr[m] is not None and oerr[m] <= 1e-6]
        checked = "oracle"
    elif ref is not None:
        ok = [m for m in modes if m == "fp64" or (res[m]["err"] is not None and res[m]["err"] <= 1e-6)]
        checked = "fp64_gpu"
    else:
        ok, checked = list(modes), None
    if not ok:
        ok, checked = list(modes), None
    best = min(ok, key=lambda m: res[m]["ms"])
    if not args.no_extras:
        extras["screening"] = time_screening(api, torch)
    if "extended" not in extras and not args.no_extras:
        extras["extended"] = time_extended(api, torch, rho_d, h, best, 8, max(args.steps // 2, 1), args.warmup)
    r = res[best]
    nch = nchunks(n, best)
    byts = stage_bytes(n, best, nch)
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in r["stages"].items() if v[1] > 0}
    dom = max((k for k in stage_ms if k in byts), key=lambda k: stage_ms[k])
    achieved = byts[dom] / (stage_ms[dom] * 1e-3) / 1e9
    traffic = load_traffic(dom, n, best)
    vol_bytes = sum(byts.values())
    b_node = (16 + 6 * (8 if best == "fp64" else 4)) + 16 + 24
    whole = load_traffic("whole_solve", n, best)
    solve_traffic = None if whole is None else whole.get("total")
    # every volume stage against the HBM roof, and the sixth-order shell
    # contraction (k_r6t) against the FP64 roof: 3 families x I^2 positions x
    # I wavenumbers, about 32 FP64 flops per step (rebuild V(k), one
    # reciprocal, five layer sums); its stage also holds the layer passes
    I = n - 2
    stage_roof = {k: {"bytes": byts[k], "ms": stage_ms[k], "GBs": byts[k] / (stage_ms[k] * 1e-3) / 1e9,
                      "frac": byts[k] / (stage_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                  for k in byts if k in stage_ms}
    if "shell_r6" in stage_ms:
        fl = 3.0 * I * I * I * 32
        stage_roof["shell_r6"] = {"flops": fl, "ms": stage_ms["shell_r6"],
                                  "TFLOPs": fl / (stage_ms["shell_r6"] * 1e-3) / 1e12,
                                  "frac": fl / (stage_ms["shell_r6"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}
    out = {
        "metric": METRIC,
        "value": npts / (r["ms"] * 1e-3) / 1e6,
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "3D %d^3 on [-1,1]^3, order 6, rho = sum of 5 seeded compact bumps "
                        "(1-|x-c|^2/w^2)^10, seed %d" % (n, args.seed),
            "grid": [n, n, n],
            "order": 6,
            "precision": best,
            "rel_err_vs_oracle": oerr[best],
            "checked_against": checked,
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": STAGE_KERNEL.get(dom, dom),
            "stage": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic["total"],
            "traffic_fetch_write": None if traffic is None else [traffic["fetch"], traffic["write"]],
            "avg_launch_ms": stage_ms[dom],
            "bytes_per_launch": byts[dom],
            # a plain device copy of 1 GiB (read + write), the rate HBM
            # delivers in practice
            "attainable_GBs": attain,
            "frac_of_attainable": achieved / attain,
        },
        "whole_solve_hbm": {
            # per-node compulsory streams: 16 + 6w B (rho in, phi out, three
            # intermediates written and read), 16 B for the second and third
            # reads of rho, 24 B for the kernel spectra read every solve
            "bytes_per_node": b_node,
            "algorithmic_GBs": b_node * npts / (r["ms"] * 1e-3) / 1e9,
            "frac": b_node * npts / (r["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            # the sum of the stage bytes of the table above
            "stage_bytes_per_step": vol_bytes,
            "stage_GBs": vol_bytes / (r["ms"] * 1e-3) / 1e9,
            # FETCH_SIZE + WRITE_SIZE over every kernel of one solve, when the
            # counters were taken on the current sources
            "counted_bytes_per_step": solve_traffic,
            "counted_GBs": None if solve_traffic is None else solve_traffic / (r["ms"] * 1e-3) / 1e9,
        },
        "stage_roofline": stage_roof,
        "modes": {
            m: {
                "mpoints_per_s": npts / (res[m]["ms"] * 1e-3) / 1e6,
                "ms_per_step": res[m]["ms"],
                "median_ms": res[m]["median_ms"],
                "rel_err_vs_oracle": oerr[m],
                "rel_err_vs_fp64": res[m]["err"],
                "plan_build_ms": res[m]["cold_ms"],
                "workspace_bytes": res[m]["workspace"],
                "table_bytes": res[m]["tables"],
                "stage_ms": {k: round(v[0] / max(v[1], 1), 5) for k, v in res[m]["stages"].items() if v[1]},
            }
            for m in modes
        },
        "source_hash": source_hash(),
    }
    out.update(extras)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
