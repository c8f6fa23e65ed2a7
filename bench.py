#!/usr/bin/env python3
"""Throughput of the non-uniform diffraction hot path on one MI355X.

Workload (N' = 2048, M = 2^20): NU-ASM_1 and NU-ASM_2 on a 1024 x 1024 plane
of pitch 4 um, wavelength 633 nm, off-axis offset o = (1 mm, 0), kernel
tolerance 1e-6, clustered point sets (70 % in a Gaussian of sigma = 0.1 W at
the centre, 30 % uniform), for z in {0.01, 0.1, 0.5} m and both the
band-limited ASM (Eq. 4) and the Fresnel (Eq. 5) transfer functions: 12 runs.
One step runs all 12 one-shot (binning of the points + operator) on inputs
already resident in HBM, recorded as one batch graph whose launch shapes and
graph form the autotuner picks before the timed steps (`--no-tune`: the
defaults).  value = 12 M / step time, in non-uniform points/s.

Prints one JSON line.  The per-kernel roofline figure comes from HIP events
the library records around every launch during a second, separately timed
pass; the CPU baseline is the FP64 oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "non-uniform pts/sec NUASM_1/2 at N'=2048, M=1M, rel-L2≤1e-5; % HBM roofline"
HBM_PEAK_GBS = 8000.0
N, G, LAM, OX, OY, TOL = 1024, 4e-6, 633e-9, 1e-3, 0.0, 1e-6
ZS = (0.01, 0.1, 0.5)
TFS = (("asm", "limited"), ("fresnel", "full"))
M = 1 << 20

# Per-launch hardware counters of the kernels (rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes scaled by a plain-copy calibration, SQ_INSTS_VALU / SQ_INSTS_MFMA)
# with the SHA-256 of the sources each kernel is built from when they were
# taken; a kernel whose sources have changed since gets no counter figures.
COUNTERS = os.path.join(ROOT, "profiles", "counters.json")
CSRC = os.path.join(ROOT, "paper_1308_6644_amd", "csrc")
POINT_STAGES = ("bin_hist", "bin_colscan", "bin_scan", "bin_scatter", "spread", "spread_reduce", "interp")
SHARED_SOURCES = ("device_common.h", "launch.h", "group.h")
# VALU issue: one wave64 instruction per SIMD every 4 cycles, 256 CUs x 4 SIMDs at 2.4 GHz
SIMDS, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4
CUS, MFMA_F32_16X16X4_CYCLES = 256, 32


def kernel_sources(stage: str):
    main = "k_points.hip" if stage in POINT_STAGES else "k_fft.hip"
    return (main,) + SHARED_SOURCES


def sources_sha256(stage: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in kernel_sources(stage):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def counter_record(stage: str):
    """Committed counters of a stage's kernel, or None when absent or taken on
    other sources."""
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)["kernels"].get(stage)
    except (OSError, ValueError, KeyError):
        return None
    if not rec or rec.get("sources_sha256") != sources_sha256(stage):
        return None
    return rec


# kernel body name in the symbol -> stage (longer names first where one
# contains another)
_STAGE_OF_BODY = (
    ("bin_hist_body", "bin_hist"), ("bin_colscan_body", "bin_colscan"), ("bin_scan_body", "bin_scan"),
    ("bin_scatter_det_body", "bin_scatter"),
    ("bin_scatter_body", "bin_scatter"), ("spread_mfma_body", "spread"), ("spread_reduce_body", "spread_reduce"),
    ("spread_body", "spread"), ("interp_body", "interp"), ("t1_rows_inv_body", "t1_rows_inv"),
    ("t1_rows_body", "t1_rows"), ("t1_cols_body", "t1_cols"), ("t2_rows_inv_body", "t2_rows_inv"),
    ("t2_rows_body", "t2_rows"), ("t2_cols_body", "t2_cols"), ("copyBuffer", "copy"))


def _counter_rows(db: str):
    """Per-dispatch counter sums of one rocprofv3 database, by stage: only the
    single-plane launches (a grouped launch covers several planes) and, for
    the copy, only the dispatches of the calibration size (the largest)."""
    import collections
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, counter_name, value from counters_collection").fetchall()
    con.close()
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for name, did, counter, value in rows:
        if "k_grouped" in name:
            continue
        stage = next((st for key, st in _STAGE_OF_BODY if key in name), None)
        if stage is not None:
            per[(stage, did)][counter] += value
    copies = [(k, d) for k, d in per.items() if k[0] == "copy"]
    if copies:
        key = "FETCH_SIZE" if "FETCH_SIZE" in copies[0][1] else "WRITE_SIZE"
        top = max(d.get(key, 0.0) for _, d in copies)
        for k, d in copies:
            if d.get(key, 0.0) < 0.9 * top:
                del per[k]
    out = collections.defaultdict(lambda: collections.defaultdict(float))
    n = collections.Counter()
    for (stage, _), d in per.items():
        n[stage] += 1
        for counter, value in d.items():
            out[stage][counter] += value
    return {st: {c: v / n[st] for c, v in d.items()} | {"launches": n[st]} for st, d in out.items()}


# The rocprofv3 passes whose databases write_counters reads (run from the
# repository root with TMPDIR=/tmp), in its argument order.
PMC_COMMANDS = [
    "rocprofv3 --pmc FETCH_SIZE SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_LDS SQ_WAVES -d gpurun_out/prof/pmcA -o p -- "
    "python3 bench.py --steps 1 --warmup 0 --profile-steps 0 --no-cpu-baseline --no-tune",
    "rocprofv3 --pmc WRITE_SIZE SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR "
    "SQ_BUSY_CYCLES SQ_WAVE_CYCLES -d gpurun_out/prof/pmcB -o p -- "
    "python3 bench.py --steps 1 --warmup 0 --profile-steps 0 --no-cpu-baseline --no-tune",
    "rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/pmcE -o p -- python3 bench.py --copy-calibration 268435456",
    "rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/pmcF -o p -- python3 bench.py --copy-calibration 268435456",
    "python3 bench.py --write-counters gpurun_out/prof/pmcA/p_results.db gpurun_out/prof/pmcB/p_results.db "
    "gpurun_out/prof/pmcE/p_results.db gpurun_out/prof/pmcF/p_results.db",
]


def write_counters(fetch_db: str, write_db: str, copy_fetch_db: str, copy_write_db: str, command=None) -> dict:
    """profiles/counters.json from four rocprofv3 --pmc databases: FETCH_SIZE
    (with the SQ counters) and WRITE_SIZE passes of the benchmark, and the same
    two counters over plain device copies of a known size, which scale them to
    bytes.  Each kernel's record carries the hash of the sources it was taken
    on, so that the benchmark only uses it while they are unchanged."""
    a, b = _counter_rows(fetch_db), _counter_rows(write_db)
    ca, cb = _counter_rows(copy_fetch_db), _counter_rows(copy_write_db)
    copy_bytes = 268435456
    fs = copy_bytes / (ca["copy"]["FETCH_SIZE"] * 1024)
    ws = copy_bytes / (cb["copy"]["WRITE_SIZE"] * 1024)
    out = {"command": command or PMC_COMMANDS,
           "calibration": {"copy_bytes": copy_bytes, "fetch_scale": fs, "write_scale": ws,
                           "copy_fetch_kib": ca["copy"]["FETCH_SIZE"], "copy_write_kib": cb["copy"]["WRITE_SIZE"]},
           "kernels": {}}
    for st in sorted(set(a) & set(b)):
        if st == "copy":
            continue
        rec = {"sources_sha256": sources_sha256(st), "launches": a[st]["launches"],
               "fetch_bytes": a[st].get("FETCH_SIZE", 0.0) * 1024 * fs,
               "write_bytes": b[st].get("WRITE_SIZE", 0.0) * 1024 * ws}
        for counter, key in (("SQ_INSTS_VALU", "valu_insts"), ("SQ_INSTS_MFMA", "mfma_insts"),
                             ("SQ_INSTS_LDS", "lds_insts"), ("SQ_WAVES", "waves"),
                             ("SQ_LDS_BANK_CONFLICT", "lds_bank_conflict_cycles"),
                             ("SQ_ACTIVE_INST_LDS", "lds_active_cycles")):
            for src in (a, b):
                if counter in src[st]:
                    rec[key] = src[st][counter]
                    break
        out["kernels"][st] = rec
    with open(COUNTERS, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return out


def tune_headline_batch(batch, specs, xs, ys, ins, outs) -> dict:
    """The autotuner on a batch (launch shapes per plane class, then the
    graph form), into a fresh cache so that a run stands alone; the summary
    with each plane's chosen shapes.  Every choice is a launch shape of the
    same arithmetic (the parity tests cover each one)."""
    import tempfile
    from paper_1308_6644_amd import tune
    t0 = time.perf_counter()
    cache = tune.TuneCache(os.path.join(tempfile.mkdtemp(prefix="nuasm_tune_"), "tune.json"))
    tuning = tune.tune_batch(batch, specs, xs, ys, ins, outs, cache, reps=3)
    tuning["seconds"] = time.perf_counter() - t0
    tuning["planes"] = {str(p): {k: v for k, v in cache.get(tune.plane_key(sp, xs[p].numel())).items() if k != "ms"}
                        for p, sp in enumerate(specs)}
    return tuning


def stage_bytes(stage: str, info: dict) -> float:
    """Algorithmic (compulsory) HBM bytes of one launch of a kernel: every
    input the kernel's job needs read once, every output written once.  M is
    the point count, L the fine-grid support side, T the number of bins, G the
    number of binning ranges, Nb the number of in-band x-frequencies (the Rect
    of Eq. 4 lets the grid passes skip the others)."""
    n, np_, L, m, T = info["N"], info["Np"], info["L"], info["M"], info["tiles"]
    m_dest = info.get("M_dest", 0)
    if m_dest:
        # type 3: interpolation at the destination points; the binning
        # stages run once per point set (the average of the two is charged)
        m_interp, m = m_dest, 0.5 * (m + m_dest)
    else:
        m_interp = m
    nb = max(0, min(info["kx_hi"], np_ // 2 - 1) - max(info["kx_lo"], -np_ // 2) + 1)
    G = max(1, -(-m // max(4096, min(65535, -(-m // 256)))))
    c = 8.0  # complex64
    return {
        "bin_hist": 16.0 * m + 2.0 * G * T,            # coordinates in, 16-bit histograms out
        # histograms in, offsets + totals + per-bin prefixes out
        "bin_colscan": 2.0 * G * T + 4.0 * G * T + 4.0 * T + 20.0 * T,
        # totals + prefixes in, bases + first chunks + chunk counts + chunk tables out
        "bin_scan": 24.0 * T + 12.0 * T + 32.0 * T,
        "bin_scatter": 16.0 * m + 4.0 * G * T + 16.0 * m,  # coordinates + offsets in, records out
        "spread": 16.0 * m + c * m + c * L * L,        # records + values in, support grid out
        "spread_reduce": 0.0,
        "t1_rows": c * L * L + c * L * nb,
        "t1_cols": c * L * nb + c * np_ * nb,
        "t1_rows_inv": c * np_ * nb + c * np_ * np_,
        "t2_rows": c * n * n + c * n * nb,
        "t2_cols": c * n * nb + c * L * nb,
        "t2_rows_inv": c * L * nb + c * L * L,
        "t3_cols": c * L * nb + c * L * nb,
        "interp": c * L * L + 16.0 * m_interp + c * m_interp,  # grid + records in, values out
    }[stage]


def make_inputs(torch, synth):
    import numpy as np
    W = N * G
    r1 = synth.rng_for(2, 0)
    x1, y1 = synth.clustered_box(r1, M, W)
    c1 = synth.unit_phase(r1, M)
    r2 = synth.rng_for(2, 1)
    x2, y2 = synth.clustered_box(r2, M, W)
    u1 = synth.unit_phase(r2, (N, N))
    host = dict(x1=x1, y1=y1, c1=c1, x2=x2, y2=y2, u1=u1)
    d = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in host.items()}
    return host, d


def cpu_baseline(host, n1=40960, n2=40960):
    """The FP64 oracle as it stands, timed on this host: NU-ASM_1 on the first
    n1 source points and NU-ASM_2 on the first n2 destination points of the
    same workload at z = 0.1 m, band-limited ASM (transfer function included)."""
    import oracle as O
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
        blas = ",".join(sorted({f"{i.get('internal_api', '?')}-{i.get('version', '?')}" for i in info
                                if i.get("user_api") == "blas"})) or blas
    except Exception:
        threads = os.cpu_count() or 1
    geo = O.Geometry(N=N, g=G, lam=LAM, z=0.1, ox=OX, oy=OY, tf="asm", band="limited")
    t0 = time.perf_counter()
    H = O.transfer(geo)
    O.nuasm1(geo, host["x1"][:n1], host["y1"][:n1], host["c1"][:n1], H)
    O.nuasm2(geo, host["u1"], host["x2"][:n2], host["y2"][:n2], H)
    dt = time.perf_counter() - t0
    return {"value": (n1 + n2) / dt, "unit": "points/s", "cores": int(threads), "kind": "oracle",
            "blas": blas, "host_cpus": os.cpu_count(),
            "sample": f"FP64 direct-sum oracle, z=0.1 m band-limited ASM, N'=2048: NU-ASM_1 on "
                      f"{n1} source points + NU-ASM_2 on {n2} destination points, {dt:.1f} s wall",
            "seconds": dt}


def batched_workload(a, torch, P, synth):
    """64 independent planes: N ~ U{256, 512, 1024, 2048}, M = floor(exp(U[ln 1e4,
    ln 2e6])) clustered points, z ~ U[0.005, 0.5] m, type ~ U{1, 2}, transfer
    function ~ U{band-limited ASM, Fresnel}, 633 nm, 4 um pitch, o = 0.  One
    step runs every plane one-shot, either as one recorded HIP graph (Batch)
    or as a sequential loop of plain plans on one stream."""
    import numpy as np
    specs, xs, ys, ins, outs = [], [], [], [], []
    for q in synth.batched_planes(g=G, tol=TOL):
        s = q["spec"]
        n, m = s["N"], q["x"].size
        specs.append(s)
        xs.append(torch.from_numpy(q["x"]).cuda())
        ys.append(torch.from_numpy(q["y"]).cuda())
        ins.append(torch.from_numpy(q["inp"]).cuda())
        outs.append(torch.empty((2 * n, 2 * n) if s["type"] == 1 else (m,), dtype=torch.complex64, device="cuda"))
    total = sum(int(x.numel()) for x in xs)
    plans = [P.Plan(defer_range_check=True, **s) for s in specs]
    batch = P.Batch(specs)
    batch.set_plane_times(False)  # throughput without completion stamps; latency measured apart

    def seq_step(ev=None):
        for i, pl in enumerate(plans):
            pl.set_points(xs[i], ys[i])
            pl.execute(ins[i], outs[i])
            if ev is not None:
                ev[i].record()

    res = {}
    tuning = None
    for mode in ("sequential", "graph", "graph_tuned"):
        if mode == "graph_tuned":
            tuning = tune_headline_batch(batch, specs, xs, ys, ins, outs)
        for _ in range(a.warmup):
            seq_step() if mode == "sequential" else batch.run(xs, ys, ins, outs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            seq_step() if mode == "sequential" else batch.run(xs, ys, ins, outs)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        # per-plane completion latency within one step
        if mode == "sequential":
            evs = [torch.cuda.Event(enable_timing=True) for _ in plans]
            s0 = torch.cuda.Event(enable_timing=True)
            s0.record()
            seq_step(evs)
            torch.cuda.synchronize()
            lat = [s0.elapsed_time(e) for e in evs]
        else:
            batch.set_plane_times(True)
            batch.run(xs, ys, ins, outs)
            lat = batch.plane_times()
            batch.set_plane_times(False)
        lat = np.asarray(lat)
        res[mode] = {"ms_per_step": ms, "points_per_s": total / (ms * 1e-3),
                     "latency_ms_p50": float(np.percentile(lat, 50)),
                     "latency_ms_p99": float(np.percentile(lat, 99))}
    if batch.check_points() != -1:
        raise RuntimeError("points outside their window")
    for pl in plans:
        pl.check_points()
    line = {"metric": "batched non-uniform pts/sec, 64 mixed planes (autotuned graph vs sequential plain plans)",
            "value": res["graph_tuned"]["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": a.steps,
            "warmup": a.warmup, "ms_per_step": res["graph_tuned"]["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "64 planes, N in {256..2048}, M log-uniform in [1e4, 2e6] clustered, "
                                   "z in [0.005, 0.5] m, mixed types and transfer functions",
                       "points_per_step": total},
            "modes": res, "speedup_vs_sequential": res["sequential"]["ms_per_step"] / res["graph_tuned"]["ms_per_step"],
            "autotuner": tuning}
    print(json.dumps(line), flush=True)
    return 0


def stage_pass(runs, seq_step, steps, torch, bytes_fn=None):
    """Run `steps` sequential steps with the library's per-launch HIP events
    on and total time, launches and algorithmic bytes per stage
    (bytes_fn(stage, info, launches) overrides stage_bytes(stage, info) x
    launches)."""
    for r in runs:
        r["plan"].set_timing(True)
    for _ in range(steps):
        seq_step()
    torch.cuda.synchronize()
    stages = {}
    per_type_ms = {1: 0.0, 2: 0.0, 3: 0.0}
    for r in runs:
        info = r["plan"].info
        for st, (ms, n) in r["plan"].read_timing().items():
            if n == 0:
                continue
            s = stages.setdefault(st, {"ms": 0.0, "launches": 0, "bytes": 0.0})
            s["ms"] += ms
            s["launches"] += n
            s["bytes"] += bytes_fn(st, info, n) if bytes_fn else stage_bytes(st, info) * n
            per_type_ms[r["type"]] += ms
        r["plan"].set_timing(False)
    return stages, per_type_ms


def roofline(stages, steps, no_counters=()):
    """Roofline object of the dominant kernel and the per-stage report.

    achieved / frac: the kernel's algorithmic bytes per launch over its
    measured average launch time against 8 TB/s of HBM.  With committed
    counters taken on the current sources it also gets the counter-measured
    HBM traffic per launch and its VALU issue fraction (SQ_INSTS_VALU x 4
    cycles over 1024 SIMDs x 2.4 GHz x the launch time); `bound` names the
    resource the counters show closest to its peak ("hbm" by counter traffic,
    or "alu" by VALU issue, in which case achieved / peak / frac are VALU lane
    instructions per second against 256 CUs x 64 lanes x 2.4 GHz)."""
    dom = max(stages, key=lambda k: stages[k]["ms"])
    ds = stages[dom]
    avg_ms = ds["ms"] / ds["launches"]
    achieved = ds["bytes"] / (ds["ms"] * 1e-3) / 1e9
    total = sum(s["ms"] for s in stages.values())
    report = {k: {"avg_us": 1e3 * v["ms"] / v["launches"], "launches_per_step": v["launches"] // steps,
                  "share": v["ms"] / total, "GBps": v["bytes"] / max(v["ms"] * 1e-3, 1e-12) / 1e9}
              for k, v in sorted(stages.items(), key=lambda kv: -kv[1]["ms"])}
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_launch_us": avg_ms * 1e3,
            "hbm_algorithmic_frac": achieved / HBM_PEAK_GBS}
    # (no_counters: stages whose kernel here is not the one the committed
    # counters were taken on)
    rec = None if dom in no_counters else counter_record(dom)
    t_launch = avg_ms * 1e-3
    if rec is not None:
        traffic = float(rec["fetch_bytes"]) + float(rec["write_bytes"])
        roof["traffic"] = traffic
        roof["hbm_counter_frac"] = traffic / t_launch / (HBM_PEAK_GBS * 1e9)
        valu = float(rec.get("valu_insts", 0.0))
        roof["valu_issue_frac"] = valu * VALU_CYCLES / (SIMDS * CLOCK_HZ * t_launch)
        if rec.get("mfma_insts") is not None:
            roof["mfma_insts_per_launch"] = float(rec["mfma_insts"])
            # v_mfma_f32_16x16x4f32 (the only matrix instruction used): 8
            # passes of 4 cycles on its SIMD's matrix core
            roof["mfma_busy_frac"] = float(rec["mfma_insts"]) * MFMA_F32_16X16X4_CYCLES / (SIMDS * CLOCK_HZ * t_launch)
        if rec.get("lds_bank_conflict_cycles") is not None:
            # LDS cycles lost to bank conflicts, per CU, over the launch
            roof["lds_conflict_frac"] = float(rec["lds_bank_conflict_cycles"]) / (CUS * CLOCK_HZ * t_launch)
        roof["counters"] = {"source": "profiles/counters.json", "sources_sha256": rec["sources_sha256"]}
        if roof["valu_issue_frac"] > max(roof["hbm_counter_frac"], roof["hbm_algorithmic_frac"]):
            lanes = SIMDS * 16 * CLOCK_HZ / 1e9  # G lane-instructions/s
            roof.update({"bound": "alu", "achieved": valu * 64 / t_launch / 1e9, "peak": lanes,
                         "unit": "Glane-inst/s", "frac": roof["valu_issue_frac"]})
    return roof, report


def copy_bandwidth(torch, nbytes=1 << 30, reps=5) -> float:
    """Device-to-device copy bandwidth (GB/s, bytes read + written), median of
    `reps` timed copies of `nbytes` after one untimed: the practical ceiling
    the roofline fraction is also stated against."""
    import statistics
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    times = []
    for i in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        if i:
            times.append(e0.elapsed_time(e1))
    del src, dst
    return 2.0 * nbytes / (statistics.median(times) * 1e-3) / 1e9


def cgh_workload(a, torch, P, synth):
    """The hologram-phase optimisation configuration: NU-ASM_2 (band-limited
    ASM) from a phase-only uniform source, N = 2048 (N' = 4096), to 2^22
    destination points in three Gaussian clusters, 532 nm, z = 0.2 m,
    tolerance 1e-6, target a sum of 32 Gaussian blobs scaled to the initial
    intensity.  The points are bound once, as in an optimisation loop.  Timed
    with HIP events: the forward operator, the hand-written adjoint (the
    type-1 pipeline with conj H and the N x N crop) on a field of the same
    size, and one whole iteration (phase to field, forward, loss, autograd
    backward through the adjoint).  value = M / iteration time."""
    import numpy as np
    Nc, Gc, lam, z, Mc = 2048, 4e-6, 532e-9, 0.2, 1 << 22
    rng = synth.rng_for(5, 1)
    x, y = synth.three_clusters(rng, Mc, Nc * Gc)
    phi0 = rng.uniform(0.0, 2.0 * np.pi, size=(Nc, Nc)).astype(np.float32)
    T = synth.gaussian_blobs(rng, x, y, Nc * Gc)
    plan = P.Plan(Nc, 2, lam, z, Gc, tf="asm", band="limited", tol=1e-6)
    plan.set_points(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
    phi = torch.from_numpy(phi0).cuda().requires_grad_(True)
    pd = phi.detach()
    u1 = torch.polar(torch.ones_like(pd), pd)
    with torch.no_grad():
        u0 = plan.execute(u1)
        s0 = float((u0.real.double() ** 2 + u0.imag.double() ** 2).sum())
    T_t = torch.from_numpy(T * (s0 / float(T.sum()))).cuda()
    out_f = torch.empty((Mc,), dtype=torch.complex64, device="cuda")
    out_a = torch.empty((Nc, Nc), dtype=torch.complex64, device="cuda")

    def forward():
        plan.execute(u1, out_f)

    def adjoint():
        plan.adjoint(u0, out_a)

    def iteration():
        phi.grad = None
        u = P.nuasm2(torch.polar(torch.ones_like(phi), phi), plan)
        r = (u.real.double() ** 2 + u.imag.double() ** 2) - T_t
        torch.sum(r * r).backward()

    def timed(fn):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / a.steps

    print(f"[bench] cgh: N'={2 * Nc}, M={Mc}", file=sys.stderr, flush=True)
    f_ms, a_ms, it_ms = timed(forward), timed(adjoint), timed(iteration)
    line = {
        "metric": "CGH iteration non-uniform pts/sec (NU-ASM_2 forward + adjoint, autograd)",
        "value": Mc / (it_ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": it_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "CGH phase optimisation: NU-ASM_2 band-limited ASM, N=2048 (N'=4096), "
                               "M=2^22 points in three Gaussian clusters, 532 nm, z=0.2 m, tol 1e-6, "
                               "points bound once",
                   "N": Nc, "Np": 2 * Nc, "M": Mc},
        "forward_ms": f_ms, "adjoint_ms": a_ms, "adjoint_over_forward": a_ms / f_ms,
        "iteration_ms": it_ms,
    }
    print(json.dumps(line), flush=True)
    return 0


def nuasm3_workload(a, torch, P, d):
    """NU-ASM_3 / NU-FRE_3 at the headline geometry: 2^20 clustered source
    points and 2^20 clustered destination points (the two point sets of the
    headline workload), z in {0.01, 0.1, 0.5} m x {band-limited ASM,
    Fresnel}: 6 runs per step, each one-shot (both point sets binned, then
    the operator), plain plans one after another on one stream.
    value = 6 (M_source + M_destination) / step time."""
    runs = []
    for z in ZS:
        for tf, band in TFS:
            spec = dict(N=N, type=3, lam=LAM, z=z, g=G, tf=tf, band=band, ox=OX, oy=OY, tol=TOL)
            plan = P.Plan(defer_range_check=True, **spec)
            out = torch.empty((M,), dtype=torch.complex64, device="cuda")
            runs.append(dict(plan=plan, out=out, type=3, z=z, tf=tf))

    def step():
        for r in runs:
            r["plan"].set_points(d["x1"], d["y1"])
            r["plan"].set_dest_points(d["x2"], d["y2"])
            r["plan"].execute(d["c1"], r["out"])

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    for r in runs:
        r["plan"].check_points()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_per_step = e0.elapsed_time(e1) / a.steps
    line = {
        "metric": "non-uniform pts/sec NU-ASM_3 (source + destination points) at N'=2048, M=1M per side",
        "value": len(runs) * 2 * M / (ms_per_step * 1e-3), "unit": "points/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "NU-ASM_3 one-shot (bin both point sets + execute), N=1024 (N'=2048), "
                               "2^20 clustered source and 2^20 clustered destination points, pitch 4 um, "
                               "633 nm, o=(1 mm, 0), z in {0.01, 0.1, 0.5} m x {band-limited ASM, Fresnel}, "
                               "tol 1e-6 (w=7), 6 runs per step",
                   "N": N, "Np": 2 * N, "M_source": M, "M_dest": M, "runs_per_step": len(runs)},
    }
    if a.profile_steps > 0:
        stages, per_type_ms = stage_pass(runs, step, a.profile_steps, torch)
        roof, report = roofline(stages, a.profile_steps)
        line.update({"roofline": roof, "stages": report,
                     "avg_run_ms": per_type_ms[3] / (a.profile_steps * len(runs))})
    print(json.dumps(line), flush=True)
    return 0


# Rayleigh-Sommerfeld direct summation: floating-point operations per source
# / destination pair as the kernel evaluates Eq. 10 (an FMA counts two):
# float64 23 (differences, rho^2, 1 + rho^2/z^2, one Newton step for
# 1/sqrt, 1 + r/|z|, one Newton step for the reciprocal, the phase and its
# reduction), float32 16 (amplitude, complex products, accumulation), and
# the four hardware estimates (rsq, rcp, sin, cos) one each.
RS_FLOPS_PER_PAIR = 23 + 16 + 4
# Vector ALU ceiling for that mix: float64 FMA and non-packed float32 FMA
# issue at the same rate, 256 CUs x 64 lanes x 2 flops x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6
PAPER_RS_S, PAPER_NUASM1_MS = 76.0, 46.0  # the paper's CPU times at N = 256 (context only)
# wave64 VALU instructions per pair of the current k_rs_direct (rocprofv3
# SQ_INSTS_VALU / (pairs / 64), profiles/rs_direct_paper_N256.md), and the
# issue ceiling: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every
# 4 cycles at 2.4 GHz
RS_VALU_PER_PAIR = 38.3
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def paper_workload(a, torch, P, synth):
    """The paper's experiment set-up (Figs. 2-5) with synthetic fields:
    256 x 256 samples, 500 nm, 5 um uniform pitch, the non-uniform plane
    sampled quadrant-wise at 0.9/0.8/0.7/1.0 x 5 um.  NU-ASM_1 (band-limited
    ASM) and NU-FRE_1 from the quadrant-sampled source to the uniform 256 x 256
    destination, against Rayleigh-Sommerfeld direct summation (Eq. 10, every
    source sample weighted by (5 um)^2) over a range of z; NU-ASM_2 from the
    uniform source to the quadrant-sampled destination at z = 8 mm.  The line's
    value is the RS kernel's pair throughput."""
    import numpy as np
    Np_, d, lam = 256, 5e-6, 500e-9
    zs = (0.008, 0.016, 0.032, 0.064, 0.128, 0.256)
    xq, yq = synth.quadrant_grid(Np_, d)
    rng = synth.rng_for(6)
    fq = synth.experiment_field(rng, xq, yq, Np_ * d)
    n = (np.arange(Np_) - Np_ // 2) * d
    X, Y = np.meshgrid(n, n, indexing="xy")
    xu, yu = X.ravel(), Y.ravel()
    fu = synth.experiment_field(synth.rng_for(6, 1), xu, yu, Np_ * d)
    t = lambda v, dt=None: torch.from_numpy(np.ascontiguousarray(v if dt is None else v.astype(dt))).cuda()
    dxq, dyq, dxu, dyu = t(xq), t(yq), t(xu), t(yu)
    cq = t(fq, np.complex64)
    cq_w = t(fq * d * d, np.complex64)
    u1 = t(fu.reshape(Np_, Np_), np.complex64)
    cu_w = t(fu * d * d, np.complex64)
    M = xq.size

    def snr(test, ref):
        ref = ref.to(torch.complex128)
        err = test.to(torch.complex128) - ref
        return float(10.0 * torch.log10(torch.sum(ref.abs() ** 2) / torch.sum(err.abs() ** 2)))

    def timed(fn, reps):
        for _ in range(max(1, a.warmup)):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    table = {}
    times = {}
    for z in zs:
        ref = P.rs_direct(dxq, dyq, cq_w, dxu, dyu, lam, z)
        row = {}
        for tf, band in (("asm", "limited"), ("fresnel", "full")):
            plan = P.Plan(Np_, 1, lam, z, d, tf=tf, band=band, tol=1e-6, crop=True)
            plan.set_points(dxq, dyq)
            out = plan.execute(cq).reshape(-1)
            row["nuasm1" if tf == "asm" else "nufre1"] = snr(out, ref)
            if z == zs[0]:
                def one_shot(plan=plan):
                    plan.set_points(dxq, dyq)
                    plan.execute(cq, out.view(Np_, Np_))
                times[f"{'nuasm1' if tf == 'asm' else 'nufre1'}_ms"] = timed(one_shot, a.steps)
        table[f"{z * 1e3:g}mm"] = row
        print(f"[bench] z = {z * 1e3:g} mm: " + ", ".join(f"{k} {v:.2f} dB" for k, v in row.items()),
              file=sys.stderr, flush=True)
    z = zs[0]
    rs_ms = timed(lambda: P.rs_direct(dxq, dyq, cq_w, dxu, dyu, lam, z), max(3, a.steps // 4))
    # NU-ASM_2 (uniform source -> quadrant-sampled destination) against two
    # Rayleigh-Sommerfeld references: the sum over the 256 x 256 source samples
    # as point sources, and the sum over the band-limited interpolant of the
    # zero-padded samples (the field the FFT methods assume) on a 4x finer grid
    U = 4
    pad = np.zeros((2 * Np_, 2 * Np_), dtype=np.complex128)
    pad[Np_ // 2:3 * Np_ // 2, Np_ // 2:3 * Np_ // 2] = fu.reshape(Np_, Np_)
    S = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(pad)))
    Sf = np.zeros((2 * U * Np_, 2 * U * Np_), dtype=np.complex128)
    o = (U - 1) * Np_
    Sf[o:o + 2 * Np_, o:o + 2 * Np_] = S
    fine = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(Sf))) * U * U
    nf_ = (np.arange(2 * U * Np_) - U * Np_) * (d / U)
    XF, YF = np.meshgrid(nf_, nf_, indexing="xy")
    dxf, dyf = t(XF.ravel()), t(YF.ravel())
    cf_w = t(fine.ravel() * (d / U) ** 2, np.complex64)
    del pad, S, Sf, fine, XF, YF
    nuasm2_rows = {}
    for z2 in zs[:3]:
        plan2 = P.Plan(Np_, 2, lam, z2, d, tf="asm", band="limited", tol=1e-6)
        plan2.set_points(dxq, dyq)
        u2 = plan2.execute(u1)
        nuasm2_rows[f"{z2 * 1e3:g}mm"] = {
            "point_rs": snr(u2, P.rs_direct(dxu, dyu, cu_w, dxq, dyq, lam, z2)),
            "fine_rs": snr(u2, P.rs_direct(dxf, dyf, cf_w, dxq, dyq, lam, z2))}
        print(f"[bench] NU-ASM_2 z = {z2 * 1e3:g} mm: " + ", ".join(
            f"{k} {v:.2f} dB" for k, v in nuasm2_rows[f"{z2 * 1e3:g}mm"].items()), file=sys.stderr, flush=True)
    pairs = float(M) * float(xu.size)
    rate = pairs / (rs_ms * 1e-3)
    achieved = rate * RS_FLOPS_PER_PAIR / 1e12
    line = {
        "metric": "Rayleigh-Sommerfeld direct summation pairs/sec, paper experiment 256x256 -> 256x256",
        "value": rate, "unit": "pairs/s", "n_gpus": 1, "steps": max(3, a.steps // 4), "warmup": a.warmup,
        "ms_per_step": rs_ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 phase / f32", "data": "synthetic",
        "config": {"workload": "256 x 256 quadrant-sampled source (0.9/0.8/0.7/1.0 x 5 um) -> 256 x 256 "
                               "uniform destination (5 um), 500 nm, z = 8 mm; synthetic blob fields "
                               "standing in for the paper's photographs",
                   "pairs": pairs},
        "roofline": {"bound": "alu", "kernel": "rs_direct", "achieved": achieved, "peak": ALU_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS, "traffic": None,
                     "flops_per_pair": RS_FLOPS_PER_PAIR, "avg_launch_us": rs_ms * 1e3,
                     "valu_issue_frac": rate * RS_VALU_PER_PAIR / 64.0 / VALU_ISSUE_PER_S},
        "experiment": {"snr_db_vs_rs": table, "nuasm2_snr_db_vs_rs": nuasm2_rows,
                       "nuasm2_fine_rs_source": f"band-limited interpolant of the zero-padded 256 x 256 samples "
                                                f"on a {2 * U * Np_} x {2 * U * Np_} grid of pitch d/{U}",
                       "nuasm1_one_shot_ms": times.get("nuasm1_ms"), "nufre1_one_shot_ms": times.get("nufre1_ms"),
                       "rs_ms": rs_ms,
                       "paper_cpu_context": {"nuasm1_ms": PAPER_NUASM1_MS, "rs_s": PAPER_RS_S}},
    }
    print(json.dumps(line), flush=True)
    return 0


def scaled_workload(a, torch, P, synth):
    """Scaled diffraction (the zoom case NU-ASM generalises): the headline's
    N = 1024 source plane (4 um, 633 nm, o = (1 mm, 0), band-limited ASM,
    tol 1e-6) propagated z = 0.1 m to a 2048 x 2048 destination grid of pitch
    2 um (a 2x zoom over the window).  One step = one one-shot run (bind the
    grid + execute).  value = destination points / step time on the grid path
    (separable interpolation, no binning); the same coordinates through the
    binned path are timed beside it."""
    import numpy as np
    n2, d2, z = 2048, G / 2, 0.1
    r = synth.rng_for(2, 1)
    u1 = torch.from_numpy(np.ascontiguousarray(synth.unit_phase(r, (N, N)))).cuda()
    spec = dict(N=N, type=2, lam=LAM, z=z, g=G, tf="asm", band="limited", ox=OX, oy=OY, tol=TOL)
    pg = P.Plan(defer_range_check=True, **spec)
    pb = P.Plan(defer_range_check=True, **spec)
    k = torch.arange(n2, dtype=torch.float64, device="cuda") - n2 // 2
    ys, xs = torch.meshgrid(k * d2, k * d2, indexing="ij")
    xs, ys = xs.contiguous().view(-1), ys.contiguous().view(-1)
    og = torch.empty(n2 * n2, dtype=torch.complex64, device="cuda")
    ob = torch.empty_like(og)

    def step_grid():
        pg.set_grid_points(n2, n2, d2)
        pg.execute(u1, og)

    def step_binned():
        pb.set_points(xs, ys)
        pb.execute(u1, ob)

    res = {}
    for name, fn in (("grid", step_grid), ("binned", step_binned)):
        for _ in range(a.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name] = e0.elapsed_time(e1) / a.steps
    pb.check_points()
    diff = float(torch.linalg.vector_norm(og - ob) / torch.linalg.vector_norm(ob))
    M2 = n2 * n2
    line = {
        "metric": "scaled ASM destination pts/sec, N'=2048 source -> 2048x2048 grid at half pitch",
        "value": M2 / (res["grid"] * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": res["grid"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "NU-ASM_2 one-shot from the N=1024 (N'=2048) 4 um source to a 2048 x 2048 "
                               "destination grid of 2 um pitch, 633 nm, z = 0.1 m, o = (1 mm, 0), band-limited "
                               "ASM, tol 1e-6",
                   "binned_path_ms": res["binned"], "speedup_vs_binned": res["binned"] / res["grid"],
                   "grid_vs_binned_rel_l2": diff},
    }
    if a.profile_steps > 0:
        runs = [dict(plan=pg, type=2)]

        def gbytes(st, info, n):
            # grid-mode interpolation (its two launches are timed as one
            # stage): support read once, grid values written once (the
            # intermediate rows are not compulsory)
            if st == "interp":
                return (8.0 * info["L"] * info["L"] + 8.0 * M2) * n
            return stage_bytes(st, info) * n
        stages, _ = stage_pass(runs, step_grid, a.profile_steps, torch, gbytes)
        # the grid interpolation kernels are not the binned ones the counters
        # describe
        roof, report = roofline(stages, a.profile_steps, no_counters=("interp",))
        line.update({"roofline": roof, "stages": report})
    print(json.dumps(line), flush=True)
    return 0


def precision_workload(a, torch, P, synth):
    """NU-ASM_2 at N = 4096 (N' = 8192) with 2^24 destination points
    (jittered pixel grid, 4x denser in a 512 x 512 region of interest),
    532 nm, z = 1 m, band-limited ASM, FP64 phase, kernel tolerances 1e-3,
    1e-6 and 1e-9: one-shot time (binning + execute) per tolerance, on the
    band-adaptive fine grid (N'' = 2048 here) and on the full 2 N' grid.
    value = points/s at tolerance 1e-6 on the band-adaptive grid."""
    import numpy as np
    Nc, Mc, lam, z = 4096, 1 << 24, 532e-9, 1.0
    print(f"[bench] generating N={Nc} M={Mc}", file=sys.stderr, flush=True)
    rng = synth.rng_for(3, 0)
    x, y = synth.jittered_roi(rng, Nc, G, M=Mc)
    u1 = synth.unit_phase(rng, (Nc, Nc))
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y).cuda()
    ud = torch.from_numpy(np.ascontiguousarray(u1)).cuda()
    del x, y, u1
    out = torch.empty(Mc, dtype=torch.complex64, device="cuda")
    res = {}
    for tol in (1e-3, 1e-6, 1e-9):
        for full in (False, True):
            plan = P.Plan(Nc, 2, lam, z, G, tf="asm", band="limited", tol=tol, defer_range_check=True,
                          full_fine_grid=full)

            def step(plan=plan):
                plan.set_points(xd, yd)
                plan.execute(ud, out)
            for _ in range(max(1, a.warmup)):
                step()
            torch.cuda.synchronize()
            plan.check_points()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = max(3, a.steps // 4)
            e0.record()
            for _ in range(reps):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            res[f"tol{tol:g}_{'full' if full else 'band'}"] = {"ms": ms, "points_per_s": Mc / (ms * 1e-3),
                                                              "Npf": plan.info["Npf"], "w": plan.info["w"]}
            print(f"[bench] tol {tol:g} {'full' if full else 'band'} grid: {ms:.3f} ms", file=sys.stderr, flush=True)
            del plan
    main_ = res["tol1e-06_band"]
    line = {
        "metric": "non-uniform pts/sec NUASM_2 at N'=8192, M=16M, z=1 m (precision-sweep configuration)",
        "value": main_["points_per_s"], "unit": "points/s", "n_gpus": 1, "steps": max(3, a.steps // 4),
        "warmup": a.warmup, "ms_per_step": main_["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "NU-ASM_2 one-shot, N=4096 (N'=8192), 2^24 jittered points with a 4x denser "
                               "512x512 ROI, 532 nm, 4 um, z = 1 m, band-limited ASM, FP64 phase",
                   "runs": res},
    }
    print(json.dumps(line), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=("graph", "sequential"), default="graph",
                    help="graph: the 12 runs of a step recorded as one HIP graph on parallel branches; "
                         "sequential: plain plans one after another on one stream")
    ap.add_argument("--workload", choices=("n2048", "batched", "nuasm3", "paper", "scaled", "precision", "cgh"),
                    default="n2048",
                    help="n2048: the 12-run N'=2048 headline workload; batched: 64 mixed planes; "
                         "nuasm3: NU-ASM_3 with 2^20 source and 2^20 destination points, 6 runs; "
                         "paper: the paper's 256 x 256 experiment against Rayleigh-Sommerfeld; "
                         "scaled: a 2x zoom to a 2048 x 2048 destination grid; precision: NU-ASM_2 at "
                         "N'=8192, M=2^24, z=1 m on the band-adaptive and the full fine grid; cgh: one "
                         "hologram-optimisation iteration at N'=4096, M=2^22 (forward, adjoint timed beside)")
    ap.add_argument("--no-tune", action="store_true",
                    help="graph mode with the default launch shapes and form (no autotuning before the "
                         "timed steps)")
    ap.add_argument("--deterministic", action="store_true",
                    help="n2048 with NUASM_DETERMINISTIC on every plan (bitwise-reproducible runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (3 times), the "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters, and exit")
    ap.add_argument("--write-counters", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write profiles/counters.json from four rocprofv3 --pmc databases (no GPU needed) "
                         "and exit")
    a = ap.parse_args(argv)
    if a.write_counters:
        out = write_counters(*a.write_counters, command=os.environ.get("NUASM_COUNTERS_COMMAND") or None)
        print(json.dumps({"kernels": sorted(out["kernels"]), "calibration": out["calibration"]}))
        return 0
    if a.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {a.gpus}). "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    import torch

    import paper_1308_6644_amd as P
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if a.copy_calibration:
        n = a.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}), flush=True)
        return 0
    P.load()
    if a.workload == "batched":
        return batched_workload(a, torch, P, synth)
    if a.workload == "paper":
        return paper_workload(a, torch, P, synth)
    if a.workload == "scaled":
        return scaled_workload(a, torch, P, synth)
    if a.workload == "precision":
        return precision_workload(a, torch, P, synth)
    if a.workload == "cgh":
        return cgh_workload(a, torch, P, synth)
    print(f"[bench] generating inputs N={N} M={M}", file=sys.stderr, flush=True)
    host, d = make_inputs(torch, synth)
    if a.workload == "nuasm3":
        return nuasm3_workload(a, torch, P, d)

    runs = []
    for z in ZS:
        for tf, band in TFS:
            for t in (1, 2):
                # the type-2 runs are never adjoined: their points are binned
                # for interpolation alone (one record per point)
                spec = dict(N=N, type=t, lam=LAM, z=z, g=G, tf=tf, band=band, ox=OX, oy=OY, tol=TOL,
                            deterministic=a.deterministic, forward_only=t == 2)
                plan = P.Plan(defer_range_check=True, **spec)
                if t == 1:
                    x, y, inp = d["x1"], d["y1"], d["c1"]
                    out = torch.empty((2 * N, 2 * N), dtype=torch.complex64, device="cuda")
                else:
                    x, y, inp = d["x2"], d["y2"], d["u1"]
                    out = torch.empty((M,), dtype=torch.complex64, device="cuda")
                runs.append(dict(plan=plan, x=x, y=y, inp=inp, out=out, type=t, z=z, tf=tf, spec=spec))

    def seq_step():
        for r in runs:
            r["plan"].set_points(r["x"], r["y"])
            r["plan"].execute(r["inp"], r["out"])

    batch = None
    tuning = None
    if a.mode == "graph":
        batch = P.Batch([r["spec"] for r in runs])
        batch.set_plane_times(False)  # no per-plane completion stamps in the timed graph
        bx = [r["x"] for r in runs]
        by = [r["y"] for r in runs]
        bi = [r["inp"] for r in runs]
        bo = [r["out"] for r in runs]
        if not a.no_tune:
            print("[bench] autotuning the batch", file=sys.stderr, flush=True)
            tuning = tune_headline_batch(batch, [r["spec"] for r in runs], bx, by, bi, bo)

        def step():
            batch.run(bx, by, bi, bo)
    else:
        step = seq_step

    print(f"[bench] warmup {a.warmup}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    if batch is not None:
        if batch.check_points() != -1:
            raise RuntimeError("points outside their window")
    else:
        for r in runs:
            r["plan"].check_points()  # every point was inside its window

    print(f"[bench] timing {a.steps} steps", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    for _ in range(a.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = e0.elapsed_time(e1) / a.steps
    value = len(runs) * M / (ms_per_step * 1e-3)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "NU-ASM_1 + NU-ASM_2 one-shot (bin + execute), N=1024 (N'=2048), M=2^20 clustered "
                        "points per run, pitch 4 um, 633 nm, o=(1 mm, 0), z in {0.01, 0.1, 0.5} m x "
                        "{band-limited ASM, Fresnel}, tol 1e-6 (w=7), 12 runs per step",
            "N": N, "Np": 2 * N, "M": M, "runs_per_step": len(runs), "phase": "f64",
            "mode": a.mode, "deterministic": a.deterministic,
            "tuning": None if tuning is None else {
                "form": "grouped" if tuning["grouped"] else f"per-plane, {tuning['branches']} branches",
                "form_ms": tuning["form_ms"], "seconds": tuning["seconds"], "planes": tuning["planes"]},
        },
        "wall_s_timed": wall,
    }
    if a.profile_steps <= 0:
        print(json.dumps(line), flush=True)
        return 0

    # execute-only time (points bound once and reused, as in the iterations of
    # a hologram optimisation): the 12 runs' execute calls on plain plans
    for r in runs:
        r["plan"].set_points(r["x"], r["y"])
    for _ in range(a.warmup):
        for r in runs:
            r["plan"].execute(r["inp"], r["out"])
    e0.record()
    for _ in range(a.steps):
        for r in runs:
            r["plan"].execute(r["inp"], r["out"])
    e1.record()
    torch.cuda.synchronize()
    ex_ms = e0.elapsed_time(e1) / a.steps
    # execute-only byte model: the whole-path model without the binning
    # (B - 44 M for type 1, B - 32 M for type 2), summed over the step's runs
    Np_ = 2 * N
    ex_bytes = sum((64.0 * M + 56.0 * Np_ * Np_ - 44.0 * M) if r["type"] == 1
                   else (56.0 * M + 44.0 * Np_ * Np_ - 32.0 * M) for r in runs)
    line["execute_only"] = {"ms_per_step": ex_ms, "points_per_s": len(runs) * M / (ex_ms * 1e-3),
                            "mode": "sequential plain plans, points bound once",
                            "model_bytes": ex_bytes,
                            "frac": ex_bytes / (ex_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}

    # second pass: per-stage HIP events recorded by the library
    print(f"[bench] per-stage timing {a.profile_steps} steps", file=sys.stderr, flush=True)
    stages, per_type_ms = stage_pass(runs, seq_step, a.profile_steps, torch)
    # the counters were taken on the default scatter, not the stable one
    roof, stage_report = roofline(stages, a.profile_steps,
                                  no_counters=("bin_scatter", "bin_colscan", "bin_hist", "bin_scan")
                                  if a.deterministic else ())
    cbw = copy_bandwidth(torch)
    roof["copy_GBps"] = cbw
    # the kernel's algorithmic bandwidth against the measured device copy
    roof["frac_of_copy"] = roof["hbm_algorithmic_frac"] * HBM_PEAK_GBS / cbw
    # whole-path byte model per type (pass-minimal): 64 M + 56 N'^2 and 56 M + 44 N'^2
    Np = 2 * N
    nruns = len(runs) // 2
    path = {}
    for t, bpp in ((1, 64.0 * M + 56.0 * Np * Np), (2, 56.0 * M + 44.0 * Np * Np)):
        t_ms = per_type_ms[t] / (a.profile_steps * nruns)
        path[f"nuasm{t}"] = {"avg_ms": t_ms, "model_bytes": bpp,
                             "frac": bpp / (t_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                             "frac_of_copy": bpp / (t_ms * 1e-3) / (cbw * 1e9)}

    line.update({"roofline": roof, "stages": stage_report, "path_model": path})
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(host)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
