"""Benchmark of the D2Q9 cascaded LBM step with consistent forcing on one GPU.

Workload: the decaying Taylor-Green vortex plus a uniform body force
(Fx, Fy) = (1e-6, 5e-7) on a periodic 4096 x 4096 lattice, u0 = 0.01,
nu = 0.01, populations stored as FP32 deviations f_i - w_i rho0, FP32
arithmetic.  A step is one collide-and-stream update of the whole lattice
(Eqs. 9-15); the library advances this lattice two fused steps per launch
(step n + 1 on a tile and its halo kept in LDS, step n + 2 from there).
Inputs are resident in HBM before timing starts.

Prints one JSON line: MLUPS, the HBM roofline of the two-step kernel (per
launch the state is read and written once: 72 algorithmic bytes per node
for two node updates) and the oracle's throughput on the host cores for a
bounded sample of the same workload.  Beside it, in the same line: the same
lattice one step per launch (72 bytes per node update), the same lattice streamed in place
(one buffer), the same lattice with FP64 and 16-bit storage, the 64 x 32
Poiseuille channel and the cache-resident 1024^2 lattice, the batch of 256 uneven Kolmogorov lattices advanced by one
persistent launch per step, and a served Poisson stream of solves with its
p50/p99 latency.

`--calibrate-copy` instead runs a plain device copy of known size (the
reference for scaling the HBM byte counters of rocprofv3).
`--traffic-summary FETCH_STEP WRITE_STEP FETCH_COPY WRITE_COPY` (CPU only)
turns the counter_collection.csv files of the four rocprofv3 --pmc runs
listed in the summary into profiles/traffic_step_f32_tg4096.json, stamped
with the hash of the kernel sources they were taken on;
`--valu-summary PMC_DIR` does the same for one run of
`--pmc SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE` (profiles/valu_step_f32_tg4096.json).
The line's roofline names the binding limit of the headline kernel: HBM
(algorithmic bytes per launch against 8 TB/s) or VALU issue (the counted
wave-instructions per launch against 256 CUs x 2.4 GHz x one wave64
instruction per clock), and carries both.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BYTES_PER_LUP = {"f64": 144, "f32": 72, "f16": 36, "bf16": 36, "f16sr": 36, "bf16sr": 36}
KERNEL_SOURCES = ["paper_1705_11092_amd/csrc/clbm_step_f32.hip",
                  "paper_1705_11092_amd/csrc/clbm_step2.h",
                  "paper_1705_11092_amd/csrc/clbm_step.h",
                  "paper_1705_11092_amd/csrc/clbm_layout.h",
                  "paper_1705_11092_amd/csrc/clbm_force.h",
                  "paper_1705_11092_amd/csrc/clbm_device.h",
                  "paper_1705_11092_amd/csrc/clbm_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_f32_tg4096.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_step_f32_tg4096.json")
# VALU issue peak: 256 CUs x 2.4 GHz x one wave64 vector instruction per CU per clock.
VALU_PEAK_G = 256 * 2.4


def kernel_hash() -> str:
    """Hash of the step kernel's sources with comments and whitespace removed,
    so that the stored counters stay valid exactly as long as the code does."""
    import re
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(storage: str, n_nodes: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("storage") != storage:
        return None
    if t.get("nodes") != n_nodes:
        return None
    return t.get("hbm_bytes_per_launch")


def measured_valu(storage: str, n_nodes: int):
    """VALU wave-instructions per launch of the two-step kernel from the
    committed rocprofv3 counter summary, or None when the kernel sources
    changed since it was taken."""
    try:
        with open(VALU_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("storage") != storage or t.get("nodes") != n_nodes:
        return None
    return t


def run_gpu(n: int, storage: str, steps: int, warmup: int, inplace: bool = False,
            pairs: bool = True, reps: int = 1):
    """Time `reps` repetitions of exactly `steps` steps each (HIP events on
    the lattice's stream, a device synchronisation on both sides of each)
    after `warmup` untimed steps.  Returns the median repetition's
    milliseconds, the wall time of all repetitions, the FP64 totals at the
    end and the list of repetitions."""
    import statistics

    import torch
    from paper_1705_11092_amd import clbm, inputs

    wl = inputs.taylor_green(n, u0=0.01, nu=0.01, F=(1e-6, 5e-7), steps=steps)
    lat = clbm.lattice_from_workload(wl, storage=storage, inplace=inplace)
    lat.step_pairs = pairs
    run_gpu.pairs = lat.step_pairs
    stream = lat.stream
    lat.step(warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    times = []
    wall0 = time.perf_counter()
    for _ in range(reps):
        torch.cuda.synchronize()
        t0.record(stream)
        lat.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        times.append(t0.elapsed_time(t1))
    wall = time.perf_counter() - wall0
    _, _, _, tot = lat.moments(fields=False)
    lat.close()
    run_gpu.reps = times
    return statistics.median(times), wall, tot


def run_small():
    """The two small workloads: the 64 x 32 Poiseuille channel (FP64, 10,000
    steps from rest, launch-bound: microseconds per step through graphs)
    and the 1024^2 Taylor-Green lattice (FP64 and FP32, 2,000 steps; its
    two buffers fit the 256 MB Infinity Cache, so its bandwidth is a
    cache-resident figure, not HBM)."""
    import torch
    from paper_1705_11092_amd import clbm, inputs

    def timed(lat, steps):
        lat.step(steps // 10)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(lat.stream)
        lat.step(steps)
        t1.record(lat.stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) * 1e3 / steps

    out = {}
    wl = inputs.poiseuille(64, 32, Fx=1e-6, tau=1.0, steps=10_000)
    lat = clbm.lattice_from_workload(wl, storage="f64")
    out["poiseuille_64x32_f64"] = {"us_per_step": round(timed(lat, 10_000), 3), "steps": 10_000}
    lat.close()
    for st in ("f64", "f32"):
        wl = inputs.taylor_green(1024, u0=0.01, nu=0.01, F=(1e-6, 5e-7), steps=2000)
        lat = clbm.lattice_from_workload(wl, storage=st)
        per_launch = 2 if lat.step_pairs else 1
        us = timed(lat, 2000)
        lat.close()
        out[f"taylor_green_1024_{st}"] = {
            "us_per_step": round(us, 3), "mlups": round(1024 * 1024 / us, 1),
            "steps_per_launch": per_launch,
            "gb_s_cache_resident": round(BYTES_PER_LUP[st] * 1024 * 1024 / per_launch / us / 1e3, 1)}
    torch.cuda.empty_cache()
    return out


def run_batch(steps: int, warmup: int, count: int = 256, variant: int = -1, reps: int = 3):
    """The batch of uneven Kolmogorov lattices (sides log-uniform in
    [32, 512], seed 0), FP32 storage, two fused steps per launch over all
    lattices (hbm_frac: 72 B per node per launch, i.e. per two updates).
    The kernel variant is the autotuner's, or `variant` when >= 0 (a
    profiler's counters would distort the autotuner's timings)."""
    import torch
    from paper_1705_11092_amd import clbm, inputs

    wls = inputs.kolmogorov_batch(count=count, seed=0, steps=steps)
    lats = [clbm.lattice_from_workload(wl, storage="f32") for wl in wls]
    b = clbm.Batch(lats)
    per_launch = 2 if lats[0].step_pairs else 1
    if variant >= 0:
        b.variant = variant
    else:
        variant = b.autotune(None)
    b.step(warmup)
    torch.cuda.synchronize()
    # The median of `reps` repetitions of `steps` steps (HIP events on the
    # batch's stream).
    times = []
    for _ in range(reps):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(b.stream)
        b.step(steps)
        t1.record(b.stream)
        torch.cuda.synchronize()
        times.append(t0.elapsed_time(t1))
    ms = sorted(times)[len(times) // 2]
    nodes = sum(wl.nx * wl.ny for wl in wls)
    b.close()
    for lat in lats:
        lat.close()
    torch.cuda.empty_cache()
    mlups = nodes * steps / (ms / 1e3) / 1e6
    return {"workload": f"{count} Kolmogorov lattices, sides log-uniform 32..512 (seed 0), f32",
            "nodes": nodes, "steps": steps, "ms_per_step": round(ms / steps, 5),
            "mlups": round(mlups, 1), "repetitions": reps, "statistic": "median",
            "steps_per_launch": per_launch,
            "hbm_frac": round(mlups * 1e6 * 72 / per_launch / 8e12, 4),
            "variant": variant}


def run_served(count: int):
    """A Poisson stream of solves at ~80 % of the measured saturation rate."""
    import torch
    from paper_1705_11092_amd import inputs
    from paper_1705_11092_amd.serve import GpuBackend, Server

    # Saturation: the same kind of stream with every request waiting at t = 0
    # (a throughput: 100 requests measure it well enough).
    sat = inputs.served_stream(count=min(count, 100), seed=2, rate=1e9)
    rep = Server(GpuBackend()).run(sat)
    mu = rep.summary()["done"] / rep.makespan
    torch.cuda.empty_cache()
    reqs = inputs.served_stream(count=count, seed=1, rate=0.8 * mu)
    rep = Server(GpuBackend()).run(reqs)
    s = rep.summary()
    torch.cuda.empty_cache()
    return {"workload": f"{count} solves, sides log-uniform 64..2048, steps log-uniform 1e3..1e5, "
                        "forcing const/kolmogorov/none, f32 or f16 (stochastic rounding) storage, "
                        "Poisson arrivals",
            "saturation_rps": round(mu, 3), "arrival_rps": round(0.8 * mu, 3),
            "p50_latency_s": round(s["p50_latency_s"], 4), "p99_latency_s": round(s["p99_latency_s"], 4),
            "mlups": round(s["mlups"], 1), "done": s["done"], "rejected": s["rejected"],
            "makespan_s": round(s["makespan_s"], 3), "max_active": s["max_active"]}


def device_copy_gbs(nbytes: int, reps: int = 5) -> float:
    """HBM bandwidth a plain device-to-device copy of nbytes reaches (bytes
    read plus bytes written per second, median of reps copies timed with
    HIP events): the achievable counterpart of the published peak."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    times = []
    for _ in range(reps):
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        b.copy_(a)
        t1.record()
        torch.cuda.synchronize()
        times.append(t0.elapsed_time(t1))
    del a, b
    torch.cuda.empty_cache()
    ms = sorted(times)[len(times) // 2]
    return 2 * nbytes / (ms / 1e3) / 1e9


def calibrate_copy(nbytes: int, reps: int):
    """A plain device-to-device copy of nbytes, reps times."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": nbytes, "reps": reps}), flush=True)


def _counter_values(path: str, name_part: str, counter: str):
    import csv
    out = []
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if name_part in row["Kernel_Name"] and row["Counter_Name"] == counter:
                out.append(float(row["Counter_Value"]))
    if not out:
        raise SystemExit(f"{path}: no {counter} rows for kernels named like {name_part!r}")
    return out


def traffic_summary(dirs, copy_bytes: int = 603979776, n: int = 4096):
    """Scale the step kernel's FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by
    what the same counters read for a plain copy of copy_bytes, and write
    the summary bench.py reports as roofline.traffic."""
    import statistics
    csvs = [os.path.join(d, "run_counter_collection.csv") for d in dirs]
    step = "k_step2<1, 0, 0, unsigned int"
    fetch = _counter_values(csvs[0], step, "FETCH_SIZE")
    write = _counter_values(csvs[1], step, "WRITE_SIZE")
    cf = statistics.median(_counter_values(csvs[2], "copyBuffer", "FETCH_SIZE"))
    cw = statistics.median(_counter_values(csvs[3], "copyBuffer", "WRITE_SIZE"))
    kib = copy_bytes / 1024.0
    fs, ws = kib / cf, kib / cw
    rd = statistics.median(fetch) * 1024.0 * fs
    wr = statistics.median(write) * 1024.0 * ws
    alg = BYTES_PER_LUP["f32"] * n * n
    base = "rocprofv3 --pmc {c} --output-format csv -d {d} -o run -- python3 bench.py {a}"
    step_args = "--steps 6 --warmup 0 --reps 1 --no-cpu-baseline --no-extra"
    copy_args = f"--calibrate-copy {copy_bytes}"
    out = {
        "kernel": "clbm::k_step2<1, 0, 0, unsigned int, Tile<64, 16, 4>> (two fused steps per launch; FP32 "
                  "deviations, constant force, consistent scheme, 64 x 16 tiles)",
        "workload": f"taylor_green_{n}x{n}_uniform_force", "storage": "f32", "nodes": n * n,
        "kernel_hash": kernel_hash(),
        "commands": [base.format(c="FETCH_SIZE", d=dirs[0], a=step_args),
                     base.format(c="WRITE_SIZE", d=dirs[1], a=step_args),
                     base.format(c="FETCH_SIZE", d=dirs[2], a=copy_args),
                     base.format(c="WRITE_SIZE", d=dirs[3], a=copy_args)],
        "fetch_kib_per_dispatch": fetch, "write_kib_per_dispatch": write,
        "copy_bytes": copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_scale": round(fs, 6), "write_scale": round(ws, 6),
        "hbm_read_bytes_per_launch": int(rd), "hbm_write_bytes_per_launch": int(wr),
        "hbm_bytes_per_launch": int(rd + wr), "algorithmic_bytes_per_launch": alg,
        "ratio_to_algorithmic": round((rd + wr) / alg, 4),
    }
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps({k: out[k] for k in ("hbm_bytes_per_launch", "ratio_to_algorithmic",
                                           "fetch_scale", "write_scale", "kernel_hash")}))


def valu_summary(d: str, n: int = 4096):
    """VALU wave-instructions, waves and clock per launch of the two-step
    kernel from one rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE run
    (its run_counter_collection.csv), written to profiles/valu_step_f32_tg4096.json
    with the hash of the kernel sources it was taken on."""
    import csv
    import statistics
    step = "k_step2<1, 0, 0, unsigned int"
    per = {}
    with open(os.path.join(d, "run_counter_collection.csv"), newline="") as fh:
        for row in csv.DictReader(fh):
            if step not in row["Kernel_Name"]:
                continue
            e = per.setdefault(row.get("Dispatch_Id") or row.get("Correlation_Id"), {})
            e[row["Counter_Name"]] = float(row["Counter_Value"])
            if row.get("Start_Timestamp") and row.get("End_Timestamp"):
                e["ns"] = float(row["End_Timestamp"]) - float(row["Start_Timestamp"])
    if not per:
        raise SystemExit(f"{d}: no counter rows for {step}")
    valu = statistics.median(e["SQ_INSTS_VALU"] for e in per.values())
    waves = statistics.median(e["SQ_WAVES"] for e in per.values())
    clocks = [e["GRBM_GUI_ACTIVE"] / 8.0 / e["ns"] for e in per.values() if e.get("ns")]
    out = {
        "kernel": "clbm::k_step2<1, 0, 0, unsigned int, Tile<64, 16, 4>> (two fused steps per launch; FP32 "
                  "deviations, constant force, consistent scheme, 64 x 16 tiles)",
        "workload": f"taylor_green_{n}x{n}_uniform_force", "storage": "f32", "nodes": n * n,
        "kernel_hash": kernel_hash(),
        "command": f"rocprofv3 --pmc SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE --output-format csv -d {d} -o run "
                   "-- python3 bench.py --steps 6 --warmup 0 --reps 1 --no-cpu-baseline --no-extra",
        "dispatches": len(per), "valu_wave_insts_per_launch": valu, "waves_per_launch": waves,
        "valu_insts_per_wave": round(valu / waves, 1),
        "valu_insts_per_node_update": round(valu * 64 / (2 * n * n), 1),
        "issue_us_at_2p4_ghz": round(valu / (256 * 2.4e9) * 1e6, 2),
        "clock_ghz": round(statistics.median(clocks), 3) if clocks else None,
    }
    with open(VALU_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def cpu_baseline(n: int, budget_s: float = 12.0):
    """The oracle on the host cores: the same 4096^2 workload, as many steps
    as fit in about budget_s seconds after one timed probe step."""
    import oracle
    from paper_1705_11092_amd import inputs

    wl = inputs.taylor_green(n, u0=0.01, nu=0.01, F=(1e-6, 5e-7), steps=1)
    fx, fy = oracle.force_field(wl.force_kind, wl.force_params, n, n)
    f = oracle.init(wl.rho, wl.ux, wl.uy, fx, fy)
    t = time.perf_counter()
    f = oracle.step(f, fx, fy, wl.s)
    one = time.perf_counter() - t
    k = max(1, min(50, int(budget_s / max(one, 1e-3))))
    t = time.perf_counter()
    oracle.run(f, fx, fy, wl.s, k)
    dt = time.perf_counter() - t
    return {"value": round(n * n * k / dt / 1e6, 3), "unit": "MLUPS",
            "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"{k} steps of the {n}x{n} FP64 oracle on the same Taylor-Green workload"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--storage", default="f32", choices=list(BYTES_PER_LUP))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the main lattice (16-bit, batch and served legs skipped)")
    ap.add_argument("--single-steps", action="store_true",
                    help="step the main lattice one step per launch (no fused pairs)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES")
    ap.add_argument("--traffic-summary", nargs=4, default=None,
                    metavar=("FETCH_STEP", "WRITE_STEP", "FETCH_COPY", "WRITE_COPY"))
    ap.add_argument("--valu-summary", default=None, metavar="PMC_DIR")
    ap.add_argument("--reps", type=int, default=0,
                    help="timed repetitions of the headline (default: at least 5 and 400 steps)")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 256-lattice batch leg (for profiling it)")
    ap.add_argument("--batch-variant", type=int, default=-1,
                    help="with --batch-only: this kernel variant instead of the autotuner's")
    args = ap.parse_args()

    if args.traffic_summary:
        traffic_summary(args.traffic_summary)
        return
    if args.valu_summary:
        valu_summary(args.valu_summary)
        return

    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy, 5)
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU path; the lattice would be split into y-slabs with one halo "
              "exchange per step.", file=sys.stderr)
        sys.exit(2)

    # The headline: reps repetitions of exactly K steps each, the median
    # repetition reported (at least 5 repetitions and 400 timed steps).
    reps = args.reps or max(5, -(-400 // max(args.steps, 1)))
    if args.batch_only:
        print(json.dumps(run_batch(max(args.steps, 2), args.warmup, variant=args.batch_variant, reps=1)),
              flush=True)
        return

    ms, wall, tot = run_gpu(args.n, args.storage, args.steps, args.warmup, pairs=not args.single_steps,
                            reps=reps)
    rep_ms = run_gpu.reps
    pairs = run_gpu.pairs
    nodes = args.n * args.n
    ms_step = ms / args.steps
    mlups = nodes / (ms_step / 1e3) / 1e6
    bpl = BYTES_PER_LUP[args.storage]
    # The dominant kernel's launch: two steps (reading and writing the state
    # once) with pairs, one step otherwise; bytes per launch bpl * nodes.
    steps_per_launch = 2 if pairs else 1
    ms_launch = ms_step * steps_per_launch
    achieved = bpl * nodes / (ms_launch / 1e3) / 1e9
    traffic = measured_traffic(args.storage, nodes) if pairs else None
    # A plain device copy of one state buffer (bpl / 2 bytes per node) gives
    # what the memory reaches in practice, beside the published peak.
    copy_gbs = device_copy_gbs(bpl // 2 * nodes)
    limits = {"hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                      "algorithmic_bytes_per_launch": bpl * nodes,
                      "device_copy_gb_s": round(copy_gbs, 1),
                      "frac_of_device_copy": round(achieved / copy_gbs, 4)}}
    valu = measured_valu(args.storage, nodes) if pairs else None
    if valu is not None:
        # VALU issue: a compute unit issues at most one wave64 vector
        # instruction per clock (FP32 arithmetic unpacked), 256 CUs at 2.4 GHz.
        per_s = valu["valu_wave_insts_per_launch"] / (ms_launch / 1e3) / 1e9
        limits["alu"] = {"achieved": round(per_s, 1), "peak": VALU_PEAK_G, "unit": "G VALU wave-instr/s",
                         "frac": round(per_s / VALU_PEAK_G, 4),
                         "valu_wave_insts_per_launch": valu["valu_wave_insts_per_launch"],
                         "clock_ghz_under_counters": valu.get("clock_ghz")}
    bound = max(limits, key=lambda k: limits[k]["frac"])
    roof = {"bound": bound, **{k: v for k, v in limits[bound].items()},
            "kernel": "k_step2 (two fused steps per launch)" if pairs else "k_step",
            "ms_per_launch": round(ms_launch, 5), "limits": limits}
    if pairs:
        # The per-update byte model (every node update reads and writes the
        # state once) does not hold for fused pairs: the state crosses HBM
        # once per two updates.
        per_update = bpl * nodes * steps_per_launch / (ms_launch / 1e3) / 1e9
        roof["per_update_model"] = {"bytes_per_update": bpl, "equivalent_gb_s": round(per_update, 1),
                                    "frac_of_hbm_peak": round(per_update / HBM_PEAK_GBS, 4),
                                    "note": "exceeds 1: the model assumes no reuse across steps"}
    line = {
        "metric": "MLUPS (D2Q9 CLBM step, consistent forcing)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": f"taylor_green_{args.n}x{args.n}_uniform_force",
                   "storage": f"{args.storage} deviations f_i - w_i rho0",
                   "nodes": nodes, "steps_per_launch": steps_per_launch,
                   "hbm_bytes_per_lup": bpl / steps_per_launch, "boundary": "periodic",
                   "u0": 0.01, "nu": 0.01, "F": [1e-6, 5e-7]},
        "roofline": roof,
        "timing": {"repetitions": reps, "steps_each": args.steps, "statistic": "median",
                   "ms_per_repetition": [round(t, 4) for t in rep_ms]},
        "wall_s": round(wall, 4),
        "mass_total": tot[0],
    }
    if not args.no_extra:
        extra = {}
        args.steps = max(args.steps, 200)  # the other legs: one repetition of at least 200 steps
        ms1, _, _ = run_gpu(args.n, args.storage, args.steps, args.warmup, pairs=False)
        m = nodes / (ms1 / args.steps / 1e3) / 1e6
        extra[f"{args.storage}_one_step_per_launch"] = {
            "mlups": round(m, 1), "ms_per_step": round(ms1 / args.steps, 5),
            "hbm_frac": round(m * 1e6 * bpl / 8e12, 4)}
        msi, _, _ = run_gpu(args.n, args.storage, args.steps, args.warmup, inplace=True)
        m = nodes / (msi / args.steps / 1e3) / 1e6
        extra[f"{args.storage}_in_place"] = {
            "mlups": round(m, 1), "ms_per_step": round(msi / args.steps, 5),
            "hbm_frac": round(m * 1e6 * bpl / 8e12, 4),
            "footprint_bytes": nodes * bpl // 2}
        for st in ("f64", "f16", "bf16", "f16sr", "bf16sr"):
            ms16, _, _ = run_gpu(args.n, st, args.steps, args.warmup)
            spl = 2 if run_gpu.pairs else 1
            m = nodes / (ms16 / args.steps / 1e3) / 1e6
            extra[st] = {"mlups": round(m, 1), "ms_per_step": round(ms16 / args.steps, 5),
                         "steps_per_launch": spl,
                         "hbm_frac": round(m * 1e6 * BYTES_PER_LUP[st] / spl / 8e12, 4)}
            if spl == 2:
                ms1, _, _ = run_gpu(args.n, st, args.steps, args.warmup, pairs=False)
                m1 = nodes / (ms1 / args.steps / 1e3) / 1e6
                extra[f"{st}_one_step_per_launch"] = {
                    "mlups": round(m1, 1), "ms_per_step": round(ms1 / args.steps, 5),
                    "hbm_frac": round(m1 * 1e6 * BYTES_PER_LUP[st] / 8e12, 4)}
        extra["batch"] = run_batch(1000, 200)
        extra.update(run_small())
        if args.serve_requests > 0:
            extra["served"] = run_served(args.serve_requests)
        line["also"] = extra
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
