"""Benchmark: MACGIC-iQUAPI path propagation on one MI355X.

One benchmark step = one whole propagation of the structured-bath workload
(two-level system, Ohmic + underdamped Brownian-oscillator bath, dk_max = 24,
mask keeping lags 0..11, theta = 1e-8, 1000 time steps, FP64, pre-merging):
reset to t = 0, 1000 time steps (step kernel + planner each), read back rho(t)
for all t.  The bath coefficients and propagator tables are built once before
timing and stay resident in HBM with the path store.

Prints one JSON line:  value = path-steps/s over the timed propagations
(path-step = one child, i.e. one group extended by one forward/backward pair
in one time step), a roofline object for the step kernel, and the CPU oracle
timed on a bounded steady-state sample of the same workload.

Roofline: the algorithmic bytes of a time step are one record per group
extended plus one per surviving child (32 B each in FP64: every merged group
is read once and every survivor is emitted once towards the merge), divided
by the kernel's mean launch time from HIP events the library records on its
stream around each launch.  The stricter state-only floor (one record per
group read + one per group stored) is reported beside it.

--copy-mib N adds one plain device-to-device copy of N MiB after the timed
work: a kernel of known traffic against which the PMC byte counters of a
profiled run are scaled.

--workload batched-scan measures the batched form: the structured bath at 64
bath parameter points (peak frequency w0 uniform in [0.5, 2], width gamma in
{0.02, 0.05, 0.1}, seeded), all propagated together for 1000 steps, one
step-kernel launch per time step; value counts the path-steps of all of them.

--workload spin-boson measures the correctness/latency configuration: an
unbiased two-level system in an Ohmic bath (alpha 0.1, wc 5, beta 5), dt 0.25,
dk_max 8, no mask (exact iQUAPI by post-merging on every lag), no filter, 100
time steps: 4^8 = 65536 groups per step at steady state.

--workload long-memory measures the long-memory configuration instead: the
same structured bath with dk_max = 40, theta = 1e-9, the mask keeping lags
0..11 exact and lags 16, 24 and 32 of the tail (80-bit histories, the
hash-table store merged through partitions; --merge hash takes the table),
1000 time steps.  Its roofline object covers the expand kernel, the largest
share of that step, with the same algorithmic bytes per step.
--precision fp32 runs the FP32 log-domain form on either workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "path-steps/sec + HBM roofline fraction at dk_max=24, theta=1e-8; time per rho(t)"
HBM_PEAK_GBS = 8000.0
CSRC = "paper_2506_03127_amd/csrc/"

# per workload: the kernel the roofline object covers, the sources it is built
# from, the committed PMC traffic record, and the oracle sample for the CPU baseline
# (cpu_skip, cpu_steps): the oracle runs steps 1..cpu_skip untimed, then times the
# next cpu_steps (a steady-state window where the workload has one)
WORKLOADS = {
    "structured-bath": {
        "kernel": "step_kernel", "kernel_label": "step_kernel<4,2>",
        "sources": [CSRC + "quapi_step.hip", CSRC + "quapi_device.h", CSRC + "quapi_host.h"],
        "traffic": "step_kernel_traffic.json", "cpu_skip": 25, "cpu_steps": 8, "max_groups": 0},
    "batched-scan": {
        "kernel": "step_kernel", "kernel_label": "step_kernel<4,2,batched>",
        "sources": [CSRC + "quapi_step.hip", CSRC + "quapi_device.h", CSRC + "quapi_host.h"],
        "traffic": "step_kernel_batched_scan_traffic.json", "cpu_skip": 25, "cpu_steps": 8, "max_groups": 0},
    "three-level": {
        "kernel": "step_kernel", "kernel_label": "step_kernel<9,4>",
        "sources": [CSRC + "quapi_step.hip", CSRC + "quapi_device.h", CSRC + "quapi_host.h"],
        "traffic": "step_kernel_three_level_traffic.json", "cpu_skip": 17, "cpu_steps": 100, "max_groups": 0},
    "spin-boson": {
        "kernel": "step_kernel", "kernel_label": "step_kernel<4,2>",
        "sources": [CSRC + "quapi_step.hip", CSRC + "quapi_device.h", CSRC + "quapi_host.h"],
        "traffic": "step_kernel_spin_boson_traffic.json", "cpu_skip": 9, "cpu_steps": 91, "max_groups": 0},
    "long-memory": {
        "kernel": "sparse_expand", "kernel_label": "sparse_expand<4,2,2>",
        "sources": [CSRC + "quapi_sparse.hip", CSRC + "quapi_sparse.h", CSRC + "quapi_device.h",
                    CSRC + "quapi_host.h"],
        "traffic": "sparse_expand_long_memory_traffic.json", "cpu_skip": 0, "cpu_steps": 15,
        "max_groups": 48 << 20},
}


# the roofline kernel of each store (the workload's entry above is the bucketed store's)
STORE_KERNELS = {
    "direct": {"kernel": "dense_step", "kernel_label": "dense_step<4,2>",
               "sources": [CSRC + "quapi_dense.hip", CSRC + "quapi_dense.h", CSRC + "quapi_device.h",
                           CSRC + "quapi_host.h"]},
    "hash": {"kernel": "sparse_expand", "kernel_label": "sparse_expand",
             "sources": [CSRC + "quapi_sparse.hip", CSRC + "quapi_sparse.h", CSRC + "quapi_device.h",
                         CSRC + "quapi_host.h"]},
    "partition": {"kernel": "sparse_expand", "kernel_label": "sparse_expand (partition merge)",
                  "sources": [CSRC + "quapi_sparse.hip", CSRC + "quapi_sparse.h", CSRC + "quapi_device.h",
                              CSRC + "quapi_host.h"]},
}
STORE_NAMES = {1: "direct", 2: "bucketed", 3: "hash", 4: "partition"}


def workload_spec(name: str, precision: str, store: str = "bucketed") -> dict:
    spec = dict(WORKLOADS[name])
    if store in STORE_KERNELS and precision != "fp32":
        spec.update(STORE_KERNELS[store])
        tag = "_partition" if store == "partition" else ""
        spec["traffic"] = f"{spec['kernel']}{tag}_{name.replace('-', '_')}_traffic.json"
    if precision == "fp32" and store == "direct":
        # the FP32 form on the direct-mapped store (contiguous two-level masks)
        spec.update(STORE_KERNELS["direct"])
        spec.update({"kernel_label": "dense_step<4,2> (FP32 form)",
                     "traffic": f"dense_step_{name.replace('-', '_')}_traffic_fp32.json"})
    elif precision == "fp32":
        # the FP32 form on the hash-table store (every other mask)
        tag = "_partition" if store == "partition" else ""
        spec.update({"kernel": "sparse_expand",
                     "kernel_label": "sparse_expand (FP32 form" + (", partition merge)" if tag else ")"),
                     "sources": WORKLOADS["long-memory"]["sources"],
                     "traffic": f"sparse_expand{tag}_{name.replace('-', '_')}_traffic_fp32.json"})
    if precision == "fp32" and name == "structured-bath":
        spec["max_groups"] = 8 << 20
    return spec


def kernel_source_hash(spec: dict) -> str:
    h = hashlib.sha256()
    for f in spec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic(spec: dict):
    """HBM bytes per launch of the roofline kernel from the committed PMC measurement,
    or None when the kernel sources changed since the counters were taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", spec["traffic"])))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash(spec):
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(wl, skip: int, steps: int) -> dict:
    """The oracle as it stands, single-threaded: steps 1..skip untimed, then the
    next `steps` time steps timed."""
    import oracle
    from oracle.eta import Bath, eta_columns
    b = wl.bath
    eta = eta_columns(Bath(b.ohmic_alpha, b.ohmic_wc, b.peaks), wl.beta, wl.dt, wl.K)
    o = oracle.Oracle(wl.H, wl.q, wl.dt, wl.K, eta, wl.rho0, mask=wl.mask, theta=wl.theta,
                      mode=oracle.PRE if wl.mode == "pre" else oracle.POST)
    if skip > 0:
        o.step(skip)
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    children = sum(o.stats(t)["n_children"] for t in range(skip + 1, skip + steps + 1))
    return {"value": children / el, "unit": "path-steps/s", "cores": 1, "kind": "oracle",
            "time_per_rho_us": 1e6 * el / steps,
            "sample": f"time steps {skip + 1}..{skip + steps} of the same workload, after {skip} untimed "
                      f"({children} path-steps, {el:.1f} s, single thread, {cpu_model()})"}


def traffic_from_counters(fetch_csv: str, write_csv: str, spec: dict, copy_mib: int) -> dict:
    """HBM bytes per launch of the roofline kernel from two rocprofv3 --pmc runs (FETCH_SIZE,
    WRITE_SIZE, KiB per dispatch) of ``bench.py --copy-mib N``: each counter is scaled by what it
    reads for that plain N-MiB device copy, whose true traffic is N MiB read and N MiB written."""
    import csv

    def read(path, counter):
        # the calibration copy is the largest dispatch of the runtime's copy kernel (a
        # device-to-device tensor copy runs as one); fills, such as the clearing of the
        # hash table, are not copies
        step, copies = [], []
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            name = r.get("Kernel_Name", "")
            if spec["kernel"] in name:
                step.append(v)
            elif "copyBuffer" in name:
                copies.append(v)
        return step, max(copies)

    f_step, f_copy = read(fetch_csv, "FETCH_SIZE")
    w_step, w_copy = read(write_csv, "WRITE_SIZE")
    rec = {"copy_bytes": copy_mib << 20}
    copy_kib = copy_mib * 1024.0
    ff, fw = copy_kib / f_copy, copy_kib / w_copy
    fetch_b = float(np.mean(f_step)) * 1024.0 * ff
    write_b = float(np.mean(w_step)) * 1024.0 * fw
    rec.update({"kernel": spec["kernel_label"], "kernel_source_sha256": kernel_source_hash(spec),
                "launches": len(f_step),
                "fetch_kib_per_launch_raw": float(np.mean(f_step)),
                "write_kib_per_launch_raw": float(np.mean(w_step)),
                "copy_fetch_kib_raw": f_copy, "copy_write_kib_raw": w_copy,
                "fetch_scale": ff, "write_scale": fw,
                "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
                "bytes_per_launch": fetch_b + write_b})
    json.dump(rec, open(os.path.join(ROOT, "profiles", spec["traffic"]), "w"), indent=1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed propagations")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-steps", type=int, default=-1,
                    help="timed time steps of the oracle sample for the CPU baseline (0: skip; "
                         "default per workload, after an untimed run into the steady state)")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="structured-bath")
    ap.add_argument("--chunk-run", type=int, default=0,
                    help="batched form: chunk run length (0: the library's tuner picks it)")
    ap.add_argument("--graph", action="store_true",
                    help="each propagation as one HIP graph (quapi_step_graph), recorded in the warm-up")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64",
                    help="fp32: the FP32 log-domain form (direct-mapped store for contiguous two-level "
                         "masks, else the hash-table merge)")
    ap.add_argument("--merge", choices=["auto", "direct", "bucketed", "hash", "partition"], default="auto",
                    help="the store (QUAPI_MERGE_*); auto: the library's choice")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="one plain device copy of this size after the timed work (PMC calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the step kernel's HBM traffic per launch from the counter files of "
                         "two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of bench.py --copy-mib; no GPU")
    args = ap.parse_args()
    if args.graph and args.warmup < 1:
        args.warmup = 1                      # the graph is recorded outside the timed region
    # the store is known once the context exists; --traffic-from names it through --merge
    spec = workload_spec(args.workload, args.precision, args.merge if args.merge != "auto" else "bucketed")
    if args.cpu_steps < 0:
        args.cpu_steps = spec["cpu_steps"]
    if args.traffic_from:
        print(json.dumps(traffic_from_counters(args.traffic_from[0], args.traffic_from[1], spec,
                                               args.copy_mib or 256)))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the path is built "
              "and measured at one GPU's share", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2506_03127_amd import quapi, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    def eta_of(b, K):
        return quapi.quapi_eta(b.ohmic_alpha, b.ohmic_wc, [x for pk in b.peaks for x in pk], wl.beta, wl.dt, K)

    stream = torch.cuda.Stream()
    precision = quapi.QUAPI_FP32_LOG if args.precision == "fp32" else quapi.QUAPI_FP64
    merge = {"auto": quapi.QUAPI_MERGE_AUTO, "direct": quapi.QUAPI_MERGE_DIRECT,
             "bucketed": quapi.QUAPI_MERGE_BUCKETED, "hash": quapi.QUAPI_MERGE_HASH,
             "partition": quapi.QUAPI_MERGE_PARTITION}[args.merge]
    baths = None
    if args.workload == "batched-scan":
        if args.precision != "fp64":
            print("the batched form is FP64", file=sys.stderr)
            sys.exit(2)
        wl, baths = workloads.batched_scan()
        etas = np.stack([eta_of(b, wl.K) for b in baths])
        prop = quapi.BatchPropagator(wl.H, wl.q, wl.dt, wl.K, etas, wl.rho0, mask=wl.mask, theta=wl.theta,
                                     mode=quapi.QUAPI_PRE, max_steps=wl.n_steps, stream=stream.cuda_stream,
                                     merge=merge)
    else:
        if args.workload == "structured-bath":
            wl = workloads.structured_bath()
        elif args.workload == "spin-boson":
            wl = workloads.spin_boson_ohmic(mode="post")
        elif args.workload == "three-level":
            wl = workloads.three_level(K=16, n_exact=6, theta=1e-8, n_steps=200)
        else:
            wl = workloads.long_memory()
        prop = quapi.Propagator(wl.H, wl.q, wl.dt, wl.K, eta_of(wl.bath, wl.K), wl.rho0, mask=wl.mask,
                                theta=wl.theta, mode=quapi.QUAPI_PRE if wl.mode == "pre" else quapi.QUAPI_POST,
                                max_steps=wl.n_steps,
                                stream=stream.cuda_stream, max_groups=spec["max_groups"], precision=precision,
                                merge=merge)
    b = wl.bath
    info = prop.info()
    store = STORE_NAMES[info["store"]]
    spec = workload_spec(args.workload, args.precision, store)
    record_bytes = info["record_bytes"]
    n_inst = info["n_instances"]
    n_t = wl.n_steps

    if wl.M == 2:
        system = {"eps": float(2 * wl.H[0, 0].real), "Delta": float(2 * wl.H[0, 1].real)}
    else:
        system = {"H_S": "seeded random Hermitian, entries ~ N(0, 0.5), seed 7", "q": [float(x) for x in wl.q]}

    chunk_run = 1
    if n_inst > 1:
        if args.chunk_run > 0:
            chunk_run = args.chunk_run
            quapi.quapi_set_chunk_run(prop.ctx, chunk_run)
        else:
            # the library's own tuner picks the chunk run length (before any timing)
            chunk_run = quapi.quapi_autotune(prop.ctx, 100)

    def run_once():
        prop.reset()
        if args.graph:
            quapi.quapi_step_graph(prop.ctx, n_t)
        else:
            quapi.quapi_step(prop.ctx, n_t)
        # rho(t) of every instance: [t][instance][M][M]
        return quapi.quapi_batch_rho_all(prop.ctx, 0, n_t + 1, n_inst, wl.M)

    for _ in range(args.warmup):
        run_once()
    torch.cuda.synchronize()
    times = []
    rho = None
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rho = run_once()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    sts = [quapi.quapi_batch_step_stats(prop.ctx, j, 1, n_t) for j in range(n_inst)]
    children = sum(s["n_children"] for st in sts for s in st)
    groups_in = np.sum([[s["n_groups"] for s in st] for st in sts], axis=0, dtype=np.float64)
    groups_out = np.sum([[s["n_stored"] for s in st] for st in sts], axis=0, dtype=np.float64)
    surv = np.sum([[s["n_survivors"] for s in st] for st in sts], axis=0, dtype=np.float64)
    total = sum(times)
    ms_per_step = 1e3 * total / len(times)
    value = children * len(times) / total
    # algorithmic bytes per time step: a record per group extended + one per surviving child
    alg_bytes = record_bytes * (groups_in + surv)
    floor_bytes = record_bytes * (groups_in + groups_out)      # state only: read + stored

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 (log domain) + f64 sums",
        "data": "synthetic (model Hamiltonian and spectral density; no dataset)",
        "config": {
            "workload": wl.name, "M": wl.M, "dk_max": wl.K,
            "mask": list(range(wl.K)) if wl.mask is None else list(wl.mask),
            "theta": wl.theta, "time_steps": n_t,
            "bath": {"ohmic_alpha": b.ohmic_alpha, "ohmic_wc": b.ohmic_wc,
                     "peaks_w0_gamma_lambda": [list(p) for p in b.peaks]},
            "beta": wl.beta, "dt": wl.dt, **system, "mode": wl.mode + "-merging",
            "precision": args.precision, "merge": {"direct": "direct-mapped store", "bucketed": "bucketed store",
                                                   "hash": "hash table",
                                                   "partition": "hash-table store, partition merge"}[store],
            "record_bytes": record_bytes, "instances": n_inst, "chunk_run": chunk_run,
            "hip_graph": bool(args.graph),
        },
        "time_per_rho_us": 1e3 * ms_per_step / n_t,
        "path_steps_per_propagation": children,
        "mean_groups_per_step": float(groups_in.mean()),
        "mean_survivors_per_step": float(surv.mean()),
        "run_hbm_fraction": float(alg_bytes.sum() / (total / len(times)) / (HBM_PEAK_GBS * 1e9)),
        "trace_final": float(np.trace(rho[-1][0]).real),
    }

    if baths is not None:
        # the bath points of the scan (the config's "bath" is the first one)
        out["config"]["scan"] = {"peak_w0_range": [min(x.peaks[0][0] for x in baths), max(x.peaks[0][0] for x in baths)],
                                 "peak_gamma_set": sorted({x.peaks[0][1] for x in baths}), "seed": 11}

    if not args.no_roofline:
        # per-launch durations of the roofline kernel: HIP events recorded by the library on
        # its stream right before and after each launch of it
        prop.reset()
        quapi.quapi_profile_begin(prop.ctx, n_t)
        quapi.quapi_step(prop.ctx, n_t)
        step_ms, plan_ms = quapi.quapi_profile_end(prop.ctx, n_t)
        mean_s = float(step_ms.mean()) * 1e-3
        per_launch_bytes = float(alg_bytes.mean())
        achieved = per_launch_bytes / mean_s / 1e9
        floor_gbs = float(floor_bytes.mean()) / mean_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(spec),
                           "kernel": spec["kernel_label"], "launches": n_t,
                           "mean_launch_us": mean_s * 1e6,
                           ("planner_mean_launch_us" if store == "bucketed" else "rest_of_step_mean_us"):
                               float(plan_ms.mean()) * 1e3,
                           "alg_bytes_per_launch": per_launch_bytes,
                           "alg_bytes": f"{record_bytes} B x (groups extended + surviving children) per step",
                           "mean_groups_per_launch": float(groups_in.mean()),
                           "mean_survivors_per_launch": float(surv.mean()),
                           "state_floor_bytes_per_launch": float(floor_bytes.mean()),
                           "state_floor_frac": floor_gbs / HBM_PEAK_GBS}

    if args.copy_mib > 0:
        import torch
        nb = args.copy_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        with torch.cuda.stream(stream):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = nb

    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(wl, spec["cpu_skip"], args.cpu_steps)

    prop.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
