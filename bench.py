"""Benchmark: sliced sparse-state contraction on one MI355X.

One step = the whole hot path over one batch of synthetic input: every slice of the
network is contracted (leaf slicing, permutes, stream and GEMM steps), summed in FP64
into psi_hat, its norm taken and 1000 bitstrings drawn.  Planning (circuit -> network ->
path, slices) happens before the timed region.

Default workload: 5x6 grid, 14 cycles, 10 sliced bonds (1024 slices), largest
intermediate <= 2^26 complex64, one group of 12 open qubits (4096 amplitudes).

Prints one JSON line (rank 0).
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

PEAK_FP32_MFMA = 157.3e12
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12


def cpu_baseline(w, flops_per_slice: float, budget_s: float = 20.0):
    """The oracle, as it stands, on a bounded sample of the same workload: as many slices
    as fit in about `budget_s` seconds (at least one), each contracted alone.  Returns the
    baseline record and the oracle amplitudes of the sampled slices by slice index."""
    import numpy as np

    from oracle import contract as ocontract
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover - informational only
        threads = os.cpu_count()
    done, t0 = 0, time.perf_counter()
    refs = {}
    while True:
        idx = done % len(w.slice_ids)
        sid = [int(w.slice_ids[idx])]
        refs[idx] = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                                sliced_bonds=w.sliced_bonds, slice_ids=sid)
        done += 1
        if time.perf_counter() - t0 > budget_s or done >= len(w.slice_ids):
            break
    dt = time.perf_counter() - t0
    per_slice = dt / done
    tflops = flops_per_slice / per_slice / 1e12
    return {"value": tflops, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{done} slice(s) of the same workload, numpy complex128 tensordot "
                      f"along the oracle's own greedy path, {per_slice:.2f} s per slice; value = "
                      f"the library's algorithmic flops per slice / oracle seconds per slice",
            "amplitudes_per_s": w.n_amplitudes / (per_slice * len(w.slice_ids))}, refs


def rel_error(got, ref) -> float:
    import numpy as np
    got, ref = np.asarray(got).reshape(-1), np.asarray(ref).reshape(-1)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def infidelity(got, ref) -> float:
    import numpy as np
    got, ref = np.asarray(got).reshape(-1), np.asarray(ref).reshape(-1)
    den = np.vdot(got, got).real * np.vdot(ref, ref).real
    return float(1.0 - abs(np.vdot(ref, got)) ** 2 / den) if den > 0 else 0.0


def slice_errors(c, refs) -> float:
    """Largest normwise relative error of single-slice contractions against the oracle."""
    worst = 0.0
    for idx, ref in refs.items():
        c.contract_range(idx, 1)
        worst = max(worst, rel_error(c.amps.cpu().numpy(), ref))
    return worst


def head_reuse(args, plain_amps, plain_amps_per_s) -> dict:
    """The same 1024-slice workload planned for head reuse (Method, Appendix B.2): slices the
    size bound needs are global, the other sliced bonds are local labels on the low slice-id
    bits, and every step above global labels only runs once per batch of 64 slices.  Timed
    over the same step (contract + sample) in complex64 and BF16x3; the amplitudes are
    compared with the plain plan's complex64 sum (the same full sum over all slices)."""
    import torch
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("sliced", mode="reuse")
    res = {"sliced_labels_local_then_global": [int(x) for x in w.plan.sliced_labels],
           "peak_log2": w.plan.cost.peak_log2}
    for name, prec in (("c64", 0), ("bf16x3", 2)):
        c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                        slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                        closed_bits=w.closed_bits, max_batch_slices=args.batch, precision=prec)
        if args.autotune:
            c.autotune(reps=2)
        n_samp = args.samples if len(w.closed_bits) == 1 else len(w.closed_bits)
        c.contract(norm=True)
        c.sample(2004, n_samp)
        steps = max(1, min(args.steps, 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            c.contract(norm=True)
            c.sample(2004, n_samp)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        amps = c.amps.cpu().numpy().copy()
        work = c.work()
        shared = sum(l.flops for l in c.launches() if l.invariant == 2)
        c.close()
        aps = w.n_amplitudes / (ms * 1e-3)
        res[name] = {"amplitudes_per_s": aps, "ms_per_step": ms,
                     "tflops": work / (ms * 1e-3) / 1e12, "flops_per_step": work,
                     "shared_flops_per_batch": shared,
                     "speedup_vs_plain_c64": aps / plain_amps_per_s,
                     "rel_err_vs_plain_c64_sum": rel_error(amps, plain_amps),
                     "infidelity_vs_plain_c64_sum": infidelity(amps, plain_amps)}
        print(f"[bench] head reuse {name}: {aps:.0f} amplitudes/s "
              f"({aps / plain_amps_per_s:.2f}x plain c64)", file=sys.stderr, flush=True)
    return res


def time_samplers(c, w, args) -> dict:
    """Wall time of the three in-group samplers on the contracted amplitudes (inverse CDF,
    the paper's Metropolis chains, frugal rejection sampling), one call each after a warm-up
    call; the bitstrings are copied to the host inside the timed call."""
    n = args.samples if len(w.closed_bits) == 1 else len(w.closed_bits)
    runs = {"inverse_cdf": lambda: c.sample(2004, n),
            "metropolis_100_steps": lambda: c.sample_metropolis(2004, n, 100),
            "frugal_m10_64_trials": lambda: c.sample_frugal(2004, n, 10.0, 64)}
    res = {"draws": n, "group_size": 1 << len(w.open_qubits)}
    for name, fn in runs.items():
        fn()
        t0 = time.perf_counter()
        fn()
        res[name + "_ms"] = 1e3 * (time.perf_counter() - t0)
    return res


def perturbed(args, plain_amps, plain_amps_per_s) -> dict:
    """The same workload with holes drilled into the circuit (Method): K = 2 per hole broken
    edges, fidelity estimate 2^-K.  Timed over the same step; the fidelity of its 4096
    amplitudes to the plain (exact) sum is reported beside the estimate."""
    import torch
    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("sliced", mode="holes")
    c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                    slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                    max_batch_slices=args.batch)
    if args.autotune:
        c.autotune(reps=2)
    n_samp = args.samples if len(w.closed_bits) == 1 else len(w.closed_bits)
    c.contract(norm=True)
    c.sample(2004, n_samp)
    steps = max(1, min(args.steps, 3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        c.contract(norm=True)
        c.sample(2004, n_samp)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    amps = c.amps.cpu().numpy().copy()
    work = c.work()
    c.close()
    K = 2 * len(w.circuit["holes"])
    aps = w.n_amplitudes / (ms * 1e-3)
    print(f"[bench] perturbed network ({K} broken edges): {aps:.0f} amplitudes/s",
          file=sys.stderr, flush=True)
    return {"holes": [int(h) for h in w.circuit["holes"]], "broken_edges": K,
            "fidelity_estimate": 2.0 ** -K,
            "fidelity_vs_exact_4096_amplitudes": 1.0 - infidelity(amps, plain_amps),
            "amplitudes_per_s": aps, "ms_per_step": ms, "flops_per_step": work,
            "tflops": work / (ms * 1e-3) / 1e12,
            "speedup_vs_plain_c64": aps / plain_amps_per_s}


def split_compare(w, args, plain_amps, refs, stream) -> dict:
    """The split-precision forms on the same workload: throughput over the same timed
    step (contract + sample) and their amplitude error against the complex64 sum and,
    slice by slice, against the oracle."""
    import torch
    from paper_2111_03011_amd.contractor import Contraction
    res = {}
    for name, prec in (("bf16x3", 2), ("fp16x3", 1)):
        c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                        slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                        closed_bits=w.closed_bits, max_batch_slices=args.batch, precision=prec)
        if args.autotune:
            c.autotune(reps=2)
        n_samp = args.samples if len(w.closed_bits) == 1 else len(w.closed_bits)
        c.contract(norm=True)
        c.sample(2004, n_samp)
        steps = max(1, min(args.steps, 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            c.contract(norm=True)
            c.sample(2004, n_samp)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        amps = c.amps.cpu().numpy().copy()
        r = {"amplitudes_per_s": w.n_amplitudes / (ms * 1e-3), "ms_per_step": ms,
             "tflops": c.stats()[0] * len(w.slice_ids) / (ms * 1e-3) / 1e12,
             "rel_err_vs_c64_sum": rel_error(amps, plain_amps),
             "infidelity_vs_c64_sum": infidelity(amps, plain_amps)}
        if refs:
            r["rel_err_vs_oracle_slices"] = slice_errors(c, refs)
        c.close()
        res[name] = r
        print(f"[bench] {name}: {r['amplitudes_per_s']:.0f} amplitudes/s, rel err vs c64 "
              f"{r['rel_err_vs_c64_sum']:.2e}", file=sys.stderr, flush=True)
    return res


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_gemm_sliced_5x6_m14_traffic.json")


def kernels_sha256():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2111_03011_amd", "csrc", "kernels.hip"), "rb").read()
    return hashlib.sha256(src).hexdigest()


def measured_traffic(args):
    """HBM bytes per k_gemm launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (calibrated against a plain 1 GiB copy), or None when they do not describe the
    kernel that runs now (different source, precision, workload or batch)."""
    try:
        rec = json.load(open(TRAFFIC_JSON))
        sha = kernels_sha256()
    except OSError:
        return None
    if (rec.get("kernels_hip_sha256") != sha or rec.get("workload") != args.workload or
            rec.get("precision") != args.precision or rec.get("batch") != args.batch):
        return None
    return rec["traffic_bytes_per_launch"]


def write_traffic(args, fetch_csv, write_csv):
    """Summarise two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE; one step of this
    bench with --copy-calibration) into the traffic record bench.py reads: KiB per dispatch
    of the dominant GEMM kernel, each counter scaled by what it reads for the plain device
    copy of known size."""
    import csv
    name = "::k_gemm<" if args.precision == "c64" else "::k_gemm_bf16x3<"

    def per_dispatch(path, counter):
        gemm, copy = {}, {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            d = r["Dispatch_Id"]
            v = float(r["Counter_Value"])
            if name in r["Kernel_Name"]:
                gemm[d] = gemm.get(d, 0.0) + v
            elif "copyBuffer" in r["Kernel_Name"]:
                copy[d] = copy.get(d, 0.0) + v
        return sum(gemm.values()) / len(gemm), len(gemm), max(copy.values())

    f_kib, n_f, f_copy = per_dispatch(fetch_csv, "FETCH_SIZE")
    w_kib, n_w, w_copy = per_dispatch(write_csv, "WRITE_SIZE")
    kib = args.copy_calibration / 1024.0
    f_fac, w_fac = kib / f_copy, kib / w_copy
    rec = {
        "kernel": name.strip(":<"), "workload": args.workload, "precision": args.precision,
        "batch": args.batch, "kernels_hip_sha256": kernels_sha256(),
        "dispatches": [n_f, n_w],
        "fetch_kib_per_launch_raw": round(f_kib, 2), "write_kib_per_launch_raw": round(w_kib, 2),
        "copy_calibration": {"bytes": args.copy_calibration, "fetch_kib": f_copy,
                             "write_kib": w_copy, "fetch_factor": round(f_fac, 4),
                             "write_factor": round(w_fac, 4)},
        "fetch_bytes_per_launch": round(f_kib * f_fac * 1024.0),
        "write_bytes_per_launch": round(w_kib * w_fac * 1024.0),
    }
    rec["traffic_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def serving_main(args):
    """Poisson request stream through libtnc's server; one JSON line with throughput and
    latency percentiles (latency = server completion time - submission time)."""
    import numpy as np
    import torch

    import synth
    from paper_2111_03011_amd.serving import Server
    from paper_2111_03011_amd.workload import serving_template

    cfg = synth.config("serving")
    rng = np.random.Generator(np.random.PCG64(cfg["seed"]))
    t = time.perf_counter()
    templates = [serving_template(cfg["seed"] * 10 + i) for i in range(args.templates)]
    print(f"[serving] planned {len(templates)} request templates in {time.perf_counter() - t:.1f} s",
          file=sys.stderr, flush=True)
    # service time of each template alone (the server otherwise idle)
    srv = Server(arena_bytes=args.arena_gb << 30, max_slots=args.slots, chunk_batches=2)
    solo = []
    for w, k in templates:
        rid = srv.submit(w.net, w.plan.path, w.plan.sliced_labels, w.slice_ids, w.open_qubits,
                         w.closed_bits, n_samples=k, seed=7,
                         max_batch_slices=args.serving_batch)
        while (r := srv.poll(rid)) is None:
            time.sleep(0.0005)
        solo.append(r["t_done"] - r["t_admit"])
    srv.close()
    print(f"[serving] solo service times (ms): {[round(1e3 * x, 1) for x in solo]}",
          file=sys.stderr, flush=True)
    R, warm = args.requests, min(cfg["warmup"], args.requests // 5)
    arrivals = np.cumsum(rng.exponential(1.0 / cfg["rate_per_s"], size=R))
    which = rng.integers(0, len(templates), size=R)
    srv = Server(arena_bytes=args.arena_gb << 30, max_slots=args.slots, chunk_batches=2)
    done, outstanding, i = {}, {}, 0
    t0 = time.perf_counter()
    while len(done) < R:
        now = time.perf_counter() - t0
        while i < R and arrivals[i] <= now:
            w, k = templates[which[i]]
            rid = srv.submit(w.net, w.plan.path, w.plan.sliced_labels, w.slice_ids,
                             w.open_qubits, w.closed_bits, n_samples=k, seed=1000 + i,
                             max_batch_slices=args.serving_batch)
            outstanding[rid] = i
            i += 1
        for rid in list(outstanding):
            r = srv.poll(rid)
            if r is not None:
                done[outstanding.pop(rid)] = r
        if now > args.serving_timeout:
            break
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    srv.close()
    meas = [done[j] for j in range(warm, R) if j in done]
    lat = np.array([1e3 * (r["t_done"] - r["t_submit"]) for r in meas])
    span = max(r["t_done"] for r in meas) - min(r["t_submit"] for r in meas)
    amps = sum(templates[which[j]][0].n_amplitudes for j in range(warm, R) if j in done)
    flops = sum(templates[which[j]][0].plan.total_flops for j in range(warm, R) if j in done)
    ns = [templates[which[j]][0].circuit["n_qubits"] for j in range(R)]
    out = {
        "metric": "contraction TFLOP/s & MFMA util; amplitudes/s; p50/p99 request latency",
        "value": len(meas) / span, "unit": "requests/s", "n_gpus": 1, "steps": len(meas),
        "warmup": warm, "ms_per_step": float(np.mean(lat)), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic (seeded circuits, Poisson arrivals)",
        "config": {"workload": f"serving: Poisson {cfg['rate_per_s']} req/s, {R} requests "
                               f"({warm} warm-up) drawn from {len(templates)} client-planned "
                               "templates: 20-36 qubits, 10-16 cycles, 256-65536 amplitudes or "
                               "1e3-1e5 samples, 2^4-2^12 slices, work <= 20 TFLOP per request",
                   "slots": args.slots, "arena_gb": args.arena_gb,
                   "batch_slices": args.serving_batch or "auto",
                   "mean_qubits": float(np.mean(ns))},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(np.mean(lat)), "max": float(np.max(lat))},
        "completed": len(done), "unfinished": R - len(done),
        "offered_rate_per_s": cfg["rate_per_s"], "achieved_rate_per_s": len(meas) / span,
        "amplitudes_per_s": amps / span, "contraction_tflops": flops / span / 1e12,
        "solo_service_ms": {"mean": 1e3 * float(np.mean([solo[j] for j in which])),
                            "min": 1e3 * min(solo), "max": 1e3 * max(solo)},
        "offered_load": cfg["rate_per_s"] * float(np.mean([solo[j] for j in which])),
        "solo_tflops": sum(t[0].plan.total_flops for t in templates) / sum(solo) / 1e12,
        "wall_s": wall,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sliced", choices=["sliced", "small", "large", "serving"])
    ap.add_argument("--requests", type=int, default=120, help="serving: requests in the stream")
    ap.add_argument("--templates", type=int, default=16, help="serving: distinct request templates")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent requests")
    ap.add_argument("--arena-gb", type=int, default=64, help="serving: device arena")
    ap.add_argument("--serving-timeout", type=float, default=150.0)
    ap.add_argument("--serving-batch", type=int, default=0,
                    help="serving: slices per launch sequence (0 = chosen per request)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--samples", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=64, help="slices per launch (hipGraph per batch)")
    ap.add_argument("--autotune", type=int, default=1, help="time tile choices per GEMM first (1/0)")
    ap.add_argument("--precision", default="c64", choices=["c64", "bf16x3", "fp16x3"])
    ap.add_argument("--perturbed", type=int, default=1,
                    help="sliced, c64: also time the workload with holes drilled (1/0)")
    ap.add_argument("--reuse", action="store_true",
                    help="large: the head-reuse mode (subtasks of 8 consecutive slices; use "
                         "--batch 8)")
    ap.add_argument("--head-reuse", type=int, default=1,
                    help="sliced, c64: also time the head-reuse plan of the same workload (1/0)")
    ap.add_argument("--split-compare", type=int, default=1,
                    help="sliced, c64: also time the split-precision forms and report their "
                         "amplitude errors (1/0)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="run one plain device copy of BYTES before the timed region (a known "
                         "reference for HBM traffic counters)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE counter files of one step "
                         "(run with --copy-calibration) into the traffic record, then exit")
    args = ap.parse_args()
    if args.write_traffic:
        if not args.copy_calibration:
            sys.exit("--write-traffic needs the --copy-calibration size the passes used")
        return write_traffic(args, *args.write_traffic)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); slices would shard "
              "across GPUs as independent blocks, which this program does not launch.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        return serving_main(args)

    import numpy as np
    import torch

    from paper_2111_03011_amd.contractor import Contraction
    from paper_2111_03011_amd.workload import config_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_plan = time.perf_counter()
    mode = "samples" if args.workload == "small" else ("reuse" if args.reuse else "default")
    w = config_workload(args.workload, mode=mode)
    t_plan = time.perf_counter() - t_plan
    print(f"[bench] planned {args.workload}: {len(w.plan.path)} steps, "
          f"{len(w.plan.sliced_labels)} sliced bonds, {len(w.slice_ids)} slices, "
          f"peak 2^{w.plan.cost.peak_log2:.0f}, {t_plan:.1f} s", file=sys.stderr, flush=True)
    c = Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                    slice_ids=w.slice_ids, open_qubits=w.open_qubits, closed_bits=w.closed_bits,
                    max_batch_slices=args.batch,
                    precision={"c64": 0, "fp16x3": 1, "bf16x3": 2}[args.precision])
    flops_slice, bytes_slice, n_steps = c.stats()
    flops_step = c.work()     # algorithmic flops one pass executes (shared steps once per batch)
    stream = torch.cuda.current_stream()

    def one_step():
        norm = c.contract(norm=True)
        bits = c.sample(2004, args.samples if len(w.closed_bits) == 1 else len(w.closed_bits))
        return norm, bits

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = c.autotune(reps=2) if args.autotune else 0
    if args.autotune:
        print(f"[bench] autotuner changed {tuned} GEMM launches", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        norm, _ = one_step()
        print(f"[bench] warmup {i}: norm {norm:.6e}", file=sys.stderr, flush=True)
    c.set_timing(True)
    c.timing(reset=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    for i in range(args.steps):
        norm, bits = one_step()
        print(f"[bench] step {i}: norm {norm:.6e}", file=sys.stderr, flush=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    kt = c.timing(reset=True)
    c.set_timing(False)

    # dominant kernel by measured time
    dom = max(kt, key=lambda k: kt[k]["ms"])
    d = kt[dom]
    if dom in ("gemm",):
        algo = d["flops"] / (d["ms"] * 1e-3) / 1e12
        if args.precision == "c64":
            # one v_mfma_f32_32x32x2f32 per complex k: matrix-core flops = algorithmic flops
            roof = {"kernel": "k_gemm (complex64 on v_mfma_f32_32x32x2f32)", "bound": "mfma",
                    "achieved": algo, "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                    "frac": algo / (PEAK_FP32_MFMA / 1e12)}
        else:
            # three products (hi*hi, hi*lo, lo*hi) per algorithmic flop; the FP16 and BF16
            # matrix instructions share one peak
            mfma = "f16" if args.precision == "fp16x3" else "bf16"
            roof = {"kernel": f"k_gemm_bf16x3 (v_mfma_f32_32x32x16_{mfma}, 3 products)",
                    "bound": "mfma", "achieved": 3 * algo, "peak": PEAK_BF16_MFMA / 1e12,
                    "unit": "TFLOP/s", "frac": 3 * algo / (PEAK_BF16_MFMA / 1e12),
                    "algorithmic_tflops": algo}
        roof.update({"traffic": measured_traffic(args), "launches_timed": d["launches"],
                     "avg_launch_ms": d["ms"] / max(d["launches"], 1),
                     "algorithmic_bytes_per_launch": d["bytes"] / max(d["launches"], 1)})
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        roof = {"kernel": f"k_{dom}", "bound": "hbm", "achieved": achieved,
                "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": achieved / (PEAK_HBM / 1e9),
                "traffic": None, "launches_timed": d["launches"],
                "avg_launch_ms": d["ms"] / max(d["launches"], 1)}
    share = {k: v["ms"] for k, v in kt.items() if v["launches"]}
    tot = sum(share.values()) or 1.0
    value = flops_step / (ms_step * 1e-3) / 1e12
    out = {
        "metric": "contraction TFLOP/s & MFMA util; amplitudes/s; p50/p99 request latency",
        "value": value,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (seeded Sycamore-like circuit; random gates, no dataset)",
        "config": {
            "workload": {
                "sliced": "5x6 grid, 14 cycles, ABCDCDAB, fSim(pi/2, pi/6), 10 sliced bonds "
                          "(1024 slices), largest intermediate <= 2^26, 12 open qubits x 1 group "
                          "(4096 amplitudes), 1000 samples",
                "small": "3x4 grid, 8 cycles, all 12 qubits open, 1000 samples",
                "large": "6x9 grid minus (0,4), 20 cycles, 256-slice subset, 2^14 groups x 6 open"
                         + (" (head reuse: 32 subtasks x 8 local slices)" if args.reuse else ""),
            }[args.workload],
            "slices": int(len(w.slice_ids)),
            "amplitudes": int(w.n_amplitudes),
            "path_steps": int(n_steps),
            "flops_per_slice": flops_slice,
            "flops_per_step": flops_step,
        },
        "amplitudes_per_s": w.n_amplitudes / (ms_step * 1e-3),
        "slices_per_s": len(w.slice_ids) / (ms_step * 1e-3),
        "autotuned_launches": tuned,
        "mfma_util_gemm": roof["frac"] if roof["bound"] == "mfma" else None,
        "time_share": {k: v / tot for k, v in share.items()},
        "roofline": roof,
    }
    out["samplers"] = time_samplers(c, w, args)
    refs = {}
    if not args.no_cpu_baseline:
        out["cpu_baseline"], refs = cpu_baseline(w, flops_slice)
        out["rel_err_vs_oracle_slices"] = slice_errors(c, refs)
    extra = args.precision == "c64" and args.workload == "sliced"
    if extra and (args.split_compare or args.head_reuse or args.perturbed):
        c.contract()
        plain = c.amps.cpu().numpy().copy()
        c.close()
        if args.split_compare:
            out["split_precision"] = split_compare(w, args, plain, refs, stream)
        if args.head_reuse:
            out["head_reuse"] = head_reuse(args, plain, out["amplitudes_per_s"])
        if args.perturbed:
            out["perturbed_network"] = perturbed(args, plain, out["amplitudes_per_s"])
    else:
        c.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
