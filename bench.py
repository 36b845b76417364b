"""Benchmark: sliced sparse-state contraction on one MI355X.

One step = the whole hot path over one pass of the workload's slice set, with the network,
targets and slice ids resident in HBM: every slice is contracted (slice leaves, stream and
GEMM steps, split-K reductions), the slices are summed in FP64 into psi_hat, its norm is
taken and bitstrings are drawn (one per group, or 1000 from a single group).  Planning
(circuit -> network -> path, slicing) happens before the timed region.

Default workload (the headline line): the 53-qubit share - 6x9 grid minus site (0,4),
20 cycles, ABCDCDAB, fSim(pi/2, pi/6), 98 sliced bonds, a fixed 256-slice subset, 2^14
groups x 6 open qubits (2^20 amplitudes), largest intermediate 2^30 complex64 (8 GiB),
four slices per launch sequence (109 GB of workspace).  `--workload sliced` runs the 5x6-grid, 14-cycle network
(1024 slices, 4096 amplitudes) as the line instead; by default it runs as extra keys of
the headline line together with the split-precision forms, head reuse and the perturbed
network.

Prints one JSON line.
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
PREC = {"c64": 0, "fp16x3": 1, "bf16x3": 2}
GOLDEN = os.path.join(ROOT, "tests", "golden")
WORKLOAD_TEXT = {
    "large": "53-qubit share: 6x9 grid minus (0,4), 20 cycles, ABCDCDAB, fSim(pi/2, pi/6), "
             "98 sliced bonds, fixed 256-slice subset, 2^14 groups x 6 open qubits "
             "(2^20 amplitudes), one draw per group",
    "sliced": "5x6 grid, 14 cycles, ABCDCDAB, fSim(pi/2, pi/6), 10 sliced bonds (1024 slices), "
              "12 open qubits x 1 group (4096 amplitudes), 1000 samples",
    "small": "3x4 grid, 8 cycles, all 12 qubits open, 1000 samples",
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info() -> dict:
    """The CPU side of the box: cores, model, memory, BLAS library and its threads."""
    import numpy as np
    info = {"nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    try:
        cfg = np.show_config(mode="dicts")
        blas = cfg["Build Dependencies"]["blas"]
        info["blas"] = f"{blas.get('name')} {blas.get('version')}"
    except Exception:
        info["blas"] = "unknown"
    try:
        from threadpoolctl import threadpool_info
        pools = threadpool_info()
        info["blas_threads"] = max([p.get("num_threads", 1) for p in pools] or [1])
        info["threadpools"] = sorted({f"{p.get('internal_api')}:{p.get('num_threads')}" for p in pools})
    except Exception:
        info["blas_threads"] = None
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
        if k in os.environ:
            info[k] = os.environ[k]
    return info


# -- stored oracle values (tests/golden, written by tests/golden/make_golden.py) -----------
def load_sliced_golden():
    """The oracle's 4096 exact amplitudes of the 5x6-grid workload (all 1024 slices)."""
    import numpy as np
    path = os.path.join(GOLDEN, "sliced_5x6_m14_full_sum.txt")
    if not os.path.exists(path):
        return None
    v = np.loadtxt(path, comments="#")
    return v[:, 0] + 1j * v[:, 1]


def load_large_golden():
    """The oracle's (slice position, group, 64 amplitudes) pairs of the 53-qubit share's
    jittered twin (per-gate angles near pi/2; at pi/2 exactly most slices of this slicing
    are exact zeros)."""
    import numpy as np
    path = os.path.join(GOLDEN, "large_53q_m20_slice_group.txt")
    if not os.path.exists(path):
        return []
    pairs, cur = [], None
    for line in open(path):
        if line.startswith("#"):
            continue
        if line.startswith("pair"):
            f = line.split()
            cur = {"pos": int(f[1]), "group": int(f[2]), "slice_id": int(f[3], 16),
                   "closed": int(f[4], 16), "amps": []}
            pairs.append(cur)
        elif line.strip():
            re, im = map(float, line.split())
            cur["amps"].append(complex(re, im))
    for p in pairs:
        p["amps"] = np.asarray(p["amps"])
    return pairs


def rel_error(got, ref) -> float:
    import numpy as np
    got, ref = np.asarray(got).reshape(-1), np.asarray(ref).reshape(-1)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def max_err_over_rms(got, ref) -> float:
    import numpy as np
    got, ref = np.asarray(got).reshape(-1), np.asarray(ref).reshape(-1)
    return float(np.max(np.abs(got - ref)) / max(np.sqrt(np.mean(np.abs(ref) ** 2)), 1e-300))


def infidelity(got, ref) -> float:
    import numpy as np
    got, ref = np.asarray(got).reshape(-1), np.asarray(ref).reshape(-1)
    den = np.vdot(got, got).real * np.vdot(ref, ref).real
    return float(1.0 - abs(np.vdot(ref, got)) ** 2 / den) if den > 0 else 0.0


def percentiles(ms) -> dict:
    import numpy as np
    a = np.asarray(ms, dtype=float)
    return {"median": float(np.median(a)), "p90": float(np.percentile(a, 90)),
            "mean": float(a.mean()), "min": float(a.min()), "max": float(a.max())}


# -- contraction helpers ----------------------------------------------------------------
def contraction(w, precision: str, batch: int):
    from paper_2111_03011_amd.contractor import Contraction
    return Contraction(w.net, w.plan.path, sliced_labels=w.plan.sliced_labels,
                       slice_ids=w.slice_ids, open_qubits=w.open_qubits,
                       closed_bits=w.closed_bits, max_batch_slices=batch,
                       precision=PREC[precision])


def n_draws(w, args) -> int:
    return args.samples if len(w.closed_bits) == 1 else len(w.closed_bits)


def timed_steps(c, w, args, steps: int, warmup: int, tag: str):
    """warmup + steps whole passes (contract all slices, FP64 sum, norm, draws); returns
    the per-step milliseconds (each step ends synchronised: the draws are copied to the
    host) and the last norm."""
    import torch
    nd = n_draws(w, args)
    for i in range(warmup):
        norm = c.contract(norm=True)
        c.sample(2004, nd)
        log(f"{tag} warmup {i}: norm {norm:.6e}")
    ms = []
    torch.cuda.synchronize()
    for i in range(steps):
        t0 = time.perf_counter()
        norm = c.contract(norm=True)
        c.sample(2004, nd)
        ms.append(1e3 * (time.perf_counter() - t0))
        log(f"{tag} step {i}: {ms[-1]:.1f} ms, norm {norm:.6e}")
    return ms, norm


def kernel_family(kind: int, config: int, precision: str) -> str:
    """Name of the HIP kernel (template family) a launch of the plan runs."""
    if kind == 1:
        if config == 6:
            return "k_gemm_outer"
        if config == 5 and precision == "c64":
            return "k_gemm_n8"
        return "k_gemm" if precision == "c64" else "k_gemm_bf16x3"
    return {2: "k_stream", 3: "k_slice_leaves", 4: "k_slice_sum", 5: "k_reduce",
            6: "k_zero_u32"}.get(kind, f"kind{kind}")


def roofline(rows, precision: str, traffic):
    """Dominant kernel by measured time (summed over its timed launches): algorithmic work
    of those launches over their summed durations (HIP event pairs on the contraction
    stream around each launch)."""
    fam = {}
    for r in rows:
        f = fam.setdefault(kernel_family(r["kind_id"], r["config"], precision),
                           {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "launches": 0})
        f["ms"] += r["ms"] * r["count"]
        f["flops"] += r["flops"] * r["count"]
        f["bytes"] += r["bytes"] * r["count"]
        f["launches"] += r["count"]
    dom = max(fam, key=lambda k: fam[k]["ms"])
    d = fam[dom]
    per = max(d["launches"], 1)
    if dom in ("k_gemm", "k_gemm_n8"):
        algo = d["flops"] / (d["ms"] * 1e-3) / 1e12
        # one v_mfma_f32_32x32x2f32 (or 16x16x4) per complex k: matrix-core flops =
        # algorithmic flops
        r = {"kernel": f"{dom} (complex64 on v_mfma_f32)", "bound": "mfma", "achieved": algo,
             "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s", "frac": algo / (PEAK_FP32_MFMA / 1e12)}
    elif dom == "k_gemm_bf16x3":
        # three products (hi*hi, hi*lo, lo*hi) per algorithmic flop; FP16 and BF16 share one
        # matrix-core peak
        algo = d["flops"] / (d["ms"] * 1e-3) / 1e12
        mf = "f16" if precision == "fp16x3" else "bf16"
        r = {"kernel": f"k_gemm_bf16x3 (v_mfma_f32_32x32x16_{mf}, 3 products)",
             "bound": "mfma", "achieved": 3 * algo, "peak": PEAK_BF16_MFMA / 1e12,
             "unit": "TFLOP/s", "frac": 3 * algo / (PEAK_BF16_MFMA / 1e12),
             "algorithmic_tflops": algo}
    else:
        gbs = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        r = {"kernel": dom, "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM / 1e9,
             "unit": "GB/s", "frac": gbs / (PEAK_HBM / 1e9)}
    r.update({"traffic": traffic, "launches_timed": d["launches"],
              "avg_launch_ms": d["ms"] / per,
              "algorithmic_flops_per_launch": d["flops"] / per,
              "algorithmic_bytes_per_launch": d["bytes"] / per,
              "time_by_kernel_ms": {k: round(v["ms"], 3) for k, v in
                                    sorted(fam.items(), key=lambda kv: -kv[1]["ms"])}})
    return r


KIND = {1: "gemm", 2: "stream", 3: "slice_leaves", 4: "slice_sum", 5: "splitk_reduce",
        6: "scale_records"}
TILE = {0: "128x64", 1: "128x16", 2: "64x32", 3: "128x128", 4: "128x32", 5: "128x8",
        6: "vector", 7: "128x128w8", 8: "256x64w8"}


def step_classes(c) -> dict:
    """Per launch of the plan (timed launches only): kind, shape, time, algorithmic
    TFLOP/s and GB/s of the launch (all the slices it processes); summarised by class - GEMMs above the FP32 ridge (MFMA-bound by
    their arithmetic intensity) and the rest (HBM-bound)."""
    rows = []
    infos = c.launches()
    for i, (ms, n) in enumerate(c.launch_timing()):
        if n == 0:
            continue
        s = infos[i]
        t = ms / n
        # per-slice work times the slices one launch processes (a full batch, or one copy
        # for steps run once per call or per batch)
        per = c.batch_slices if s.invariant == 0 else 1
        s.flops *= per
        s.bytes *= per
        inten = s.flops / max(s.bytes, 1.0)
        rows.append({"i": i, "kind": KIND.get(s.kind, str(s.kind)), "kind_id": s.kind,
                     "config": s.config, "flops": s.flops, "bytes": s.bytes, "inv": s.invariant,
                     "rows": s.rows, "m": s.m, "n": s.n, "k": s.k,
                     "tile": TILE.get(s.config, "-") if s.kind == 1 else "-",
                     "splits": s.k_splits, "row_mode": s.row_mode, "ms": t, "count": n,
                     "tflops": s.flops / (t * 1e-3) / 1e12 if t > 0 else 0.0,
                     "gbs": s.bytes / (t * 1e-3) / 1e9 if t > 0 else 0.0,
                     "intensity": inten,
                     "mfma_bound": s.kind == 1 and inten >= PEAK_FP32_MFMA / PEAK_HBM})
    out = {}
    for cls, sel in (("mfma_bound_gemm", lambda r: r["mfma_bound"]),
                     ("hbm_bound", lambda r: not r["mfma_bound"])):
        rs = [r for r in rows if sel(r)]
        ms = sum(r["ms"] * r["count"] for r in rs)
        fl = sum(r["tflops"] * r["ms"] * r["count"] for r in rs)
        by = sum(r["gbs"] * r["ms"] * r["count"] for r in rs)
        out[cls] = {"launch_types": len(rs), "ms": ms,
                    "tflops": fl / ms if ms else 0.0, "gbs": by / ms if ms else 0.0}
    tot = sum(v["ms"] for v in out.values()) or 1.0
    for v in out.values():
        v["time_share"] = v["ms"] / tot
    out["mfma_bound_gemm"]["frac_of_fp32_peak"] = out["mfma_bound_gemm"]["tflops"] / (PEAK_FP32_MFMA / 1e12)
    out["hbm_bound"]["frac_of_hbm_peak"] = out["hbm_bound"]["gbs"] / (PEAK_HBM / 1e9)
    return out, rows


def write_step_table(path: str, rows, title: str) -> None:
    with open(path, "w") as f:
        f.write(f"# {title}\n\n")
        f.write("| launch | kind | inv | rows | M | N | K | tile | splits | row mode | ms | "
                "TFLOP/s | GB/s | flop/B | bound |\n")
        f.write("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|\n")
        for r in sorted(rows, key=lambda r: -r["ms"] * r["count"]):
            f.write(f"| {r['i']} | {r['kind']} | {r['inv']} | {r['rows']} | {r['m']} | {r['n']} | "
                    f"{r['k']} | {r['tile']} | {r['splits']} | {r['row_mode']} | {r['ms']:.4f} | "
                    f"{r['tflops']:.1f} | {r['gbs']:.0f} | {r['intensity']:.1f} | "
                    f"{'mfma' if r['mfma_bound'] else 'hbm'} |\n")


# -- the CPU oracle, timed (the only place the benchmark runs oracle code) -----------------
def cpu_baseline_sliced(w, flops_per_slice: float, budget_s: float = 20.0):
    """The oracle, as it stands, on as many single slices of the workload as fit in about
    `budget_s` seconds (at least one).  Returns the record and the oracle amplitudes of the
    sampled slices by slice position."""
    from oracle import contract as ocontract
    done, t0, refs = 0, time.perf_counter(), {}
    while True:
        idx = done % len(w.slice_ids)
        refs[idx] = ocontract.sparse_amplitudes(w.circuit, w.open_qubits, w.closed_bits,
                                                sliced_bonds=w.sliced_bonds,
                                                slice_ids=[int(w.slice_ids[idx])])
        done += 1
        if time.perf_counter() - t0 > budget_s or done >= len(w.slice_ids):
            break
    per_slice = (time.perf_counter() - t0) / done
    hi = host_info()
    return {"value": w.n_amplitudes / (per_slice * len(w.slice_ids)), "unit": "amplitudes/s",
            "cores": hi.get("blas_threads") or hi["nproc"], "kind": "oracle",
            "sample": f"{done} slice(s) of the same workload, numpy complex128 tensordot along "
                      f"the oracle's own greedy path, {per_slice:.2f} s per slice; value = the "
                      "workload's amplitudes / (oracle seconds per slice x its slices)",
            "seconds_per_slice": per_slice,
            "tflops_equivalent": flops_per_slice / per_slice / 1e12,
            "host": hi}, refs


def cpu_baseline_large(w, flops_per_slice: float, pos: int = 0, group: int = 0):
    """The oracle, as it stands, on one (slice, group) pair of the 53-qubit share: its own
    network for that group (closed outputs fixed), the pair's slice fixed, its own seeded
    random-greedy path (path search not timed), numpy complex128 tensordot.  Every pair has
    the same structure, so the oracle's rate in the bench's unit is the pair's amplitudes
    over (its time x the number of slices summed); its flop rate is reported beside it."""
    from oracle import contract as ocontract
    from oracle import network as onetwork
    circ, n = w.circuit, w.circuit["n_qubits"]
    sigma, cb = int(w.slice_ids[pos]), int(w.closed_bits[group])
    closed = [q for q in range(n) if q not in set(w.open_qubits)]
    net = onetwork.build_network(circ, {q: (cb >> (n - 1 - q)) & 1 for q in closed})
    fixed = {net.bond_label[tuple(b)]: (sigma >> bi) & 1 for bi, b in enumerate(w.sliced_bonds)}
    tensors, labels = net.sliced(fixed)
    path = ocontract.random_greedy_path(labels, 5101)
    macs, ls = 0.0, [set(l) for l in labels]
    for i, j in path:
        macs += 2.0 ** len(ls[i] | ls[j])
        ls[i] = ls[i] ^ ls[j]
    t0 = time.perf_counter()
    out = ocontract.contract_path(tensors, labels, path, [net.out_label[q] for q in w.open_qubits])
    sec = time.perf_counter() - t0
    rate = 8.0 * macs / sec
    hi = host_info()
    return {"value": out.size / (sec * len(w.slice_ids)), "unit": "amplitudes/s",
            "cores": hi.get("blas_threads") or hi["nproc"], "kind": "oracle",
            "sample": f"one (slice, group) pair of the same workload (slice position {pos}, group "
                      f"{group}): its {out.size} amplitudes of one slice in {sec:.1f} s "
                      f"({8 * macs:.3e} oracle flops); value = {out.size} / ({sec:.1f} s x "
                      f"{len(w.slice_ids)} slices), amplitudes summed over the slice subset",
            "oracle_pair_seconds": sec, "oracle_tflops": rate / 1e12,
            "host": hi}, {(pos, group): out.reshape(-1)}


# -- extra keys ---------------------------------------------------------------------------
def pair_errors(c, w, pairs) -> dict:
    """Single (slice, group) pairs of the contraction against stored oracle values:
    normwise relative error and max |error| / rms of the 64 amplitudes."""
    worst, worst_max = 0.0, 0.0
    for p in pairs:
        assert int(w.slice_ids[p["pos"]]) == p["slice_id"], "stored pair names another slice"
        assert int(w.closed_bits[p["group"]]) == p["closed"], "stored pair names another group"
        c.contract_range(p["pos"], 1)
        got = c.amps[p["group"]].cpu().numpy()
        worst = max(worst, rel_error(got, p["amps"]))
        worst_max = max(worst_max, max_err_over_rms(got, p["amps"]))
    return {"pairs": len(pairs), "rel_err": worst, "max_err_over_rms": worst_max}


def twin_pair_errors(w, name, pairs) -> dict:
    """pair_errors on the jittered twin of the workload (same plan and slices, per-gate
    angles near pi/2), one slice contracted at a time (results do not depend on the batch)."""
    import synth
    from paper_2111_03011_amd.workload import jittered_twin
    j = synth.config("large")["parity_jitter"]
    tw = jittered_twin(w, j["theta_jitter"], j["jitter_seed"])
    c = contraction(tw, name, 1)
    c.autotune(reps=1)
    res = pair_errors(c, tw, pairs)
    c.close()
    return res


def large_forms(args, c64_amps, c64_aps, pairs, batch: int) -> dict:
    """The split-precision forms of the 53-qubit share (same plan, slices, batch): one timed
    whole pass each, amplitudes/s, difference from the complex64 sum, error against the
    stored oracle pairs."""
    import torch
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("large", mode="default" if args.plain_path else "branch")
    res = {}
    for name in ("bf16x3", "fp16x3"):
        c = contraction(w, name, batch)
        if args.autotune:
            c.autotune(reps=1)
        c.contract_range(0, batch)
        torch.cuda.synchronize()
        ms, _ = timed_steps(c, w, args, 1, 0, f"large {name}")
        amps = c.amps.cpu().numpy().copy()
        r = {"amplitudes_per_s": w.n_amplitudes / (ms[0] * 1e-3), "ms_per_step": ms[0],
             "ms_per_slice": ms[0] / len(w.slice_ids),
             "tflops": c.work() / (ms[0] * 1e-3) / 1e12,
             "speedup_vs_c64": (w.n_amplitudes / (ms[0] * 1e-3)) / c64_aps,
             "rel_err_vs_c64_sum": rel_error(amps, c64_amps),
             "infidelity_vs_c64_sum": infidelity(amps, c64_amps)}
        c.close()
        if pairs:
            r["vs_oracle_pairs_jittered_twin"] = twin_pair_errors(w, name, pairs)
        res[name] = r
        log(f"large {name}: {r['amplitudes_per_s']:.0f} amplitudes/s "
            f"({r['speedup_vs_c64']:.2f}x c64), rel diff vs c64 {r['rel_err_vs_c64_sum']:.2e}")
    return res


def large_reuse(args, c64_aps) -> dict:
    """Head reuse on the 53-qubit share (Method; Appendix B.2): the branch-merged path and
    the plan's sliced bonds, the three cheapest on the low slice-id bits, 256 slices as 32
    subtasks x 8 local values; every step above the 95 global labels runs once per batch of
    8."""
    import torch
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("large", mode="reuse")
    res = {"subtasks": len(w.slice_ids) // 8, "local_slices": 8}
    for name in ("c64", "bf16x3", "fp16x3"):
        c = contraction(w, name, 8)
        if args.autotune:
            c.autotune(reps=1)
        c.contract_range(0, 8)
        torch.cuda.synchronize()
        ms, _ = timed_steps(c, w, args, 1, 0, f"large reuse {name}")
        aps = w.n_amplitudes / (ms[0] * 1e-3)
        res[name] = {"amplitudes_per_s": aps, "ms_per_step": ms[0],
                     "ms_per_slice": ms[0] / len(w.slice_ids),
                     "executed_tflops": c.work() / (ms[0] * 1e-3) / 1e12,
                     "speedup_vs_plain_c64": aps / c64_aps,
                     "workspace_gb": c.ws_bytes / 1e9}
        c.close()
        log(f"large reuse {name}: {aps:.0f} amplitudes/s ({aps / c64_aps:.2f}x plain c64)")
    return res


def large_plain_path(args, merged_aps, batch: int = 4) -> dict:
    """The 53-qubit share on the plain path (the planner's path before branch merging; same
    sliced bonds and slices; four slices per launch sequence, as its 2^30 intermediates
    allow): one timed whole pass per form, against the branch-merged complex64 rate of the
    headline."""
    import torch
    from paper_2111_03011_amd.workload import config_workload
    w0 = config_workload("large")
    w = config_workload("large", mode="branch")
    res = {"flops_per_slice_plain": w0.plan.cost.flops_per_slice,
           "flops_per_slice_branch_merged": w.plan.cost.flops_per_slice}
    for name in ("c64", "bf16x3", "fp16x3"):
        c = contraction(w0, name, batch)
        if args.autotune:
            c.autotune(reps=1)
        c.contract_range(0, batch)
        torch.cuda.synchronize()
        ms, _ = timed_steps(c, w0, args, 1, 0, f"large plain path {name}")
        aps = w0.n_amplitudes / (ms[0] * 1e-3)
        res[name] = {"amplitudes_per_s": aps, "ms_per_step": ms[0],
                     "ms_per_slice": ms[0] / len(w0.slice_ids),
                     "tflops": c.work() / (ms[0] * 1e-3) / 1e12,
                     "branch_merged_c64_speedup": merged_aps / aps,
                     "workspace_gb": c.ws_bytes / 1e9}
        c.close()
        log(f"large plain path {name}: {ms[0] / len(w0.slice_ids):.2f} ms per slice")
        torch.cuda.empty_cache()
    return res


def large_zigzag(args, tail_start: int = 19, count: int = 4) -> dict:
    """The zigzag tail order (Method; Appendix E) on the 53-qubit share: the planner's total
    work of a zigzag plan with its own slicing against the plain plans, and a zigzag plan
    that slices the plain plan's bonds plus those its bound needs, run with the plain path
    on that same slicing over the same `count` slices of the jittered twin (their sums must
    agree; at pi/2 exactly the slices are structural zeros)."""
    import numpy as np
    import torch
    import synth
    from paper_2111_03011_amd import planner
    from paper_2111_03011_amd.workload import config_workload, jittered_twin, zigzag_pair
    w = config_workload("large")
    jit = synth.config("large")["parity_jitter"]
    twin = jittered_twin(w, jit["theta_jitter"], jit["jitter_seed"])
    zz = planner.zigzag_plan(w.net, w.open_qubits, w.closed_bits, tail_start, 30, trials=4,
                             seed=1919)
    wz, wp = zigzag_pair(twin, tail_start, 30, count, 1919)
    free = planner.find_plan(w.net, w.open_qubits, w.closed_bits, max_log2=30, n_sliced=None,
                             trials=4, seed=5)
    res = {"tail_start": tail_start,
           "planned_total_flops_log2": {"zigzag_own_slicing": float(np.log2(zz.total_flops)),
                                        "plain_fewest_slices": float(np.log2(free.total_flops)),
                                        "plain_98_bonds": float(np.log2(w.plan.total_flops))},
           "sliced_bonds": {"zigzag_own": len(zz.sliced_labels), "plain_fewest": len(free.sliced_labels),
                            "zigzag_on_plain": len(wz.plan.sliced_labels)},
           "slices_run": count}
    sums = {}
    for tag, ww in (("zigzag", wz), ("plain_path", wp)):
        c = contraction(ww, "c64", 1)
        c.contract_range(0, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.contract()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        sums[tag] = c.amps.cpu().numpy().copy()
        res[tag] = {"ms_per_slice": ms / count, "planned_flops_per_slice": ww.plan.cost.flops_per_slice,
                    "peak_log2": ww.plan.cost.peak_log2, "launches": len(c.launches()),
                    "tflops": c.work() / (ms * 1e-3) / 1e12}
        c.close()
        log(f"zigzag extra, {tag}: {ms / count:.1f} ms per slice")
    res["sum_rel_diff"] = rel_error(sums["zigzag"], sums["plain_path"])
    return res


def xeb_vs_exact(c, w, exact, n_samples: int, seed: int) -> float:
    """Linear XEB (Appendix D) of n_samples draws from the contraction's amplitudes, scored
    with the exact probabilities |psi(s)|^2 of the stored state-vector amplitudes."""
    import numpy as np
    bits = c.sample(seed, n_samples)
    n, opn = w.circuit["n_qubits"], w.open_qubits
    mu = np.zeros(len(bits), dtype=np.int64)
    for t, q in enumerate(opn):
        mu |= ((bits.astype(np.int64) >> (n - 1 - q)) & 1) << (len(opn) - 1 - t)
    p = np.abs(exact[mu]) ** 2
    return float(2.0 ** n * p.mean() - 1.0)


def sliced_extra(args, refs=None) -> dict:
    """The 5x6-grid, 14-cycle network (1024 slices, 4096 amplitudes) in every form: the
    plain complex64 pass at 64 slices per launch (graph replays), BF16x3 and FP16x3 with
    their amplitude error, infidelity and XEB change against the exact (FP64 state-vector)
    amplitudes, the head-reuse plan and the perturbed network."""
    import numpy as np
    import torch
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("sliced")
    exact = load_sliced_golden()
    res = {"workload": WORKLOAD_TEXT["sliced"], "batch": 64, "peak_log2": w.plan.cost.peak_log2}
    amps_by = {}
    for name in ("c64", "bf16x3", "fp16x3"):
        c = contraction(w, name, 64)
        if args.autotune:
            c.autotune(reps=2)
        if name == "c64":
            c.set_timing(True)
            c.timing(reset=True)
        ms, _ = timed_steps(c, w, args, 3, 1, f"sliced {name}")
        r = {"ms_per_step": percentiles(ms), "amplitudes_per_s": w.n_amplitudes / (np.median(ms) * 1e-3),
             "tflops": c.work() / (np.median(ms) * 1e-3) / 1e12}
        if name == "c64":
            r["roofline"] = roofline(step_classes(c)[1], "c64", None)
            c.timing(reset=True)
            c.set_timing(False)
        c.contract()
        amps = c.amps.cpu().numpy()[0].copy()
        amps_by[name] = amps
        if exact is not None:
            r["rel_err_vs_oracle_full_sum"] = rel_error(amps, exact)
            r["max_err_over_rms_vs_oracle"] = max_err_over_rms(amps, exact)
            r["infidelity_vs_oracle"] = infidelity(amps, exact)
            r["xeb_1024_samples"] = xeb_vs_exact(c, w, exact, 1024, 3001)
        if name != "c64":
            r["speedup_vs_c64"] = r["amplitudes_per_s"] / res["c64"]["amplitudes_per_s"]
            if exact is not None:
                r["delta_xeb_vs_c64"] = r["xeb_1024_samples"] - res["c64"]["xeb_1024_samples"]
        if exact is not None and name == "c64":
            # draws from the exact amplitudes themselves (uploaded into the same buffer)
            c.amps.copy_(torch.from_numpy(exact.reshape(1, -1)).to(c.amps.device))
            res["xeb_1024_samples_exact_amplitudes"] = xeb_vs_exact(c, w, exact, 1024, 3001)
        c.close()
        res[name] = r
        log(f"sliced {name}: {r['amplitudes_per_s']:.0f} amplitudes/s"
            + (f", rel err vs oracle {r['rel_err_vs_oracle_full_sum']:.2e}" if exact is not None else ""))
    if exact is not None:
        for name in ("c64", "bf16x3", "fp16x3"):
            res[name]["delta_xeb_vs_exact"] = (res[name]["xeb_1024_samples"]
                                               - res["xeb_1024_samples_exact_amplitudes"])
    plain_aps = res["c64"]["amplitudes_per_s"]
    if args.head_reuse:
        res["head_reuse"] = sliced_reuse(args, amps_by["c64"], plain_aps)
    if args.perturbed:
        res["perturbed_network"] = perturbed(args, amps_by["c64"] if exact is None else exact, plain_aps)
    return res


def sliced_reuse(args, plain_amps, plain_aps) -> dict:
    """The 1024-slice workload planned for head reuse: 4 global bonds (size bound) and 6
    local ones on the low slice-id bits; steps above the global labels once per 64."""
    import numpy as np
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("sliced", mode="reuse")
    res = {"peak_log2": w.plan.cost.peak_log2}
    for name in ("c64", "bf16x3"):
        c = contraction(w, name, 64)
        if args.autotune:
            c.autotune(reps=2)
        ms, _ = timed_steps(c, w, args, 3, 1, f"sliced reuse {name}")
        amps = c.amps.cpu().numpy()[0].copy()
        aps = w.n_amplitudes / (np.median(ms) * 1e-3)
        res[name] = {"amplitudes_per_s": aps, "ms_per_step": float(np.median(ms)),
                     "executed_tflops": c.work() / (np.median(ms) * 1e-3) / 1e12,
                     "speedup_vs_plain_c64": aps / plain_aps,
                     "rel_err_vs_plain_c64_sum": rel_error(amps, plain_amps)}
        c.close()
    return res


def perturbed(args, exact_amps, plain_aps) -> dict:
    """The 1024-slice workload with holes drilled into the circuit (Method): K = 2 broken
    edges per hole, fidelity estimate 2^-K, measured against the exact amplitudes."""
    import numpy as np
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload("sliced", mode="holes")
    c = contraction(w, "c64", 64)
    if args.autotune:
        c.autotune(reps=2)
    ms, _ = timed_steps(c, w, args, 3, 1, "perturbed")
    amps = c.amps.cpu().numpy()[0].copy()
    work = c.work()
    c.close()
    K = 2 * len(w.circuit["holes"])
    aps = w.n_amplitudes / (np.median(ms) * 1e-3)
    return {"holes": [int(h) for h in w.circuit["holes"]], "broken_edges": K,
            "fidelity_estimate": 2.0 ** -K,
            "fidelity_vs_exact_4096_amplitudes": 1.0 - infidelity(amps, exact_amps),
            "amplitudes_per_s": aps, "ms_per_step": float(np.median(ms)),
            "flops_per_step": work, "speedup_vs_plain_c64": aps / plain_aps}


def time_samplers(c, w, args) -> dict:
    """Wall time of the three in-group samplers on the contracted amplitudes (inverse CDF,
    the paper's Metropolis chains, frugal rejection sampling), one call each after a warm-up
    call; the bitstrings are copied to the host inside the timed call."""
    n = n_draws(w, args)
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


# -- HBM traffic of the dominant kernel (rocprofv3 counter passes, summarised offline) -----
def traffic_json(workload: str, precision: str) -> str:
    name = {"large": "large_53q_m20", "sliced": "sliced_5x6_m14", "small": "small_3x4_m8"}[workload]
    return os.path.join(ROOT, "profiles", f"k_gemm_{name}_{precision}_traffic.json")


def kernels_sha256():
    import hashlib
    src = open(os.path.join(ROOT, "paper_2111_03011_amd", "csrc", "kernels.hip"), "rb").read()
    return hashlib.sha256(src).hexdigest()


def headline_mode(args) -> str:
    """Workload mode of the timed run: the 53-qubit share runs its branch-merged path
    (planner.merge_branches) unless --plain-path or --reuse asks otherwise."""
    if args.workload == "small":
        return "samples"
    if args.reuse:
        return "reuse"
    if args.workload == "large" and not args.plain_path:
        return "branch"
    return "default"


def measured_traffic(args, batch: int):
    """HBM bytes per launch of the dominant GEMM kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (calibrated against a plain device copy), or None when
    they do not describe the kernel that runs now (other source, precision, workload, path,
    batch or launch program)."""
    try:
        rec = json.load(open(traffic_json(args.workload, args.precision)))
        sha = kernels_sha256()
    except OSError:
        return None
    if (rec.get("kernels_hip_sha256") != sha or rec.get("workload") != args.workload or
            rec.get("precision") != args.precision or rec.get("batch") != batch or
            rec.get("mode", "default") != headline_mode(args)):
        return None
    if rec.get("launch_shapes_sha256") != launch_shapes_sha256(args, batch):
        return None
    return rec["traffic_bytes_per_launch"]


def launch_shapes_sha256(args, batch: int) -> str:
    """Fingerprint of the launch program the timed run compiles (kind, shape, tile and
    split of every launch, before autotuning), so that a counter record is used only for
    the launch mix it was taken on; planner and compiler changes alter it as kernel changes
    alter the source hash.  Compiled on the host: no device is touched."""
    import hashlib
    from paper_2111_03011_amd import tnc
    from paper_2111_03011_amd.workload import config_workload
    w = config_workload(args.workload, mode=headline_mode(args))
    prec = {"c64": tnc.TNC_C64, "bf16x3": tnc.TNC_BF16X3, "fp16x3": tnc.TNC_FP16X3}[args.precision]
    h = tnc.tnc_net_create(0, w.net.n_qubits, w.net.ranks(), w.net.flat_labels(),
                           w.net.flat_data(), w.net.out_label)
    try:
        tnc.tnc_net_set_path(h, w.plan.path)
        tnc.set_slices_any(h, w.plan.sliced_labels, w.slice_ids)
        tnc.tnc_net_set_targets(h, w.open_qubits, w.closed_bits)
        p = tnc.tnc_plan_create(h, prec, batch)
        try:
            rows = []
            for i in range(tnc.tnc_plan_n_launches(p)):
                l = tnc.tnc_plan_launch_info(p, i)
                rows.append((l.kind, l.invariant, l.rows, l.m, l.n, l.k, l.config, l.k_splits))
        finally:
            tnc.tnc_plan_destroy(p)
    finally:
        tnc.tnc_net_destroy(h)
    return hashlib.sha256(repr(rows).encode()).hexdigest()


def write_traffic(args, batch: int, fetch_csv, write_csv):
    """Summarise two rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE; a short run of this
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
        "mode": headline_mode(args),
        "batch": batch, "kernels_hip_sha256": kernels_sha256(),
        "launch_shapes_sha256": launch_shapes_sha256(args, batch),
        "slices_profiled": args.max_slices or "all", "dispatches": [n_f, n_w],
        "fetch_kib_per_launch_raw": round(f_kib, 2), "write_kib_per_launch_raw": round(w_kib, 2),
        "copy_calibration": {"bytes": args.copy_calibration, "fetch_kib": f_copy,
                             "write_kib": w_copy, "fetch_factor": round(f_fac, 4),
                             "write_factor": round(w_fac, 4)},
        "fetch_bytes_per_launch": round(f_kib * f_fac * 1024.0),
        "write_bytes_per_launch": round(w_kib * w_fac * 1024.0),
    }
    rec["traffic_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    with open(traffic_json(args.workload, args.precision), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


def summarise_stats(path: str) -> None:
    """Markdown table of a rocprofv3 --stats kernel summary (kernel_stats.csv), one line per
    kernel template instance and one per kernel family (template arguments dropped)."""
    import csv
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0

    def short(name):
        # "void tnc::(anonymous namespace)::k_gemm<2, 2, ...>(tnc::GemmArgs)" -> "k_gemm<2, 2, ...>"
        import re
        m = re.search(r"(k_\w+|__amd_\w+)(<[^()]*>)?", name)
        return (m.group(1) + (m.group(2) or "")) if m else name

    fam = {}
    print("| kernel | calls | total ms | avg us | share % |")
    print("|---|---|---|---|---|")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        n, calls, t = short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"])
        f = fam.setdefault(n.split("<")[0].split("(")[0], [0, 0.0])
        f[0] += calls
        f[1] += t
        if t / tot >= 0.001:
            print(f"| `{n}` | {calls} | {t / 1e6:.2f} | {t / calls / 1e3:.2f} | {100 * t / tot:.2f} |")
    print("\n| kernel family | calls | total ms | avg us | share % |")
    print("|---|---|---|---|---|")
    for n, (calls, t) in sorted(fam.items(), key=lambda kv: -kv[1][1]):
        print(f"| `{n}` | {calls} | {t / 1e6:.2f} | {t / calls / 1e3:.2f} | {100 * t / tot:.2f} |")


def xeb_vs_group_size(args) -> dict:
    """Linear XEB of one draw per group against the group size l (Appendix D): the 5x6-grid,
    14-cycle circuit, 2048 seeded groups whose l = 2^j amplitudes vary the last j qubits,
    contracted on the GPU (complex64, all slices) and sampled with the GPU samplers (inverse
    CDF inside each group, Metropolis chains of 100 steps, frugal rejection with m = 10).
    Draws are scored with the contraction's own amplitudes, p(s) = |psi(s)|^2 (the circuit
    is unitary, so no normalisation).  'in_group_exact' is the expectation of inverse-CDF
    sampling computed from the amplitudes; for Porter-Thomas amplitudes it is near
    (l - 1) / (l + 1)."""
    import numpy as np
    import torch
    import synth
    from paper_2111_03011_amd.workload import config_workload, make_workload
    base = config_workload("sliced")
    circ, n, L = base.circuit, base.circuit["n_qubits"], 2048
    res = {"workload": "5x6 grid, 14 cycles (30 qubits), 2048 groups, complex64", "rows": []}
    for j in range(7):
        open_q = list(range(n - j, n))
        closed = synth.group_targets(n, open_q, L, 2002)
        w = make_workload(circ, open_q, closed, max_log2=28, trials=4, seed=2005)
        c = contraction(w, "c64", 8)
        t0 = time.perf_counter()
        c.contract()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0)
        amps = c.amps.cpu().numpy().reshape(L, -1)
        p = np.abs(amps) ** 2
        row = {"l": 1 << j, "sliced": len(w.plan.sliced_labels), "contract_ms": ms,
               "tflops": c.work() / (ms * 1e-3) / 1e12,
               "in_group_exact": float(2.0 ** n * np.mean((p ** 2).sum(1) / p.sum(1)) - 1.0),
               "porter_thomas": ((1 << j) - 1) / ((1 << j) + 1)}
        draws = {"inverse_cdf": c.sample(11, L), "metropolis_100": c.sample_metropolis(12, L, 100),
                 "frugal_m10": c.sample_frugal(13, L, 10.0, 64)}
        for name, bits in draws.items():
            mu = np.zeros(L, dtype=np.int64)
            for t, q in enumerate(open_q):
                mu |= ((bits.astype(np.int64) >> (n - 1 - q)) & 1) << (len(open_q) - 1 - t)
            row[name] = float(2.0 ** n * p[np.arange(L), mu].mean() - 1.0)
        c.close()
        res["rows"].append(row)
        log(f"XEB vs l: l={1 << j}: " + ", ".join(f"{k} {v:.3f}" for k, v in row.items()
                                                  if isinstance(v, float)))
    return res


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
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["large", "sliced", "small", "serving"])
    ap.add_argument("--precision", default="c64", choices=["c64", "bf16x3", "fp16x3"])
    ap.add_argument("--batch", type=int, default=0,
                    help="slices per launch sequence (0 = the workload's own: 64 for large, "
                         "4 for large --plain-path, 8 for large --reuse, 64 for sliced)")
    ap.add_argument("--reuse", action="store_true",
                    help="large: the head-reuse mode (32 subtasks x 8 local slices)")
    ap.add_argument("--samples", type=int, default=1000)
    ap.add_argument("--autotune", type=int, default=1, help="time tile choices per GEMM first (1/0)")
    ap.add_argument("--extras", type=int, default=1,
                    help="large, c64: also the split-precision forms and head reuse of the same "
                         "share, and the 5x6-grid network in every form (1/0)")
    ap.add_argument("--head-reuse", type=int, default=1, help="5x6 network: also the reuse plan")
    ap.add_argument("--perturbed", type=int, default=1, help="5x6 network: also the drilled one")
    ap.add_argument("--plain-path", action="store_true",
                    help="large: time the plain path instead of the branch-merged one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--step-table", metavar="PATH", help="write the per-launch timing table")
    ap.add_argument("--max-slices", type=int, default=0,
                    help="profiling runs only: contract the first N slices of the subset")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="run one plain device copy of BYTES before the timed region (a known "
                         "reference for HBM traffic counters)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE counter files of a run "
                         "with --copy-calibration into the traffic record, then exit")
    ap.add_argument("--summarise-stats", metavar="KERNEL_STATS_CSV",
                    help="print a markdown summary of a rocprofv3 --stats kernel file, then exit")
    ap.add_argument("--xeb-vs-l", action="store_true",
                    help="print the XEB-against-group-size study of the 5x6 network, then exit")
    ap.add_argument("--requests", type=int, default=400, help="serving: requests in the stream")
    ap.add_argument("--templates", type=int, default=16, help="serving: distinct request templates")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent requests")
    ap.add_argument("--arena-gb", type=int, default=64, help="serving: device arena")
    ap.add_argument("--serving-timeout", type=float, default=150.0)
    ap.add_argument("--serving-batch", type=int, default=0,
                    help="serving: slices per launch sequence (0 = chosen per request)")
    args = ap.parse_args()
    large_batch = 8 if args.reuse else (4 if args.plain_path else 64)
    batch = args.batch or {"large": large_batch, "sliced": 64, "small": 1}.get(args.workload, 1)
    if args.summarise_stats:
        return summarise_stats(args.summarise_stats)
    if args.write_traffic:
        if not args.copy_calibration:
            sys.exit("--write-traffic needs the --copy-calibration size the passes used")
        return write_traffic(args, batch, *args.write_traffic)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); slices would shard "
              "across GPUs as independent blocks, which this program does not launch.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        return serving_main(args)
    if args.xeb_vs_l:
        print(json.dumps(xeb_vs_group_size(args)), flush=True)
        return

    import dataclasses

    import numpy as np
    import torch

    from paper_2111_03011_amd.workload import config_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_plan = time.perf_counter()
    mode = headline_mode(args)
    w = config_workload(args.workload, mode=mode)
    if args.max_slices:
        w = dataclasses.replace(w, slice_ids=w.slice_ids[:args.max_slices])
    t_plan = time.perf_counter() - t_plan
    log(f"planned {args.workload}: {len(w.plan.path)} steps, {len(w.plan.sliced_labels)} sliced "
        f"bonds, {len(w.slice_ids)} slices, peak 2^{w.plan.cost.peak_log2:.0f}, {t_plan:.1f} s")
    c = contraction(w, args.precision, batch)
    flops_slice, bytes_slice, n_steps = c.stats()
    flops_step = c.work()     # algorithmic flops one pass executes (shared steps once per batch)
    log(f"workspace {c.ws_bytes / 1e9:.1f} GB, {flops_step / 1e12:.1f} TFLOP per pass")
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = c.autotune(reps=1 if args.workload == "large" else 2) if args.autotune else 0
    log(f"autotuner changed {tuned} GEMM launches")
    for i in range(args.warmup):
        norm = c.contract(norm=True)
        c.sample(2004, n_draws(w, args))
        log(f"warmup {i}: norm {norm:.6e}")
    c.set_timing(True)
    c.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms, norm = timed_steps(c, w, args, args.steps, 0, "timed")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    kt = c.timing(reset=False)
    classes, table = step_classes(c)
    c.timing(reset=True)
    c.set_timing(False)
    if args.step_table:
        write_step_table(args.step_table, table,
                         f"per-launch times, {args.workload} workload, {args.precision}, batch {batch}")
    roof = roofline(table, args.precision, measured_traffic(args, batch))
    share = {k: v["ms"] for k, v in kt.items() if v["launches"]}
    tot = sum(share.values()) or 1.0
    aps = w.n_amplitudes / (ms_step * 1e-3)
    out = {
        "metric": "contraction TFLOP/s & MFMA util; amplitudes/s; p50/p99 request latency",
        "value": aps,
        "unit": "amplitudes/s",
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
            "workload": WORKLOAD_TEXT[args.workload]
                        + (" (head reuse: 32 subtasks x 8 local slices)" if args.reuse else "")
                        + (" (branch-merged path)" if mode == "branch" else ""),
            "slices": int(len(w.slice_ids)),
            "amplitudes": int(w.n_amplitudes),
            "largest_intermediate_log2": float(w.plan.cost.peak_log2),
            "slices_per_launch": int(c.batch_slices),
            "path_steps": int(n_steps),
            "flops_per_slice": flops_slice,
            "flops_per_step": flops_step,
            "workspace_gb": c.ws_bytes / 1e9,
        },
        "step_ms": percentiles(ms),
        "contraction_tflops": flops_step / (ms_step * 1e-3) / 1e12,
        "slices_per_s": len(w.slice_ids) / (ms_step * 1e-3),
        "ms_per_slice": ms_step / len(w.slice_ids),
        "autotuned_launches": tuned,
        "mfma_util_gemm": roof["frac"] if roof["bound"] == "mfma" else None,
        "time_share": {k: v / tot for k, v in share.items()},
        "step_classes": classes,
        "roofline": roof,
        "samplers": time_samplers(c, w, args),
    }
    c.contract()
    main_amps = c.amps.cpu().numpy().copy()
    if args.workload == "sliced" and not args.max_slices:
        exact = load_sliced_golden()
        if exact is not None:
            out["rel_err_vs_oracle_full_sum"] = rel_error(main_amps[0], exact)
            out["max_err_over_rms_vs_oracle"] = max_err_over_rms(main_amps[0], exact)
    if not args.no_cpu_baseline:
        if args.workload == "large":
            out["cpu_baseline"], refs = cpu_baseline_large(w, flops_slice)
        else:
            out["cpu_baseline"], refs = cpu_baseline_sliced(w, flops_slice)
            worst = 0.0
            for idx, ref in refs.items():
                c.contract_range(idx, 1)
                worst = max(worst, rel_error(c.amps.cpu().numpy(), ref))
            out["rel_err_vs_oracle_slices"] = worst
    c.close()
    del c
    torch.cuda.empty_cache()
    if args.workload == "large" and not args.max_slices and not args.reuse:
        pairs = load_large_golden()
        if pairs:
            out["vs_oracle_pairs_jittered_twin"] = twin_pair_errors(w, args.precision, pairs)
    if args.extras and args.workload == "large" and args.precision == "c64" and not args.reuse \
            and not args.max_slices:
        out["split_precision"] = large_forms(args, main_amps, aps, load_large_golden(), batch)
        torch.cuda.empty_cache()
        if args.head_reuse:
            out["head_reuse"] = large_reuse(args, aps)
            torch.cuda.empty_cache()
        if mode == "branch":
            out["plain_path"] = large_plain_path(args, aps)
            torch.cuda.empty_cache()
        out["zigzag_tail"] = large_zigzag(args)
        torch.cuda.empty_cache()
        out["sliced_5x6_m14"] = sliced_extra(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
