"""Benchmark: top-k multidimensional motif search on one MI355X.

One step = index construction (window statistics, r estimate, MFMA projection
and packing) plus the full traversal (prefix sorts, enumeration, verification,
pool, stopping rule) over the resident synthetic series. Prints one JSON line.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload rw8_1m]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBps": 8000.0,
    "mfma_TFLOPs": {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp8": 5000.0},
    # 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one op per
    # lane per clock (the fp32 figure, 157.3 TFLOP/s, counts an FMA as two
    # and two ops per lane per clock)
    "alu_TOPs": 256 * 4 * 16 * 2.4e9 / 1e12,
}
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = {"enum": "paper_2502_14446_amd/csrc/k_search.hip",
                  "proj": "paper_2502_14446_amd/csrc/k_hash.hip"}
METRIC = "top-k motif time-to-solution (s) + hashed subseq·dims/s, BF16 vs FP32 path"
HBM_KERNELS = ("sort_scatter", "sort_hist", "sort_scan", "enum", "verify", "stats")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def code_sha(kernel: str) -> str | None:
    """SHA-256 of the kernel's source with comments removed and whitespace
    collapsed: an edit to comments alone leaves it (and the compiled code)
    unchanged."""
    src = KERNEL_SOURCES.get(kernel)
    if not src:
        return None
    with open(os.path.join(ROOT, src), encoding="utf-8") as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()


def measured_traffic(kernel: str, workload: str) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or None when
    there is none or the kernel's code changed since it was taken."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+): (\S+)$", line.strip())
            if m:
                vals[m.group(1)] = m.group(2)
    if vals.get("code_sha256") != code_sha(kernel):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def calibrate_copy(nbytes: int, reps: int) -> int:
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)
    return 0


def cpu_baseline(series, p, seed: int, n_cpu: int, r_scale: float) -> dict:
    import oracle
    x = series.x[:, :n_cpu]
    t0 = time.perf_counter()
    res = oracle.lsh_pipeline(x, p["w"], p["d"], p["k"], p["delta"], seed,
                              mem_limit=p["mem_limit"], elem_bytes=4, r_scale=r_scale)
    dt = time.perf_counter() - t0
    ns = n_cpu - p["w"] + 1
    return {"value": ns * p["D"] / dt, "unit": "subseq·dims/s", "cores": 1, "kind": "oracle",
            "sample": (f"first {n_cpu} points of the same series, same d/k/delta/K/L/seed/r; the "
                       f"oracle's complete search (hash + traversal"
                       f"{' + exact fallback' if res.get('fallback') else ''}) took {dt:.2f} s, "
                       f"stop ({res['i_stop']},{res['J_stop']}), single-threaded C")}


def bench_batch(args, torch, mm, synth) -> int:
    """Many independent series through momenti_topk_batch: one step is the
    whole batch; also timed with one worker for comparison."""
    spec = dict(synth.BATCHES[args.workload])
    spec_r = spec.pop("r_scale", 1.0)
    ser = synth.batch_workload(synth.BATCH_SEED, **spec)
    jobs = [dict(series=torch.from_numpy(x.as_dtype()).to("cuda:0"), w=q["w"], d=q["d"], k=q["k"],
                 delta=q["delta"]) for x, q in ser]
    torch.cuda.synchronize()
    units = sum((q["n"] - q["w"] + 1) * q["D"] for _, q in ser)
    r_scale = args.r_scale if args.r_scale > 0 else spec_r
    kw = dict(mem_limit=8 << 30, seed=0x15A004, max_pairs=args.max_pairs, r_scale=r_scale)

    def run(workers):
        res, rc = mm.topk_batch(jobs, workers=workers, **kw)
        return res, rc

    for wi in range(args.warmup):
        run(args.workers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for si in range(args.steps):
        res, rc = run(args.workers)
        log(f"[bench] batch step {si}: rc {rc}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    t1 = time.perf_counter()
    run(1)
    ms1 = (time.perf_counter() - t1) * 1000.0
    st = [r[2] for r in res]
    planted = sum(len({(m.p1, m.p2) for m in x.motifs} & {(g["a"], g["b"]) for g in r[0]})
                  for (x, _), r in zip(ser, res))
    out = {
        "metric": METRIC, "value": units / (ms / 1000.0), "unit": "subseq·dims/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "series": len(jobs), "workers": args.workers,
                   "max_pairs": args.max_pairs, "r_scale": r_scale,
                   **{k: v for k, v in spec.items() if k != "count"}},
        "series_per_s": len(jobs) / (ms / 1000.0), "ms_one_worker": ms1,
        "status_counts": {str(v): st.count(v) for v in sorted(set(st))},
        "planted_recovered": planted, "planted_total": sum(len(x.motifs) for x, _ in ser),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rw8_1m")
    ap.add_argument("--proj", default=None, help="projection precision (default: the workload's)")
    ap.add_argument("--cpu-n", type=int, default=2000,
                    help="points of the series the CPU oracle is timed on (about 25 s on one core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--r-scale", type=float, default=0.0,
                    help="r as a multiple of the section 6.1 estimate (default: the workload's)")
    ap.add_argument("--max-pairs", type=float, default=5e13,
                    help="work budget in colliding pairs per round group (0: none)")
    ap.add_argument("--workers", type=int, default=4, help="series in flight (batch workloads)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the method has no multi-GPU path here); "
              f"got --gpus {args.gpus}", file=sys.stderr)
        return 2
    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy, 4)

    import torch
    from paper_2502_14446_amd import momenti as mm
    from paper_2502_14446_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload in synth.BATCHES:
        return bench_batch(args, torch, mm, synth)
    s, p = synth.workload(args.workload)
    proj = args.proj or p["proj"]
    seed = synth.LSH_SEED[args.workload]
    log(f"[bench] workload {args.workload}: D={s.D} n={s.n} w={p['w']} d={p['d']} k={p['k']} "
        f"delta={p['delta']} proj={proj}")
    x = torch.from_numpy(s.as_dtype()).to("cuda:0")
    torch.cuda.synchronize()
    r_scale = args.r_scale if args.r_scale > 0 else p.get("r_scale", 1.0)
    plan = mm.Plan(s.n, s.D, p["w"], "f32" if s.dtype == "f32" else "f64", p["mem_limit"],
                   device_series=True, seed=seed, proj=proj, profile=0 if args.no_profile else 2,
                   r_scale=r_scale, max_pairs=args.max_pairs)

    def step():
        plan.hash(x)
        return plan.search(p["d"], p["k"], p["delta"])

    for wi in range(args.warmup):
        got, rep, rc = step()
        log(f"[bench] warmup {wi}: tts {rep['t_hash_ms'] + rep['t_search_ms']:.1f} ms, "
            f"stop ({rep['i_stop']},{rep['j_stop']})")
    plan.profile(clear=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for si in range(args.steps):
        got, rep, rc = step()
        reps.append(rep)
        log(f"[bench] step {si}: hash {rep['t_hash_ms']:.2f} ms, search {rep['t_search_ms']:.1f} ms, "
            f"stop ({rep['i_stop']},{rep['j_stop']}), cand {rep['n_cand']}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    ns = s.n - p["w"] + 1
    units = ns * s.D
    prm = plan.params()
    prof_t, prof = {}, {}
    if not args.no_profile:
        # the timed steps carry HIP events around the pair enumeration only
        # (the dominant kernel); one more step, untimed, times every kernel
        prof_t = plan.profile(clear=True)
        plan.set_profile(1)
        step()
        prof = plan.profile(clear=True)
    plan.close()

    planted = {(m.p1, m.p2) for m in s.motifs}
    found = {(m["a"], m["b"]) for m in got}
    out = {
        "metric": METRIC, "value": units / (ms / 1000.0), "unit": "subseq·dims/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": proj, "data": "synthetic",
        "config": {"workload": args.workload, "D": s.D, "n": s.n, "w": p["w"], "d": p["d"],
                   "k": p["k"], "delta": p["delta"], "mem_limit": p["mem_limit"],
                   "series": s.dtype, "proj": proj, "K": 8, "L_used": prm["L"], "r_scale": r_scale},
        "tts_s": ms / 1000.0,
        "hash_subseq_dims_per_s": units / (sum(r["t_hash_ms"] for r in reps) / len(reps) / 1000.0),
        "hash_ms": sum(r["t_hash_ms"] for r in reps) / len(reps),
        "stop": [rep["i_stop"], rep["j_stop"]], "r": prm["r"], "status": rc,
        "n_cand": rep["n_cand"], "n_collisions": rep["n_collisions"],
        "planted_recovered": f"{len(planted & found)}/{len(planted)}",
    }
    if prof:
        ranked = sorted(((v["ms"], k) for k, v in prof.items() if v["launches"]), reverse=True)
        out["kernel_ms_per_step"] = {k: round(v["ms"], 3) for k, v in prof.items() if v["launches"]}
        dom = ranked[0][1]
        # the dominant kernel's figures over the timed region when it was timed
        # there (the enumeration), else from the extra step
        live = dom in prof_t and prof_t[dom]["launches"] > 0
        v = prof_t[dom] if live else prof[dom]
        nsteps = args.steps if live else 1
        avg_ms = v["ms"] / v["launches"]
        sec = v["ms"] / 1000.0
        if dom == "proj":
            bound, unit, peak = "mfma", "TFLOP/s", PEAKS["mfma_TFLOPs"][proj]
            ach = v["flops"] / sec / 1e12
        elif dom == "enum":
            # the pair screen is 32-bit integer VALU work
            bound, unit, peak = "alu", "TOP/s", PEAKS["alu_TOPs"]
            ach = v["flops"] / sec / 1e12
        else:
            bound, unit, peak = "hbm", "GB/s", PEAKS["hbm_GBps"]
            ach = v["bytes"] / sec / 1e9
        out["roofline"] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                           "traffic": measured_traffic(dom, args.workload), "kernel": dom,
                           "avg_launch_ms": avg_ms, "launches_per_step": v["launches"] / nsteps,
                           "timed_region": live,
                           "algorithmic_bytes_per_launch": v["bytes"] / v["launches"],
                           "algorithmic_ops_per_launch": v["flops"] / v["launches"]}
        pj = prof.get("proj")
        if pj and pj["launches"]:
            ach = pj["flops"] / (pj["ms"] / 1000.0) / 1e12
            out["proj_mfma"] = {"achieved_TFLOPs": ach, "peak": PEAKS["mfma_TFLOPs"][proj],
                                "frac": ach / PEAKS["mfma_TFLOPs"][proj]}
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on the first {args.cpu_n} points")
        out["cpu_baseline"] = cpu_baseline(s, p, seed, args.cpu_n, r_scale)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
