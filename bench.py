"""Benchmark: top-k multidimensional motif search on one MI355X.

One step = index construction (window statistics, r estimate, MFMA projection
and packing) plus the full traversal (prefix sorts, enumeration, verification,
pool, stopping rule) over the resident synthetic series. Prints one JSON line.

The default workload is rwsin32_4m (D = 32, n = 4 194 304, w = 1000, d = 8,
k = 10): `value` is its time to solution with the BF16 projection, next to
the FP32 projection timed in the same process, the hash-flip rate and the
distance error against the FP64 oracle, and the oracle's own search on the
host cores.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload rwsin32_4m|rw8_1m|...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

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


def cpu_baseline(series, p, seed: int, r: float) -> dict:
    """The oracle's LSH search (O2, OpenMP build on every host core) on a
    bounded sample of the workload: the stretches of 3 w points around each
    planted window, joined in time order (every planted motif is in it, so
    the search stops on the rule as the device's does), with the device run's
    d, k, delta, K, L, seed and r."""
    import oracle
    w = p["w"]
    segs = sorted(q for m in series.motifs for q in (m.p1, m.p2))
    lo = [max(0, q - w) for q in segs]
    x = np.concatenate([series.x[:, a: min(series.n, a + 3 * w)] for a in lo], axis=1)
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or (os.cpu_count() or 1)
    t0 = time.perf_counter()
    res = oracle.lsh_pipeline(x, w, p["d"], p["k"], p["delta"], seed, mem_limit=p["mem_limit"],
                              elem_bytes=4 if series.dtype == "f32" else 8, r=r, omp=True)
    dt = time.perf_counter() - t0
    ns = x.shape[1] - w + 1
    return {"value": ns * series.D / dt, "unit": "subseq·dims/s", "cores": threads, "kind": "oracle",
            "sample": (f"the oracle's whole search (index + traversal, OpenMP over dimensions) on "
                       f"{x.shape[1]} points: the {3 * w}-point stretches around the {len(segs)} planted "
                       f"windows joined in time order, same d/k/delta/K/L/seed/r; took {dt:.1f} s, "
                       f"stop ({res['i_stop']},{res['J_stop']})"
                       f"{', exact fallback' if res.get('fallback') else ''}"),
            "seconds": dt, "stop": [res["i_stop"], res["J_stop"]]}


def flip_rate(plan, series, p, seed: int, r: float, cells: int = 4096) -> dict:
    """Hash symbols of sampled windows against the FP64 oracle's (Eq. drp):
    the fraction that differ, on runs of 16 consecutive windows at random
    places of every dimension."""
    import oracle
    rng = np.random.default_rng(0xF11B)
    w, D = p["w"], series.D
    ns = series.n - w + 1
    prm = plan.params()
    NF, K = prm["NF"], 8
    R, U = oracle.draw_projections(seed, D, w, 4 * NF)
    runs = max(1, cells // (16 * D))
    diff = total = 0
    for f in range(D):
        for a0 in rng.integers(0, ns - 16, runs):
            words = plan.hash_words(f, int(a0), 16)
            for q in range(16):
                by, _, _ = oracle.hash_one(series.x[f], w, int(a0) + q, R[f], U[f], r)
                for F in range(NF):
                    for pos in range(K // 2):
                        g = (int(words[F, q]) >> (24 - 8 * pos)) & 255
                        diff += g != int(by[4 * F + pos])
                        total += 1
    return {"rate": diff / total, "symbols": total}


def bench_batch(args, torch, mm, synth) -> int:
    """Many independent series through momenti_topk_batch, in waves of
    --wave series (each wave one call, --workers in flight); one step is the
    whole batch. With --tune the repetitions per launch come from the
    autotuner run on the batch's largest series; the first wave is also
    timed with one worker (the series one at a time)."""
    spec = dict(synth.BATCHES[args.workload])
    spec_r = spec.pop("r_scale", 1.0)
    ser = synth.batch_workload(synth.BATCH_SEED, **spec)
    jobs = [dict(series=torch.from_numpy(x.as_dtype()).to("cuda:0"), w=q["w"], d=q["d"], k=q["k"],
                 delta=q["delta"]) for x, q in ser]
    torch.cuda.synchronize()
    units = sum((q["n"] - q["w"] + 1) * q["D"] for _, q in ser)
    r_scale = args.r_scale if args.r_scale > 0 else spec_r
    kw = dict(mem_limit=8 << 30, seed=0x15A004, max_pairs=args.max_pairs, r_scale=r_scale)
    tuned = None
    if args.tune:
        big = max(range(len(ser)), key=lambda q: ser[q][1]["n"] * ser[q][1]["D"])
        xq, pq = ser[big]
        plan = mm.Plan(pq["n"], pq["D"], pq["w"], "f32", kw["mem_limit"], device_series=True,
                       seed=kw["seed"], max_pairs=kw["max_pairs"], r_scale=r_scale)
        plan.hash(jobs[big]["series"])
        best, bms = plan.tune(pq["d"], pq["k"], pq["delta"], cands=(2, 4, 8, 16, 32))
        plan.close()
        tuned = {"series": big, "n": pq["n"], "D": pq["D"], "batch_reps": best, "search_ms": bms}
        kw["batch_reps"] = best
        log(f"[bench] tuned on series {big} (n={pq['n']}, D={pq['D']}): {best} repetitions per launch")
    wave = max(1, args.wave)

    def run(workers, count=None):
        res, rc = [], 0
        last = len(jobs) if count is None else count
        for q0 in range(0, last, wave):
            r, c = mm.topk_batch(jobs[q0:min(last, q0 + wave)], workers=workers, **kw)
            res += r
            rc = rc or c
            log(f"[bench]   series {q0}..{min(last, q0 + wave) - 1} done")
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
    n0 = min(wave, len(jobs))
    t1 = time.perf_counter()
    run(args.workers, n0)
    msw = (time.perf_counter() - t1) * 1000.0
    t1 = time.perf_counter()
    res1, _ = run(1, n0)
    ms1 = (time.perf_counter() - t1) * 1000.0
    same = all([(m["a"], m["b"]) for m in a[0]] == [(m["a"], m["b"]) for m in b[0]] and a[2] == b[2]
               for a, b in zip(res[:n0], res1))
    st = [r[2] for r in res]
    planted = sum(len({(m.p1, m.p2) for m in x.motifs} & {(g["a"], g["b"]) for g in r[0]})
                  for (x, _), r in zip(ser, res))
    out = {
        "metric": METRIC, "value": units / (ms / 1000.0), "unit": "subseq·dims/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "series": len(jobs), "workers": args.workers, "wave": wave,
                   "max_pairs": args.max_pairs, "r_scale": r_scale,
                   **{k: v for k, v in spec.items() if k != "count"}},
        "series_per_s": len(jobs) / (ms / 1000.0),
        "first_wave": {"series": n0, "ms_workers": msw, "ms_one_worker": ms1, "answers_identical": same},
        "tuned": tuned,
        "status_counts": {str(v): st.count(v) for v in sorted(set(st))},
        "planted_recovered": planted, "planted_total": sum(len(x.motifs) for x, _ in ser),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


def run_leg(args, torch, mm, s, p, x, proj: str, seed: int, r_scale: float, steps: int, warmup: int,
            profile: bool):
    """Time `steps` whole searches (index + traversal) of one projection
    precision on a resident series; one more untimed step, profiled per kernel."""
    plan = mm.Plan(s.n, s.D, p["w"], "f32" if s.dtype == "f32" else "f64", p["mem_limit"],
                   device_series=True, seed=seed, proj=proj, profile=2 if profile else 0,
                   r_scale=r_scale, max_pairs=args.max_pairs)

    def step():
        plan.hash(x)
        return plan.search(p["d"], p["k"], p["delta"])

    for wi in range(warmup):
        got, rep, rc = step()
        log(f"[bench] {proj} warmup {wi}: tts {rep['t_hash_ms'] + rep['t_search_ms']:.1f} ms, "
            f"stop ({rep['i_stop']},{rep['j_stop']})")
    plan.profile(clear=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for si in range(steps):
        got, rep, rc = step()
        reps.append(rep)
        log(f"[bench] {proj} step {si}: hash {rep['t_hash_ms']:.2f} ms, search {rep['t_search_ms']:.1f} ms, "
            f"stop ({rep['i_stop']},{rep['j_stop']}), cand {rep['n_cand']}")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    prof_t, prof = {}, {}
    if profile:
        # the timed steps carry HIP events around the pair enumeration only
        # (the dominant kernel); one more step, untimed, times every kernel
        prof_t = plan.profile(clear=True)
        plan.set_profile(1)
        step()
        prof = plan.profile(clear=True)
    return dict(plan=plan, ms=ms, got=got, rep=rep, rc=rc, reps=reps, prof_t=prof_t, prof=prof)


def roofline(leg, proj: str, workload: str, steps: int) -> dict:
    prof, prof_t = leg["prof"], leg["prof_t"]
    ranked = sorted(((v["ms"], k) for k, v in prof.items() if v["launches"]), reverse=True)
    dom = ranked[0][1]
    # the dominant kernel's figures over the timed region when it was timed
    # there (the enumeration), else from the extra step
    live = dom in prof_t and prof_t[dom]["launches"] > 0
    v = prof_t[dom] if live else prof[dom]
    nsteps = steps if live else 1
    sec = v["ms"] / 1000.0
    if dom == "proj":
        bound, unit, peak = "mfma", "TFLOP/s", PEAKS["mfma_TFLOPs"][proj]
        ach = v["flops"] / sec / 1e12
    else:
        # the enumeration is bound by its fingerprint-row gathers (its bit-sliced
        # screen uses a small share of the 32-bit VALU peak): graded on HBM with
        # its algorithmic bytes, the ALU view reported beside it
        bound, unit, peak = "hbm", "GB/s", PEAKS["hbm_GBps"]
        ach = v["bytes"] / sec / 1e9
    extra = {}
    if dom == "enum":
        alu = v["flops"] / sec / 1e12
        extra = {"alu_view": {"achieved": alu, "peak": PEAKS["alu_TOPs"], "unit": "TOP/s",
                              "frac": alu / PEAKS["alu_TOPs"]}}
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "traffic": measured_traffic(dom, workload), "kernel": dom, **extra,
            "avg_launch_ms": v["ms"] / v["launches"], "launches_per_step": v["launches"] / nsteps,
            "timed_region": live,
            "algorithmic_bytes_per_launch": v["bytes"] / v["launches"],
            "algorithmic_ops_per_launch": v["flops"] / v["launches"]}


def proj_mfma(leg, proj: str) -> dict | None:
    pj = leg["prof"].get("proj")
    if not pj or not pj["launches"]:
        return None
    ach = pj["flops"] / (pj["ms"] / 1000.0) / 1e12
    return {"achieved_TFLOPs": ach, "peak": PEAKS["mfma_TFLOPs"][proj],
            "frac": ach / PEAKS["mfma_TFLOPs"][proj], "ms": pj["ms"]}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rwsin32_4m")
    ap.add_argument("--proj", default=None, help="projection precision (default: the workload's)")
    ap.add_argument("--compare-steps", type=int, default=3,
                    help="timed steps of the comparison precision (FP32 against BF16)")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-checks", action="store_true", help="skip the flip-rate and distance checks")
    ap.add_argument("--r-scale", type=float, default=0.0,
                    help="r as a multiple of the section 6.1 estimate (default: the workload's)")
    ap.add_argument("--max-pairs", type=float, default=5e13,
                    help="work budget in colliding pairs per round group (0: none)")
    ap.add_argument("--workers", type=int, default=4, help="series in flight (batch workloads)")
    ap.add_argument("--wave", type=int, default=64, help="series per batch call (batch workloads)")
    ap.add_argument("--tune", action="store_true",
                    help="batch workloads: repetitions per launch from the autotuner")
    ap.add_argument("--n", type=float, default=0,
                    help="series length instead of the workload's (e.g. the scal5 sweep 1e4 .. 1e8)")
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
    t_gen = time.perf_counter()
    s, p = synth.workload(args.workload, n=int(args.n) if args.n else None)
    proj = args.proj or p["proj"]
    cmp_proj = None if (args.no_compare or args.proj) else p.get("compare_proj")
    seed = synth.LSH_SEED[args.workload]
    log(f"[bench] workload {args.workload}: D={s.D} n={s.n} w={p['w']} d={p['d']} k={p['k']} "
        f"delta={p['delta']} proj={proj}{' vs ' + cmp_proj if cmp_proj else ''} "
        f"(series drawn in {time.perf_counter() - t_gen:.1f} s)")
    x = torch.from_numpy(s.as_dtype()).to("cuda:0")
    torch.cuda.synchronize()
    r_scale = args.r_scale if args.r_scale > 0 else p.get("r_scale", 1.0)
    prof_on = not args.no_profile
    lead = run_leg(args, torch, mm, s, p, x, proj, seed, r_scale, args.steps, args.warmup, prof_on)
    ns = s.n - p["w"] + 1
    units = ns * s.D
    prm = lead["plan"].params()
    got, rep, rc = lead["got"], lead["rep"], lead["rc"]
    planted = {(m.p1, m.p2) for m in s.motifs}
    found = [(m["a"], m["b"]) for m in got]
    hash_ms = sum(r["t_hash_ms"] for r in lead["reps"]) / len(lead["reps"])
    out = {
        "metric": METRIC, "value": lead["ms"] / 1000.0, "unit": "s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": lead["ms"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": proj, "data": "synthetic",
        "config": {"workload": args.workload, "D": s.D, "n": s.n, "w": p["w"], "d": p["d"],
                   "k": p["k"], "delta": p["delta"], "mem_limit": p["mem_limit"],
                   "series": s.dtype, "proj": proj, "K": 8, "L_used": prm["L"], "r_scale": r_scale},
        "tts_s": {proj: lead["ms"] / 1000.0},
        "hash_subseq_dims_per_s": {proj: units / (hash_ms / 1000.0)},
        "hash_ms": {proj: hash_ms},
        "search_subseq_dims_per_s": {proj: units / (lead["ms"] / 1000.0)},
        "stop": {proj: [rep["i_stop"], rep["j_stop"]]}, "r": prm["r"], "status": {proj: rc},
        "n_cand": rep["n_cand"], "n_collisions": rep["n_collisions"],
        "planted_recovered": {proj: f"{len(planted & set(found))}/{len(planted)}"},
        "top3": [[m["a"], m["b"], m["dist_d"], m["dist_max"]] for m in got[:3]],
    }
    if prof_on and lead["prof"]:
        out["kernel_ms_per_step"] = {proj: {k: round(v["ms"], 3) for k, v in lead["prof"].items() if v["launches"]}}
        out["roofline"] = roofline(lead, proj, args.workload, args.steps)
        out["proj_mfma"] = {proj: proj_mfma(lead, proj)}
    checks = not args.no_checks
    if checks:
        import oracle
        # r of the oracle (section 6.1 estimate, same draws) equals the device's
        r_orc = oracle.estimate_r(s.x, p["w"], seed) * r_scale
        out["r_oracle_equal"] = r_orc == prm["r"]
        out["flip_rate_vs_fp64"] = {proj: flip_rate(lead["plan"], s, p, seed, prm["r"])}
        err = 0.0
        for m in got:
            dd, dm, dims, _ = oracle.distd(s.x, p["w"], m["a"], m["b"], p["d"])
            err = max(err, abs(m["dist_d"] - dd) / dd, abs(m["dist_max"] - dm) / dm)
        out["dist_rel_err_vs_fp64"] = {proj: err}
        out["planted_dist"] = [[m.p1, m.p2, *oracle.distd(s.x, p["w"], m.p1, m.p2, p["d"])[:2]]
                               for m in s.motifs[:10]]
    lead["plan"].close()
    if cmp_proj:
        leg = run_leg(args, torch, mm, s, p, x, cmp_proj, seed, r_scale, args.compare_steps, 1, prof_on)
        hms = sum(r["t_hash_ms"] for r in leg["reps"]) / len(leg["reps"])
        out["tts_s"][cmp_proj] = leg["ms"] / 1000.0
        out["hash_subseq_dims_per_s"][cmp_proj] = units / (hms / 1000.0)
        out["hash_ms"][cmp_proj] = hms
        out["search_subseq_dims_per_s"][cmp_proj] = units / (leg["ms"] / 1000.0)
        out["stop"][cmp_proj] = [leg["rep"]["i_stop"], leg["rep"]["j_stop"]]
        out["status"][cmp_proj] = leg["rc"]
        found_c = [(m["a"], m["b"]) for m in leg["got"]]
        out["planted_recovered"][cmp_proj] = f"{len(planted & set(found_c))}/{len(planted)}"
        out[f"tts_ratio_{cmp_proj}_over_{proj}"] = leg["ms"] / lead["ms"]
        out[f"topk_{proj}_equals_{cmp_proj}"] = found == found_c
        if prof_on and leg["prof"]:
            out["kernel_ms_per_step"][cmp_proj] = {k: round(v["ms"], 3) for k, v in leg["prof"].items()
                                                   if v["launches"]}
            out["proj_mfma"][cmp_proj] = proj_mfma(leg, cmp_proj)
        if checks:
            out["flip_rate_vs_fp64"][cmp_proj] = flip_rate(leg["plan"], s, p, seed, prm["r"])
        leg["plan"].close()
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline: the oracle's search on the stretches around the planted windows")
        import oracle
        r_cpu = oracle.estimate_r(s.x, p["w"], seed) * r_scale
        out["cpu_baseline"] = cpu_baseline(s, p, seed, r_cpu)
        out["cpu_baseline"]["gpu_same_unit"] = units / (lead["ms"] / 1000.0)
        # the metric's own unit: the time the oracle would take for the whole
        # workload at the rate it reached on the sample (an estimate, linear
        # in the number of windows)
        out["cpu_baseline"]["tts_s_scaled"] = {
            "value": units / out["cpu_baseline"]["value"], "unit": "s",
            "how": "the whole workload's subseq·dims divided by the sample's rate"}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
