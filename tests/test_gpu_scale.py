"""Parity of the HIP path with the oracle on the code paths that full-size
workloads take and small cases do not:

* segments longer than several sort tiles (cross-tile scan and scatter),
  with a ragged last tile;
* D = 128 (32-word fingerprint rows kept partly in LDS / memory, the verifier's
  dimensions 64..127);
* BF16 / FP8 projections whose rows take several LDS chunks (w = 300, 333, 1000);
* a pool of verified pairs too small for TOP (eviction, restart with a larger pool);
* searches under a memory cap that splits a round group and enumerates one
  repetition in parts, and repeated searches on one plan within the cap;
* the batch entry point against the oracle;
* the benchmark's workloads at full size: rw8_1m against its exact top-10,
  rwsin32_4m (BF16 and FP32) against the oracle's distances, hash bands and
  planted motifs.

Tolerances as in test_gpu_parity.py: candidates, TOP after every step, the stop
step and motif indices identical; distances within 1e-9 relative.
"""
import math

import numpy as np
import pytest

from paper_2502_14446_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_14446_amd import momenti as mm  # noqa: E402
from test_gpu_parity import (_band, _check_symbols, _lowp_band, _oracle_sets, _oracle_symbols,  # noqa: E402
                             _plan, _unpack)


def _mem_limit(n, D, w, L, elem, slack):
    """mem_limit that leaves `slack` bytes over the L-repetition index and the
    fixed reserve (the formula of momenti_prepare)."""
    ns = n - w + 1
    m = math.isqrt(L - 1) + 1 if L > 1 else 1
    nl, nr = -(-L // m), min(L, m)
    return n * D * elem + 48 * ns * D + (64 << 20) + 4 * ns * D * (nl + nr) + slack


def _compare_steps(ref, tr, K, Lu):
    last = (K - ref["i_stop"]) * Lu + ref["J_stop"] - 1 if ref["i_stop"] else K * Lu - 1
    osets = _oracle_sets(ref["cand"])
    gsets = _oracle_sets(tr["cand"])
    for step in range(last + 1):
        want = osets.get(step, set())
        if step >= Lu:                           # round i < K: pairs seen at prefix i+1 are skipped
            want = want - osets.get(step - Lu, set())
        assert gsets.get(step, set()) == want, f"step {step}"
        assert tr["top_size"][step] == ref["top_size"][step], f"step {step}"
        n = ref["top_size"][step]
        assert np.array_equal(tr["top_pairs"][step, :n], ref["top_pairs"][step, :n]), f"step {step}"


def _compare_motifs(got, want):
    assert [(m["a"], m["b"]) for m in got] == [(m["a"], m["b"]) for m in want]
    for g, o in zip(got, want):
        assert g["dist_d"] == pytest.approx(o["dist_d"], rel=1e-9)
        assert g["dist_max"] == pytest.approx(o["dist_max"], rel=1e-9)
        assert g["dims"] == o["dims"]


def _traverse(orc, s, w, seed, K, L, k, d, delta, rule, mem_limit=1 << 30, inject=True,
              oracle_fallback=True, trace_cap=4_000_000, **kw):
    """Search on the device (FP64 hash, or the oracle's index injected) with a
    trace, and the oracle's search over the same index."""
    plan, _ = _plan(s, dict(w=w, mem_limit=mem_limit), "f64", seed, K=K, L=L, stop=rule, **kw)
    prm = plan.params()
    Lu, r = prm["L"], prm["r"]
    assert r == orc.estimate_r(s.x, w, seed) * kw.get("r_scale", 1.0)
    R, U = orc.draw_projections(seed, s.D, w, 4 * prm["NF"])
    words = orc.pack(orc.hash_all(s.x, w, R, U, r), prm["NF"], K)
    if inject:
        plan.set_hashes(words)
    else:                                        # the device's own FP64 index must be the oracle's
        assert np.array_equal(plan.hashes(), words)
    plan.set_trace(trace_cap, k)
    got, rep, rc = plan.search(d, k, delta)
    tr = plan.trace()
    plan.close()
    code = {"tensor": orc.STOP_TENSOR, "lemma52": orc.STOP_LEMMA52, "rigorous": orc.STOP_RIGOROUS}[rule]
    ref = orc.lsh_search(s.x, w, d, k, delta, words, K, Lu, r, rule=code, trace=True, cand_cap=trace_cap,
                         fallback=oracle_fallback)
    assert (rep["i_stop"], rep["j_stop"]) == (ref["i_stop"], ref["J_stop"])
    _compare_steps(ref, tr, K, Lu)
    return got, rep, rc, ref


# --------------------------------------------------------------------------- sort tiles
def test_traversal_segments_span_several_sort_tiles(orc):
    # n_s = 13 951 windows: three full 4096-element sort tiles and a ragged
    # fourth in every segment; K = 4 and a vanishing delta traverse every
    # round down to 1 (360 000 candidates), the final answer is the exact one
    s = synth.make_series(91, 4, 14000, 50, 2, 2, noise=0.05, dtype="f64")
    ns = s.n - 50 + 1
    assert ns > 3 * 4096 and ns % 4096 != 0
    got, rep, rc, ref = _traverse(orc, s, 50, 13, 4, 6, 2, 2, 1e-300, "lemma52", oracle_fallback=False)
    assert rc == mm.OK_FALLBACK and ref["i_stop"] == 0 and len(ref["cand"]) > 100_000
    _compare_motifs(got, orc.topk_exact_sweep(s.x, 50, 2, 2))


# --------------------------------------------------------------------------- D = 128
def test_traversal_and_answer_with_128_dimensions(orc):
    # D = 128, d = 16: fingerprint rows of 32 words (8 kept in registers, the
    # rest read back), and the verifier's dimensions 64..127; the device hashes
    # the series itself (FP64, equal to the oracle's index) and stops where
    # the oracle stops, after 170 000 candidates in round 1
    s = synth.make_series(92, 128, 1500, 30, 2, 20, noise=0.02, dtype="f64")
    got, rep, rc, ref = _traverse(orc, s, 30, 14, 8, 12, 2, 16, 0.1, "lemma52", inject=False, r_scale=8.0)
    assert rc == mm.OK and ref["i_stop"] >= 1
    _compare_motifs(got, ref["motifs"])
    assert any(f >= 64 for m in got for f in m["dims"])   # chosen dimensions past the first 64


# --------------------------------------------------------------------------- low precision
@pytest.mark.parametrize("proj", ["bf16", "fp8"])
@pytest.mark.parametrize("w,D,n", [(300, 3, 2400), (333, 3, 2400), (1000, 2, 5000)])
def test_lowp_hash_with_several_lds_chunks(orc, proj, w, D, n):
    # projection rows staged through LDS in chunks of 64 steps of t: 5, 6 and
    # 16 chunks (w = 333 is not a multiple of the chunk)
    s = synth.make_series(100 + w, D, n, w, 1, min(2, D), dtype="f32")
    p = dict(w=w, mem_limit=1 << 30)
    seed = 78
    plan, _ = _plan(s, p, proj, seed)
    prm = plan.params()
    R, U = orc.draw_projections(seed, s.D, w, 4 * prm["NF"])
    r = prm["r"]
    assert r == orc.estimate_r(s.x, w, seed)
    by, pre, sab, amb = [], [], [], []
    for f in range(s.D):
        b_, p_, s_, a_ = orc.hash_dim_lowp(s.x[f], w, R[f], U[f], r, proj)
        by.append(b_); pre.append(p_); sab.append(s_); amb.append(a_)
    by, pre, sab, amb = map(np.array, (by, pre, sab, amb))
    gsym = _unpack(plan.hashes(), 8)
    bad_out, bad_in, near, diff = _check_symbols(gsym, by, pre, _lowp_band(w, pre, sab, amb, r, proj), 8)
    print(f"{proj} w={w}: symbols={by.size} band={near} differing={diff}")
    assert bad_out == 0 and bad_in == 0
    ref, _, _ = _oracle_symbols(orc, s.x, w, R, U, r)
    flips = float(np.mean(gsym != ref))
    predicted = float(np.mean(by != ref))
    print(f"{proj} w={w}: flip rate vs FP64 = {flips:.4f} (emulation {predicted:.4f})")
    assert abs(flips - predicted) <= near / ref.size
    plan.close()


@pytest.mark.parametrize("proj,w", [("bf16", 7616), ("fp8", 8192)])
def test_lowp_hash_at_the_longest_windows(orc, proj, w):
    # the longest windows whose work-group tile fits the CU's LDS: BF16 up to
    # w = 7616 (163 456 of 163 840 bytes), FP8 up to the ABI's 8192; one
    # window more is refused when the plan is made
    s = synth.make_series(300 + w % 97, 1, w + 700, w, 0, 0, dtype="f32")
    p = dict(w=w, mem_limit=1 << 30)
    seed = 79
    plan, _ = _plan(s, p, proj, seed)
    prm = plan.params()
    R, U = orc.draw_projections(seed, s.D, w, 4 * prm["NF"])
    r = prm["r"]
    assert r == orc.estimate_r(s.x, w, seed)
    by, pre, sab, amb = orc.hash_dim_lowp(s.x[0], w, R[0], U[0], r, proj)
    gsym = _unpack(plan.hashes(), 8)
    bad_out, bad_in, near, diff = _check_symbols(gsym, by[None], pre[None], _lowp_band(w, pre, sab, amb, r, proj)[None], 8)
    print(f"{proj} w={w}: symbols={by.size} band={near} differing={diff}")
    assert bad_out == 0 and bad_in == 0
    plan.close()
    if proj == "bf16":
        longer = synth.make_series(301, 1, w + 64 + 700, w + 64, 0, 0, dtype="f32")
        with pytest.raises(mm.MomentiError) as e:
            _plan(longer, dict(w=w + 64, mem_limit=1 << 30), proj, seed)
        assert e.value.code == mm.E_ARG and "at most 7616" in str(e.value)


@pytest.mark.parametrize("proj", ["f64", "f32"])
def test_longest_window_end_to_end(orc, proj):
    # w = 8192, the longest window the ABI takes (statistics, the r sample and
    # the projection tile at their largest): r equal to the oracle's, symbols
    # within their bands (at this w the FP32 bound, linear in w, is wider than
    # half a symbol, so for FP32 that part checks little: 15 of 162 036
    # symbols differ from the FP64 hash), and with the FP64 projection (bit-exact symbols) the
    # search's answer and stop step equal to the oracle's (Algorithm 1) and
    # its motif to the exact one; non-trivial pairs lie more than w / 2 apart,
    # so the 4 501 windows hold one motif and the search ends in the exact
    # answer (the diagonal sweep, n_s > 4096)
    w, k = 8192, 1
    s = synth.make_series(0x8192, 1, w + 4500, w, 0, 0, dtype=proj)
    p = dict(w=w, mem_limit=1 << 30)
    seed = 81
    plan, _ = _plan(s, p, proj, seed, L=20)
    prm = plan.params()
    assert prm["L"] == 20
    r = orc.estimate_r(s.x, w, seed)
    assert prm["r"] == r
    R, U = orc.draw_projections(seed, s.D, w, 4 * prm["NF"])
    ref, pre, sab = _oracle_symbols(orc, s.x, w, R, U, r)
    gsym = _unpack(plan.hashes(), 8)
    bad_out, bad_in, near, diff = _check_symbols(gsym, ref, pre, _band(proj, w, pre, sab, r), 8)
    print(f"{proj} w={w}: symbols={ref.size} band={near} differing={diff}")
    assert bad_out == 0 and bad_in == 0
    got, rep, rc = plan.search(1, k, 0.1)
    plan.close()
    ex = orc.topk_exact(s.x, w, 1, k)
    assert len(ex) == k and len(got) == k
    if proj == "f64":
        assert diff == 0
        res = orc.lsh_pipeline(s.x, w, 1, k, 0.1, seed, L_max=20, mem_limit=1 << 30)
        assert (rep["i_stop"], rep["j_stop"]) == (res["i_stop"], res["J_stop"])
        assert [(m["a"], m["b"]) for m in got] == [(m["a"], m["b"]) for m in res["motifs"]]
        if res["i_stop"] == 0:
            assert [(m["a"], m["b"]) for m in got] == [(m["a"], m["b"]) for m in ex]
    for m in got:
        dd, dm, dims, _ = orc.distd(s.x, w, m["a"], m["b"], 1)
        assert m["dist_d"] == pytest.approx(dd, rel=1e-9) and tuple(m["dims"]) == dims
    assert got[0]["dist_d"] >= ex[0]["dist_d"] * (1 - 1e-9)


# --------------------------------------------------------------------------- pool
def test_pool_too_small_for_top_restarts_to_the_oracle_answer(orc):
    # a pool of k = 3 verified pairs: the best pairs are neighbours of one
    # planted motif along its diagonal, so TOP over the pool has fewer than k
    # picks while pairs were dropped; the search restarts with larger pools
    # and still takes every step the oracle (unbounded set of pairs) takes
    s = synth.make_series(21, 5, 2500, 40, 3, 2, dtype="f64")
    got, rep, rc, ref = _traverse(orc, s, 40, 5, 8, 30, 3, 2, 0.05, "lemma52", pool_size=3)
    assert rep["pool_overflow"] >= 1
    _compare_motifs(got, ref["motifs"])


# --------------------------------------------------------------------------- memory cap
def _storm_series():
    # two noisy sinusoids of period 20: windows a whole number of periods apart
    # are close, so every round holds hundreds of thousands of candidates
    rng = np.random.default_rng(5)
    n, P = 3000, 20
    t = np.arange(n)
    x = np.stack([np.sin(2 * np.pi * t / P + f) + 0.1 * rng.standard_normal(n) for f in range(2)])
    return synth.Series(np.ascontiguousarray(x), 30, [], "f64")


def test_memory_cap_splits_groups_and_enumerates_steps_in_parts(orc):
    # 1 MiB over the fixed reserve: the first round group (rounds 4..1, one
    # sort) would store 1.7 M verified records, so it is split into single
    # rounds; a round-1 repetition has 640 000 candidates, more than the
    # candidate buffer that fits, so it is enumerated in parts. Every step
    # still matches the oracle, and the answer is the exact one.
    s = _storm_series()
    lim = _mem_limit(s.n, 2, 30, 2, 8, 1 << 20)
    got, rep, rc, ref = _traverse(orc, s, 30, 31, 4, 2, 3, 1, 1e-300, "lemma52", mem_limit=lim,
                                  r_scale=10.0, merge_pairs=1e12)
    assert rc == mm.OK_FALLBACK
    assert rep["group_splits"] >= 1 and rep["step_parts"] >= 2, rep
    assert rep["peak_bytes"] <= lim
    _compare_motifs(got, ref["motifs"])


def test_constant_series_under_a_small_cap(orc):
    # every window flat: all 690 000 pairs collide everywhere at distance 0;
    # the first step is enumerated in parts and the search stops there with
    # the exact answer (ties broken by (a, b))
    x = np.full((2, 1200), 2.5)
    s = synth.Series(x, 16, [], "f64")
    lim = _mem_limit(1200, 2, 16, 4, 8, 1 << 20)
    plan, _ = _plan(s, dict(w=16, mem_limit=lim), "f64", 3, K=4, L=4)
    got, rep, rc = plan.search(2, 3, 0.1)
    plan.close()
    ex = orc.topk_exact(x, 16, 2, 3)
    assert rc == mm.OK and rep["step_parts"] >= 2 and rep["peak_bytes"] <= lim
    assert [(m["a"], m["b"]) for m in got] == [(m["a"], m["b"]) for m in ex]
    assert all(m["dist_d"] == 0.0 for m in got)


def test_repeated_searches_stay_within_the_cap(orc):
    # searches with other d (other block sizes) on one plan: the blocks it
    # holds plus those it keeps for reuse never exceed mem_limit, and each
    # search answers as a fresh plan does
    s = synth.make_series(71, 6, 200_000, 50, 3, 3, noise=0.02, dtype="f32")
    lim = _mem_limit(s.n, 6, 50, 200, 4, 8 << 20)
    p = dict(w=50, mem_limit=lim)

    def key(res):
        got, rep, rc = res
        return (rc, [(m["a"], m["b"], m["dist_d"], m["dims"]) for m in got], rep["i_stop"], rep["j_stop"])

    plan, _ = _plan(s, p, "f32", 12)
    for d, k in ((3, 3), (2, 3), (4, 2), (3, 3)):
        res = plan.search(d, k, 0.05)
        assert res[1]["peak_bytes"] <= lim, (d, k, res[1]["peak_bytes"], lim)
        fresh, _ = _plan(s, p, "f32", 12)
        want = key(fresh.search(d, k, 0.05))
        fresh.close()
        assert key(res) == want, (d, k)
    plan.close()


# --------------------------------------------------------------------------- batch
def test_batch_matches_the_oracle(orc):
    # every job of a batch of uneven series (D, n, w, d and k all differ) gives
    # the oracle's answer and stop step: FP64 projection, close planted motifs
    # and r at 3 times the estimate, so that the searches stop on the rule
    spec = [(61, 3, 3000, 40, 2, 2), (62, 6, 5200, 60, 2, 2), (63, 4, 2600, 50, 1, 1),
            (64, 9, 4100, 32, 3, 2), (65, 5, 6400, 80, 2, 3), (66, 12, 3300, 45, 3, 2)]
    jobs, ser = [], []
    for seed, D, n, w, d, k in spec:
        s = synth.make_series(seed, D, n, w, k, d, noise=0.02, dtype="f32")
        ser.append(s)
        jobs.append(dict(series=torch.from_numpy(s.as_dtype()).to("cuda"), w=w, d=d, k=k, delta=0.1))
    res, rc = mm.topk_batch(jobs, mem_limit=1 << 30, workers=3, seed=77, proj="f64", r_scale=3.0)
    assert rc == mm.OK
    for s, j, (got, rep, st) in zip(ser, jobs, res):
        ref = orc.lsh_pipeline(s.x, j["w"], j["d"], j["k"], j["delta"], 77, mem_limit=1 << 30, elem_bytes=4,
                               r_scale=3.0)
        assert st == (mm.OK_FALLBACK if ref["fallback"] else mm.OK)
        assert (rep["i_stop"], rep["j_stop"]) == (ref["i_stop"], ref["J_stop"])
        _compare_motifs(got, ref["motifs"])


# --------------------------------------------------------------------------- exact answer at full size
def _collision_steps(orc, x, w, seed, r, L, K, a, b, d, stop):
    """Steps (i, J) up to `stop` at which windows a and b collide in at least d
    dimensions by the oracle's hash: `sure` where every symbol involved is
    outside the FP32 guard band (the device's FP32 symbols equal the oracle's
    there), `maybe` where some are inside it."""
    D = x.shape[0]
    m, nl, nr = orc.tensor_shape(L)
    R, U = orc.draw_projections(seed, D, w, 4 * (nl + nr))
    sym, amb = {}, {}
    for q in (a, b):
        for f in range(D):
            by, pre, sab = orc.hash_one(x[f], w, q, R[f], U[f], r)
            band = 2.0 * 2.0 ** -24 * ((w + 4) * sab / r + 3.0 * (np.abs(pre) + 1.0))
            frac = pre - np.floor(pre)
            sym[q, f] = by
            amb[q, f] = np.minimum(frac, 1.0 - frac) <= band
    sure, maybe = [], []
    i_stop, J_stop = stop
    for i in range(K, 0, -1):
        for J in range(1, L + 1):
            if i < i_stop or (i == i_stop and J > J_stop):
                return sure, maybe
            j = J - 1
            cols = [4 * (j // m) + q // 2 if q % 2 == 0 else 4 * (nl + j % m) + q // 2 for q in range(i)]
            w_sure = w_maybe = 0
            for f in range(D):
                eq = all(sym[a, f][c] == sym[b, f][c] for c in cols)
                fuzzy = any(amb[a, f][c] or amb[b, f][c] for c in cols)
                w_sure += eq and not fuzzy
                w_maybe += eq or fuzzy
            if w_sure >= d:
                sure.append((i, J))
            elif w_maybe >= d:
                maybe.append((i, J))
    return sure, maybe


def test_bench_workload_answer_against_the_exact_golden(orc):
    # rw8_1m (D = 8, n = 1e6, w = 300, d = 3, k = 10, FP32 projection, 8 GB cap:
    # the workload and launch configuration of the benchmark) against its exact
    # top-10, written by the oracle's diagonal sweep (tests/golden/make_golden.py).
    # The search may miss a motif with probability <= delta (Lemma 5.3). Greedy
    # over the verified pairs takes the golden motifs in order up to the first
    # one it lacks; that one must never have collided in >= d dimensions at a
    # step the search traversed (else it was verified and greedy would take it).
    # Picks after a miss may differ without further claim.
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "rw8_1m_top10.json")) as fh:
        golden = json.load(fh)
    s, p = synth.workload("rw8_1m")
    assert golden["data_seed"] == synth.DATA_SEED["rw8_1m"] and golden["params"]["n"] == s.n
    seed = synth.LSH_SEED["rw8_1m"]
    plan, _ = _plan(s, p, "f32", seed)
    prm = plan.params()
    got, rep, rc = plan.search(p["d"], p["k"], p["delta"])
    words = plan.hashes()
    plan.close()
    assert rc == mm.OK and len(got) == p["k"]
    want = [(g[0], g[1]) for g in golden["motifs"]]
    have = [(m["a"], m["b"]) for m in got]
    first = 0
    while first < len(want) and have[first] == want[first]:
        g = golden["motifs"][first]
        assert got[first]["dist_d"] == pytest.approx(g[2], rel=1e-9)
        assert got[first]["dist_max"] == pytest.approx(g[3], rel=1e-9)
        assert list(got[first]["dims"]) == g[4]
        first += 1
    print(f"search answer = golden on its first {first} of {len(want)} motifs; stop {rep['i_stop'], rep['j_stop']}")
    if first == len(want):
        return
    a, b = want[first]
    assert (a, b) not in have[first:], "golden motif verified but placed out of order"
    sure, maybe = _collision_steps(orc, s.x.astype(np.float64), p["w"], seed, prm["r"], prm["L"], 8, a, b,
                                   p["d"], (rep["i_stop"], rep["j_stop"]))
    print(f"golden motif {first} ({a}, {b}) missed: sure collisions {sure[:5]}, inside the band {maybe[:5]}")
    assert not sure, f"golden motif ({a}, {b}) collided in >= d dimensions at {sure[:3]} but was not reported"
    # the same with the device's own symbols of the two windows (checked against
    # the oracle's within the FP32 band first): no step up to the stop had the
    # pair colliding in >= d dimensions, so the search never had it to verify
    m, nl, _ = orc.tensor_shape(prm["L"])
    R, U = orc.draw_projections(seed, s.D, p["w"], 4 * prm["NF"])
    for q in (a, b):
        for f in range(s.D):
            by, pre, sab = orc.hash_one(s.x[f].astype(np.float64), p["w"], q, R[f], U[f], prm["r"])
            dev = np.array([(int(words[f, c // 4, q]) >> (24 - 8 * (c % 4))) & 255 for c in range(4 * prm["NF"])],
                           dtype=np.uint8)
            bo, bi, _, _ = _check_symbols(dev[None, None], by[None, None], pre[None, None],
                                          _band("f32", p["w"], pre, sab, prm["r"])[None, None], 8)
            assert bo == 0 and bi == 0
    for i in range(8, rep["i_stop"] - 1, -1):
        for J in range(1, prm["L"] + 1):
            if i == rep["i_stop"] and J > rep["j_stop"]:
                break
            W = sum(orc.prefix(words, prm["L"], f, J - 1, a, i) == orc.prefix(words, prm["L"], f, J - 1, b, i)
                    for f in range(s.D))
            assert W < p["d"], f"device index: ({a}, {b}) collides in {W} dimensions at ({i}, {J})"


# --------------------------------------------------------------------------- the headline workload
def test_headline_workload_bf16_against_fp32_and_the_oracle(orc):
    # rwsin32_4m (D = 32, n = 4 194 304, w = 1000, d = 8, k = 10, random walks
    # mixed with sinusoids, r x4): the benchmark's workload and launch
    # configuration, BF16 projection against FP32. Its exact top-10 is out of
    # reach here (about 2.8e14 pair-dimensions), so the test checks what holds
    # at any size:
    #  * r is the oracle's estimate (section 6.1) times the workload's factor;
    #  * sampled symbols (runs of 16 windows in every dimension, with windows at
    #    the series' ends): FP32 within its band of the oracle's FP64 hash,
    #    BF16 within its band of the rounded-input emulation;
    #  * both precisions stop at the same step with the same k motifs, whose
    #    dist_d, dist_max and dimensions are the oracle's FP64 d-dimensional
    #    distance of each pair (Eq. distdmax);
    #  * every planted motif is among them.
    s, p = synth.workload("rwsin32_4m")
    seed = synth.LSH_SEED["rwsin32_4m"]
    w, D = p["w"], s.D
    ns = s.n - w + 1
    x64 = s.x.astype(np.float64)
    r_want = orc.estimate_r(x64, w, seed) * p["r_scale"]
    rng = np.random.default_rng(0x4EAD)
    starts = [[0, ns - 16] + [int(a) for a in rng.integers(0, ns - 16, 2)] for _ in range(D)]
    answers = {}
    for proj in ("bf16", "f32"):
        plan, _ = _plan(s, p, proj, seed, r_scale=p["r_scale"])
        prm = plan.params()
        assert prm["r"] == r_want
        R, U = orc.draw_projections(seed, D, w, 4 * prm["NF"])
        for f in range(D):
            for a0 in starts[f]:
                xs = x64[f, a0: a0 + 16 + w - 1]
                gsym = _unpack(plan.hash_words(f, a0, 16)[None], 8)[0]
                if proj == "f32":
                    by, pre, sab = orc.hash_dim(xs, w, R[f], U[f], prm["r"])
                    band = _band("f32", w, pre, sab, prm["r"])
                else:
                    by, pre, sab, amb = orc.hash_dim_lowp(xs, w, R[f], U[f], prm["r"], proj)
                    band = _lowp_band(w, pre, sab, amb, prm["r"], proj)
                bad_out, bad_in, _, _ = _check_symbols(gsym, by, pre, band, 8)
                assert bad_out == 0 and bad_in == 0, (proj, f, a0)
        got, rep, rc = plan.search(p["d"], p["k"], p["delta"])
        plan.close()
        assert rc == mm.OK and len(got) == p["k"], (proj, rc, len(got))
        answers[proj] = ([(m["a"], m["b"]) for m in got], (rep["i_stop"], rep["j_stop"]))
        for m in got:
            dd, dm, dims, _ = orc.distd(x64, w, m["a"], m["b"], p["d"])
            assert m["dist_d"] == pytest.approx(dd, rel=1e-9) and m["dist_max"] == pytest.approx(dm, rel=1e-9)
            assert tuple(m["dims"]) == dims
        assert [m["dist_d"] for m in got] == sorted(m["dist_d"] for m in got)
        planted = {(q.p1, q.p2) for q in s.motifs}
        assert planted <= set(answers[proj][0]), (proj, planted - set(answers[proj][0]))
    assert answers["bf16"] == answers["f32"]
    print(f"rwsin32_4m: BF16 and FP32 answer alike, stop {answers['bf16'][1]}, {len(s.motifs)} planted found")


# --------------------------------------------------------------------------- exact answer on the device
@pytest.mark.parametrize("case", ["no_top", "partial_top", "flat", "dims96"])
def test_exact_fallback_sweep_equals_the_oracle(orc, case):
    # no step stops (LEMMA52 with a vanishing delta), so the answer is the
    # exact top-k over every pair, which the device computes by sweeping the
    # diagonals of the pair matrix past 4096 windows; the oracle's own sweep
    # (itself pinned to the brute force) gives the reference
    if case == "no_top":
        # 70 000 windows and a tiny r: nothing collides, TOP is empty, the cut
        # starts from the first candidates the sweep buffers
        s = synth.make_series(95, 4, 70_050, 50, 3, 2, dtype="f32")
        w, d, k, K, L, rs = 50, 2, 3, 8, 2, 0.02
    elif case == "partial_top":
        # the traversal's TOP (rounds 2 and 1 of two repetitions) sets the cut
        s = synth.make_series(96, 4, 70_050, 50, 3, 2, dtype="f32")
        w, d, k, K, L, rs = 50, 2, 3, 2, 2, 1.0
    elif case == "flat":
        # flat stretches (normal forms of zeros), each in one dimension only, so
        # that no pair is at distance 0 in d = 2 dimensions (which would stop)
        s = synth.make_series(97, 3, 20_000, 40, 2, 2, dtype="f32")
        s.x[0, 5000:5400] = 1.25
        s.x[1, 12000:12300] = 7.0
        s.x[2, 15000:15200] = -3.0
        w, d, k, K, L, rs = 40, 2, 4, 8, 2, 0.02
    else:
        # D = 96: two dimensions per lane in the sweep
        s = synth.make_series(98, 96, 6000, 40, 2, 10, noise=0.02, dtype="f32")
        w, d, k, K, L, rs = 40, 8, 2, 8, 2, 0.02
    p = dict(w=w, mem_limit=1 << 30)
    plan, _ = _plan(s, p, "f32", 5, K=K, L=L, stop="lemma52", r_scale=rs)
    got, rep, rc = plan.search(d, k, 1e-300)
    plan.close()
    assert rc == mm.OK_FALLBACK and rep["fallback"] == 1
    want = orc.topk_exact_sweep(s.x, w, d, k)
    _compare_motifs(got, want)


# --------------------------------------------------------------------------- anytime answers, delta modes, rules
def test_rigorous_rule_matches_the_oracle(orc):
    # the rigorous tensoring bound as the stopping rule: every step, TOP and
    # the stop step as the oracle's search with the same rule; each motif's
    # reported failure bound is the oracle's bound at the stop step
    s = synth.make_series(21, 5, 2500, 40, 3, 2, noise=0.02, dtype="f64")
    got, rep, rc, ref = _traverse(orc, s, 40, 5, 8, 60, 3, 2, 0.1, "rigorous", r_scale=2.0)
    assert rc == mm.OK and ref["i_stop"] >= 1
    _compare_motifs(got, ref["motifs"])
    plan_r = orc.estimate_r(s.x, 40, 5) * 2.0
    for m in got:
        want = orc.fail_bound(orc.collision_prob(m["dist_max"], plan_r) ** 2, ref["i_stop"], ref["J_stop"], 8,
                              rep["L_used"], orc.STOP_RIGOROUS)
        assert m["fail_prob"] == pytest.approx(want, rel=1e-9, abs=1e-300)
    assert rep["fail_bound"] == got[-1]["fail_prob"] <= 0.1


def test_joint_delta_is_the_per_motif_rule_at_delta_over_k(orc):
    # Lemma 5.4: with delta_mode "joint" the rule runs at delta / k
    s = synth.make_series(22, 4, 3000, 40, 3, 2, noise=0.02, dtype="f64")
    p = dict(w=40, mem_limit=1 << 30)
    plan, _ = _plan(s, p, "f64", 6, delta_mode="joint")
    got, rep, rc = plan.search(2, 3, 0.3)
    plan.close()
    ref = orc.lsh_pipeline(s.x, 40, 2, 3, 0.1, 6, mem_limit=1 << 30)
    assert (rep["i_stop"], rep["j_stop"]) == (ref["i_stop"], ref["J_stop"])
    _compare_motifs(got, ref["motifs"])
    assert rep["fail_bound"] <= 0.1


def test_step_budget_returns_top_with_its_failure_bounds(orc):
    # an anytime answer after 7 steps: TOP as the oracle has it after its 7th
    # step, each motif with the rule's bound at that step (section 4: the
    # search can be stopped at any time with the error probabilities)
    s = synth.make_series(23, 5, 2500, 40, 3, 2, dtype="f64")
    plan, _ = _plan(s, dict(w=40, mem_limit=1 << 30), "f64", 5, K=8, L=30, stop="lemma52", max_steps=7)
    prm = plan.params()
    got, rep, rc = plan.search(2, 3, 1e-6)
    plan.close()
    assert rc == mm.OK_PARTIAL and rep["n_steps"] == 7
    R, U = orc.draw_projections(5, s.D, 40, 4 * prm["NF"])
    words = orc.pack(orc.hash_all(s.x, 40, R, U, prm["r"]), prm["NF"], 8)
    ref = orc.lsh_search(s.x, 40, 2, 3, 1e-6, words, 8, prm["L"], prm["r"], rule=orc.STOP_LEMMA52, trace=True)
    n = ref["top_size"][6]
    assert [(m["a"], m["b"]) for m in got] == [tuple(v) for v in ref["top_pairs"][6, :n]]
    for m in got:        # step 7 is round 8, repetition 7
        want = orc.fail_bound(orc.collision_prob(m["dist_max"], prm["r"]) ** 2, 8, 7, 8, prm["L"], orc.STOP_LEMMA52)
        assert m["fail_prob"] == pytest.approx(want, rel=1e-9)
    assert rep["fail_bound"] == (got[2]["fail_prob"] if len(got) == 3 else 1.0)


# --------------------------------------------------------------------------- several dimensionalities
@pytest.mark.parametrize("case", ["planted", "mostly_fallback"])
def test_multi_d_search_answers_each_d_as_its_own_search(orc, case):
    # section 6.3: one traversal for d = 1..4; each d stops at the step of a
    # search for that d alone, with its answer, and that is the oracle's
    # search over the same index. "planted": d = 1, 2, 3 stop in rounds 8, 7
    # and 4, d = 4 never stops and gets the exact answer after the
    # traversal; "mostly_fallback": only d = 1 stops
    if case == "planted":
        s = synth.make_series(31, 5, 3000, 40, 3, 3, noise=0.02, dtype="f64")
        w, seed, K, k, L, delta, rule, r_scale = 40, 8, 8, 3, 40, 0.1, "tensor", 2.0
    else:
        s = synth.make_series(32, 4, 1200, 30, 2, 1, noise=0.05, dtype="f64")
        w, seed, K, k, L, delta, rule, r_scale = 30, 9, 8, 2, 20, 0.1, "lemma52", 3.0
    d_lo, d_hi = 1, 4
    plan, _ = _plan(s, dict(w=w, mem_limit=1 << 30), "f64", seed, K=K, L=L, stop=rule, r_scale=r_scale)
    prm = plan.params()
    R, U = orc.draw_projections(seed, s.D, w, 4 * prm["NF"])
    words = orc.pack(orc.hash_all(s.x, w, R, U, prm["r"]), prm["NF"], K)
    plan.set_hashes(words)
    multi = plan.search_multi(d_lo, d_hi, k, delta)
    single = {d: plan.search(d, k, delta) for d in range(d_lo, d_hi + 1)}
    again = plan.search_multi(d_lo, d_hi, k, delta)       # the plan's blocks reused: same answers
    plan.close()
    code = {"tensor": orc.STOP_TENSOR, "lemma52": orc.STOP_LEMMA52}[rule]
    statuses = []
    for d in range(d_lo, d_hi + 1):
        got, rep, st = multi[d]
        sg, srep, src = single[d]
        statuses.append(st)
        assert st == src, f"d={d}"
        assert (rep["i_stop"], rep["j_stop"]) == (srep["i_stop"], srep["j_stop"]), f"d={d}"
        assert rep["fallback"] == srep["fallback"]
        _compare_motifs(got, sg)
        assert [m["fail_prob"] for m in got] == pytest.approx([m["fail_prob"] for m in sg], rel=1e-12)
        ref = orc.lsh_search(s.x, w, d, k, delta, words, K, prm["L"], prm["r"], rule=code)
        assert (rep["i_stop"], rep["j_stop"]) == (ref["i_stop"], ref["J_stop"]), f"d={d}"
        _compare_motifs(got, ref["motifs"])
        g2, r2, s2 = again[d]
        assert s2 == st and (r2["i_stop"], r2["j_stop"]) == (rep["i_stop"], rep["j_stop"])
        _compare_motifs(g2, got)
    want = [mm.OK] * 3 + [mm.OK_FALLBACK] if case == "planted" else [mm.OK] + [mm.OK_FALLBACK] * 3
    assert statuses == want


def test_multi_d_search_with_one_d_and_a_step_budget(orc):
    # d_lo = d_hi is momenti_search; a step budget ends every open d at that
    # step with TOP as it stands there (the single searches' anytime answers)
    s = synth.make_series(33, 4, 2500, 40, 3, 2, dtype="f64")
    plan, _ = _plan(s, dict(w=40, mem_limit=1 << 30), "f64", 5, K=8, L=30, stop="lemma52")
    one = plan.search_multi(2, 2, 3, 0.1)[2]
    ref = plan.search(2, 3, 0.1)
    plan.close()
    assert one[2] == ref[2] and (one[1]["i_stop"], one[1]["j_stop"]) == (ref[1]["i_stop"], ref[1]["j_stop"])
    _compare_motifs(one[0], ref[0])
    plan, _ = _plan(s, dict(w=40, mem_limit=1 << 30), "f64", 5, K=8, L=30, stop="lemma52", max_steps=7)
    multi = plan.search_multi(1, 3, 3, 1e-6)
    single = {d: plan.search(d, 3, 1e-6) for d in (1, 2, 3)}
    plan.close()
    for d in (1, 2, 3):
        got, rep, st = multi[d]
        assert st == single[d][2] == mm.OK_PARTIAL and rep["n_steps"] == 7
        _compare_motifs(got, single[d][0])
        assert [m["fail_prob"] for m in got] == pytest.approx([m["fail_prob"] for m in single[d][0]], rel=1e-12)


# --------------------------------------------------------------------------- autotuning
def test_tuner_keeps_the_answer_and_the_plan_uses_its_choice(orc):
    # repetitions per launch change the cost only: the tuner checks every
    # candidate's answer against the first and keeps the fastest; the next
    # search runs with it and gives the oracle's answer and stop step
    s = synth.make_series(34, 5, 3000, 40, 3, 2, noise=0.02, dtype="f64")
    plan, _ = _plan(s, dict(w=40, mem_limit=1 << 30), "f64", 8, K=8, L=40, stop="tensor", r_scale=2.0)
    best, ms = plan.tune(2, 3, 0.1, cands=(1, 3, 8, 40))
    got, rep, rc = plan.search(2, 3, 0.1)
    prm = plan.params()
    plan.close()
    assert best in (1, 3, 8, 40) and ms > 0.0 and rep["batch_reps"] == best
    ref = orc.lsh_pipeline(s.x, 40, 2, 3, 0.1, 8, L_max=40, mem_limit=1 << 30, r_scale=2.0)
    assert (rep["i_stop"], rep["j_stop"]) == (ref["i_stop"], ref["J_stop"]) and rc == mm.OK
    _compare_motifs(got, ref["motifs"])
    assert prm["L"] == 40


# --------------------------------------------------------------------------- full size, FP8
def _collided_steps(words_a, words_b, nl, m, K, L, d, stop):
    """Steps (i, J) up to `stop` at which two windows' prefixes are equal in
    >= d dimensions, from their index words ([D][NF] each, four symbols to a
    word, position 0 most significant; the key interleaves left and right)."""
    hits = []
    i_stop, J_stop = stop
    for i in range(K, max(i_stop, 1) - 1, -1):
        nlft, nrgt = (i + 1) // 2, i // 2
        for J in range(1, L + 1):
            if i == i_stop and J > J_stop:
                break
            j = J - 1
            l, r = j // m, nl + j % m
            eq = ((words_a[:, l] ^ words_b[:, l]) >> np.uint32(32 - 8 * nlft)) == 0
            if nrgt:
                eq &= ((words_a[:, r] ^ words_b[:, r]) >> np.uint32(32 - 8 * nrgt)) == 0
            if int(eq.sum()) >= d:
                hits.append((i, J))
    return hits


def test_fp8_workload_misses_only_pairs_that_never_collided(orc):
    # rw128_1m (D = 128, n = 1e6, w = 500, d = 16, k = 50, FP8 projection, r x6) in
    # the benchmark's configuration: every planted motif missing from the answer
    # either never collided in >= d dimensions at a step the search traversed,
    # by the device's own index words of its two windows (so it was never a
    # candidate), or is ranked out by the answer (worse than the k-th, or
    # overlapping a better pick). A missing pair that collided would have been
    # verified and placed by the greedy TOP.
    s, p = synth.workload("rw128_1m")
    seed = synth.LSH_SEED["rw128_1m"]
    plan, _ = _plan(s, p, "fp8", seed, r_scale=p["r_scale"])
    got, rep, rc = plan.search(p["d"], p["k"], p["delta"])
    prm = plan.params()
    assert rc == mm.OK and len(got) == p["k"]
    m, nl, _ = orc.tensor_shape(prm["L"])
    picks = [(g["a"], g["b"]) for g in got]
    kth = got[-1]["dist_d"]
    unexplained = []
    for mt in s.motifs:
        a, b = mt.p1, mt.p2
        if (a, b) in picks:
            continue
        wa = np.stack([plan.hash_words(f, a, 1)[:, 0] for f in range(s.D)]).astype(np.uint32)
        wb = np.stack([plan.hash_words(f, b, 1)[:, 0] for f in range(s.D)]).astype(np.uint32)
        hits = _collided_steps(wa, wb, nl, m, 8, prm["L"], p["d"], (rep["i_stop"], rep["j_stop"]))
        if not hits:
            continue
        dd = orc.distd(s.x, p["w"], a, b, p["d"])[0]
        overlaps = any(2 * abs(u - v) <= p["w"] for u in (a, b) for (x, y) in picks for v in (x, y))
        if dd <= kth and not overlaps:
            unexplained.append(((a, b), hits[:3], dd))
    plan.close()
    assert not unexplained, f"planted pairs that collided but are missing: {unexplained}"
