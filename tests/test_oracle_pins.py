"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a published known-answer
vector, a closed form, an invariance of the definitions, a brute force written
differently (vectorised numpy over all pairs), a statistical law, or a number
worked out by hand.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats as sstats

from paper_2502_14446_amd import synth


# --------------------------------------------------------------------------- RNG
def test_philox_known_answers(orc):
    # Known-answer vectors published with Random123 (Salmon et al., SC'11) for
    # Philox4x32 with 10 rounds.
    assert orc.philox([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert orc.philox([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert orc.philox([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_gauss_and_uniform_streams_have_their_laws(orc):
    z = np.array([orc.gauss(1234, t, c, 0, 0) for t in range(200) for c in range(100)])
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    assert sstats.kstest(z, "norm").pvalue > 1e-4
    u = np.array([orc.uniform(99, c, f, 0, 1) for c in range(200) for f in range(100)])
    assert u.min() >= 0 and u.max() < 1
    assert sstats.kstest(u, "uniform").pvalue > 1e-4
    # distinct counters give distinct draws; the same counter the same draw
    assert orc.gauss(5, 1, 2, 3, 0) == orc.gauss(5, 1, 2, 3, 0)
    assert orc.gauss(5, 1, 2, 3, 0) != orc.gauss(5, 2, 1, 3, 0)
    assert orc.gauss(5, 1, 2, 3, 0) != orc.gauss(6, 1, 2, 3, 0)


# --------------------------------------------------------------------------- section 3.1
def test_window_stats_are_population_moments(orc):
    rng = np.random.default_rng(0)
    for w in (2, 7, 50, 301):
        x = rng.standard_normal(w) * 3 + 100
        mu, sg, flat = orc.window_stats(x)
        assert mu == pytest.approx(np.mean(x), rel=1e-14)
        assert sg == pytest.approx(np.std(x), rel=1e-12)     # numpy's default is the population std
        assert not flat
    mu, sg, flat = orc.window_stats(np.full(40, 0.1))
    assert flat                                              # constant window
    mu, sg, flat = orc.window_stats(np.zeros(40))
    assert flat and sg == 0.0


def test_dist_closed_forms(orc):
    rng = np.random.default_rng(1)
    w = 64
    x = np.cumsum(rng.standard_normal(w))
    # scale and offset invariance of the z-normalised distance
    assert orc.dist(x, 3.5 * x - 17.0) == pytest.approx(0.0, abs=1e-12)
    # a mirrored window is at the largest possible distance 2 sqrt(w)
    assert orc.dist(x, -x) == pytest.approx(2 * math.sqrt(w), rel=1e-13)
    # Pearson identity dist^2 = 2 w (1 - corr)
    y = np.cumsum(rng.standard_normal(w))
    corr = np.corrcoef(x, y)[0, 1]
    assert orc.dist(x, y) ** 2 == pytest.approx(2 * w * (1 - corr), rel=1e-12)
    # flat window: its normal form is all zeros, so the distance is ||x_hat|| = sqrt(w)
    assert orc.dist(np.full(w, 2.0), y) == pytest.approx(math.sqrt(w), rel=1e-13)
    assert orc.dist(np.full(w, 2.0), np.full(w, -5.0)) == 0.0


def _np_znorm_windows(xf, w):
    win = np.lib.stride_tricks.sliding_window_view(xf, w)
    mu = win.mean(axis=1, keepdims=True)
    sd = win.std(axis=1, keepdims=True)
    return (win - mu) / sd


def _np_dist_matrix(x, w):
    """[D][ns][ns] z-normalised distances, vectorised."""
    out = []
    for xf in x:
        z = _np_znorm_windows(xf, w)
        g = z @ z.T
        sq = np.diag(g)[:, None] + np.diag(g)[None, :] - 2 * g
        out.append(np.sqrt(np.maximum(sq, 0.0)))
    return np.array(out)


def test_distd_equals_exhaustive_subset_minimum(orc):
    rng = np.random.default_rng(2)
    D, n, w = 6, 120, 16
    x = np.cumsum(rng.standard_normal((D, n)), axis=1)
    for (a, b, d) in [(0, 40, 1), (5, 77, 2), (10, 100, 3), (3, 60, 6), (20, 90, 4)]:
        per = np.array([orc.dist(x[f, a:a + w], x[f, b:b + w]) for f in range(D)])
        best = min(itertools.combinations(range(D), d), key=lambda F: (sum(per[list(F)]), F))
        dd, dm, dims, per_o = orc.distd(x, w, a, b, d)
        assert dd == pytest.approx(sum(per[list(best)]), rel=1e-13)
        assert dims == best
        assert dm == pytest.approx(max(per[list(best)]), rel=1e-13)


def _np_all_pairs(x, w, d):
    """All non-trivial pairs with dist_d, from an independent numpy computation."""
    Dm = _np_dist_matrix(x, w)
    D, ns, _ = Dm.shape
    a, b = np.triu_indices(ns, 1)
    keep = 2 * (b - a) > w
    a, b = a[keep], b[keep]
    per = np.sort(Dm[:, a, b], axis=0)
    return a, b, per[:d].sum(axis=0)


def _compatible(p, q, w):
    return all(2 * abs(u - v) > w for u in p for v in q)


def test_topk_exact_is_the_greedy_non_overlapping_choice(orc):
    rng = np.random.default_rng(3)
    D, n, w, d = 3, 170, 12, 2
    x = np.cumsum(rng.standard_normal((D, n)), axis=1)
    for k in (1, 3, 6):
        got = orc.topk_exact(x, w, d, k)
        a, b, dd = _np_all_pairs(x, w, d)
        order = np.lexsort((b, a, dd))
        keys = list(zip(dd[order], a[order], b[order]))
        picks = [(m["a"], m["b"]) for m in got]
        # distances agree with the independent computation
        for m in got:
            ref = dd[(a == m["a"]) & (b == m["b"])][0]
            assert m["dist_d"] == pytest.approx(ref, rel=1e-9)
        # picks are non-trivial, mutually non-overlapping and in increasing order
        assert all(2 * (q - p) > w for p, q in picks)
        assert all(_compatible(picks[s], picks[t], w) for s in range(len(picks)) for t in range(s))
        # every better pair that was passed over overlaps an earlier pick, and
        # the next pick is the first pair compatible with all previous ones
        chosen = []
        for (dist, p, q) in keys:
            if len(chosen) == len(picks):
                break
            if all(_compatible((p, q), c, w) for c in chosen):
                assert (p, q) == picks[len(chosen)]
                chosen.append((p, q))
        assert chosen == picks
        assert len(picks) == k


def test_topk_exact_finds_the_planted_motif(orc):
    s, p = synth.workload("tiny")
    got = orc.topk_exact(s.x, p["w"], p["d"], 1)
    m = s.motifs[0]
    assert (got[0]["a"], got[0]["b"]) == (m.p1, m.p2)
    assert got[0]["dims"] == m.dims


def test_topk_exact_returns_fewer_when_pairs_run_out(orc):
    rng = np.random.default_rng(4)
    x = np.cumsum(rng.standard_normal((2, 60)), axis=1)
    got = orc.topk_exact(x, 20, 1, 10)
    # 41 windows, exclusion 10: at most a handful of disjoint pairs exist
    assert 0 < len(got) < 10
    picks = [(m["a"], m["b"]) for m in got]
    a, b, _ = _np_all_pairs(x, 20, 1)
    # no remaining pair is compatible with all picks
    assert not any(all(_compatible((p, q), c, 20) for c in picks) for p, q in zip(a, b))


# --------------------------------------------------------------------------- Eq. drp, Eq. 423
def test_hash_value_hand_examples(orc):
    import ctypes as C
    lib = orc.lib()

    def h(z, R, U, r):
        z = np.array(z, dtype=np.float64); R = np.array(R, dtype=np.float64)
        pre, sab = C.c_double(), C.c_double()
        byte = lib.orc_hash_value(z.ctypes.data_as(C.c_void_p), len(z), R.ctypes.data_as(C.c_void_p),
                                  1, U, r, C.byref(pre), C.byref(sab))
        return byte, pre.value, sab.value

    # dot = 0.5 - 0.25 + 0.5 - 1 = -0.25; b = 0.5 * 0.25; u = (-0.25 + 0.125) / 0.5 = -0.25
    assert h([1, -1, 0.5, -0.5], [0.5, 0.25, 1, 2], 0.25, 0.5) == (127, -0.25, 2.25)
    # dot = 3; b = 0.25 * 0.75 = 0.1875; u = 3.1875 / 0.25 = 12.75 -> h = 12 -> byte 140
    assert h([1, 2], [1, 1], 0.75, 0.25)[:2] == (140, 12.75)
    # dot = -50; r = 0.25 -> u = -200 + 0 -> h = -200 -> (-72) mod 256 = 184
    assert h([-50.0], [1.0], 0.0, 0.25)[0] == 184
    # dot = 40, r = 0.25, U = 0.5 -> u = 160.5 -> h = 160 -> 288 mod 256 = 32
    assert h([40.0], [1.0], 0.5, 0.25)[0] == 32


def _f32_values(rng, count):
    """float32-representable values over many binades, both signs."""
    mant = rng.uniform(1.0, 2.0, count)
    expo = rng.integers(-30, 10, count)
    v = mant * np.exp2(expo) * rng.choice([-1.0, 1.0], count)
    return v.astype(np.float32).astype(np.float64)


def test_round_fmt_matches_torch_bfloat16(orc):
    # round-to-nearest-even to bfloat16 (8 significant bits): torch's float32 ->
    # bfloat16 conversion is an independent implementation of the format
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(40)
    v = _f32_values(rng, 600_000)
    # exact midpoints between neighbouring bfloat16 values (ties go to even)
    lead = np.exp2(rng.integers(-20, 20, 200_000).astype(np.float64))
    k = rng.integers(128, 256, 200_000).astype(np.float64)
    ties = (k + 0.5) * lead / 128.0 * rng.choice([-1.0, 1.0], 200_000)
    # values one float32 ulp on either side of a midpoint
    near = np.concatenate([np.nextafter(ties.astype(np.float32), np.float32(np.inf)),
                           np.nextafter(ties.astype(np.float32), np.float32(-np.inf))]).astype(np.float64)
    allv = np.concatenate([v, ties, near, [0.0, -0.0, 1.0, -1.0, 3.0e38]])
    got = orc.round_fmt_array(allv, "bf16")
    want = torch.from_numpy(allv.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(got, want)


def test_round_fmt_matches_torch_e4m3(orc):
    # OCP FP8 E4M3: 4 significant bits, bias 7, subnormal quantum 2^-9. torch's
    # float8_e4m3fn conversion is independent; it returns NaN for values that
    # round above 448 (no saturation), so the comparison stops below 464.
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(41)
    v = _f32_values(rng, 600_000)
    v = v[np.abs(v) < 464.0]
    # every subnormal midpoint and normal midpoint, both signs
    sub = (np.arange(0, 16) + 0.5) * 2.0 ** -9
    nrm = np.array([(8 + m + 0.5) * 2.0 ** (e - 3) for e in range(-6, 9) for m in range(8)])
    nrm = nrm[nrm < 464.0]
    ties = np.concatenate([sub, nrm, -sub, -nrm])
    near = np.concatenate([np.nextafter(ties.astype(np.float32), np.float32(np.inf)),
                           np.nextafter(ties.astype(np.float32), np.float32(-np.inf))]).astype(np.float64)
    grid = np.arange(-4096, 4097) * 2.0 ** -13            # dense sweep of the subnormal range
    allv = np.concatenate([v, ties, near, grid, [0.0, 448.0, -448.0, 463.9]])
    allv = allv[np.abs(allv) < 464.0]
    got = orc.round_fmt_array(allv, "fp8")
    want = torch.from_numpy(allv.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(got, want)


def test_round_fmt_hand_values(orc):
    r = lambda v, f: orc.round_fmt(v, f)   # noqa: E731
    # e4m3: ties to even in the subnormal range, the smallest quantum 2^-9
    assert r(2.0 ** -9, "fp8") == 2.0 ** -9
    assert r(2.0 ** -10, "fp8") == 0.0                 # halfway to 2^-9: even (zero)
    assert r(3 * 2.0 ** -10, "fp8") == 2.0 ** -8       # 1.5 quanta: even (2 quanta)
    assert r(0.75 * 2.0 ** -9, "fp8") == 2.0 ** -9
    assert r(7.5 * 2.0 ** -9, "fp8") == 2.0 ** -6      # up into the normal range
    assert r(1.0625, "fp8") == 1.0 and r(1.1875, "fp8") == 1.25
    # e4m3 saturates at the largest finite value 448 (464 is a tie: even, 448)
    assert r(448.0, "fp8") == 448.0 and r(464.0, "fp8") == 448.0
    assert r(470.0, "fp8") == 448.0 and r(1e4, "fp8") == 448.0 and r(-1e4, "fp8") == -448.0
    # bfloat16: 8 significant bits, ties to even
    assert r(1.0 + 2.0 ** -8, "bf16") == 1.0
    assert r(1.0 + 3 * 2.0 ** -8, "bf16") == 1.0 + 2.0 ** -6
    assert r(-(1.0 + 2.0 ** -8 + 2.0 ** -20), "bf16") == -(1.0 + 2.0 ** -7)


def _lowp_one(orc, z, R, U, r, fmt):
    import ctypes as C
    lib = orc.lib()
    z = np.array(z, dtype=np.float64); R = np.array(R, dtype=np.float64)
    pre, sab, amb = C.c_double(), C.c_double(), C.c_double()
    byte = lib.orc_hash_value_lowp(z.ctypes.data_as(C.c_void_p), len(z), R.ctypes.data_as(C.c_void_p),
                                   1, U, r, orc.FMT[fmt], C.byref(pre), C.byref(sab), C.byref(amb))
    return byte, pre.value, sab.value, amb.value


def test_hash_value_lowp_hand_examples(orc):
    # bfloat16, worked by hand with dyadic values:
    #   Q(z) = [1 (1 + 2^-8 is a tie), 2, -0.5], Q(a) = [1, 0.75, 1 + 2^-6 (1 + 3 2^-8 is a tie)]
    #   Q(a).Q(z) = 1 + 1.5 - 0.5078125 = 1.9921875; r = 2^-8, b = r / 2
    #   u = (1.9921875 + 2^-9) 256 = 510.5 -> h = 510 -> (510 + 128) mod 256 = 126
    # (unrounded inputs would give u = 512 -> 128). The first sample sits on a
    # midpoint, so the ambiguity is |Q(a_0)| gap = 2^-7.
    byte, pre, sab, amb = _lowp_one(orc, [1 + 2 ** -8, 2.0, -0.5], [1.0, 0.75, 1 + 3 * 2 ** -8],
                                    0.5, 2.0 ** -8, "bf16")
    assert (byte, pre, sab, amb) == (126, 510.5, 3.0078125, 2.0 ** -7)
    # e4m3: Q(z) = [1 (tie), 6 2^-9 (subnormal, exact), 2^-8 (3 2^-10 is a subnormal
    # tie), 3], Q(a) = [2, 1, 0.3125 (0.3 rounded on the 2^-5 grid), -0.5]
    #   Q(a).Q(z) = 2 + 0.01171875 + 0.001220703125 - 1.5 = 0.512939453125
    #   r = 2^-6, b = r / 4: u = 33.078125 -> h = 33 -> byte 161 (unrounded: 41 -> 169)
    #   ambiguity: 2 * 2^-3 (first sample) + 0.3125 * 2^-9 (third) = 0.2506103515625
    byte, pre, sab, amb = _lowp_one(orc, [1.0625, 6 * 2 ** -9, 3 * 2 ** -10, 3.0], [2.0, 1.0, 0.3, -0.5],
                                    0.25, 2.0 ** -6, "fp8")
    assert (byte, pre, sab, amb) == (161, 33.078125, 3.512939453125, 0.2506103515625)


def test_collision_probability_matches_monte_carlo(orc):
    # For a ~ N(0, I) and b ~ U[0, r), two points at distance R collide iff
    # floor((s + b) / r) == floor(b / r) with s = a . (y - x) ~ N(0, R^2).
    rng = np.random.default_rng(5)
    N = 1_000_000
    for r, R in [(1.0, 0.3), (1.0, 1.0), (0.68, 0.25), (2.0, 5.0)]:
        s = rng.standard_normal(N) * R
        b = rng.uniform(0, r, N)
        hit = np.mean(np.floor((s + b) / r) == np.floor(b / r))
        p = orc.collision_prob(R, r)
        assert abs(hit - p) < 5 * math.sqrt(p * (1 - p) / N), (r, R, hit, p)
    assert orc.collision_prob(0.0, 1.0) == 1.0
    t = 1e-4
    assert orc.collision_prob(1.0 / t, 1.0) == pytest.approx(t / math.sqrt(2 * math.pi), rel=1e-3)
    ps = [orc.collision_prob(R, 0.7) for R in np.linspace(0.01, 10, 50)]
    assert all(u > v for u, v in zip(ps, ps[1:]))


# --------------------------------------------------------------------------- section 6.1
def test_tensor_shape_and_repetition_map(orc):
    assert orc.tensor_shape(200) == (15, 14, 15)
    assert orc.tensor_shape(196) == (14, 14, 14)
    assert orc.tensor_shape(1) == (1, 1, 1)
    assert orc.tensor_shape(2) == (2, 1, 2)
    for L in (1, 2, 7, 16, 50, 200):
        m, nl, nr = orc.tensor_shape(L)
        pairs = {(j // m, j % m) for j in range(L)}
        assert len(pairs) == L                           # every repetition has its own (l, r)
        assert max(l for l, _ in pairs) == nl - 1
        assert max(r for _, r in pairs) == nr - 1
        assert m * m >= L and (m - 1) * (m - 1) < L


def test_pack_and_interleaved_prefix(orc):
    L = 4                              # m = 2, two left and two right functions
    m, nl, nr = orc.tensor_shape(L)
    NF = nl + nr
    by = np.zeros((1, 1, 4 * NF), dtype=np.uint8)
    by[0, 0, 0:4] = [0xA1, 0xA2, 0xA3, 0xA4]             # left 0
    by[0, 0, 4:8] = [0xC1, 0xC2, 0xC3, 0xC4]             # left 1
    by[0, 0, 8:12] = [0xB1, 0xB2, 0xB3, 0xB4]            # right 0
    by[0, 0, 12:16] = [0xD1, 0xD2, 0xD3, 0xD4]           # right 1
    words = orc.pack(by, NF, 8)
    assert [hex(v) for v in words[0, :, 0]] == ["0xa1a2a3a4", "0xc1c2c3c4", "0xb1b2b3b4", "0xd1d2d3d4"]
    assert orc.prefix(words, L, 0, 0, 0, 8) == 0xA1B1A2B2A3B3A4B4
    assert orc.prefix(words, L, 0, 0, 0, 3) == 0xA1B1A2
    assert orc.prefix(words, L, 0, 1, 0, 2) == 0xA1D1      # j = 1 -> (l, r) = (0, 1)
    assert orc.prefix(words, L, 0, 2, 0, 4) == 0xC1B1C2B2  # j = 2 -> (1, 0)
    assert orc.prefix(words, L, 0, 3, 0, 1) == 0xC1
    w4 = orc.pack(by, NF, 4)                                # K = 4 keeps two symbols per half
    assert hex(int(w4[0, 0, 0])) == "0xa1a20000"


def test_L_used_hand_values(orc):
    # n = 1000, D = 2, w = 100, 8-byte samples: n_s = 901,
    # fixed = 16000 + 16*901*2 + 32*901*2 + 64 MiB = 67211360 bytes,
    # index(L) = 4*901*2*(left + right) = 7208 * (left + right).
    base = 67211360
    assert orc.L_used(1000, 2, 100, 200, 8, base + 7208 * 29) == 200
    assert orc.L_used(1000, 2, 100, 200, 8, base + 7208 * 29 - 1) == 196   # 14 + 14 functions
    assert orc.L_used(1000, 2, 100, 200, 8, base + 7208 * 2) == 1
    assert orc.L_used(1000, 2, 100, 200, 8, base + 7208 * 2 - 1) == 0


def test_r_is_invariant_to_per_dimension_affine_maps(orc):
    rng = np.random.default_rng(6)
    x = np.cumsum(rng.standard_normal((3, 3000)), axis=1)
    r1 = orc.estimate_r(x, 64, 77)
    y = x * np.array([[2.0], [0.5], [4.0]]) + np.array([[1e3], [-7.0], [0.25]])
    assert orc.estimate_r(y, 64, 77) == pytest.approx(r1, rel=1e-9)
    # the projections of unit-norm-sqrt(w) windows on N(0, I) vectors are N(0, w):
    # the range of ~3*2950*8 of them is about 2 sqrt(2 ln N) standard deviations
    N = 3 * 2937 * 8
    expect = 2 * math.sqrt(2 * math.log(N)) * math.sqrt(64) / 256
    assert 0.7 * expect < r1 < 1.2 * expect


# --------------------------------------------------------------------------- Algorithm 2
def test_fail_bound_hand_values(orc):
    T, L52 = orc.STOP_TENSOR, orc.STOP_LEMMA52
    # p = 1/2, i = K = 8, J = 20, L = 200 (m = 15): (1 - 1/16)^(20 div 15) * (1 - 1/16)^(20 mod 15)
    assert orc.fail_bound(0.5, 8, 20, 8, 200, T) == pytest.approx(0.9375 ** 6, rel=1e-15)
    # i = 7 < K: P_t(3.5, 20) * P_t(4, 180) = (15/16)^1 (7/8)^5 * (15/16)^(12 + 0)
    assert orc.fail_bound(0.5, 7, 20, 8, 200, T) == pytest.approx(0.9375 * 0.875 ** 5 * 0.9375 ** 12, rel=1e-14)
    # round 1: the right half contributes no symbol; its factor is 1, so
    # J = 1: P_t(1/2, 1) = (1 - p)^0 = 1; P_t(1, 199) = (1 - p)^13 (1 - p)^4
    assert orc.fail_bound(0.3, 1, 1, 8, 200, T) == pytest.approx(0.7 ** 17, rel=1e-14)
    # J = 20: P_t(1/2, 20) = (1 - p)^1; P_t(1, 180) = (1 - p)^12 (1 - p)^0
    assert orc.fail_bound(0.5, 1, 20, 8, 200, T) == pytest.approx(0.5 ** 13, rel=1e-14)
    # taken literally, (1 - p^0)^(J mod m) vanishes as soon as J mod m > 0
    TL = orc.STOP_TENSOR_LITERAL
    assert orc.fail_bound(0.3, 1, 1, 8, 200, TL) == 0.0
    assert orc.fail_bound(0.5, 1, 15, 8, 200, TL) == pytest.approx(0.5 ** 18, rel=1e-14)
    # rounds above 1 are the same under both readings
    assert orc.fail_bound(0.5, 7, 20, 8, 200, TL) == orc.fail_bound(0.5, 7, 20, 8, 200, T)
    # Lemma 5.2 form: (1 - p^i)^J (1 - p^(i+1))^(L - J)
    assert orc.fail_bound(0.5, 8, 3, 8, 200, L52) == pytest.approx((1 - 2 ** -8) ** 3, rel=1e-15)
    assert orc.fail_bound(0.5, 2, 10, 8, 20, L52) == pytest.approx(0.75 ** 10 * 0.875 ** 10, rel=1e-15)
    # a pair at distance 0 collides always: nothing can have been missed
    assert orc.stop(0.0, 0.7, 3, 8, 1, 8, 200, T, 1e-9)


# --------------------------------------------------------------------------- Algorithm 1
def _np_prefix(words, L, f, j, i):
    m = int(math.ceil(math.sqrt(L) - 1e-12))
    while m * m < L:
        m += 1
    _, nl, _ = (m, -(-L // m), min(L, m))
    left = words[f, j // m].astype(np.uint64)
    right = words[f, nl + j % m].astype(np.uint64)
    v = np.zeros_like(left)
    for q in range(i):
        src = left if q % 2 == 0 else right
        sym = (src >> np.uint64(24 - 8 * (q // 2))) & np.uint64(255)
        v = (v << np.uint64(8)) | sym
    return v


def test_step_candidates_match_all_pairs_brute_force(orc):
    rng = np.random.default_rng(7)
    D, n, w, d, k = 3, 400, 20, 2, 2
    x = np.cumsum(rng.standard_normal((D, n)), axis=1)
    res = orc.lsh_pipeline(x, w, d, k, 1e-300, seed=11, K=4, L_max=9, rule=orc.STOP_LEMMA52,
                           trace=True)
    assert res["fallback"]                                   # delta this small never stops
    words, L = res["words"], res["L"]
    ns = n - w + 1
    a, b = np.triu_indices(ns, 1)
    keep = 2 * (b - a) > w
    a, b = a[keep], b[keep]
    cand = res["cand"]
    for i in range(4, 0, -1):
        for j in range(L):
            step = (4 - i) * L + j
            W = np.zeros(a.size, dtype=np.int64)
            for f in range(D):
                pf = _np_prefix(words, L, f, j, i)
                W += pf[a] == pf[b]
            want = set(zip(a[W >= d].tolist(), b[W >= d].tolist()))
            got = cand[cand[:, 0] == step]
            assert set(zip(got[:, 1].tolist(), got[:, 2].tolist())) == want, (i, j)
    # the exhausted search answers with the exact top-k
    assert [(m["a"], m["b"]) for m in res["motifs"]] == \
        [(m["a"], m["b"]) for m in orc.topk_exact(x, w, d, k)]


def test_lsh_search_returns_the_exact_answer_on_the_tiny_workload(orc):
    s, p = synth.workload("tiny")
    res = orc.lsh_pipeline(s.x, p["w"], p["d"], p["k"], p["delta"], seed=synth.LSH_SEED["tiny"],
                           mem_limit=p["mem_limit"])
    ex = orc.topk_exact(s.x, p["w"], p["d"], p["k"])
    assert [(m["a"], m["b"]) for m in res["motifs"]] == [(m["a"], m["b"]) for m in ex]


def test_lsh_search_stops_on_a_close_planted_motif(orc):
    # noise 0.02 instead of 0.05: the motif is close enough for the bound to
    # reach delta before round 1
    s = synth.make_series(0xD00D01, 4, 2000, 50, 1, 2, noise=0.02, min_gap=500)
    res = orc.lsh_pipeline(s.x, 50, 2, 1, 0.1, seed=synth.LSH_SEED["tiny"], mem_limit=1 << 30)
    ex = orc.topk_exact(s.x, 50, 2, 1)
    assert [(m["a"], m["b"]) for m in res["motifs"]] == [(m["a"], m["b"]) for m in ex]
    assert (ex[0]["a"], ex[0]["b"]) == (s.motifs[0].p1, s.motifs[0].p2)
    assert not res["fallback"] and res["i_stop"] > 1
    # the stopping rule holds at the reported step, and not one step earlier
    # (with TOP as it stood after that earlier step)
    m = res["motifs"][-1]
    i, J, L = res["i_stop"], res["J_stop"], res["L"]
    assert orc.stop(m["dist_max"], res["r"], 2, i, J, 8, L, orc.STOP_TENSOR, 0.1)
    tr = orc.lsh_search(s.x, 50, 2, 1, 0.1, res["words"], 8, L, res["r"], rule=orc.STOP_TENSOR,
                        trace=True)
    assert (tr["i_stop"], tr["J_stop"]) == (i, J)
    step = (8 - i) * L + J - 1
    assert step >= 1
    pi, pJ = (i, J - 1) if J > 1 else (i + 1, L)
    # one step earlier the rule fails: TOP is short of k, or its bound exceeds delta
    assert tr["top_size"][step - 1] < 1 or \
        not orc.stop(tr["top_distmax"][step - 1], res["r"], 2, pi, pJ, 8, L, orc.STOP_TENSOR, 0.1)


@pytest.mark.parametrize("rule", ["tensor", "lemma52"])
def test_lsh_recall_is_at_least_one_minus_delta(orc, rule):
    # Lemma 5.3: each returned motif is the true one with probability >= 1 - delta.
    # The instances are chosen so that the search stops on the rule itself (a
    # close motif, noise 0.02, and r at 3 times the section 6.1 estimate): a run
    # that ends in the exact fallback cannot miss, so the fallback share is
    # bounded too, else the recall would be 1 by construction.
    delta, runs = 0.05, 200
    code = orc.STOP_TENSOR if rule == "tensor" else orc.STOP_LEMMA52
    misses = fallbacks = 0
    for seed in range(runs):
        s = synth.make_series(1000 + seed, 3, 500, 24, 1, 2, noise=0.02)
        res = orc.lsh_pipeline(s.x, 24, 2, 1, delta, seed=seed, K=8, L_max=16, rule=code,
                               r_scale=3.0)
        ex = orc.topk_exact(s.x, 24, 2, 1)
        fallbacks += res["fallback"]
        misses += (res["motifs"][0]["a"], res["motifs"][0]["b"]) != (ex[0]["a"], ex[0]["b"])
    assert fallbacks <= 0.1 * runs, fallbacks
    # failures are at most Binomial(runs, delta); allow 3 standard deviations
    assert misses <= runs * delta + 3 * math.sqrt(runs * delta * (1 - delta)), misses


# ----------------------------------------------------------------------------- Example 4.1
from example_4_1 import example_4_1_scenario  # noqa: E402


def test_example_4_1_control_flow(orc):
    fx, s, words, r, pairs, top = example_4_1_scenario(orc)
    prm, ex = fx["parameters"], fx["expected"]
    K, L = prm["K"], prm["L"]
    res = orc.lsh_search(s.x, 40, prm["d"], prm["k"], prm["delta"], words, K, L, r,
                         rule=orc.STOP_LEMMA52, trace=True)
    assert [res["i_stop"], res["J_stop"]] == ex["stops_at"]
    assert [(m["a"], m["b"]) for m in res["motifs"]] == [pairs[top]]
    p = orc.collision_prob(res["motifs"][0]["dist_max"], r) ** prm["d"]
    for i, J in ex["rule_does_not_hold_at"]:
        assert orc.fail_bound(p, i, J, K, L, orc.STOP_LEMMA52) > prm["delta"]
    # every traversed step sees both motifs (weight 2) and keeps the closer one
    last = (K - res["i_stop"]) * L + res["J_stop"] - 1
    cand = res["cand"]
    for step in range(last + 1):
        got = {(int(x), int(y)) for _, x, y in cand[cand[:, 0] == step]}
        assert got == set(pairs), step
        assert res["top_size"][step] == 1
        assert tuple(res["top_pairs"][step, 0]) == pairs[top]


# ----------------------------------------------------------------------------- O1-fast
@pytest.mark.parametrize("seed,D,n,w,d,k", [
    (3, 3, 1200, 40, 2, 3), (5, 4, 3000, 51, 2, 5), (9, 6, 2500, 33, 3, 4), (11, 1, 2000, 64, 1, 6),
    (13, 5, 4800, 100, 5, 3)])
def test_sweep_equals_brute_force(orc, seed, D, n, w, d, k):
    # the diagonal sweep (a filter, every kept pair recomputed by the brute
    # force's own definition) returns the brute force's answer, with a small
    # pool so that the certification and the retry path are exercised
    s = synth.make_series(seed, D, n, w, 2, d)
    ex = orc.topk_exact(s.x, w, d, k)
    for pool in (64, 4096):
        info = {}
        sw = orc.topk_exact_sweep(s.x, w, d, k, pool=pool, omp=False, info=info)
        assert [(m["a"], m["b"], m["dist_d"], m["dist_max"], m["dims"]) for m in sw] == \
            [(m["a"], m["b"], m["dist_d"], m["dist_max"], m["dims"]) for m in ex]
        # the filter's error is far inside the margin the certificate uses
        assert info["max_err"] < 1e-6 * info["eps"]


def test_sweep_with_flat_windows_and_threads(orc):
    # flat stretches (their normal forms are zeros: distance 0 between two of
    # them, sqrt(w) to any other window) and the OpenMP build
    rng = np.random.default_rng(17)
    x = np.cumsum(rng.standard_normal((3, 1500)), axis=1)
    x[0, 200:330] = 4.0
    x[0, 900:1000] = -2.0
    x[1, 210:320] = 1.5          # dimensions 0 and 1 flat together in two places
    x[1, 905:990] = 7.0
    x[2, 600:700] = 0.5          # a flat stretch in one dimension only
    ex = orc.topk_exact(x, 30, 2, 4)
    assert ex[0]["dist_d"] == 0.0                       # flat in two dimensions at both windows
    for omp in (False, True):
        sw = orc.topk_exact_sweep(x, 30, 2, 4, pool=256, omp=omp)
        assert [(m["a"], m["b"], m["dist_d"], m["dims"]) for m in sw] == \
            [(m["a"], m["b"], m["dist_d"], m["dims"]) for m in ex]


def test_openmp_build_gives_the_same_search(orc):
    # the CPU baseline's build (OpenMP over dimensions and distances) runs the
    # same steps: same candidates, same TOP after every step, same answer
    s = synth.make_series(21, 5, 2500, 40, 3, 2)
    res = orc.lsh_pipeline(s.x, 40, 2, 3, 0.05, seed=5, K=8, L_max=30, rule=orc.STOP_LEMMA52, trace=True)
    par = orc.lsh_search(s.x, 40, 2, 3, 0.05, res["words"], 8, res["L"], res["r"], rule=orc.STOP_LEMMA52,
                         trace=True, omp=True)
    assert (par["i_stop"], par["J_stop"]) == (res["i_stop"], res["J_stop"])
    assert np.array_equal(par["cand"], res["cand"])
    assert np.array_equal(par["top_size"], res["top_size"])
    assert [(m["a"], m["b"], m["dist_d"]) for m in par["motifs"]] == \
        [(m["a"], m["b"], m["dist_d"]) for m in res["motifs"]]


# ----------------------------------------------------------------------------- rigorous tensoring bound
def _mc_tensored_failure(p, i, J, K, L, N, rng):
    """Monte Carlo of the failure event of the tensored index: every half-
    function gets an independent collision depth G with P(G >= s) = p^s;
    repetition j (left j div m, right j mod m) collides at prefix length i'
    when the left depth reaches ceil(i'/2) and the right depth floor(i'/2).
    Failure: no repetition j < J collides at prefix i, and (below round K) no
    repetition collides at prefix i + 1."""
    m = math.isqrt(L - 1) + 1 if L > 1 else 1
    nl, nr = -(-L // m), min(L, m)
    Dl = rng.geometric(1.0 - p, size=(N, nl)) - 1      # P(Dl >= s) = p^s
    Er = rng.geometric(1.0 - p, size=(N, nr)) - 1
    fail = np.ones(N, dtype=bool)
    for j in range(L):
        l, r = j // m, j % m
        for ii in ([i] if j < J else []) + ([i + 1] if i < K else []):
            fail &= ~((Dl[:, l] >= (ii + 1) // 2) & (Er[:, r] >= ii // 2))
    return fail.mean()


@pytest.mark.parametrize("p,i,J,K,L", [
    (0.5, 3, 20, 8, 200), (0.3, 1, 7, 8, 200), (0.85, 6, 1, 8, 200), (0.6, 2, 50, 8, 50),
    (0.9, 8, 5, 8, 30), (0.4, 4, 16, 8, 16), (0.7, 5, 33, 8, 40), (0.55, 1, 12, 4, 12)])
def test_rigorous_bound_equals_the_geometric_depth_model(orc, p, i, J, K, L):
    rng = np.random.default_rng(int(p * 1000) + 31 * i + J)
    N = 400_000
    mc = _mc_tensored_failure(p, i, J, K, L, N, rng)
    v = orc.fail_bound(p, i, J, K, L, orc.STOP_RIGOROUS)
    sig = math.sqrt(max(v * (1 - v), 1e-12) / N)
    assert abs(mc - v) <= 5 * sig + 1e-9, (mc, v)


def test_rigorous_bound_special_cases(orc):
    R = orc.STOP_RIGOROUS
    # one repetition: Lemma 5.2's (1 - p^i)
    assert orc.fail_bound(0.5, 8, 1, 8, 1, R) == pytest.approx(1 - 0.5 ** 8, rel=1e-15)
    # (below round K the one repetition at prefix i + 1 adds nothing: a collision
    # there is one at prefix i)
    assert orc.fail_bound(0.7, 5, 1, 8, 1, R) == pytest.approx(1 - 0.7 ** 5, rel=1e-15)
    # p = 1: every pair collides, nothing can be missed; p = 0: nothing collides
    assert orc.fail_bound(1.0, 3, 5, 8, 200, R) == 0.0
    assert orc.fail_bound(0.0, 3, 5, 8, 200, R) == 1.0
    # more repetitions never raise the bound
    vals = [orc.fail_bound(0.6, 4, J, 8, 200, R) for J in range(1, 201)]
    assert all(u >= v - 1e-15 for u, v in zip(vals, vals[1:]))
