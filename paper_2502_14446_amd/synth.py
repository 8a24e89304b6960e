"""Seeded synthetic inputs: random walks with planted multidimensional motifs.

This module only draws data. It holds none of the motif-search arithmetic
(no normalisation, hashing or distances), so both the CPU oracle side and the
GPU side of the test suite can take their inputs from it.

Recipe (paper section 7.5 uses random walks with planted patterns for its
scalability study; the real datasets of its Table "dataset" are not used):

* every dimension is a random walk, the cumulative sum of N(0, 1) steps;
* optionally a sinusoid of random period is added to each dimension;
* a motif is planted by writing the same w-1 random-walk increments into the
  increment sequence at two window positions p1 < p2 in each of its chosen
  dimensions, re-integrating (so the series stays continuous), and then
  adding independent N(0, noise^2) noise to both copies;
* all planted windows are pairwise at least ``2 w`` apart.

Series are laid out ``[D][n]`` (each dimension contiguous), float64; FP32
workloads are produced by rounding once, so every consumer sees the same values.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Motif:
    dims: Tuple[int, ...]
    p1: int
    p2: int


@dataclasses.dataclass
class Series:
    x: np.ndarray            # [D][n] float64 (already rounded to fp32 when dtype == "f32")
    w: int
    motifs: List[Motif]
    dtype: str               # "f64" or "f32"

    @property
    def D(self) -> int:
        return self.x.shape[0]

    @property
    def n(self) -> int:
        return self.x.shape[1]

    def as_dtype(self) -> np.ndarray:
        """The series in its storage dtype, C-contiguous [D][n]."""
        if self.dtype == "f32":
            return np.ascontiguousarray(self.x.astype(np.float32))
        return np.ascontiguousarray(self.x)


def random_walk(rng: np.random.Generator, D: int, n: int) -> np.ndarray:
    return np.cumsum(rng.standard_normal((D, n)), axis=1)


def add_sinusoids(rng: np.random.Generator, x: np.ndarray,
                  period_lo: float = 50.0, period_hi: float = 5000.0) -> np.ndarray:
    D, n = x.shape
    t = np.arange(n, dtype=np.float64)
    out = x.copy()
    for f in range(D):
        period = math.exp(rng.uniform(math.log(period_lo), math.log(period_hi)))
        phase = rng.uniform(0.0, 2.0 * math.pi)
        amp = rng.uniform(0.5, 2.0) * math.sqrt(period)
        out[f] += amp * np.sin(2.0 * math.pi * t / period + phase)
    return out


def choose_positions(rng: np.random.Generator, n: int, w: int, count: int,
                     min_gap: int = 0, max_tries: int = 100000) -> List[Tuple[int, int]]:
    """Pick ``count`` (p1, p2) pairs; every planted window is >= 2w from every other."""
    n_s = n - w + 1
    taken: List[int] = []
    out: List[Tuple[int, int]] = []
    gap = max(2 * w, min_gap)
    for _ in range(max_tries):
        if len(out) == count:
            break
        p1, p2 = sorted(int(v) for v in rng.integers(0, n_s, size=2))
        if p2 - p1 < gap:
            continue
        if any(abs(p - q) < 2 * w for p in (p1, p2) for q in taken):
            continue
        taken += [p1, p2]
        out.append((p1, p2))
    if len(out) != count:
        raise ValueError(f"cannot place {count} motifs of length {w} in n={n}")
    return out


def plant(rng: np.random.Generator, x: np.ndarray, w: int, motifs: Sequence[Motif],
          noise: float) -> np.ndarray:
    """Plant each motif in increment space, re-integrate, then add noise to both copies."""
    inc = np.diff(x, axis=1)
    for m in motifs:
        for f in m.dims:
            snippet = rng.standard_normal(w - 1)
            inc[f, m.p1:m.p1 + w - 1] = snippet
            inc[f, m.p2:m.p2 + w - 1] = snippet
    out = np.concatenate([x[:, :1], x[:, :1] + np.cumsum(inc, axis=1)], axis=1)
    for m in motifs:
        for f in m.dims:
            out[f, m.p1:m.p1 + w] += noise * rng.standard_normal(w)
            out[f, m.p2:m.p2 + w] += noise * rng.standard_normal(w)
    return out


def plant_sine(rng: np.random.Generator, x: np.ndarray, w: int, motifs: Sequence[Motif],
               noise: float) -> np.ndarray:
    """Plant each motif as a sinusoid (period uniform in [w/10, w/2], amplitude
    1, random phase; one shape per dimension of the motif) written over both
    windows from the series' level at the window start, then add independent
    N(0, noise^2) noise to both copies."""
    out = x.copy()
    t = np.arange(w, dtype=np.float64)
    for m in motifs:
        for f in m.dims:
            period = rng.uniform(w / 10.0, w / 2.0)
            phase = rng.uniform(0.0, 2.0 * math.pi)
            shape = np.sin(2.0 * math.pi * t / period + phase)
            for p in (m.p1, m.p2):
                out[f, p:p + w] = out[f, p] + shape - shape[0] + noise * rng.standard_normal(w)
    return out


def make_series(seed: int, D: int, n: int, w: int, n_motifs: int, motif_dims: int,
                noise: float = 0.05, dtype: str = "f64", sinusoids: bool = False,
                min_gap: int = 0, motif: str = "walk") -> Series:
    rng = np.random.default_rng(seed)
    x = random_walk(rng, D, n)
    if sinusoids:
        x = add_sinusoids(rng, x)
    motifs: List[Motif] = []
    if n_motifs > 0:
        pos = choose_positions(rng, n, w, n_motifs, min_gap=min_gap)
        for p1, p2 in pos:
            dims = tuple(sorted(int(v) for v in rng.choice(D, size=motif_dims, replace=False)))
            motifs.append(Motif(dims, p1, p2))
        x = plant_sine(rng, x, w, motifs, noise) if motif == "sine" else plant(rng, x, w, motifs, noise)
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
    return Series(np.ascontiguousarray(x), w, motifs, dtype)


# The workloads the method is exercised on (sizes and distributions of the
# paper-scale problems; everything synthetic and seeded).
WORKLOADS = {
    # tiny plain case: D=4, n=2000, w=50, d=2, k=1, one motif in 2 dims, >=500 apart
    "tiny": dict(D=4, n=2000, w=50, d=2, k=1, delta=0.1, n_motifs=1, motif_dims=2,
                 dtype="f64", proj="f64", min_gap=500, mem_limit=1 << 30),
    # plain method at scale: D=8, n=1e6, w=300, d=3, k=10, delta=0.05, 8 GB cap, fp32
    "rw8_1m": dict(D=8, n=1_000_000, w=300, d=3, k=10, delta=0.05, n_motifs=10,
                   motif_dims=3, dtype="f32", proj="f32", mem_limit=8_000_000_000),
    # precision: D=32, n=4,194,304, w=1000, d=8, k=10, random walks + sinusoids;
    # r at r_scale times the estimate (with the estimate itself no step stops
    # above round 1 for these distances and d)
    "rwsin32_4m": dict(D=32, n=4_194_304, w=1000, d=8, k=10, delta=0.05, n_motifs=10,
                       motif_dims=8, dtype="f32", proj="bf16", compare_proj="f32", sinusoids=True,
                       mem_limit=64_000_000_000, r_scale=4.0),
    # large fp8: D=128, n=1e6, w=500, d=16, k=50, delta=0.01, 64 GB cap
    "rw128_1m": dict(D=128, n=1_000_000, w=500, d=16, k=50, delta=0.01, n_motifs=50,
                     motif_dims=16, dtype="f32", proj="fp8", mem_limit=64_000_000_000, r_scale=6.0),
    # the paper's scalability series (section 7, "Scalability"): D=5 random
    # walk, one sinusoidal motif of length 300 in 2 dimensions with Gaussian
    # noise, the top-1 2-dimensional motif; n from 1e4 to 1e8 (--n). Noise
    # 0.04 (per-dimension distance of the planted pair about 1.4) and r at 4
    # times the estimate: with the estimate itself no step stops above the
    # exact fallback at n = 2e4
    "scal5": dict(D=5, n=1_000_000, w=300, d=2, k=1, delta=0.1, n_motifs=1, motif_dims=2,
                  dtype="f32", proj="f32", motif="sine", noise=0.04, r_scale=4.0,
                  mem_limit=200_000_000_000),
}

DATA_SEED = {"tiny": 0xD00D01, "rw8_1m": 0xD00D02, "rwsin32_4m": 0xD00D03, "rw128_1m": 0xD00D05,
             "scal5": 0xD00D06}
LSH_SEED = {"tiny": 0x15A001, "rw8_1m": 0x15A002, "rwsin32_4m": 0x15A003, "rw128_1m": 0x15A005,
            "scal5": 0x15A006}


def workload(name: str, n: int | None = None, seed: int | None = None) -> Tuple[Series, dict]:
    """Series and parameters of a named workload (optionally at a reduced length n).
    With MOMENTI_SERIES_CACHE set to a directory, the drawn series is kept
    there (.npy) and loaded on later calls: the same values, drawn once."""
    p = dict(WORKLOADS[name])
    nn = p["n"] if n is None else n
    sd = DATA_SEED[name] if seed is None else seed
    cache = os.environ.get("MOMENTI_SERIES_CACHE")
    path = os.path.join(cache, f"{name}_{nn}_{sd:x}.npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path)
        motifs = [Motif(tuple(int(v) for v in row[2:] if v >= 0), int(row[0]), int(row[1]))
                  for row in z["motifs"]]
        s = Series(z["x"], p["w"], motifs, p["dtype"])
    else:
        s = make_series(sd, p["D"], nn, p["w"], p["n_motifs"], p["motif_dims"], dtype=p["dtype"],
                        sinusoids=p.get("sinusoids", False), min_gap=p.get("min_gap", 0),
                        noise=p.get("noise", 0.05), motif=p.get("motif", "walk"))
        if path:
            os.makedirs(cache, exist_ok=True)
            width = 2 + max((len(m.dims) for m in s.motifs), default=0)
            rows = np.full((len(s.motifs), width), -1, dtype=np.int64)
            for q, m in enumerate(s.motifs):
                rows[q, :2 + len(m.dims)] = [m.p1, m.p2, *m.dims]
            np.savez(path + ".tmp.npz", x=s.x, motifs=rows)
            os.replace(path + ".tmp.npz", path)
    p["n"] = nn
    return s, p


def batch_workload(seed: int, count: int = 512, n_lo: int = 10_000, n_hi: int = 500_000,
                   D_lo: int = 3, D_hi: int = 64, k: int = 5, n_motifs: int = 2):
    """Many independent series of uneven length and width: n log-uniform in
    [n_lo, n_hi], D uniform in [D_lo, D_hi], w in {50, 100, 200}, d = ceil(D/4),
    n_motifs planted motifs each."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))
        D = int(rng.integers(D_lo, D_hi + 1))
        w = int(rng.choice([50, 100, 200]))
        d = (D + 3) // 4
        ser = make_series(seed + 1 + s, D, n, w, n_motifs, d, dtype="f32")
        out.append((ser, dict(D=D, n=n, w=w, d=d, k=k, delta=0.1)))
    return out


# The many-series workloads: a fleet of independent series (k = 5 with two
# planted motifs, D up to 64: most searches need very long traversals), and a variant
# whose series can stop (k = planted motifs = 3, D in 5..16 so that d >= 2,
# r at 6 times the estimate: with the estimate itself half of them do not
# stop above the exact fallback or the work budget).
BATCHES = {
    "batch64": dict(count=64, n_lo=10_000, n_hi=200_000, D_lo=5, D_hi=16, k=3, n_motifs=3, r_scale=6.0),
    "batch64_k5": dict(count=64),
    # the fleet at full size: 512 series, n log-uniform in
    # [1e4, 5e5], D in 3..64, w in {50, 100, 200}, d = ceil(D / 4), k = 5,
    # two planted motifs each; r at 6 times the estimate
    "batch512": dict(count=512, r_scale=6.0),
}
BATCH_SEED = 0xD00D04
