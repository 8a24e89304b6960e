"""ctypes driver of the C oracle (``momenti_oracle.c``). Test infrastructure only.

Every function takes and returns numpy arrays; the arithmetic lives in the C
file, each routine there citing the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "build", "lib", "philox", "gauss", "uniform", "window_stats", "stats", "dist", "distd",
    "topk_exact", "topk_exact_sweep", "tensor_shape", "L_used", "draw_projections", "estimate_r", "hash_dim",
    "hash_one", "hash_all", "pack", "prefix", "collision_prob", "fail_bound", "stop", "lsh_search",
    "lsh_pipeline", "STOP_TENSOR", "STOP_LEMMA52", "STOP_TENSOR_LITERAL", "STOP_RIGOROUS", "FLAT_REL", "round_fmt", "round_fmt_array", "hash_dim_lowp", "FMT",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "momenti_oracle.c"), os.path.join(_HERE, "o1fast.c")]
_LIB = os.path.join(_HERE, "_build", "libmomenti_oracle.so")
# the same sources with OpenMP: the CPU baseline (all host cores) and the
# golden-file sweeps; identical results, the sequential build is the checker
_LIB_OMP = os.path.join(_HERE, "_build", "libmomenti_oracle_omp.so")

STOP_TENSOR = 0
STOP_LEMMA52 = 1
STOP_TENSOR_LITERAL = 2
STOP_RIGOROUS = 3
FLAT_REL = 1e-8


def _stale(path: str) -> bool:
    return not os.path.exists(path) or os.path.getmtime(path) < max(os.path.getmtime(s) for s in _SRCS)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction), once
    sequential (the checker) and once with OpenMP."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    flags = ["-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fPIC"]
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or _stale(out):
            tmp = out + ".tmp"
            objs = []
            for src in _SRCS:
                # the sweep's fixed-width loops over diagonals vectorise at -O3
                opt = "-O3" if src.endswith("o1fast.c") else "-O2"
                obj = tmp + "." + os.path.basename(src) + ".o"
                subprocess.check_call(["gcc", opt, *flags, *extra, "-c", "-o", obj, src])
                objs.append(obj)
            subprocess.check_call(["gcc", "-shared", *extra, "-o", tmp, *objs, "-lm"])
            for obj in objs:
                os.remove(obj)
            os.replace(tmp, out)
    return _LIB


class Motif(C.Structure):
    _fields_ = [("a", C.c_int64), ("b", C.c_int64), ("dist_d", C.c_double),
                ("dist_max", C.c_double), ("dims", C.c_uint64 * 2)]


class LshCtl(C.Structure):
    _fields_ = [("K", C.c_int32), ("L", C.c_int32), ("rule", C.c_int32), ("no_fallback", C.c_int32),
                ("r", C.c_double),
                ("cand", C.POINTER(C.c_int64)), ("cand_cap", C.c_int64), ("cand_count", C.c_int64),
                ("top_size", C.POINTER(C.c_int32)), ("top_pairs", C.POINTER(C.c_int64)),
                ("top_distmax", C.POINTER(C.c_double)),
                ("i_stop", C.c_int32), ("J_stop", C.c_int32),
                ("n_verified", C.c_int64), ("n_collisions", C.c_int64)]


_libs = {}


def lib(omp: bool = False):
    """The sequential oracle (omp=False, the checker) or its OpenMP build."""
    if omp not in _libs:
        path = _LIB_OMP if omp else _LIB
        if _stale(path):
            build(force=True)
        L = C.CDLL(path)
        P = C.POINTER
        d, i32, i64, u64 = C.c_double, C.c_int32, C.c_int64, C.c_uint64
        vp = C.c_void_p
        sig = {
            "orc_philox4x32_10": (None, [vp, vp, vp]),
            "orc_gauss": (d, [u64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
            "orc_uniform": (d, [u64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]),
            "orc_window_stats": (None, [vp, i32, P(d), P(d), P(i32)]),
            "orc_stats": (None, [vp, i64, i32, i32, vp, vp, vp]),
            "orc_dist": (d, [vp, vp, i32]),
            "orc_distd": (None, [vp, i64, i32, i32, i64, i64, i32, P(d), P(d), vp, vp]),
            "orc_topk_exact": (i32, [vp, i64, i32, i32, i32, i32, vp]),
            "orc_tensor_shape": (None, [i32, P(i32), P(i32), P(i32)]),
            "orc_L_used": (i32, [i64, i32, i32, i32, i32, u64]),
            "orc_draw_projections": (None, [u64, i32, i32, i32, vp, vp]),
            "orc_estimate_r": (d, [vp, i64, i32, i32, u64]),
            "orc_hash_value": (i32, [vp, i32, vp, i64, d, d, P(d), P(d)]),
            "orc_hash_dim": (None, [vp, i64, i32, vp, vp, i32, d, vp, vp, vp]),
            "orc_hash_one": (None, [vp, i32, i64, vp, vp, i32, d, vp, vp, vp]),
            "orc_hash_all": (None, [vp, i64, i32, i32, vp, vp, i32, d, vp]),
            "orc_topk_exact_sweep": (i32, [vp, i64, i32, i32, i32, i32, i64, vp, vp]),
            "orc_pack": (None, [vp, i64, i32, i32, i32, vp]),
            "orc_round_fmt": (d, [d, i32]),
            "orc_round_fmt_array": (None, [vp, i64, i32, vp]),
            "orc_hash_value_lowp": (i32, [vp, i32, vp, i64, d, d, i32, P(d), P(d), P(d)]),
            "orc_hash_dim_lowp": (None, [vp, i64, i32, vp, vp, i32, d, i32, vp, vp, vp, vp]),
            "orc_prefix": (u64, [vp, i64, i32, i32, i32, i32, i32, i64, i32]),
            "orc_collision_prob": (d, [d, d]),
            "orc_fail_bound": (d, [d, i32, i32, i32, i32, i32]),
            "orc_stop": (i32, [d, d, i32, i32, i32, i32, i32, i32, d]),
            "orc_lsh_search": (i32, [vp, i64, i32, i32, i32, i32, d, vp, P(LshCtl), vp]),
            "orc_motif_size": (i32, []),
            "orc_ctl_size": (i32, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        assert L.orc_motif_size() == C.sizeof(Motif)
        assert L.orc_ctl_size() == C.sizeof(LshCtl)
        _libs[omp] = L
    return _libs[omp]


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ----------------------------------------------------------------------------- RNG
def philox(ctr, key) -> List[int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(o))
    return [int(v) for v in o]


def gauss(seed: int, c0: int, c1: int, c2: int, purpose: int) -> float:
    return lib().orc_gauss(seed, c0, c1, c2, purpose)


def uniform(seed: int, c0: int, c1: int, c2: int, purpose: int) -> float:
    return lib().orc_uniform(seed, c0, c1, c2, purpose)


# ----------------------------------------------------------------------------- section 3.1
def window_stats(xw) -> tuple:
    xw = _f64(xw)
    mu, sg, fl = C.c_double(), C.c_double(), C.c_int32()
    lib().orc_window_stats(_p(xw), len(xw), C.byref(mu), C.byref(sg), C.byref(fl))
    return mu.value, sg.value, bool(fl.value)


def stats(x, w: int):
    x = _f64(x)
    D, n = x.shape
    ns = n - w + 1
    mu = np.zeros((D, ns)); sg = np.zeros((D, ns)); fl = np.zeros((D, ns), dtype=np.int32)
    lib().orc_stats(_p(x), n, D, w, _p(mu), _p(sg), _p(fl))
    return mu, sg, fl.astype(bool)


def dist(xa, xb) -> float:
    xa, xb = _f64(xa), _f64(xb)
    return lib().orc_dist(_p(xa), _p(xb), len(xa))


def distd(x, w: int, a: int, b: int, d: int):
    """(dist_d, dist_max, sorted dims tuple, per-dimension distances)."""
    x = _f64(x)
    D, n = x.shape
    dd, dm = C.c_double(), C.c_double()
    mask = np.zeros(2, dtype=np.uint64)
    per = np.zeros(D)
    lib().orc_distd(_p(x), n, D, w, a, b, d, C.byref(dd), C.byref(dm), _p(mask), _p(per))
    dims = tuple(f for f in range(D) if (int(mask[f >> 6]) >> (f & 63)) & 1)
    return dd.value, dm.value, dims, per


def _motifs(arr, count) -> List[dict]:
    out = []
    for m in arr[:count]:
        dims = tuple(f for f in range(128) if (int(m.dims[f >> 6]) >> (f & 63)) & 1)
        out.append(dict(a=int(m.a), b=int(m.b), dist_d=float(m.dist_d), dist_max=float(m.dist_max),
                        dims=dims))
    return out


def topk_exact(x, w: int, d: int, k: int) -> List[dict]:
    x = _f64(x)
    D, n = x.shape
    arr = (Motif * max(k, 1))()
    got = lib().orc_topk_exact(_p(x), n, D, w, d, k, C.cast(arr, C.c_void_p))
    if got < 0:
        raise MemoryError("oracle brute force could not allocate")
    return _motifs(arr, got)


def topk_exact_sweep(x, w: int, d: int, k: int, pool: int = 1 << 16, omp: bool = True,
                     info: Optional[dict] = None) -> List[dict]:
    """The answer of topk_exact by a diagonal sweep (o1fast.c), for long inputs."""
    x = _f64(x)
    D, n = x.shape
    arr = (Motif * max(k, 1))()
    inf = np.zeros(5)
    got = lib(omp).orc_topk_exact_sweep(_p(x), n, D, w, d, k, pool, C.cast(arr, C.c_void_p), _p(inf))
    if got == -1:
        raise MemoryError("oracle sweep could not allocate")
    if got < 0:
        raise RuntimeError("oracle sweep could not certify its answer")
    if info is not None:
        info.update(theta=inf[0], eps=inf[1], pool=int(inf[2]), passes=int(inf[3]), max_err=inf[4])
    return _motifs(arr, got)


# ----------------------------------------------------------------------------- sections 3.2, 6.1
def tensor_shape(L: int):
    m, nl, nr = C.c_int32(), C.c_int32(), C.c_int32()
    lib().orc_tensor_shape(L, C.byref(m), C.byref(nl), C.byref(nr))
    return m.value, nl.value, nr.value


def L_used(n: int, D: int, w: int, L_max: int, elem_bytes: int, mem_limit: int) -> int:
    return lib().orc_L_used(n, D, w, L_max, elem_bytes, mem_limit)


def draw_projections(seed: int, D: int, w: int, Ccols: int):
    R = np.zeros((D, w, Ccols)); U = np.zeros((D, Ccols))
    lib().orc_draw_projections(seed, D, w, Ccols, _p(R), _p(U))
    return R, U


def estimate_r(x, w: int, seed: int) -> float:
    x = _f64(x)
    D, n = x.shape
    return lib().orc_estimate_r(_p(x), n, D, w, seed)


def hash_dim(xf, w: int, Rf, Uf, r: float, want_pre: bool = True):
    xf, Rf, Uf = _f64(xf), _f64(Rf), _f64(Uf)
    n = len(xf); ns = n - w + 1; Cc = Rf.shape[1]
    by = np.zeros((ns, Cc), dtype=np.uint8)
    pre = np.zeros((ns, Cc)) if want_pre else None
    sab = np.zeros((ns, Cc)) if want_pre else None
    lib().orc_hash_dim(_p(xf), n, w, _p(Rf), _p(Uf), Cc, r, _p(by),
                       _p(pre) if want_pre else None, _p(sab) if want_pre else None)
    return by, pre, sab


def hash_one(xf, w: int, a: int, Rf, Uf, r: float):
    xf, Rf, Uf = _f64(xf), _f64(Rf), _f64(Uf)
    Cc = Rf.shape[1]
    by = np.zeros(Cc, dtype=np.uint8); pre = np.zeros(Cc); sab = np.zeros(Cc)
    lib().orc_hash_one(_p(xf), w, a, _p(Rf), _p(Uf), Cc, r, _p(by), _p(pre), _p(sab))
    return by, pre, sab


FMT = {"bf16": 2, "fp8": 3}


def round_fmt(v: float, fmt: str) -> float:
    return lib().orc_round_fmt(v, FMT[fmt])


def round_fmt_array(v, fmt: str) -> np.ndarray:
    v = _f64(v).ravel()
    out = np.empty_like(v)
    lib().orc_round_fmt_array(_p(v), v.size, FMT[fmt], _p(out))
    return out


def hash_dim_lowp(xf, w: int, Rf, Uf, r: float, fmt: str):
    """Symbols, pre-floor values, sum |.| and ambiguity bound of the rounded-input projection."""
    xf, Rf, Uf = _f64(xf), _f64(Rf), _f64(Uf)
    n = len(xf); ns = n - w + 1; Cc = Rf.shape[1]
    by = np.zeros((ns, Cc), dtype=np.uint8)
    pre = np.zeros((ns, Cc)); sab = np.zeros((ns, Cc)); amb = np.zeros((ns, Cc))
    lib().orc_hash_dim_lowp(_p(xf), n, w, _p(Rf), _p(Uf), Cc, r, FMT[fmt], _p(by), _p(pre),
                            _p(sab), _p(amb))
    return by, pre, sab, amb


def pack(bytes_: np.ndarray, NF: int, K: int) -> np.ndarray:
    """bytes_ [D][n_s][4*NF] -> words [D][NF][n_s] (uint32)."""
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    D, ns, _ = b.shape
    words = np.zeros((D, NF, ns), dtype=np.uint32)
    lib().orc_pack(_p(b), ns, D, NF, K, _p(words))
    return words


def prefix(words, L: int, f: int, j: int, a: int, i: int) -> int:
    words = np.ascontiguousarray(words, dtype=np.uint32)
    D, NF, ns = words.shape
    m, nl, _ = tensor_shape(L)
    return int(lib().orc_prefix(_p(words), ns, NF, nl, m, f, j, a, i))


# ----------------------------------------------------------------------------- Eq. 423, Alg. 2
def collision_prob(R: float, r: float) -> float:
    return lib().orc_collision_prob(R, r)


def fail_bound(p: float, i: int, J: int, K: int, L: int, rule: int = STOP_TENSOR) -> float:
    return lib().orc_fail_bound(p, i, J, K, L, rule)


def stop(dist_max: float, r: float, d: int, i: int, J: int, K: int, L: int, rule: int,
         delta: float) -> bool:
    return bool(lib().orc_stop(dist_max, r, d, i, J, K, L, rule, delta))


# ----------------------------------------------------------------------------- Algorithm 1
def lsh_search(x, w: int, d: int, k: int, delta: float, words, K: int, L: int, r: float,
               rule: int = STOP_TENSOR, trace: bool = False, cand_cap: int = 2_000_000,
               omp: bool = False, fallback: bool = True) -> Dict:
    """Algorithm 1 over a given index. fallback=False skips the exact answer
    when no step stops (motifs is then empty; the steps are still traced)."""
    x = _f64(x)
    D, n = x.shape
    words = np.ascontiguousarray(words, dtype=np.uint32)
    ctl = LshCtl()
    ctl.K, ctl.L, ctl.rule, ctl.r = K, L, rule, r
    ctl.no_fallback = 0 if fallback else 1
    keep = []
    if trace:
        cand = np.zeros((cand_cap, 3), dtype=np.int64)
        tsz = np.zeros(K * L, dtype=np.int32)
        tpairs = np.zeros((K * L, max(k, 1), 2), dtype=np.int64)
        tdm = np.zeros(K * L)
        keep = [cand, tsz, tpairs, tdm]
        ctl.cand = cand.ctypes.data_as(C.POINTER(C.c_int64))
        ctl.cand_cap = cand_cap
        ctl.top_size = tsz.ctypes.data_as(C.POINTER(C.c_int32))
        ctl.top_pairs = tpairs.ctypes.data_as(C.POINTER(C.c_int64))
        ctl.top_distmax = tdm.ctypes.data_as(C.POINTER(C.c_double))
    arr = (Motif * max(k, 1))()
    got = lib(omp).orc_lsh_search(_p(x), n, D, w, d, k, delta, _p(words), C.byref(ctl),
                                  C.cast(arr, C.c_void_p))
    out = dict(motifs=_motifs(arr, got), i_stop=ctl.i_stop, J_stop=ctl.J_stop,
               n_verified=ctl.n_verified, n_collisions=ctl.n_collisions,
               fallback=(ctl.i_stop == 0))
    if trace:
        cand, tsz, tpairs, tdm = keep
        cnt = int(ctl.cand_count)
        if cnt > cand_cap:
            raise RuntimeError(f"candidate trace truncated ({cnt} > {cand_cap})")
        out.update(cand=cand[:cnt].copy(), top_size=tsz, top_pairs=tpairs, top_distmax=tdm)
    return out


def hash_all(x, w: int, R, U, r: float, omp: bool = False) -> np.ndarray:
    """Symbols [D][n_s][C] of every window of every dimension (Eq. drp)."""
    x, R, U = _f64(x), _f64(R), _f64(U)
    D, n = x.shape
    Cc = R.shape[2]
    by = np.zeros((D, n - w + 1, Cc), dtype=np.uint8)
    lib(omp).orc_hash_all(_p(x), n, D, w, _p(R), _p(U), Cc, r, _p(by))
    return by


def lsh_pipeline(x, w: int, d: int, k: int, delta: float, seed: int, K: int = 8,
                 L_max: int = 200, mem_limit: Optional[int] = None, elem_bytes: int = 8,
                 r: Optional[float] = None, rule: int = STOP_TENSOR, trace: bool = False,
                 r_scale: float = 1.0, omp: bool = False) -> Dict:
    """The whole method: L under the memory cap, draws, r, hashes, packing, search.
    Without an explicit r, r is r_scale times the section 6.1 estimate. omp
    runs the OpenMP build of the oracle (same results)."""
    x = _f64(x)
    D, n = x.shape
    L = L_max if mem_limit is None else L_used(n, D, w, L_max, elem_bytes, mem_limit)
    if L < 1:
        raise MemoryError("memory limit below the smallest index")
    m, nl, nr = tensor_shape(L)
    NF = nl + nr
    Ccols = 4 * NF
    R, U = draw_projections(seed, D, w, Ccols)
    rr = estimate_r(x, w, seed) * (r_scale if r_scale > 0 else 1.0) if r is None else float(r)
    by = hash_all(x, w, R, U, rr, omp=omp)
    words = pack(by, NF, K)
    res = lsh_search(x, w, d, k, delta, words, K, L, rr, rule=rule, trace=trace, omp=omp)
    res.update(L=L, r=rr, words=words, R=R, U=U, NF=NF, m=m, n_left=nl)
    return res
