"""Python binding of libmomenti (include/momenti.h): argument marshalling only.

Every step of the search runs in the HIP library; this module converts
arguments (numpy host arrays or torch device tensors), calls the C ABI and
turns results into Python objects. It never computes anything itself and has
no fallback: without a built ``libmomenti.so`` every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmomenti.so")

OK, OK_FALLBACK, OK_PARTIAL = 0, 1, 2
E_ARG, E_NOMEM, E_DEVICE, E_STATE, E_UNSUPPORTED = -1, -2, -3, -4, -5
F64, F32 = 0, 1
PROJ = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3}
STOP = {"tensor": 0, "lemma52": 1, "tensor_literal": 2, "rigorous": 3}
DELTA_MODE = {"per_motif": 0, "joint": 1}

EXPORTS = [
    "momenti_default_opts", "momenti_prepare", "momenti_hash", "momenti_search", "momenti_topk",
    "momenti_destroy", "momenti_last_error", "momenti_get_params", "momenti_get_stats",
    "momenti_get_hashes", "momenti_set_hashes", "momenti_set_trace", "momenti_get_profile",
    "momenti_set_profile",
    "momenti_topk_batch", "momenti_get_hash_words", "momenti_search_noalloc",
    "momenti_search_multi", "momenti_tune",
]


class Opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("K", C.c_int32), ("L", C.c_int32), ("r", C.c_double),
                ("r_scale", C.c_double),
                ("proj", C.c_int32), ("stop_rule", C.c_int32), ("series_on_device", C.c_int32),
                ("pool_size", C.c_int32), ("batch_reps", C.c_int32), ("profile", C.c_int32),
                ("merge_pairs", C.c_double), ("max_pairs", C.c_double), ("stream", C.c_void_p),
                ("delta_mode", C.c_int32), ("max_steps", C.c_int32), ("max_ms", C.c_double)]


class Job(C.Structure):
    _fields_ = [("series", C.c_void_p), ("n", C.c_int64), ("dtype", C.c_int32), ("D", C.c_int32),
                ("w", C.c_int32), ("d", C.c_int32), ("k", C.c_int32), ("delta", C.c_double)]


class KProf(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("launches", C.c_int64), ("ms", C.c_double),
                ("bytes", C.c_double), ("flops", C.c_double)]


class Motif(C.Structure):
    _fields_ = [("a", C.c_int64), ("b", C.c_int64), ("dist_d", C.c_double),
                ("dist_max", C.c_double), ("dims", C.c_uint64 * 2), ("fail_prob", C.c_double)]


class Report(C.Structure):
    _fields_ = [("t_hash_ms", C.c_double), ("t_search_ms", C.c_double),
                ("i_stop", C.c_int32), ("j_stop", C.c_int32), ("L_used", C.c_int32),
                ("K", C.c_int32), ("r", C.c_double), ("n_steps", C.c_int64),
                ("n_collisions", C.c_int64), ("n_cand", C.c_int64), ("n_verified", C.c_int64),
                ("peak_bytes", C.c_uint64), ("fallback", C.c_int32), ("pool_overflow", C.c_int32),
                ("batch_reps", C.c_int32), ("first_group_lo", C.c_int32),
                ("budget_round", C.c_int32), ("max_run", C.c_int32),
                ("group_splits", C.c_int32), ("step_parts", C.c_int32), ("fail_bound", C.c_double)]


class MomentiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"momenti error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmomenti.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, P = C.c_void_p, C.POINTER
        i32, i64, u64, d = C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "momenti_default_opts": (None, [P(Opts)]),
            "momenti_prepare": (i32, [P(vp), i64, i32, i32, i32, u64, P(Opts)]),
            "momenti_hash": (i32, [vp, vp]),
            "momenti_search": (i32, [vp, i32, i32, d, P(Motif), P(i32), P(Report)]),
            "momenti_search_noalloc": (i32, [vp, i32, i32, d, P(Motif), P(i32), P(Report)]),
            "momenti_search_multi": (i32, [vp, i32, i32, i32, d, P(Motif), P(i32), P(i32), P(Report)]),
            "momenti_tune": (i32, [vp, i32, i32, d, P(i32), i32, P(i32), P(d)]),
            "momenti_topk": (i32, [vp, i32, i64, i32, i32, i32, i32, d, u64, P(Opts), P(Motif),
                                   P(i32), P(Report)]),
            "momenti_destroy": (None, [vp]),
            "momenti_last_error": (C.c_char_p, []),
            "momenti_get_params": (i32, [vp, P(d), P(i32), P(i32), P(i32)]),
            "momenti_get_stats": (i32, [vp, vp, vp, C.c_size_t]),
            "momenti_get_hashes": (i32, [vp, vp, C.c_size_t]),
            "momenti_set_hashes": (i32, [vp, vp, C.c_size_t]),
            "momenti_get_hash_words": (i32, [vp, i32, i64, i64, vp]),
            "momenti_set_trace": (i32, [vp, vp, i64, vp, vp, vp, i64, i32]),
            "momenti_get_profile": (i32, [vp, P(KProf), i32, P(i32), i32]),
            "momenti_set_profile": (i32, [vp, i32]),
            "momenti_topk_batch": (i32, [P(Job), i32, u64, P(Opts), i32, P(Motif), P(i32), P(i32),
                                         P(Report)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise MomentiError(rc, lib().momenti_last_error().decode())
    return rc


def make_opts(seed: int = 0x5EED, K: int = 8, L: int = 200, r: float = 0.0, proj: str = "f32",
              stop: str = "tensor", series_on_device: bool = False, pool_size: int = 0,
              batch_reps: int = 0, profile: int = 0, stream: Optional[int] = None,
              r_scale: float = 1.0, max_pairs: float = 0.0, merge_pairs: float = 0.0,
              delta_mode: str = "per_motif", max_steps: int = 0, max_ms: float = 0.0) -> Opts:
    o = Opts()
    lib().momenti_default_opts(C.byref(o))
    o.seed, o.K, o.L, o.r, o.r_scale, o.max_pairs = seed, K, L, r, r_scale, max_pairs
    o.delta_mode, o.max_steps, o.max_ms = DELTA_MODE[delta_mode], max_steps, max_ms
    o.merge_pairs = merge_pairs
    o.proj, o.stop_rule = PROJ[proj], STOP[stop]
    o.series_on_device = 1 if series_on_device else 0
    o.pool_size, o.batch_reps = pool_size, batch_reps
    o.profile = int(profile)
    o.stream = stream
    return o


def _motifs(arr, count: int) -> List[Dict]:
    out = []
    for m in arr[:count]:
        dims = tuple(f for f in range(128) if (int(m.dims[f >> 6]) >> (f & 63)) & 1)
        out.append(dict(a=int(m.a), b=int(m.b), dist_d=float(m.dist_d),
                        dist_max=float(m.dist_max), dims=dims, fail_prob=float(m.fail_prob)))
    return out


def _report(r: Report) -> Dict:
    return {name: getattr(r, name) for name, _ in Report._fields_}


def _torch_stream_handle() -> Optional[int]:
    import torch
    return torch.cuda.current_stream().cuda_stream


class Plan:
    """A prepared search (momenti_prepare); owns the device index."""

    def __init__(self, n: int, D: int, w: int, dtype: str = "f32", mem_limit: int = 8 << 30,
                 device_series: bool = False, **opts):
        if device_series and "stream" not in opts:
            opts["stream"] = _torch_stream_handle()
        self.opts = make_opts(series_on_device=device_series, **opts)
        self.n, self.D, self.w = n, D, w
        self.dtype = dtype
        self.device_series = device_series
        self._series_ref = None
        h = C.c_void_p()
        _check(lib().momenti_prepare(C.byref(h), n, D, w, F64 if dtype == "f64" else F32,
                                     mem_limit, C.byref(self.opts)))
        self.h = h
        self._trace_bufs = None

    # -- lifecycle
    def close(self) -> None:
        if getattr(self, "h", None):
            lib().momenti_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- calls
    def hash(self, series) -> None:
        """series: numpy [D][n] (host plan) or a contiguous torch CUDA tensor (device plan)."""
        if self.device_series:
            assert series.is_cuda and series.is_contiguous()
            want = "torch.float64" if self.dtype == "f64" else "torch.float32"
            assert str(series.dtype) == want, f"series dtype {series.dtype} != {want}"
            assert tuple(series.shape) == (self.D, self.n)
            self._series_ref = series
            ptr = C.c_void_p(series.data_ptr())
        else:
            arr = np.ascontiguousarray(series, dtype=np.float64 if self.dtype == "f64" else np.float32)
            assert arr.shape == (self.D, self.n)
            self._series_ref = arr
            ptr = arr.ctypes.data_as(C.c_void_p)
        _check(lib().momenti_hash(self.h, ptr))

    def search(self, d: int, k: int, delta: float) -> Tuple[List[Dict], Dict, int]:
        arr = (Motif * max(k, 1))()
        got = C.c_int32()
        rep = Report()
        rc = _check(lib().momenti_search(self.h, d, k, delta, arr, C.byref(got), C.byref(rep)))
        return _motifs(arr, got.value), _report(rep), rc

    def search_noalloc(self, d: int, k: int, delta: float) -> Tuple[List[Dict], Dict, int]:
        """momenti_search_noalloc: the same search, its buffers in the library's scratch area."""
        arr = (Motif * max(k, 1))()
        got = C.c_int32()
        rep = Report()
        rc = _check(lib().momenti_search_noalloc(self.h, d, k, delta, arr, C.byref(got), C.byref(rep)))
        return _motifs(arr, got.value), _report(rep), rc

    def search_multi(self, d_lo: int, d_hi: int, k: int, delta: float) -> Dict[int, Tuple[List[Dict], Dict, int]]:
        """momenti_search_multi: {d: (motifs, report, status)} for every d in [d_lo, d_hi]."""
        nd = max(d_hi - d_lo + 1, 1)
        arr = (Motif * (nd * max(k, 1)))()
        got = (C.c_int32 * nd)()
        status = (C.c_int32 * nd)()
        reps = (Report * nd)()
        _check(lib().momenti_search_multi(self.h, d_lo, d_hi, k, delta, arr, got, status, reps))
        return {d_lo + q: (_motifs(arr[q * k:(q + 1) * k], got[q]), _report(reps[q]), status[q])
                for q in range(nd)}

    def tune(self, d: int, k: int, delta: float, cands=(4, 8, 16, 32)) -> Tuple[int, float]:
        """momenti_tune: the fastest repetitions per launch among cands (kept by the plan)."""
        arr = (C.c_int32 * len(cands))(*cands)
        best, ms = C.c_int32(), C.c_double()
        _check(lib().momenti_tune(self.h, d, k, delta, arr, len(cands), C.byref(best), C.byref(ms)))
        return best.value, ms.value

    def params(self) -> Dict:
        r, L, nl, nr = C.c_double(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().momenti_get_params(self.h, C.byref(r), C.byref(L), C.byref(nl), C.byref(nr)))
        return dict(r=r.value, L=L.value, n_left=nl.value, n_right=nr.value,
                    NF=nl.value + nr.value)

    def stats(self) -> Tuple[np.ndarray, np.ndarray]:
        ns = self.n - self.w + 1
        mu = np.zeros((self.D, ns)); isg = np.zeros((self.D, ns))
        _check(lib().momenti_get_stats(self.h, mu.ctypes.data_as(C.c_void_p),
                                       isg.ctypes.data_as(C.c_void_p), mu.size))
        return mu, isg

    def hashes(self) -> np.ndarray:
        ns = self.n - self.w + 1
        NF = self.params()["NF"]
        out = np.zeros((self.D, NF, ns), dtype=np.uint32)
        _check(lib().momenti_get_hashes(self.h, out.ctypes.data_as(C.c_void_p), out.size))
        return out

    def hash_words(self, f: int, a0: int, count: int) -> np.ndarray:
        """Index words [n_left + n_right][count] of windows a0 .. a0+count-1 of dimension f."""
        out = np.zeros((self.params()["NF"], count), dtype=np.uint32)
        _check(lib().momenti_get_hash_words(self.h, f, a0, count, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_hashes(self, words: np.ndarray) -> None:
        words = np.ascontiguousarray(words, dtype=np.uint32)
        _check(lib().momenti_set_hashes(self.h, words.ctypes.data_as(C.c_void_p), words.size))

    def profile(self, clear: bool = False) -> Dict[str, Dict]:
        """Per-kernel totals (launches, ms, algorithmic bytes, flops) when profiling is on."""
        recs = (KProf * 32)()
        n = C.c_int32()
        _check(lib().momenti_get_profile(self.h, recs, 32, C.byref(n), 1 if clear else 0))
        return {r.name.decode(): dict(launches=r.launches, ms=r.ms, bytes=r.bytes, flops=r.flops)
                for r in recs[:n.value]}

    def set_profile(self, mode: int) -> None:
        """0 off, 1 every kernel launch, 2 only the pair enumeration."""
        _check(lib().momenti_set_profile(self.h, int(mode)))

    def set_trace(self, cand_cap: int, k: int) -> None:
        K, L = self.opts.K, self.params()["L"]
        steps = K * L
        cand = np.zeros((cand_cap, 3), dtype=np.int64)
        cnt = np.zeros(1, dtype=np.int64)
        tsz = np.zeros(steps, dtype=np.int32)
        tpairs = np.zeros((steps, k, 2), dtype=np.int64)
        self._trace_bufs = (cand, cnt, tsz, tpairs)
        _check(lib().momenti_set_trace(self.h, cand.ctypes.data_as(C.c_void_p), cand_cap,
                                       cnt.ctypes.data_as(C.c_void_p), tsz.ctypes.data_as(C.c_void_p),
                                       tpairs.ctypes.data_as(C.c_void_p), steps, k))

    def trace(self) -> Dict:
        cand, cnt, tsz, tpairs = self._trace_bufs
        c = int(cnt[0])
        if c > cand.shape[0]:
            raise RuntimeError(f"trace truncated ({c} > {cand.shape[0]})")
        return dict(cand=cand[:c].copy(), top_size=tsz.copy(), top_pairs=tpairs.copy())


def topk(series, w: int, d: int, k: int, delta: float, mem_limit: int = 8 << 30,
         dtype: str = "f32", **opts) -> Tuple[List[Dict], Dict, int]:
    """One call: prepare + hash + search + destroy (momenti_topk)."""
    if hasattr(series, "is_cuda") and series.is_cuda:
        with Plan(series.shape[1], series.shape[0], w, dtype, mem_limit, device_series=True,
                  **opts) as p:
            p.hash(series)
            return p.search(d, k, delta)
    arr = np.ascontiguousarray(series, dtype=np.float64 if dtype == "f64" else np.float32)
    o = make_opts(**opts)
    out = (Motif * max(k, 1))()
    got = C.c_int32()
    rep = Report()
    rc = _check(lib().momenti_topk(arr.ctypes.data_as(C.c_void_p), F64 if dtype == "f64" else F32,
                                   arr.shape[1], arr.shape[0], w, d, k, delta, mem_limit,
                                   C.byref(o), out, C.byref(got), C.byref(rep)))
    return _motifs(out, got.value), _report(rep), rc


def topk_batch(jobs, mem_limit: int = 8 << 30, workers: int = 4, dtype: str = "f32",
               **opts) -> Tuple[List[Tuple[List[Dict], Dict, int]], int]:
    """Many independent series at once (momenti_topk_batch). jobs: sequence of
    dicts with keys series ([D][n] numpy array, or torch CUDA tensors for all
    jobs), w, d, k, delta. Returns ([(motifs, report, status) per job], rc)."""
    on_dev = [hasattr(j["series"], "is_cuda") and j["series"].is_cuda for j in jobs]
    if any(on_dev) and not all(on_dev):
        raise ValueError("either every series is a CUDA tensor or none is")
    dev = bool(jobs) and all(on_dev)
    keep = []
    arr = (Job * max(len(jobs), 1))()
    for q, j in enumerate(jobs):
        x = j["series"]
        if dev:
            x = x.contiguous()
            ptr = x.data_ptr()
        else:
            x = np.ascontiguousarray(x, dtype=np.float64 if dtype == "f64" else np.float32)
            ptr = x.ctypes.data
        keep.append(x)
        arr[q] = Job(ptr, x.shape[1], F64 if dtype == "f64" else F32, x.shape[0], j["w"], j["d"],
                     j["k"], j["delta"])
    if dev:
        import torch
        torch.cuda.synchronize()
    opts.pop("stream", None)
    o = make_opts(series_on_device=dev, **opts)
    total = sum(j["k"] for j in jobs)
    out = (Motif * max(total, 1))()
    n_out = (C.c_int32 * max(len(jobs), 1))()
    status = (C.c_int32 * max(len(jobs), 1))()
    not_run = -(1 << 30)
    for q in range(len(jobs)):
        status[q] = not_run
    reps = (Report * max(len(jobs), 1))()
    rc = lib().momenti_topk_batch(arr, len(jobs), mem_limit, C.byref(o), workers, out, n_out, status, reps)
    # an error before any job ran (bad arguments of the call) raises; a job's
    # own error is left in its status, beside the other jobs' answers
    if rc < 0 and all(status[q] == not_run for q in range(len(jobs))):
        _check(rc)
    res, off = [], 0
    for q, j in enumerate(jobs):
        res.append((_motifs(out[off:off + j["k"]], n_out[q]), _report(reps[q]), int(status[q])))
        off += j["k"]
    return res, rc
