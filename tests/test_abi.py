"""The C ABI library loads and exports every entry point its header declares
(no GPU needed: only dlopen and symbol lookup), and the binding fails loudly
without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "momenti.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(momenti_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("momenti_prepare", "momenti_hash", "momenti_search", "momenti_topk",
                 "momenti_destroy", "momenti_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2502_14446_amd import momenti as mm
    if not os.path.exists(mm.LIB_PATH):
        from paper_2502_14446_amd import build
        build.build()
    lib = ctypes.CDLL(mm.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(mm.EXPORTS) == _declared()


def test_argument_errors_are_reported_without_touching_a_gpu():
    from paper_2502_14446_amd import momenti as mm
    lib = mm.lib()
    h = ctypes.c_void_p()
    o = mm.make_opts()
    # n shorter than w + 1
    assert lib.momenti_prepare(ctypes.byref(h), 10, 2, 50, 1, 1 << 30, ctypes.byref(o)) == mm.E_ARG
    assert b"shorter" in lib.momenti_last_error()
    # odd K
    o.K = 5
    assert lib.momenti_prepare(ctypes.byref(h), 1000, 2, 50, 1, 1 << 30, ctypes.byref(o)) == mm.E_ARG
    o.K = 8
    # more repetitions than the projection's 128 hash columns serve (L <= 256)
    o.L = 257
    assert lib.momenti_prepare(ctypes.byref(h), 1000, 2, 50, 1, 1 << 30, ctypes.byref(o)) == mm.E_ARG
    assert b"L=257 outside [1, 256]" in lib.momenti_last_error()
    o.L = 200
    # mem_limit below the one-repetition index
    assert lib.momenti_prepare(ctypes.byref(h), 1000, 2, 50, 1, 1 << 20, ctypes.byref(o)) == mm.E_NOMEM
    # the BF16 projection's work-group tile (four shifted copies of the series
    # tile and two chunks of projection rows) must fit a CU's 160 KiB of LDS:
    # w <= 7616 with 128 hash columns (refused before the device is touched)
    ob = mm.make_opts(proj="bf16")
    assert lib.momenti_prepare(ctypes.byref(h), 9000, 1, 8192, 1, 1 << 30, ctypes.byref(ob)) == mm.E_ARG
    assert b"too long for the BF16 projection" in lib.momenti_last_error()
    assert b"at most 7616" in lib.momenti_last_error()
    # search on a NULL plan
    out = (mm.Motif * 1)()
    n = ctypes.c_int32()
    assert lib.momenti_search(None, 1, 1, 0.1, out, ctypes.byref(n), None) == mm.E_ARG


def test_batch_argument_errors_are_reported_without_touching_a_gpu():
    from paper_2502_14446_amd import momenti as mm
    lib = mm.lib()
    o = mm.make_opts()
    out = (mm.Motif * 4)()
    n = (ctypes.c_int32 * 2)()
    st = (ctypes.c_int32 * 2)()
    jobs = (mm.Job * 2)()
    # no jobs: nothing to do
    assert lib.momenti_topk_batch(jobs, 0, 1 << 30, ctypes.byref(o), 2, out, n, st, None) == mm.OK
    assert lib.momenti_topk_batch(jobs, -1, 1 << 30, ctypes.byref(o), 2, out, n, st, None) == mm.E_ARG
    assert lib.momenti_topk_batch(None, 2, 1 << 30, ctypes.byref(o), 2, out, n, st, None) == mm.E_ARG
    jobs[0].k = jobs[1].k = 2
    assert lib.momenti_topk_batch(jobs, 2, 1 << 30, ctypes.byref(o), 0, out, n, st, None) == mm.E_ARG
    assert b"workers" in lib.momenti_last_error()
    jobs[1].k = 0
    assert lib.momenti_topk_batch(jobs, 2, 1 << 30, ctypes.byref(o), 2, out, n, st, None) == mm.E_ARG
    assert b"job 1" in lib.momenti_last_error()


def test_batch_binding_raises_for_errors_of_the_call():
    # bad arguments of the call itself raise (no job ran); a job's own error
    # would be returned in its status instead
    import numpy as np
    from paper_2502_14446_amd import momenti as mm
    jobs = [dict(series=np.zeros((2, 100), dtype=np.float32), w=10, d=1, k=1, delta=0.1)]
    with pytest.raises(mm.MomentiError) as e:
        mm.topk_batch(jobs, workers=0)
    assert e.value.code == mm.E_ARG and "workers" in str(e.value)


def test_binding_refuses_to_run_without_the_library(monkeypatch):
    from paper_2502_14446_amd import momenti as mm
    monkeypatch.setattr(mm, "LIB_PATH", "/nonexistent/libmomenti.so")
    monkeypatch.setattr(mm, "_lib", None)
    with pytest.raises(RuntimeError):
        mm.lib()
