"""momenti_search_noalloc (every traversal buffer in the library's static
scratch area, no device allocation) answers as momenti_search does on the
same plan: motif indices, FP64 distances, dimensions, status and stop step
identical, on two calls in a row, the second with a smaller input; an input
whose traversal cannot fit the scratch area is refused with E_NOMEM."""
import numpy as np
import pytest

from paper_2502_14446_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2502_14446_amd import momenti as mm  # noqa: E402


def _key(res):
    got, rep, rc = res
    return (rc, [(m["a"], m["b"], m["dist_d"], m["dist_max"], m["dims"]) for m in got],
            rep["i_stop"], rep["j_stop"], rep["n_cand"])


def _plan(s, w, proj="f32", mem_limit=1 << 30):
    x = torch.from_numpy(s.as_dtype()).to("cuda")
    plan = mm.Plan(s.n, s.D, w, "f32", mem_limit, device_series=True, seed=0x5EED, proj=proj)
    plan.hash(x)
    return plan, x


def test_noalloc_search_matches_search_on_two_calls():
    cases = [(201, 6, 40_000, 60, 2, 3), (202, 4, 6_000, 40, 2, 2)]   # the second input is smaller
    for seed, D, n, w, d, k in cases:
        s = synth.make_series(seed, D, n, w, k, d, noise=0.02, dtype="f32")
        plan, x = _plan(s, w)
        got = plan.search_noalloc(d, k, 0.1)
        want = plan.search(d, k, 0.1)
        again = plan.search_noalloc(d, k, 0.1)    # the plan's own buffers are untouched by it
        plan.close()
        assert _key(got) == _key(want), (seed, _key(got), _key(want))
        assert _key(again) == _key(want)
        assert got[1]["peak_bytes"] <= 256 << 20
        assert [(m["a"], m["b"]) for m in got[0]] and got[2] in (mm.OK, mm.OK_FALLBACK)


def test_noalloc_search_refuses_an_input_beyond_the_scratch_area():
    # 3 million windows in 8 dimensions: one repetition's sort buffers alone
    # need more than the 256 MiB area
    s = synth.make_series(203, 8, 3_000_000, 100, 0, 0, dtype="f32")
    plan, x = _plan(s, 100, mem_limit=16 << 30)
    with pytest.raises(mm.MomentiError) as e:
        plan.search_noalloc(3, 2, 0.1)
    plan.close()
    assert e.value.code == mm.E_NOMEM and "scratch" in str(e.value)
