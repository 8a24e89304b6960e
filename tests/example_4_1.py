"""The scenario of the paper's worked example (section 4, Example 4.1), shared
by the oracle's pin and the GPU parity test. Inputs only: a seeded series,
an index in which exactly the two motifs collide, and the width r; no part
of the method's arithmetic beyond calls into the oracle."""
import json
import math
import os

import numpy as np

from paper_2502_14446_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def example_4_1_scenario(orc):
    """Series, injected index and r reproducing the scenario of Example 4.1
    (section 4): two motifs in D = 2 dimensions are the only colliding pairs,
    at every prefix length and repetition; r puts p = P(dist_max)^d of the
    closer motif where the Lemma 5.2 bound first reaches delta at (3, 2)."""
    fx = json.load(open(os.path.join(GOLDEN, "example_4_1.json")))
    prm = fx["parameters"]
    K, L, D, d = prm["K"], prm["L"], prm["D"], prm["d"]
    w, n = 40, 1200
    s = synth.make_series(0xE41, D, n, w, 2, D, min_gap=200)
    ns = n - w + 1
    m, nl, nr = orc.tensor_shape(L)
    NF = nl + nr
    # every window's prefix of length >= 2 is its own: left symbols carry the
    # low byte of its index, right symbols the high byte
    by = np.zeros((D, ns, 4 * NF), dtype=np.uint8)
    a = np.arange(ns)
    for fn in range(NF):
        by[:, :, 4 * fn] = (a & 255) if fn < nl else (a >> 8) & 255
    pairs = [(mt.p1, mt.p2) for mt in s.motifs]
    for p1, p2 in pairs:
        by[:, p2, :] = by[:, p1, :]
    words = orc.pack(by, NF, K)
    dd = [orc.distd(s.x, w, p1, p2, d) for p1, p2 in pairs]
    top = min(range(2), key=lambda q: (dd[q][0], pairs[q]))
    P_target = math.sqrt(0.888)
    lo, hi = 1e-6, 1e6
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if orc.collision_prob(dd[top][1], mid) < P_target:
            lo = mid
        else:
            hi = mid
    return fx, s, words, hi, pairs, top
