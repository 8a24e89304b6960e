"""Write the exact top-k of a full-size workload as a golden file.

The answer comes from the CPU oracle only (oracle.topk_exact_sweep: the
definitions of section 3.1 evaluated over every non-trivial pair, with the
diagonal sweep as a filter and every kept pair recomputed by the brute-force
definition); the input from the seeded generator. Nothing here touches the
GPU library.

    python tests/golden/make_golden.py rw8_1m      # about 30 min on 6 cores
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def main(name: str) -> None:
    import oracle
    from paper_2502_14446_amd import synth

    s, p = synth.workload(name)
    t0 = time.time()
    info: dict = {}
    top = oracle.topk_exact_sweep(s.x, p["w"], p["d"], p["k"], pool=1 << 14, omp=True, info=info)
    dt = time.time() - t0
    out = {
        "what": f"exact top-{p['k']} motifs of the {name} workload (section 3.1 definitions: "
                "dist_d over every non-trivial pair, greedy non-overlapping choice in "
                "(dist_d, a, b) order)",
        "workload": name,
        "data_seed": synth.DATA_SEED[name],
        "params": {k: p[k] for k in ("D", "n", "w", "d", "k")},
        "series_dtype": p["dtype"],
        "planted": [[m.p1, m.p2, list(m.dims)] for m in s.motifs],
        "motifs": [[m["a"], m["b"], m["dist_d"], m["dist_max"], list(m["dims"])] for m in top],
        "certificate": {"theta": info["theta"], "eps": info["eps"], "pool": info["pool"],
                        "passes": info["passes"], "max_filter_error": info["max_err"]},
        "seconds": round(dt, 1),
        "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
    }
    path = os.path.join(HERE, f"{name}_top{p['k']}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {dt:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "rw8_1m")
