"""Write the stored expected values for the full-size single-group workloads.

Calls only the CPU oracle (oracle/) and the seeded input generators.  Run from
the repository root:  python tests/golden/make_golden.py
Each N=12 enumeration (479,001,600 orderings) takes about a minute on 8 cores.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import cmodel  # noqa: E402
from oracle import model as M  # noqa: E402
from paper_1806_10113_amd import workloads as W  # noqa: E402


def summary(tasks, m):
    t0 = time.time()
    s = cmodel.exhaustive(tasks, m)
    wall = time.time() - t0
    n = len(tasks)
    h = M.heuristic(tasks, m)
    return {
        "model": {"q": m.q, "p_htd": m.p_htd, "p_dth": m.p_dth, "dma_engines": m.dma_engines},
        "tasks_ns": [[int(v) for v in row] for row in tasks],
        "min_ns": s["min_ns"], "argmin_rank": s["argmin_rank"],
        "max_ns": s["max_ns"], "argmax_rank": s["argmax_rank"],
        "sum": str(s["sum"]), "count": s["count"], "mean_ns": s["mean_ns"],
        "fingerprint": str(s["fingerprint"]),
        "best": list(M.nth_permutation(n, s["argmin_rank"])),
        "worst": list(M.nth_permutation(n, s["argmax_rank"])),
        "heuristic": h, "heuristic_ns": M.simulate(tasks, h, m),
        "oracle_wall_s": round(wall, 2), "oracle_threads": s["threads"],
    }


def main():
    out = {}
    out["uniform_n8_seed0"] = summary(W.single_group_uniform(8, 0), M.DEFAULT)
    out["uniform_n8_seed0_paper_rates"] = summary(W.single_group_uniform(8, 0), M.PAPER_EXAMPLE)
    out["mixed_n12_seed1"] = summary(W.single_group_mixed(12, 1), M.DEFAULT)
    # one DMA engine (Section 3.2, launch scheme for such devices)
    one = M.Model(4, 3, 3, 1)
    out["uniform_n8_seed0_one_dma"] = summary(W.single_group_uniform(8, 0), one)
    out["mixed_n12_seed1_one_dma"] = summary(W.single_group_mixed(12, 1), one)
    with open(os.path.join(HERE, "single_group_summaries.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: {kk: v[kk] for kk in ("min_ns", "max_ns", "mean_ns", "oracle_wall_s")}
                      for k, v in out.items()}))


if __name__ == "__main__":
    main()
