"""Write the stored expected values for the full-size workloads.

Calls only the CPU oracle (oracle/) and the seeded input generators.  Run from
the repository root:

    python tests/golden/make_golden.py [single] [n13] [batch] [memory]

(no argument: all).  single: the N = 8 and N = 12 groups
(single_group_summaries.json; an N = 12 enumeration takes one to two minutes
on 8 cores); n13: the two N = 13 groups (6,227,020,800 orderings each, about
20-30 minutes each on 8 cores; added to the same file); batch: every group of
the 4,096-group batch under both launch schemes (batch_4096_seed2.npz, about
10 minutes each); memory: the N = 12 group under a device-memory limit at five
capacities and both schemes (memory_n12_summaries.json, about two minutes
each).
"""
import json
import math
import os
import sys
import time

import numpy as np

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


def single(out):
    out["uniform_n8_seed0"] = summary(W.single_group_uniform(8, 0), M.DEFAULT)
    out["uniform_n8_seed0_paper_rates"] = summary(W.single_group_uniform(8, 0), M.PAPER_EXAMPLE)
    out["mixed_n12_seed1"] = summary(W.single_group_mixed(12, 1), M.DEFAULT)
    # one DMA engine (Section 3.2, launch scheme for such devices)
    one = M.Model(4, 3, 3, 1)
    out["uniform_n8_seed0_one_dma"] = summary(W.single_group_uniform(8, 0), one)
    out["mixed_n12_seed1_one_dma"] = summary(W.single_group_mixed(12, 1), one)


def n13(out):
    out["mixed_n13_seed7"] = summary(W.single_group_mixed(13, 7), M.DEFAULT)
    out["mixed_n13_seed1_one_dma"] = summary(W.single_group_mixed(13, 1), M.Model(4, 3, 3, 1))


BATCH_FIELDS = ("min_ns", "argmin_rank", "max_ns", "argmax_rank", "sum_lo", "sum_hi", "fingerprint",
                "heur_ns")


def batch():
    """Every group of the batch of 4,096 groups with N uniform in [4, 10]
    (seed 2, one DK/DT label per group): exhaustive summary and Algorithm 1."""
    b = W.batch_groups(4096, 4, 10, seed=2)
    arrays = {}
    for name, m in (("two_dma", M.DEFAULT), ("one_dma", M.Model(4, 3, 3, 1))):
        cols = {k: np.zeros(b.n_groups, dtype=np.uint64) for k in BATCH_FIELDS}
        heur = np.full((b.n_groups, 16), 0xFF, dtype=np.uint8)
        t0 = time.time()
        for g in range(b.n_groups):
            tasks = b.group(g)
            s = cmodel.exhaustive(tasks, m)
            h = M.heuristic(tasks, m)
            vals = {"min_ns": s["min_ns"], "argmin_rank": s["argmin_rank"], "max_ns": s["max_ns"],
                    "argmax_rank": s["argmax_rank"], "sum_lo": s["sum"] & ((1 << 64) - 1),
                    "sum_hi": s["sum"] >> 64, "fingerprint": s["fingerprint"],
                    "heur_ns": M.simulate(tasks, h, m)}
            for k in BATCH_FIELDS:
                cols[k][g] = vals[k]
            heur[g, :len(h)] = h
        for k in BATCH_FIELDS:
            arrays[f"{name}_{k}"] = cols[k]
        arrays[f"{name}_heur"] = heur
        print(f"batch {name}: {time.time() - t0:.0f} s", flush=True)
    arrays["sizes"] = np.asarray(b.sizes(), dtype=np.int32)
    np.savez_compressed(os.path.join(HERE, "batch_4096_seed2.npz"), **arrays)


def mem_summary(tasks, mem, cap, m, chunk=40_000_000):
    """Summary over every ordering under the memory limit, from the oracle's
    per-ordering times taken in rank chunks."""
    n = len(tasks)
    R = math.factorial(n)
    mn = mx = None
    amin = amax = 0
    total = 0
    fp = np.uint64(0)
    t0 = time.time()
    with np.errstate(over="ignore"):
        for lo in range(0, R, chunk):
            hi = min(R, lo + chunk)
            T = cmodel.mem_times(tasks, mem, cap, m, lo=lo, hi=hi)
            i = int(np.argmin(T))
            if mn is None or T[i] < mn:
                mn, amin = int(T[i]), lo + i
            j = int(np.argmax(T))
            if mx is None or T[j] > mx:
                mx, amax = int(T[j]), lo + j
            total += int(T.sum(dtype=np.int64))
            r = np.arange(lo, hi, dtype=np.uint64)
            fp = fp + np.sum((np.uint64(2) * r + np.uint64(1)) * T.astype(np.uint64), dtype=np.uint64)
    from oracle import memory as MM
    h = MM.heuristic(tasks, mem, cap, m)
    return {"model": {"q": m.q, "p_htd": m.p_htd, "p_dth": m.p_dth, "dma_engines": m.dma_engines},
            "capacity": int(cap), "min_ns": mn, "argmin_rank": amin, "max_ns": mx, "argmax_rank": amax,
            "sum": str(total), "count": R, "fingerprint": str(int(fp)),
            "heuristic": h, "heuristic_ns": MM.simulate(tasks, mem, cap, h, m),
            "oracle_wall_s": round(time.time() - t0, 1)}


def memory():
    t = W.single_group_mixed(12, 1)
    mem = W.footprints(t)
    out = {"tasks_ns": [[int(v) for v in row] for row in t], "mem_bytes": [int(v) for v in mem], "cases": {}}
    for dma in (2, 1):
        m = M.Model(4, 3, 3, dma)
        for frac in (1.0, 0.6, 0.4, 0.25, 0.0):
            cap = W.capacity_fraction(mem, frac)
            out["cases"][f"dma{dma}_cap{frac:g}"] = mem_summary(t, mem, cap, m)
            print(f"memory dma{dma} cap{frac:g} done", flush=True)
            with open(os.path.join(HERE, "memory_n12_summaries.json"), "w") as f:
                json.dump(out, f, indent=1)


def main():
    want = set(sys.argv[1:]) or {"single", "n13", "batch", "memory"}
    path = os.path.join(HERE, "single_group_summaries.json")
    if want & {"single", "n13"}:
        out = json.load(open(path)) if os.path.exists(path) else {}
        if "single" in want:
            single(out)
        if "n13" in want:
            n13(out)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps({k: {kk: v[kk] for kk in ("min_ns", "max_ns", "mean_ns", "oracle_wall_s")}
                          for k, v in out.items()}))
    if "batch" in want:
        batch()
    if "memory" in want:
        memory()


if __name__ == "__main__":
    main()
