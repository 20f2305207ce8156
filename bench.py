"""Benchmark: exhaustive evaluation of every launch ordering of one task group.

Workload: one group of N=12 tasks (6 dominant-kernel: K log-uniform 1-20 ms,
HtD/DtH 0.1-2 ms; 6 dominant-transfer: ranges swapped), int64 ns, seed 1;
overlap rates 3/4.  One step = all 12! = 479,001,600 orderings evaluated and
reduced to best / worst / mean (one exhaustive call) plus the ordering
heuristic for the same group.  Inputs are resident in HBM before timing.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one short JSON line (the headline, with a summary of the extra
measurements); the full record of the extras is written to --extras-out.
Only one GPU is used; --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "orderings evaluated/sec at N=12 (exact); groups/sec + p99 latency, N≤16"
N = 12
SEED = 1

# MI355X: 256 CUs x 128 32-bit VALU lanes per clock x 2.4 GHz = 78.6e12
# lane-ops/s (the same lane rate as the 157.3 TFLOP/s FP32 vector figure,
# which counts an FMA as two operations); the integer issue probe reaches 1.92
# of the 2 wave-instructions per CU-clock this implies.
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# VALU lane-ops per ordering issued by exhaustive_kernel<u32, M=5> on this
# workload: SQ_INSTS_VALU per launch x 64 lanes / 12! (rocprofv3 counter run
# recorded in profiles/exhaustive_n12_counters.txt).
VALU_LANE_OPS_PER_ORDERING = 175.89
# Share of lanes active per issued VALU instruction of that kernel on this
# workload: SQ_THREAD_CYCLES_VALU / (64 x SQ_ACTIVE_INST_VALU) from a counter
# run (profiles/exhaustive_n12_lane_utilisation.txt).  Issued lane-ops times
# this share are the lane-ops that did work for some ordering; lanes masked off
# in a divergent step do none.
VALU_LANE_UTILISATION = 0.5805
# Integer operations the method needs per ordering of that workload, counted
# by `python opcount.py` (a transcription of the chain form of the windows and
# the walk over the last five positions, each statement priced at its 32-bit
# ALU operations, lanes counted on their own: 2.77 windows, 1.32 DtHs crossed
# and 0.23 gaps of the DtH engine per ordering, the set-major prefix decode).
ALG_OPS_PER_ORDERING = 110.6
# HBM bytes per launch: FETCH_SIZE x 2.000 + WRITE_SIZE x 1.000, each scaled by
# what the counter reads for a 256 MiB device copy (same profile file).
TRAFFIC_BYTES_PER_LAUNCH = 833_346_406


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target duration of the CPU-oracle baseline sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the batched, learned-proposal and serving measurements")
    p.add_argument("--extras", default="all",
                   help="comma-separated subset of: batch, one_dma, rounds, memory, proposal, serving, hw, "
                        "train (the network's training alone; proposal and serving train it too) "
                        "(default all)")
    p.add_argument("--train-pairs", type=float, default=2e7,
                   help="exact (ordering, time) pairs used to train the proposal network")
    p.add_argument("--train-batch", type=int, default=65536,
                   help="pairs per training step (the forward/backward kernel takes 128 rows per block, "
                        "so 32,768 or more fill the 256 CUs)")
    p.add_argument("--train-lr", type=float, default=1e-3, help="Adam learning rate (a quarter of it in the "
                                                                 "last third of the steps)")
    p.add_argument("--train-epochs", type=int, default=3, help="passes over the training pairs")
    p.add_argument("--eval-groups", type=int, default=1024)
    p.add_argument("--serve-seconds", type=float, default=10.0)
    p.add_argument("--hw-unit-ms", type=float, default=10.0,
                   help="time unit of the synthetic tasks run on the device (0: skip that validation)")
    p.add_argument("--calibrate-valu", action="store_true",
                   help="also run the integer issue probe (for the ALU peak, read with counters)")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="also run a 256 MiB device copy (for HBM counter calibration)")
    p.add_argument("--extras-out", default=os.path.join("gpurun_out", "bench_extras.json"),
                   help="file that receives the full record of the extra measurements "
                        "(the headline line carries a short summary of them)")
    return p.parse_args()


def cpu_baseline(tasks, seconds: float):
    """The C oracle on a bounded prefix of the rank range, all host threads."""
    from oracle import cmodel
    from oracle import model as M
    threads = cmodel.default_threads()
    # calibrate on a short run, then size the sample to ~`seconds`
    probe = 200_000 * threads
    t0 = time.perf_counter()
    cmodel.exhaustive(tasks, M.DEFAULT, lo=0, hi=probe, threads=threads)
    dt = time.perf_counter() - t0
    rate = probe / max(dt, 1e-9)
    count = int(min(math.factorial(N), max(probe, rate * seconds)))
    t0 = time.perf_counter()
    cmodel.exhaustive(tasks, M.DEFAULT, lo=0, hi=count, threads=threads)
    dt = time.perf_counter() - t0
    # the same simulator on one thread, over a tenth of the sample's ranks
    one = max(1, count // (10 * threads))
    t1 = time.perf_counter()
    cmodel.exhaustive(tasks, M.DEFAULT, lo=0, hi=one, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": count / dt, "unit": "orderings/s", "cores": threads, "kind": "oracle",
            "sample": f"ranks 0..{count - 1} of the N=12 group ({count / math.factorial(N):.2%} "
                      f"of 12!), plain C event simulator, {threads} threads, {dt:.1f} s",
            "single_thread_value": one / dt1, "cpu_model": _cpu_model(),
            "host_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "thread_cap": "16: the host CPU share of one GPU on this machine"}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def batch_extra(dev, reps: int = 5):
    """4,096 groups, N uniform in [4, 10], seed 2: all orderings of every group
    plus the heuristic, one graph replay per batch."""
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    b = W.batch_groups(4096, 4, 10, seed=2)
    tasks = torch.as_tensor(b.tasks).to(dev)
    offs = torch.as_tensor(b.offs).to(dev)
    plan = tgo.Plan(tgo.DEFAULT, max_groups=b.n_groups)
    desc = plan.autotune(tasks, offs)
    out = plan.run(tasks, offs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(reps):
        plan.run(tasks, offs, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    st = tgo.read_summaries(out)
    bad = sum(1 for x in st if x["status"] != 0)
    orderings = int(sum(math.factorial(int(n)) for n in b.sizes()))
    plan.close()
    return {"workload": "4096 groups, N~U{4..10}, DK/DT per group, seed 2: exhaustive + heuristic",
            "ms_per_batch": ms, "groups_per_s": b.n_groups / (ms / 1e3),
            "orderings_per_s": orderings / (ms / 1e3), "orderings": orderings,
            "bad_status": bad, "plan": desc}


def one_dma_extra(dev, reps: int = 10):
    """The one-DMA launch scheme (HtDs before DtHs on one transfer engine):
    N=12 mixed group (checked against the oracle's stored enumeration), an
    N=13 group, and the 4,096-group batch."""
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    model = tgo.Model(2, 3, 3, dma_engines=1)
    stream = torch.cuda.current_stream()
    out = {}
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "single_group_summaries.json")))
    for n in (12, 13):
        t = torch.as_tensor(W.single_group_mixed(n, SEED)).to(dev)
        summ, _ = tgo.exhaustive(t, model, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            tgo.exhaustive(t, model, summary=summ, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        s = tgo.read_summary(summ)
        rec = {"ms": ms, "orderings_per_s": math.factorial(n) / (ms / 1e3), "min_ns": s["min_ns"],
               "max_ns": s["max_ns"], "mean_ns": s["mean_ns"], "status": s["status"]}
        if n == 12:
            g = gold["mixed_n12_seed1_one_dma"]
            rec["matches_oracle"] = bool(s["min_ns"] == g["min_ns"] and s["argmin_rank"] == g["argmin_rank"]
                                         and s["sum"] == int(g["sum"])
                                         and s["fingerprint"] == int(g["fingerprint"]))
        out[f"exhaustive_n{n}"] = rec
    b = W.batch_groups(4096, 4, 10, seed=2)
    tasks, offs = torch.as_tensor(b.tasks).to(dev), torch.as_tensor(b.offs).to(dev)
    plan = tgo.Plan(model, max_groups=b.n_groups)
    desc = plan.autotune(tasks, offs)
    res = plan.run(tasks, offs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        plan.run(tasks, offs, res)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    orderings = int(sum(math.factorial(int(n)) for n in b.sizes()))
    bad = sum(1 for x in tgo.read_summaries(res) if x["status"] != 0)
    plan.close()
    out["batch"] = {"ms_per_batch": ms, "groups_per_s": b.n_groups / (ms / 1e3),
                    "orderings_per_s": orderings / (ms / 1e3), "bad_status": bad,
                    "plan": {"m_by_n": desc.get("m_by_n"), "lane_mult": desc.get("lane_mult"),
                             "blocks": desc.get("blocks")}}
    return out


def rounds_extra(dev, seed: int = 11):
    """Section 6.2 in the model: T workers x R dependent tasks drawn from each
    BK benchmark; NoReorder over every ordering vs the Heuristic setup.
    Speedups are against the worst NoReorder ordering, as in the paper's
    figures (best, median, geometric mean, heuristic)."""
    import numpy as np
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    stream = torch.cuda.current_stream()
    out = {}
    total_orderings, total_ms = 0, 0.0
    for T, R in ((4, 1), (4, 2), (4, 4), (6, 1), (6, 2), (8, 1)):
        for bi, bk in enumerate(W.PAPER_BENCHMARKS):
            tasks = torch.as_tensor(W.rounds_experiment(bk, T, R, seed + 100 * bi + 10 * T + R)).to(dev)
            summ, po, groups = tgo.rounds(tasks, T, R, tgo.DEFAULT, per_order=True, stream=stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            tgo.rounds(tasks, T, R, tgo.DEFAULT, summary=summ, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            s = tgo.read_summary(summ)
            times = po.cpu().numpy().astype(np.float64)
            worst = float(s["max_ns"])
            count = math.factorial(T) ** R
            total_orderings += count
            total_ms += ms
            out[f"T{T}_R{R}_{bk}"] = {
                "orderings": count, "ms": ms, "status": s["status"],
                "speedup_best": worst / s["min_ns"], "speedup_median": worst / float(np.median(times)),
                "speedup_geomean": worst / float(np.exp(np.log(times).mean())),
                "speedup_heuristic": worst / s["heur_ns"],
                "heuristic_groups": len(tgo.read_groups(groups)),
            }
    return {"cases": out, "orderings": total_orderings, "ms": total_ms,
            "orderings_per_s": total_orderings / (total_ms / 1e3)}


def memory_extra(dev):
    """Task groups under a device-memory limit: the N = 12 group (footprint
    = bytes moved at 57 GB/s) with capacities from its whole footprint down
    to its largest task.  Per capacity and launch scheme: every ordering
    (tgo_exhaustive_mem, timed with HIP events), speedups against the worst
    ordering, and what ignoring the limit costs (the best ordering without
    it, evaluated under it)."""
    import numpy as np
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    stream = torch.cuda.current_stream()
    t_np = W.single_group_mixed(12, seed=1)
    mem_np = W.footprints(t_np)
    tasks, mem = torch.as_tensor(t_np).to(dev), torch.as_tensor(mem_np).to(dev)
    out, total_ms, total_ord = {}, 0.0, 0
    for dma in (2, 1):
        model = tgo.Model(2, 3, 3, dma)
        free, _ = tgo.exhaustive(tasks, model)
        free = tgo.read_summary(free)
        for frac in (1.0, 0.6, 0.4, 0.25, 0.0):
            cap = W.capacity_fraction(mem_np, frac)
            summ, _ = tgo.exhaustive_mem(tasks, mem, cap, model, stream=stream)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(3):
                tgo.exhaustive_mem(tasks, mem, cap, model, summary=summ, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            s = tgo.read_summary(summ)
            order = torch.as_tensor(np.asarray([free["best"]], dtype=np.uint8)).to(dev)
            t_free = int(tgo.evaluate_mem(tasks, mem, cap, order, model).cpu()[0])
            total_ms += ms
            total_ord += s["count"]
            out[f"dma{dma}_cap{frac:g}"] = {
                "capacity_bytes": cap, "ms": ms, "orderings_per_s": s["count"] / (ms / 1e3),
                "status": s["status"], "min_ns": s["min_ns"], "max_ns": s["max_ns"], "mean_ns": s["mean_ns"],
                "heur_ns": s["heur_ns"], "speedup_best": s["max_ns"] / s["min_ns"],
                "speedup_heuristic": s["max_ns"] / s["heur_ns"],
                "unlimited_best_under_limit_ns": t_free,
                "unlimited_best_vs_best_pct": 100.0 * (t_free / s["min_ns"] - 1.0)}
    return {"workload": "N=12 mixed group (seed 1), footprint = (h + d) x 57 B/ns, total "
                        f"{int(mem_np.sum())} B", "cases": out,
            "orderings_per_s": total_ord / (total_ms / 1e3)}


def hw_validation_extra(dev, unit_ms: float):
    """The model against real HtD / kernel / DtH tasks on this device
    (Sections 4.2, 4.3): fitted rates, overlap-model errors, and the mean
    prediction error over every ordering of each BK benchmark."""
    from paper_1806_10113_amd import validate
    r = validate.run(dev, unit_ms=unit_ms, reps=3)
    out = {"unit_ms": unit_ms, "transfers": r["transfers"], "kernel": r["kernel"], "overlap": r["overlap"],
           "rounds": r["rounds"], "kernel_alu": r["kernel_alu"], "interference": r["interference"],
           "memory": [{k: v for k, v in m.items() if k != "per_ordering"} for m in r["memory"]]}
    for sc in ("two_dma", "one_dma_scheme", "two_dma_alu_kernels"):
        out[sc] = {"geomean_err_pct": r[sc]["geomean_err_pct"],
                   "benchmarks": {b: {k: v[k] for k in ("mean_err_pct", "max_err_pct", "measured_speedup_best",
                                                          "measured_speedup_heuristic",
                                                          "measured_time_of_predicted_best_vs_best_pct")}
                                  for b, v in r[sc]["benchmarks"].items()}}
    return out


def train_surrogate(dev, pairs_total: float, seed: int = 1003, batch: int = 8192, lr: float = 1e-3,
                    epochs: int = 1):
    """Train the proposal network on exact pairs from groups of N in [8, 16]
    (`epochs` passes over the pairs, each in its own shuffled order)."""
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    per = 1024
    groups = max(64, int(pairs_total // per))
    b = W.batch_groups(groups, 8, 16, seed=seed, per_task_label=True)
    tasks, offs = torch.as_tensor(b.tasks).to(dev), torch.as_tensor(b.offs).to(dev)
    t0 = time.perf_counter()
    orders, gid, T, status = tgo.pairs(tasks, offs, per, seed=seed)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    sur = tgo.Surrogate(max_rows=max(1 << 16, batch), max_groups=max(4096, groups))
    sur.init(seed)
    P = orders.shape[0]
    per_epoch = P // batch
    steps = per_epoch * epochs
    # one shuffle of the whole set per epoch, up front; every step then takes
    # a contiguous slice (no per-step gathers)
    gen = torch.Generator().manual_seed(seed)
    shuffled = []
    for _ in range(epochs):
        perm = torch.randperm(P, generator=gen).to(dev)
        shuffled.append((orders[perm].contiguous(), gid[perm].contiguous(), T[perm].contiguous()))
    del orders, gid, T
    torch.cuda.synchronize()
    orders, gid, T = shuffled[0]
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    sur.train_step(tasks, offs, orders[:batch], gid[:batch], T[:batch], lr, loss=loss)
    first = float(loss.cpu()[0])
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for i in range(1, steps):
        rate = lr if i < steps * 2 // 3 else lr / 4
        orders, gid, T = shuffled[i // per_epoch]
        sl = slice((i % per_epoch) * batch, (i % per_epoch + 1) * batch)
        sur.train_step(tasks, offs, orders[sl], gid[sl], T[sl], rate, loss=loss)
    e1.record(stream)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    # forward 2 x 143,616 FLOP per row; backward: activation gradients of
    # layers 3 and 2 (2 x 2 x 65,536) and the weight gradients (2 x 143,360)
    flop_row = 2 * 143616 + 2 * 2 * 65536 + 2 * 143360
    del shuffled
    return sur, {"pairs": int(P), "train_groups": groups, "steps": steps, "batch": batch, "epochs": epochs,
                 "lr": lr,
                 "pairs_s": t_pairs, "train_s": t_train, "loss_first": first,
                 "loss_last": float(loss.cpu()[0]), "us_per_step": 1e3 * ms / max(1, steps - 1),
                 "train_flop_per_s": flop_row * batch * (steps - 1) / (ms / 1e3),
                 "flop_per_row": flop_row}


def surrogate_extra(dev, sur, n_groups: int):
    """1,024 groups of N=16 (per-task DK/DT, seed 3): learned proposal vs the
    plain exact-evaluation search (heuristic + uniformly sampled orderings)."""
    import torch
    from paper_1806_10113_amd import tgo, workloads as W
    ev = W.fixed_size_groups(n_groups, 16, seed=3)
    tasks, offs = torch.as_tensor(ev.tasks).to(dev), torch.as_tensor(ev.offs).to(dev)

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    res = {}
    sur_runs = {}
    for S in (1 << 10, 1 << 12, 1 << 14, 1 << 16, 1 << 18, 1_000_000):
        r, t = timed(lambda: sur.search(tasks, offs, samples=S, topk=64, seed=31))
        sur_runs[S] = (tgo.read_search(r), t)
    plain_runs = {}
    for B in (1 << 12, 1 << 14, 1 << 16, 1 << 18, 1 << 20):
        r, t = timed(lambda: tgo.random_search(tasks, offs, samples=B, seed=32))
        plain_runs[B] = (tgo.read_search(r), t)
    ablation, _ = timed(lambda: tgo.random_search(tasks, offs, samples=64, seed=33))
    ablation = tgo.read_search(ablation)

    def mean_best(rs):
        return sum(x["best_ns"] for x in rs) / len(rs)

    def gap(a, b):  # mean over groups of (T_a - T_b) / T_b, percent
        return 100.0 * sum((x["best_ns"] - y["best_ns"]) / y["best_ns"] for x, y in zip(a, b)) / len(a)

    res["surrogate"] = {str(S): {"s": t, "groups_per_s": n_groups / t, "mean_best_ns": mean_best(r),
                                 "from_heuristic": sum(x["from_heuristic"] for x in r)}
                        for S, (r, t) in sur_runs.items()}
    res["plain"] = {str(B): {"s": t, "groups_per_s": n_groups / t, "mean_best_ns": mean_best(r)}
                    for B, (r, t) in plain_runs.items()}
    # equal wall time: the plain budget whose time is closest to each surrogate run
    eq = {}
    for S, (r, t) in sur_runs.items():
        B = min(plain_runs, key=lambda b: abs(math.log(plain_runs[b][1] / t)))
        eq[str(S)] = {"plain_samples": B, "time_ratio": plain_runs[B][1] / t,
                      "gap_pct_vs_plain": gap(r, plain_runs[B][0])}
    res["equal_time"] = eq
    # the plain search at its largest budget vs every surrogate run
    Bmax = max(plain_runs)
    res["vs_plain_max"] = {str(S): {"gap_pct": gap(r, plain_runs[Bmax][0]),
                                    "speedup_groups_per_s": plain_runs[Bmax][1] / t}
                           for S, (r, t) in sur_runs.items()}
    res["plain_max_samples"] = Bmax
    # ablation: the network's 64 candidates vs 64 uniformly sampled ones
    r16 = sur_runs[1 << 16][0]
    res["ablation_candidates"] = {
        "network_better": sum(x["cand_best_ns"] < y["cand_best_ns"] for x, y in zip(r16, ablation)),
        "random_better": sum(x["cand_best_ns"] > y["cand_best_ns"] for x, y in zip(r16, ablation)),
        "gap_pct_network_vs_random": 100.0 * sum((x["cand_best_ns"] - y["cand_best_ns"]) / y["cand_best_ns"]
                                                 for x, y in zip(r16, ablation)) / n_groups}
    res["heuristic_mean_ns"] = sum(x["heur_ns"] for x in r16) / n_groups
    return res


SERVE_CFG = {"streams": 4, "max_batch": 256, "max_batch_large": 64, "samples": 4096, "topk": 64,
             "budget_bytes": 8 << 30, "window_us": 300}
SERVE_P99_TARGET_US = 5000.0  # the latency at which serving capacity is stated


def _serve_run(sur, arr, warm_s: float, **over):
    """Replay one arrival trace in real time; latency figures over arrivals
    after the first warm_s seconds."""
    import numpy as np
    from paper_1806_10113_amd import tgo
    cfg = tgo.server_config(**{**SERVE_CFG, **over})
    srv = tgo.Server(tgo.DEFAULT, cfg, sur)
    t0 = time.perf_counter()
    out = srv.replay(arr.batch.tasks, arr.batch.offs, arr.t_ns)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    keep = arr.t_ns >= arr.t_ns[0] + int(warm_s * 1e9)
    lat = (out["t_done_ns"] - out["t_arrive_ns"])[keep] / 1e3
    wait = (out["t_admit_ns"] - out["t_arrive_ns"])[keep] / 1e3
    small = (out["path"] == 0)[keep]
    span = (out["t_done_ns"].max() - out["t_arrive_ns"].min()) / 1e9
    pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None  # noqa: E731
    return {"requests": int(len(out)), "achieved_groups_per_s": len(out) / span, "wall_s": wall,
            "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
            "p50_us_exhaustive": pct(lat[small], 50), "p99_us_exhaustive": pct(lat[small], 99),
            "p50_us_proposal": pct(lat[~small], 50), "p99_us_proposal": pct(lat[~small], 99),
            "p99_admission_wait_us": pct(wait, 99),
            "bad_status": int((out["status"] != 0).sum()), "batches": st["batches"],
            "max_queued": st["max_queued"], "max_in_use_bytes": st["max_in_use_bytes"],
            "base_bytes": st["base_bytes"], "ring_rows": st["ring_rows"], "budget_bytes": st["budget_bytes"]}


def serving_extra(dev, sur, seconds: float):
    """Config 5: Poisson arrivals at 20,000 groups/s, N ~ U{4..16}, per-task
    DK/DT, seed 4, for `seconds`; then the offered load is raised (streams
    drawn from a fixed pool of 50,000 such groups) until the server saturates,
    and one run at 20,000/s has a budget that binds."""
    from paper_1806_10113_amd import workloads as W
    arr = W.poisson_arrivals(20_000.0, seconds, 4, 16, seed=4)
    warm_s = min(1.0, 0.25 * seconds)  # the first second (or quarter) is warm-up
    res = {"offered_groups_per_s": 20_000.0, **_serve_run(sur, arr, warm_s),
           "latency_window": f"arrivals after the first {warm_s:g} s of a {seconds:g} s trace",
           "config": dict(SERVE_CFG)}
    # capacity: offered load doubled until the server falls behind (achieved
    # below 95 % of offered)
    pool = W.batch_groups(50_000, 4, 16, seed=5, per_task_label=True)
    sweep, capacity, sustained = [], None, None
    cap_lo, cap_hi = None, None  # offered loads around the capacity point

    def run_at(rate, refine):
        nonlocal capacity, sustained
        a = W.poisson_stream(rate, 1.5, pool, seed=6)
        r = {"offered_groups_per_s": rate, "refine": refine, **_serve_run(sur, a, 0.5)}
        sweep.append(r)
        keeps_up = r["achieved_groups_per_s"] >= 0.95 * rate and r["bad_status"] == 0
        if keeps_up:
            sustained = max(sustained or 0.0, r["achieved_groups_per_s"])
        ok = keeps_up and r["p99_us"] <= SERVE_P99_TARGET_US
        if ok:
            capacity = max(capacity or 0.0, r["achieved_groups_per_s"])
        return keeps_up, ok

    rate = 20_000.0
    while rate <= 640_000.0:
        keeps_up, ok = run_at(rate, False)
        if ok:
            cap_lo = rate
        elif cap_hi is None:
            cap_hi = rate
        if not keeps_up:
            break
        rate *= 2
    # three bisection steps between the last load that met the p99 target and
    # the first that did not
    if cap_lo is not None and cap_hi is not None:
        for _ in range(3):
            mid = round(0.5 * (cap_lo + cap_hi), -3)
            if mid <= cap_lo or mid >= cap_hi:
                break
            _, ok = run_at(mid, True)
            if ok:
                cap_lo = mid
            else:
                cap_hi = mid
    res["capacity_sweep"] = sweep
    res["capacity_groups_per_s"] = capacity
    res["sustained_groups_per_s"] = sustained
    res["capacity_rule"] = (f"offered load doubled from 20,000/s (1.5 s traces, latency over arrivals "
                            f"after 0.5 s) until the server falls below 95 % of it, then three bisection "
                            f"steps between the last load served with p99 <= {SERVE_P99_TARGET_US:g} us and "
                            f"the first that was not: capacity = the largest load served with p99 <= "
                            f"{SERVE_P99_TARGET_US:g} us, sustained = the largest load served at any latency")
    # a budget that binds: the server's own memory plus 512 task rows
    tight = res["base_bytes"] + 512 * 24
    a = W.poisson_stream(20_000.0, 2.0, pool, seed=8)
    res["binding_budget"] = {"offered_groups_per_s": 20_000.0, **_serve_run(sur, a, 0.5, budget_bytes=tight)}
    return res


def extras_summary(extras: dict) -> dict:
    """A few figures of each extra measurement for the headline line (the
    full record goes to its own file)."""
    def pick(d, *keys):
        if not isinstance(d, dict):
            return None
        if "error" in d:
            return {"error": str(d["error"])[:160]}
        return {k: d.get(k) for k in keys if k in d}

    out = {}
    if "batch" in extras:
        out["batch"] = pick(extras["batch"], "groups_per_s", "orderings_per_s", "ms_per_batch", "bad_status")
    if "one_dma" in extras:
        d = extras["one_dma"]
        if isinstance(d, dict) and "error" not in d:
            out["one_dma"] = {k: pick(d.get(k), "orderings_per_s", "ms_per_batch", "ms", "groups_per_s",
                                      "matches_oracle")
                              for k in ("exhaustive_n12", "exhaustive_n13", "batch")}
        else:
            out["one_dma"] = pick(d)
    if "rounds" in extras:
        out["rounds"] = pick(extras["rounds"], "orderings_per_s", "orderings")
    if "memory" in extras:
        out["memory"] = pick(extras["memory"], "orderings_per_s")
    if "proposal_training" in extras:
        out["proposal_training"] = pick(extras["proposal_training"], "pairs", "steps", "us_per_step",
                                        "train_flop_per_s", "loss_last")
    if "proposal_n16" in extras:
        d = extras["proposal_n16"]
        if isinstance(d, dict) and "error" not in d:
            # per sample count S: [gap % to the plain search at equal time,
            # gap % to the largest plain search, speedup over it]
            eq, mx = d.get("equal_time") or {}, d.get("vs_plain_max") or {}
            out["proposal_n16"] = {
                "per_S": {S: [round(eq[S]["gap_pct_vs_plain"], 3), round(mx[S]["gap_pct"], 3),
                              round(mx[S]["speedup_groups_per_s"], 2)] for S in mx if S in eq},
                "per_S_fields": "gap_pct_equal_time, gap_pct_vs_plain_max, speedup_vs_plain_max",
                "plain_max_samples": d.get("plain_max_samples"),
                "network_better_than_random": (d.get("ablation_candidates") or {}).get("network_better")}
        else:
            out["proposal_n16"] = pick(d)
    if "serving" in extras:
        out["serving"] = pick(extras["serving"], "offered_groups_per_s", "achieved_groups_per_s", "p50_us",
                              "p99_us", "bad_status", "capacity_groups_per_s", "sustained_groups_per_s")
    if "hw_validation" in extras:
        d = extras["hw_validation"]
        if isinstance(d, dict) and "error" not in d:
            out["hw_validation"] = {sc: (d.get(sc) or {}).get("geomean_err_pct")
                                    for sc in ("two_dma", "one_dma_scheme", "two_dma_alu_kernels")}
        else:
            out["hw_validation"] = pick(d)
    return _round(out)


def _round(x):
    """Floats to 4 significant digits (the headline line stays short)."""
    if isinstance(x, float):
        return float(f"{x:.4g}")
    if isinstance(x, dict):
        return {k: _round(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_round(v) for v in x]
    return x


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the path is measured on a single MI355X "
              "(several GPUs would split the rank range; that is not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1806_10113_amd import tgo, workloads as W

    dev = torch.device("cuda:0")
    tasks_np = W.single_group_mixed(N, SEED)
    tasks = torch.as_tensor(tasks_np).to(dev)
    offs = torch.tensor([0, N], dtype=torch.int32, device=dev)
    model = tgo.DEFAULT
    stream = torch.cuda.current_stream()
    summary = torch.empty(tgo.SUMMARY_DTYPE.itemsize, dtype=torch.uint8, device=dev)

    if args.calibrate_valu:
        # 8,192 blocks x 256 threads x 2,000 x 16 x 8 x 2 instructions
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tgo.valu_probe(8192, 2000, stream)
        e0.record(stream)
        tgo.valu_probe(8192, 2000, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        lane_ops = 8192 * 256 * 2000 * 16 * 8 * 2
        print(json.dumps({"valu_probe_ms": e0.elapsed_time(e1),
                          "valu_probe_tops": lane_ops / (e0.elapsed_time(e1) / 1e3) / 1e12}), file=sys.stderr)
    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    # One stream: the process keeps few streams alive, because HIP maps them
    # onto 4 hardware queues and the device validation below needs its HtD
    # and DtH streams on queues of their own (a second stream for Algorithm 1
    # here, kept alive by torch's stream pool, made those copies serialise).
    def step(ev_pair=None):
        if ev_pair is not None:
            ev_pair[0].record(stream)
        tgo.exhaustive(tasks, model, summary=summary, stream=stream)
        if ev_pair is not None:
            ev_pair[1].record(stream)
        tgo.heuristic(tasks, offs, model, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    k = args.steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for i in range(k):
        step(evs[i])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    launch_ms = [a.elapsed_time(b) for a, b in evs]
    avg_launch_ms = sum(launch_ms) / k

    # the answer must be the oracle's (stored full enumeration)
    s = tgo.read_summary(summary)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "single_group_summaries.json")))["mixed_n12_seed1"]
    ok = (s["status"] == 0 and s["min_ns"] == gold["min_ns"] and s["argmin_rank"] == gold["argmin_rank"]
          and s["max_ns"] == gold["max_ns"] and s["sum"] == int(gold["sum"])
          and s["fingerprint"] == int(gold["fingerprint"]))
    if not ok:
        print(json.dumps({"error": "result differs from the oracle", "got": s}), file=sys.stderr)
        sys.exit(1)

    orderings = math.factorial(N)
    ms_per_step = total_ms / k
    value = orderings * k / (total_ms / 1e3)

    roof = {"bound": "alu", "unit": "TOP/s", "peak": VALU_PEAK_TOPS}
    if VALU_LANE_OPS_PER_ORDERING is not None:
        achieved = VALU_LANE_OPS_PER_ORDERING * orderings / (avg_launch_ms / 1e3) / 1e12
        roof.update({"achieved": achieved, "frac": achieved / VALU_PEAK_TOPS,
                     "lane_utilisation": VALU_LANE_UTILISATION,
                     "achieved_active_lanes": achieved * VALU_LANE_UTILISATION,
                     "frac_alg": achieved * VALU_LANE_UTILISATION / VALU_PEAK_TOPS,
                     "alg_ops_per_ordering": ALG_OPS_PER_ORDERING,
                     "frac_alg_opcount": ALG_OPS_PER_ORDERING * orderings / (avg_launch_ms / 1e3) / 1e12
                                         / VALU_PEAK_TOPS,
                     "frac_note": "frac = issued VALU lane-ops (counter run) / peak; frac_alg counts "
                                  "only the lanes active in each issued instruction; frac_alg_opcount = "
                                  "the method's counted integer ops per ordering (opcount.py) / peak"})
    else:
        roof.update({"achieved": None, "frac": None})
    roof["traffic"] = TRAFFIC_BYTES_PER_LAUNCH
    roof["launch_ms"] = avg_launch_ms
    roof["kernel"] = "exhaustive_kernel<u32, M=5>"
    roof["launch_ms_note"] = "HIP events around the exhaustive call (time-path classify, main kernel, idle 64-bit twin, finalize)"
    roof["hbm_gbs"] = TRAFFIC_BYTES_PER_LAUNCH / (avg_launch_ms / 1e3) / 1e9

    out = {
        "metric": METRIC, "value": value, "unit": "orderings/s", "n_gpus": 1, "steps": k,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "exhaustive N=12 (6 DK + 6 DT, log-uniform, seed 1), all 479,001,600 "
                               "orderings -> min/argmin/max/argmax/mean, plus Algorithm-1 heuristic",
                   "group_size": N, "orderings_per_step": orderings, "overlap_rates": "3/4, 3/4",
                   "time_path": "32-bit (bound checked on device; identical to int64)"},
        "roofline": roof,
        # the model's own work unit: 3N command completions per ordering
        "event_steps_per_s": value * 3 * N,
        "min_ns": s["min_ns"], "mean_ns": s["mean_ns"],
    }
    if not args.no_extras:
        want = set(args.extras.split(",")) if args.extras != "all" else \
            {"batch", "one_dma", "rounds", "memory", "proposal", "serving", "hw"}
        extras = {}
        device_ok = [True]

        def run_extra(name, fn, *a):
            # an extra that fails is reported in its place and the headline
            # line still prints; after a device-side error no further GPU
            # work is started in this process
            if not device_ok[0]:
                extras[name] = {"error": "skipped after a device error in an earlier extra"}
                return None
            try:
                t0 = time.perf_counter()
                r = fn(*a)
                extras[name] = r
                print(json.dumps({"extra_done": name, "s": round(time.perf_counter() - t0, 1)}), file=sys.stderr,
                      flush=True)
                return r
            except Exception as e:  # noqa: BLE001 - reported, not swallowed
                msg = f"{type(e).__name__}: {e}"
                extras[name] = {"error": msg}
                print(json.dumps({"extra_failed": name, "error": msg}), file=sys.stderr, flush=True)
                dev_err = (isinstance(e, tgo.TgoError) and e.code == tgo.TGO_EDEVICE) or \
                    ("HIP error" in str(e) or "CUDA error" in str(e))
                if dev_err:
                    device_ok[0] = False
                return None

        for name, fn in (("batch", batch_extra), ("one_dma", one_dma_extra), ("rounds", rounds_extra),
                         ("memory", memory_extra)):
            if name in want:
                run_extra(name, fn, dev)
        if want & {"proposal", "serving", "train"}:
            trained = run_extra("proposal_training", lambda: train_surrogate(dev, args.train_pairs, batch=args.train_batch,
                                                                             lr=args.train_lr, epochs=args.train_epochs))
            if trained is not None:
                sur, tr = trained
                extras["proposal_training"] = tr
                if "proposal" in want:
                    run_extra("proposal_n16", surrogate_extra, dev, sur, args.eval_groups)
                if "serving" in want:
                    run_extra("serving", serving_extra, dev, sur, args.serve_seconds)
                sur.close()
        if "hw" in want and args.hw_unit_ms > 0:
            run_extra("hw_validation", hw_validation_extra, dev, args.hw_unit_ms)
        out["extras_summary"] = extras_summary(extras)
        path = args.extras_out
        try:
            os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
            with open(path, "w") as f:
                json.dump(extras, f, indent=1)
            out["extras_file"] = path
        except OSError as e:
            out["extras_file"] = f"not written: {e}"
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(tasks_np, args.cpu_seconds)
    line = json.dumps(out)
    if len(line) > 4000:  # the headline must stay one short line; drop the summary before anything else
        out.pop("extras_summary", None)
        line = json.dumps(out)
    print(line, flush=True)


if __name__ == "__main__":
    main()
