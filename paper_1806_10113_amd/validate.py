"""Validation of the temporal execution model on the device it runs on
(Sections 4.2 and 4.3): calibrate the command-time models, measure real task
groups launched with the Section 3.2 schemes, and compare with the model's
prediction for every ordering.

Steps (each measurement is the median of ``reps`` runs):
  1. Transfers: solo HtD and DtH times over a range of sizes, fitted to a line
     (latency + bytes / bandwidth) with tgo_fit_line.
  2. Overlap (Section 4.2.1): an HtD and a DtH of equal size issued together
     (and with the DtH delayed to overlap 75 / 50 / 25 % of the HtD); the
     overlap rates rho_htd, rho_dth come from tgo_fit_overlap over the fully
     overlapped runs and give the model's p/q (q = 1024).  Each experiment's
     total is predicted by tgo_evaluate with the fitted rates (partial
     overlap, the model), with no slowdown (non-overlapped model) and with
     both transfers slowed for their whole length (fully overlapped model).
  3. Kernel (Eq. 1): T = eta * m + gamma with m = floats scaled x passes.
  4. Task groups: the synthetic tasks T0..T7 of Section 4.3 (fractions of a
     time unit, 10 ms in the paper) built from the fitted models, every
     ordering of each benchmark BK0..BK100 run on the device, and the model's
     prediction for every ordering (tgo_exhaustive with the tasks' measured
     solo command times) compared with the measured makespan.
  5. Dependent tasks (Section 6.2): NoReorder orderings and a proxy running
     the Heuristic setup, against tgo_rounds.
  6. A device-memory limit: six of the synthetic tasks with their buffers
     counted against a capacity, run with tgo_hw_run_mem, against
     tgo_exhaustive_mem, with memory-streaming and with register-resident
     task kernels.
  7. Transfer speed under a concurrent kernel of each kind (the model has
     transfers and kernels independent).

Everything that runs on the device goes through the C ABI (tgo_hw_*,
tgo_evaluate, tgo_exhaustive); this module only orchestrates and summarises.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import tgo
from . import workloads as W

MB = 1 << 20
Q_LOG2 = 10  # fitted rates are expressed as p / 1024


def _median_run(hw, tasks, order, dma, reps):
    runs = [hw.run(tasks, order, dma) for _ in range(reps)]
    totals = [r[0] for r in runs]
    i = int(np.argsort(totals)[len(totals) // 2])
    return totals[i], runs[i][1]


def _one(htd=0, dth=0, elems=0, iters=0, kind=tgo.HW_KERNEL_HBM):
    t = np.zeros(1, dtype=tgo.HW_TASK_DTYPE)
    t["htd_bytes"], t["dth_bytes"], t["kern_elems"], t["kern_iters"] = htd, dth, elems, iters
    t["kern_kind"] = kind
    return t


def calibrate_transfers(hw, sizes_mb, reps):
    out = {}
    for kind, c in (("htd", 0), ("dth", 2)):
        xs, ys = [], []
        for mb in sizes_mb:
            b = int(mb * MB)
            task = _one(htd=b) if kind == "htd" else _one(dth=b)
            _, times = _median_run(hw, task, [0], 2, reps)
            xs.append(b)
            ys.append(float(times[0]["end_ns"][c] - times[0]["start_ns"][c]))
        slope, icept = tgo.fit_line(xs, ys)
        out[kind] = {"ns_per_byte": slope, "latency_ns": icept, "gb_per_s": 1.0 / slope,
                     "sizes_bytes": xs, "ns": ys}
    return out


def calibrate_kernel(hw, elems, iters_list, reps, kind=tgo.HW_KERNEL_HBM):
    xs, ys = [], []
    for it in iters_list:
        _, times = _median_run(hw, _one(elems=elems, iters=it, kind=kind), [0], 2, reps)
        xs.append(float(elems) * it)
        ys.append(float(times[0]["end_ns"][1] - times[0]["start_ns"][1]))
    eta, gamma = tgo.fit_line(xs, ys)
    return {"eta_ns_per_elem_pass": eta, "gamma_ns": gamma, "m": xs, "ns": ys}


def overlap_experiments(hw, sizes_mb, reps, dev):
    """Fig. overlap_error on this device."""
    import torch
    solo, full, records = [], [], []
    for mb in sizes_mb:
        b = int(mb * MB)
        sh = int(np.median([t[1] - t[0] for t in (hw.overlap(b, 0, 0) for _ in range(reps))]))
        sd = int(np.median([t[3] - t[2] for t in (hw.overlap(0, b, 0) for _ in range(reps))]))
        for frac in (1.0, 0.75, 0.5, 0.25, 0.0):
            delay = int(round((1.0 - frac) * sh))
            runs = [hw.overlap(b, b, delay) for _ in range(reps)]
            tot = [max(t[1], t[3]) - t[0] for t in runs]
            t = runs[int(np.argsort(tot)[len(tot) // 2])]
            records.append({"mb": mb, "overlap": frac, "times": [int(v) for v in t], "solo": [sh, sd]})
            if frac == 1.0:
                full.append(t)
                solo.append([sh, sd])
    note = None
    try:
        rho_h, rho_d = tgo.fit_overlap(np.array(full), np.array(solo))
    except tgo.TgoError as e:
        if e.code != tgo.TGO_EINVAL:
            raise
        # the device ran the HtD and the DtH one after the other in every
        # experiment that started them together: no slowdown can be fitted,
        # so the rates stay at solo speed and the report says so
        rho_h = rho_d = 1.0
        note = "no HtD/DtH overlap observed on this device: rates left at solo speed (p = q)"
    q = 1 << Q_LOG2
    p_h = int(min(q, max(1, round(rho_h * q))))
    p_d = int(min(q, max(1, round(rho_d * q))))
    fitted = tgo.Model(Q_LOG2, p_h, p_d)
    flat = tgo.Model(Q_LOG2, q, q)
    errs = {"partial": [], "non_overlapped": [], "fully_overlapped": []}
    # the two transfers as a two-task group: task 0 = (0, delay, d): its
    # kernel holds the DtH back until the measured DtH start; task 1 = (h, 0, 0)
    tasks = []
    for rec in records:
        t = rec["times"]
        h, d = rec["solo"]
        off = t[2] - t[0]
        tasks.append(np.array([[0, max(0, off), d], [h, 0, 0]], dtype=np.int64))
    order = torch.tensor([[0, 1]], dtype=torch.uint8, device=dev)
    for rec, tk in zip(records, tasks):
        t = rec["times"]
        meas = max(t[1], t[3]) - t[0]
        td = torch.as_tensor(tk).to(dev)
        pred_p = int(tgo.evaluate(td, order, fitted).cpu()[0])
        pred_n = int(tgo.evaluate(td, order, flat).cpu()[0])
        h, d = rec["solo"]
        off = max(0, t[2] - t[0])
        pred_f = max(h / rho_h, off + d / rho_d)
        for k, v in (("partial", pred_p), ("non_overlapped", pred_n), ("fully_overlapped", pred_f)):
            e = abs(v - meas) / meas
            errs[k].append(e)
        rec.update({"measured_ns": int(meas), "pred_partial_ns": pred_p, "pred_non_overlapped_ns": pred_n,
                    "pred_fully_overlapped_ns": pred_f})
    summary = {k: {"mean_pct": 100 * float(np.mean(v)), "max_pct": 100 * float(np.max(v))}
               for k, v in errs.items()}
    return {"rho_htd": rho_h, "rho_dth": rho_d, "model": [Q_LOG2, p_h, p_d], "errors": summary,
            "note": note, "records": records}, fitted


def build_task(frac, unit_ns, xfer, kern, elems):
    """Commands sized for (h, k, d) = frac * unit from the fitted models."""
    h_ns, k_ns, d_ns = (f * unit_ns for f in frac)
    hb = max(0, int((h_ns - xfer["htd"]["latency_ns"]) / xfer["htd"]["ns_per_byte"]))
    db = max(0, int((d_ns - xfer["dth"]["latency_ns"]) / xfer["dth"]["ns_per_byte"]))
    it = max(1, int(round((k_ns - kern["gamma_ns"]) / (kern["eta_ns_per_elem_pass"] * elems))))
    return hb, db, it


def validate_benchmarks(hw, dev, xfer, kern, model, unit_ns, elems, reps, dma_engines=2,
                        kind=tgo.HW_KERNEL_HBM):
    """Fig. prediction_error on this device: every ordering of each benchmark
    (task kernels of the given kind, sized with its calibration `kern`)."""
    import torch
    out = {}
    mdl = tgo.Model(model.q_log2, model.p_htd, model.p_dth, dma_engines)
    for bk, names in W.PAPER_BENCHMARKS.items():
        tasks = np.zeros(4, dtype=tgo.HW_TASK_DTYPE)
        for i, nm in enumerate(names):
            hb, db, it = build_task(W.PAPER_TASKS_UNITS[nm], unit_ns, xfer, kern, elems)
            tasks[i] = (hb, db, elems, it, kind)
        # measured solo command times feed the model
        solo = np.zeros((4, 3), dtype=np.int64)
        for i in range(4):
            _, tm = _median_run(hw, tasks[i:i + 1], [0], 2, reps)
            solo[i] = tm[0]["end_ns"] - tm[0]["start_ns"]
        solo_dev = torch.as_tensor(solo).to(dev)
        summ, po = tgo.exhaustive(solo_dev, mdl, per_order=True)
        horder, _ = tgo.heuristic(solo_dev, torch.tensor([0, 4], dtype=torch.int32, device=dev), mdl)
        pred = po.cpu().numpy()
        s = tgo.read_summary(summ)
        heur = [int(v) for v in horder.cpu().numpy()[0, :4]]
        meas = np.zeros(24, dtype=np.int64)
        for rk, order in enumerate(itertools.permutations(range(4))):
            meas[rk], _ = _median_run(hw, tasks, list(order), dma_engines, reps)
        err = np.abs(pred - meas) / meas
        heur_rank = tgo.rank(heur)
        out[bk] = {
            "solo_ns": solo.tolist(), "pred_ns": pred.tolist(), "measured_ns": meas.tolist(),
            "mean_err_pct": 100 * float(err.mean()), "max_err_pct": 100 * float(err.max()),
            "measured_speedup_best": float(meas.max() / meas.min()),
            "measured_speedup_heuristic": float(meas.max() / meas[heur_rank]),
            "predicted_best_rank": int(s["argmin_rank"]), "measured_best_rank": int(np.argmin(meas)),
            "measured_time_of_predicted_best_vs_best_pct":
                100 * float(meas[s["argmin_rank"]] / meas.min() - 1.0),
        }
    geo = math.exp(np.mean([math.log(max(v["mean_err_pct"], 1e-9)) for v in out.values()]))
    return {"benchmarks": out, "geomean_err_pct": geo}


def validate_rounds(hw, dev, xfer, kern, model, unit_ns, elems, reps, workers=4, rounds=2, bk="BK50",
                    seed=0, sample=24, dma_engines=2):
    """Section 6.2 on the device: workers x dependent tasks drawn from a BK
    benchmark, NoReorder orderings (a seeded sample plus the predicted best
    and worst) run with the dependencies and compared with tgo_rounds."""
    import torch
    T, R = workers, rounds
    units = W.rounds_experiment(bk, T, R, seed)
    names = {tuple(int(round(f * W.PAPER_UNIT_NS)) for f in W.PAPER_TASKS_UNITS[k]): k
             for k in W.PAPER_TASKS_UNITS}
    tasks = np.zeros(T * R, dtype=tgo.HW_TASK_DTYPE)
    for x, row in enumerate(units):
        hb, db, it = build_task(W.PAPER_TASKS_UNITS[names[tuple(int(v) for v in row)]], unit_ns, xfer, kern, elems)
        tasks[x] = (hb, db, elems, it, 0)
    solo = np.zeros((T * R, 3), dtype=np.int64)
    for x in range(T * R):
        _, tm = _median_run(hw, tasks[x:x + 1], [0], 2, reps)
        solo[x] = tm[0]["end_ns"] - tm[0]["start_ns"]
    mdl = tgo.Model(model.q_log2, model.p_htd, model.p_dth, dma_engines)
    summ, po, _ = tgo.rounds(torch.as_tensor(solo).to(dev), T, R, mdl, per_order=True)
    pred = po.cpu().numpy()
    s = tgo.read_summary(summ)
    count = len(pred)
    rng = np.random.default_rng(seed)
    ranks = sorted(set(rng.choice(count, size=min(sample, count), replace=False).tolist())
                   | {int(s["argmin_rank"]), int(s["argmax_rank"])})
    tf = math.factorial(T)
    errs, meas = [], {}
    for rk in ranks:
        seq, rem = [], rk
        perms = []
        for _ in range(R):
            rem, d = divmod(rem, tf)
            perms.append(tgo.unrank(T, d))
        perms = perms[::-1]
        seq = [w * R + r for r, p in enumerate(perms) for w in p]
        runs = [hw.run_rounds(tasks, T, R, seq, dma_engines)[0] for _ in range(reps)]
        m = int(np.median(runs))
        meas[rk] = m
        errs.append(abs(int(pred[rk]) - m) / m)
    # the Heuristic setup with a real proxy, against the model's prediction
    hruns = [hw.run_proxy(tasks, solo, T, R, mdl) for _ in range(reps)]
    htot = [h[0] for h in hruns]
    hmed = hruns[int(np.argsort(htot)[len(htot) // 2])]
    model_seq = [int(v) for v in s["heur"][:T * R]]
    return {"workers": T, "rounds": R, "benchmark": bk, "orderings": count, "measured": len(ranks),
            "heuristic_setup_measured_ns": int(hmed[0]), "heuristic_setup_predicted_ns": int(s["heur_ns"]),
            "heuristic_setup_err_pct": 100 * abs(int(s["heur_ns"]) - hmed[0]) / hmed[0],
            "heuristic_setup_same_order": hmed[1] == model_seq,
            "measured_speedup_heuristic_vs_worst": meas[int(s["argmax_rank"])] / hmed[0],
            "measured_speedup_best_vs_worst": meas[int(s["argmax_rank"])] / meas[int(s["argmin_rank"])],
            "mean_err_pct": 100 * float(np.mean(errs)), "max_err_pct": 100 * float(np.max(errs)),
            "predicted_best_ns": int(s["min_ns"]), "measured_at_predicted_best_ns": meas[int(s["argmin_rank"])],
            "predicted_worst_ns": int(s["max_ns"]), "measured_at_predicted_worst_ns": meas[int(s["argmax_rank"])]}


MEMORY_TASKS = ("T0", "T4", "T5", "T6", "T1", "T7")


def interference(hw, xfer, kern, elems, reps, kind, mb=256):
    """A transfer alone and under a concurrent kernel of the given kind (long
    enough to cover it): the transfer's speed under the kernel as a fraction
    of its solo speed.  The model of Section 4.2 has transfers and kernels
    run independently (a rate of 1)."""
    b = int(mb * MB)
    solo_ns = {"htd": xfer["htd"]["latency_ns"] + b * xfer["htd"]["ns_per_byte"],
               "dth": xfer["dth"]["latency_ns"] + b * xfer["dth"]["ns_per_byte"]}
    it = max(1, int(round(2.5 * max(solo_ns.values()) / (kern["eta_ns_per_elem_pass"] * elems))))
    k = _one(elems=elems, iters=it, kind=kind)
    out = {"kernel_kind": kind, "bytes": b}
    for name, tasks, order, x, c in (("htd", np.concatenate([k, _one(htd=b)]), [0, 1], 1, 0),
                                     ("dth", np.concatenate([_one(dth=b), k]), [0, 1], 0, 2)):
        _, alone = _median_run(hw, tasks[x:x + 1], [0], 2, reps)
        _, tm = _median_run(hw, tasks, order, 2, reps)
        t_alone = int(alone[0]["end_ns"][c] - alone[0]["start_ns"][c])
        t_with = int(tm[x]["end_ns"][c] - tm[x]["start_ns"][c])
        ks, ke = int(tm[1 - x]["start_ns"][1]), int(tm[1 - x]["end_ns"][1])
        covered = ks <= int(tm[x]["start_ns"][c]) + 50_000 and ke >= int(tm[x]["end_ns"][c])
        out[name] = {"alone_ns": t_alone, "with_kernel_ns": t_with, "rate": t_alone / t_with,
                     "kernel_covers_transfer": bool(covered)}
    return out


def validate_memory(hw, dev, xfer, kern, model, unit_ns, elems, reps, frac=0.4, names=MEMORY_TASKS, seed=0,
                    sample=16, dma_engines=2, kind=tgo.HW_KERNEL_HBM):
    """A task group under a device-memory limit on the device: each task's
    footprint is its bytes moved (input + output buffers), the capacity a
    fraction of the group's total.  A seeded sample of orderings plus the
    predicted best, worst and Algorithm 1's ordering run with tgo_hw_run_mem
    and compared with tgo_exhaustive_mem's prediction; the predicted best
    ordering without the limit is run under it too."""
    import torch
    n = len(names)
    tasks = np.zeros(n, dtype=tgo.HW_TASK_DTYPE)
    for i, nm in enumerate(names):
        hb, db, it = build_task(W.PAPER_TASKS_UNITS[nm], unit_ns, xfer, kern, elems)
        tasks[i] = (hb, db, elems, it, kind)
    mem = (tasks["htd_bytes"] + tasks["dth_bytes"]).astype(np.int64)
    cap = W.capacity_fraction(mem, frac)
    solo = np.zeros((n, 3), dtype=np.int64)
    for i in range(n):
        _, tm = _median_run(hw, tasks[i:i + 1], [0], 2, reps)
        solo[i] = tm[0]["end_ns"] - tm[0]["start_ns"]
    mdl = tgo.Model(model.q_log2, model.p_htd, model.p_dth, dma_engines)
    sd, md = torch.as_tensor(solo).to(dev), torch.as_tensor(mem).to(dev)
    summ, po = tgo.exhaustive_mem(sd, md, cap, mdl, per_order=True)
    pred = po.cpu().numpy()
    s = tgo.read_summary(summ)
    free, _ = tgo.exhaustive(sd, mdl)
    free = tgo.read_summary(free)
    count = len(pred)
    rng = np.random.default_rng(seed)
    heur = [int(v) for v in s["heur"][:n]]
    ranks = sorted(set(rng.choice(count, size=min(sample, count), replace=False).tolist())
                   | {int(s["argmin_rank"]), int(s["argmax_rank"]), tgo.rank(heur), int(free["argmin_rank"])})

    def measure(order):
        runs = [hw.run_mem(tasks, order, mem, cap, dma_engines)[0] for _ in range(reps)]
        return int(np.median(runs))

    meas = {rk: measure(tgo.unrank(n, rk)) for rk in ranks}
    errs = [abs(int(pred[rk]) - m) / m for rk, m in meas.items()]
    worst = meas[int(s["argmax_rank"])]
    return {"tasks": list(names), "kernel_kind": kind, "dma_engines": dma_engines,
            "capacity_frac": frac, "capacity_bytes": cap, "footprint_bytes": mem.tolist(),
            "orderings": count, "measured": len(ranks),
            "mean_err_pct": 100 * float(np.mean(errs)), "max_err_pct": 100 * float(np.max(errs)),
            "predicted_best_ns": int(s["min_ns"]), "measured_at_predicted_best_ns": meas[int(s["argmin_rank"])],
            "predicted_worst_ns": int(s["max_ns"]), "measured_at_predicted_worst_ns": worst,
            "heuristic_predicted_ns": int(s["heur_ns"]), "heuristic_measured_ns": meas[tgo.rank(heur)],
            "measured_speedup_best_vs_worst": worst / meas[int(s["argmin_rank"])],
            "measured_speedup_heuristic_vs_worst": worst / meas[tgo.rank(heur)],
            "unlimited_best_predicted_under_limit_ns": int(pred[int(free["argmin_rank"])]),
            "unlimited_best_measured_under_limit_ns": meas[int(free["argmin_rank"])],
            "unlimited_min_ns": int(free["min_ns"]),
            "per_ordering": [[rk, int(pred[rk]), m] for rk, m in sorted(meas.items())]}


def run(dev=None, unit_ms: float = 10.0, reps: int = 3, quick: bool = False):
    import torch
    dev = dev or torch.device("cuda:0")
    sizes = [8, 16, 32, 64] if quick else [16, 32, 64, 128, 256, 512]
    iters = [1, 2, 4, 8, 16, 32] if quick else [1, 2, 4, 8, 16, 32, 64, 128]
    elems = 1 << 24
    unit_ns = unit_ms * 1e6
    hw = tgo.HwRunner(4, int(max(sizes) * MB), elems)
    try:
        xfer = calibrate_transfers(hw, sizes, reps)
        kern = calibrate_kernel(hw, elems, iters, reps)
        kern_alu = calibrate_kernel(hw, elems, [max(1, i // 4) for i in iters], reps, tgo.HW_KERNEL_ALU)
        interf = [interference(hw, xfer, k, elems, reps, kind, mb=min(256, max(sizes)))
                  for k, kind in ((kern, tgo.HW_KERNEL_HBM), (kern_alu, tgo.HW_KERNEL_ALU))]
        ov, model = overlap_experiments(hw, sizes[-3:], reps, dev)
        need = max(build_task(f, unit_ns, xfer, kern, elems)[i]
                   for f in W.PAPER_TASKS_UNITS.values() for i in (0, 1))
        if need > int(max(sizes) * MB):
            hw.close()
            hw = tgo.HwRunner(4, need, elems)
        res2 = validate_benchmarks(hw, dev, xfer, kern, model, unit_ns, elems, reps, 2)
        res1 = validate_benchmarks(hw, dev, xfer, kern, model, unit_ns, elems, reps, 1)
        res2a = validate_benchmarks(hw, dev, xfer, kern_alu, model, unit_ns, elems, reps, 2, tgo.HW_KERNEL_ALU)
        hw.close()
        hw = tgo.HwRunner(8, need, elems)
        rounds = [validate_rounds(hw, dev, xfer, kern, model, unit_ns, elems, reps, 4, 2, bk,
                                  sample=8 if quick else 24)
                  for bk in (("BK25",) if quick else ("BK25", "BK50", "BK75"))]
        cases = (((0.4, 2, tgo.HW_KERNEL_HBM), (0.4, 2, tgo.HW_KERNEL_ALU)) if quick else
                 ((0.25, 2, tgo.HW_KERNEL_HBM), (0.4, 2, tgo.HW_KERNEL_HBM), (0.6, 2, tgo.HW_KERNEL_HBM),
                  (0.4, 1, tgo.HW_KERNEL_HBM), (0.4, 2, tgo.HW_KERNEL_ALU), (0.6, 2, tgo.HW_KERNEL_ALU),
                  (0.4, 1, tgo.HW_KERNEL_ALU)))
        memory = [validate_memory(hw, dev, xfer, kern if kind == tgo.HW_KERNEL_HBM else kern_alu, model, unit_ns,
                                  elems, reps, frac, dma_engines=dma, sample=6 if quick else 16, kind=kind)
                  for frac, dma, kind in cases]
    finally:
        hw.close()
    return {"unit_ms": unit_ms, "reps": reps,
            "transfers": {k: {kk: v[kk] for kk in ("gb_per_s", "latency_ns")} for k, v in xfer.items()},
            "kernel": {k: kern[k] for k in ("eta_ns_per_elem_pass", "gamma_ns")},
            "kernel_alu": {k: kern_alu[k] for k in ("eta_ns_per_elem_pass", "gamma_ns")},
            "interference": interf,
            "overlap": {k: ov[k] for k in ("rho_htd", "rho_dth", "model", "errors", "note")},
            "overlap_records": ov["records"],
            "two_dma": res2, "one_dma_scheme": res1, "two_dma_alu_kernels": res2a, "rounds": rounds,
            "memory": memory}
