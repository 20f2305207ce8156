"""Algorithmic operation count of the exhaustive enumeration (measurement aid).

Counts, on the CPU, the integer operations that the window formulation of the
model (Section 4.1 simulator, overlap rates of Section 4.2.1) and the
prefix-sharing walk over the last M positions need per ordering: windows,
DtH events inside windows, rate changes, tails and the per-ordering
bookkeeping, each priced at the 32-bit ALU operations its statement needs
(listed in COSTS).  Lanes are counted on their own: the lockstep of a wave
(a wave runs as many event iterations as its busiest lane) is reported
separately, as the ratio of wave-lockstep to lane iterations.

The result prices the headline kernel's useful work: algorithmic ops per
ordering x orderings per second / the ALU peak is the roofline fraction of
work that some ordering needed, next to the issued fraction that the counters
give.  It is a transcription for counting only: no library code calls it and
it is not a reference for results (the CPU oracle is; tests/test_opcount.py
checks this transcription's times against it).

    python opcount.py [--subtrees 3000] [--waves 40]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

from paper_1806_10113_amd import workloads as W

# ALU operations per statement of the formulation (32-bit integer or select)
COSTS = {
    "window_setup": 6,     # idle DtH learns its kernel end (2 compares, select); HtD work, end estimate (select, add)
    "loop_test": 1,        # next DtH event before the HtD end?
    "event": 16,           # cursor, slot address, start test (3), rate test, overlapped-work split (3), slack,
                           # next event (4), DtH solo time
    "rate_change": 11,     # exact HtD work left (select, sub, mul, sub), two ceilings (3 + 2), new estimate (2)
    "window_end": 6,       # kernel end (max, add), its lateness against the DtH prefix (sub, max), DtH prefix, slot
    "tail": 2,             # max(emax + dpre, ...) when the DtH engine is idle at the last HtD end
    "tail_running": 11,    # running DtH's work left and its end, when busy
    "leaf": 12,            # min / max with rank, 64-bit sum, 64-bit rank-weighted sum
    "child": 9,            # next task from the nibble list (2), leaf index (2), remaining list (5)
    "prefix_position": 10,  # factorial digit (div, mul, sub), nibble extract and list splice
    "subtree": 16,         # list init, rank of the subtree, fold into the lane accumulators
}


class Rates:
    def __init__(self, q_log2=2, p_h=3, p_d=3):
        self.q_log2, self.p_h, self.p_d = q_log2, p_h, p_d


def tables(tasks, r):
    q = 1 << r.q_log2
    H, D = [], []
    for h, k, d in tasks:
        H.append((int(h), -(-q * int(h) // r.p_h), int(k), int(d)))
        D.append(-(-q * int(d) // r.p_d))
    return H, D


INF = 1 << 62


class Lane:
    __slots__ = ("t", "ck", "dev", "slack", "dpre", "dthru", "emax", "i", "drun")

    def __init__(self):
        self.t = self.ck = 0
        self.dev = INF
        self.slack = self.dpre = self.dthru = 0
        self.emax = -INF
        self.i = 0
        self.drun = False

    def copy(self):
        c = Lane.__new__(Lane)
        for f in Lane.__slots__:
            setattr(c, f, getattr(self, f))
        return c


class Counter:
    def __init__(self):
        self.ops = 0
        self.windows = 0
        self.events = 0
        self.rate_changes = 0

    def add(self, key, n=1):
        self.ops += COSTS[key] * n


def window(s, j, x, H, D, Q, r, put, cnt, iters_out=None):
    """Window j of the formulation (HtD of task x at position j); returns T
    only through the lane state, counts operations into cnt."""
    q = 1 << r.q_log2
    h, hp, k, d = H[x]
    cnt.add("window_setup")
    cnt.windows += 1
    if not s.drun and s.i == j - 1:
        s.dev = s.ck
    jlast = j - 1 if j > 0 else 0
    uh = h << r.q_log2
    th0 = s.t
    eh = s.t + (hp if s.drun else h)
    it = 0
    while True:
        cnt.add("loop_test")
        ev = s.dev
        if not ev < eh:
            break
        it += 1
        cnt.add("event")
        cnt.events += 1
        inew = s.i + (1 if s.drun else 0)
        ck_n, dp_n = Q[inew if put else min(inew, jlast)]
        start = inew < j and ck_n <= ev
        if start != s.drun:
            cnt.add("rate_change")
            cnt.rate_changes += 1
            uh -= (r.p_h if s.drun else q) * (ev - th0)
            th0 = ev
            cp = -(-uh // r.p_h)
            cq = -(-uh // q)
            eh = ev + (cp if start else cq)
        w = r.p_d * dp_n
        if start:
            s.dthru += w >> r.q_log2
            s.slack = w & (q - 1)
            s.dev = ev + dp_n
        else:
            s.dev = ck_n if inew < j else INF
        s.drun = start
        s.i = inew
    cnt.add("window_end")
    s.t = eh
    s.ck = max(eh, s.ck) + k
    s.emax = max(s.emax, s.ck - s.dpre)
    s.dpre += d
    if put:
        Q[j] = (s.ck, D[x])
    if iters_out is not None:
        iters_out.append(it)


def tail(s, r, cnt):
    q = 1 << r.q_log2
    T = s.emax + s.dpre
    if s.drun:
        cnt.add("tail_running")
        pw = r.p_d * (s.dev - s.t)
        ud = pw - s.slack if pw > s.slack else 0
        T = max(T, s.t + (-(-ud // q)) + (s.dpre - s.dthru))
    else:
        cnt.add("tail")
    return T


def walk_subtree(tasks, sub, M, r, cnt, trace=None):
    """The orderings of subtree `sub` (ranks sub*M! ..), as one lane walks
    them; returns their times in rank order.  trace (optional) receives the
    event-iteration count of every window in walk order."""
    n = len(tasks)
    H, D = tables(tasks, r)
    Q = [(0, 0)] * n
    cnt.add("subtree")
    rest = list(range(n))
    s = Lane()
    plen = n - M
    blk = math.factorial(n - 1) // math.factorial(M)
    rem = sub
    for i in range(plen):
        cnt.add("prefix_position")
        c = rem // blk
        rem -= c * blk
        if i + 1 < plen:
            blk //= n - 1 - i
        x = rest.pop(c)
        window(s, i, x, H, D, Q, r, True, cnt, trace)
    out = []

    def level(s, L, rest):
        j = n - L
        for ci in range(L):
            cnt.add("child")
            x = rest[ci]
            s2 = s.copy()
            window(s2, j, x, H, D, Q, r, L > 1, cnt, trace)
            if L == 1:
                cnt.add("leaf")
                out.append(tail(s2, r, cnt))
            else:
                level(s2, L - 1, rest[:ci] + rest[ci + 1:])

    level(s, M, rest)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--subtrees", type=int, default=3000)
    ap.add_argument("--waves", type=int, default=40)
    args = ap.parse_args()
    tasks = W.single_group_mixed(12, 1)
    n, M = 12, 4
    r = Rates()
    nsub = math.factorial(n) // math.factorial(M)
    rng = np.random.default_rng(0)
    cnt = Counter()
    subs = rng.choice(nsub, size=args.subtrees, replace=False)
    for sidx in subs:
        walk_subtree(tasks, int(sidx), M, r, cnt)
    orderings = args.subtrees * math.factorial(M)
    # lockstep of waves: 64 lanes take 64 consecutive subtrees
    lane_iters, wave_iters = 0, 0
    starts = rng.choice(nsub - 64, size=args.waves, replace=False)
    for s0 in starts:
        traces = []
        for lane in range(64):
            tr = []
            walk_subtree(tasks, int(s0) + lane, M, r, Counter(), tr)
            traces.append(tr)
        arr = np.array(traces)  # every lane walks the same tree shape
        lane_iters += arr.sum()
        wave_iters += 64 * arr.max(axis=0).sum()
    res = {
        "group": "mixed N=12, seed 1, overlap 3/4, two DMA engines",
        "M": M, "subtrees": args.subtrees, "orderings": orderings,
        "alg_ops_per_ordering": cnt.ops / orderings,
        "windows_per_ordering": cnt.windows / orderings,
        "events_per_ordering": cnt.events / orderings,
        "rate_changes_per_ordering": cnt.rate_changes / orderings,
        "lockstep_iterations_ratio": float(wave_iters / lane_iters),
        "costs": COSTS,
    }
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
