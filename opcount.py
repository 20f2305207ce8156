"""Algorithmic operation count of the exhaustive enumeration (measurement aid).

Counts, on the CPU, the integer operations that the chain form of the model
(Section 4.1 simulator, overlap rates of Section 4.2.1: every DtH that starts
before the last HtD ends runs at the overlapped rate, so its start and end are
appended to a chain once its kernel's end is known) and the prefix-sharing
walk over the last M positions need per ordering: windows, DtHs crossed
inside a window, gaps of the DtH engine, starts from idle, chain appends,
tails and the per-ordering bookkeeping, each priced at the 32-bit ALU
operations its statement needs (listed in COSTS).  Lanes are counted on their
own: the lockstep of a wave (a wave runs as many loop iterations as its
busiest lane) is reported separately, as the ratio of wave-lockstep to lane
iterations.

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
    "window_setup": 6,     # cursor on the chain?, running at t?, idle end estimate, starts inside?, select
    "start": 6,            # DtH starts inside the window: work left (sub, shift, sub), busy estimate (ceil, add)
    "loop_test": 1,        # running DtH ends before the estimate?
    "crossing": 10,        # its solo time (sub, mul, shift, add), cursor, slot index and address, gap test (3)
    "gap": 18,             # exact work left (sub, mul, sub), idle estimate (3), start test (2), work and
                           # busy estimate if it starts (3 + 4), four selects
    "window_end": 6,       # kernel end (max, add), its lateness against the DtH prefix (sub, max), DtH prefix,
                           # running flag
    "append": 6,           # chain entry (max, add), slot address, cursor refresh (compare, two selects)
    "tail": 2,             # emax + dpre when no DtH runs at the last HtD end
    "tail_running": 7,     # work moved by the running DtH (sub, mul, shift), solo times left (sub, add), max
    "leaf": 12,            # min / max with rank, 64-bit sum, 64-bit rank-weighted sum
    "child": 9,            # next task from the nibble list (2), leaf index (2), remaining list (5)
    "prefix_position": 13,  # factorial digit (div, mul, sub), nibble extract and list splice,
                            # lexicographic digit (mask, popcount, multiply-add)
    "subtree": 64,         # set-major index split, the prefix's task set (one binomial step per task),
                           # fold into the lane accumulators with ties to the lower rank
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
    """State at the start of a window; S, E is the chain (shared by copies,
    like the per-lane queue: entry j is written by the window of position j)."""
    __slots__ = ("t", "ck", "emax", "dpre", "elast", "cs", "ce", "dcross", "c", "run", "S", "E")

    def __init__(self, n):
        self.t = self.ck = self.dpre = self.elast = self.cs = self.ce = self.dcross = self.c = 0
        self.emax = -INF
        self.run = False
        self.S = [0] * n
        self.E = [0] * n

    def copy(self):
        c = Lane.__new__(Lane)
        for f in Lane.__slots__:
            setattr(c, f, getattr(self, f))
        return c


class Counter:
    def __init__(self):
        self.ops = 0
        self.windows = 0
        self.events = 0        # DtHs crossed inside windows
        self.rate_changes = 0  # gaps of the DtH engine inside windows

    def add(self, key, n=1):
        self.ops += COSTS[key] * n


def window(s, j, x, H, D, r, put, cnt, iters_out=None):
    """Window j (HtD of task x at position j) of the chain form; the lane
    state advances in place, operations are counted into cnt."""
    q = 1 << r.q_log2
    h, hp, k, d = H[x]
    cnt.add("window_setup")
    cnt.windows += 1
    i, S, E, dsum = s.c, s.cs, s.ce, s.dcross
    rc, u, ecmp = s.t, h << r.q_log2, E
    if not i < j:
        eb, ecmp = s.t + h, INF
    elif S < s.t:
        eb = s.t + hp
    else:
        ei = s.t + h
        if S < ei:
            cnt.add("start")
            u -= (S - s.t) << r.q_log2
            rc = S
            eb = S + -(-u // r.p_h)
        else:
            eb, ecmp = ei, INF
    it = 0
    while True:
        cnt.add("loop_test")
        if not ecmp < eb:
            break
        it += 1
        cnt.add("crossing")
        cnt.events += 1
        dsum += (r.p_d * (E - S)) >> r.q_log2
        ep = E
        i += 1
        S, E = s.S[min(i, j - 1)], s.E[min(i, j - 1)]
        ecmp = E
        if i >= j or S != ep:
            cnt.add("gap")
            cnt.rate_changes += 1
            u -= r.p_h * (ep - rc)
            rc = ep
            ei = rc + -(-u // q)
            if i < j and S < ei:
                u -= (S - rc) << r.q_log2
                rc = S
                eb = rc + -(-u // r.p_h)
            else:
                eb, ecmp = ei, INF
    cnt.add("window_end")
    s.c, s.cs, s.ce, s.dcross, s.run = i, S, E, dsum, ecmp != INF
    s.t = eb
    s.ck = max(eb, s.ck) + k
    s.emax = max(s.emax, s.ck - s.dpre)
    s.dpre += d
    if put:
        cnt.add("append")
        sj = max(s.elast, s.ck)
        s.S[j], s.E[j] = sj, sj + D[x]
        s.elast = s.E[j]
        if s.c == j:
            s.cs, s.ce = s.S[j], s.E[j]
    if iters_out is not None:
        iters_out.append(it)


def tail(s, r, cnt):
    T = s.emax + s.dpre
    if s.run:
        cnt.add("tail_running")
        T = max(T, s.t + (s.dpre - s.dcross) - ((r.p_d * (s.t - s.cs)) >> r.q_log2))
    else:
        cnt.add("tail")
    return T


def walk_subtree(tasks, sub, M, r, cnt, trace=None):
    """The orderings of subtree `sub` (ranks sub*M! ..), as one lane walks
    them; returns their times in rank order.  trace (optional) receives the
    loop iterations (DtHs crossed) of every window in walk order."""
    n = len(tasks)
    H, D = tables(tasks, r)
    cnt.add("subtree")
    rest = list(range(n))
    s = Lane(n)
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
        window(s, i, x, H, D, r, True, cnt, trace)
    out = []

    def level(s, L, rest):
        j = n - L
        for ci in range(L):
            cnt.add("child")
            x = rest[ci]
            s2 = s.copy()
            window(s2, j, x, H, D, r, L > 1, cnt, trace)
            if L == 1:
                cnt.add("leaf")
                out.append(tail(s2, r, cnt))
            else:
                level(s2, L - 1, rest[:ci] + rest[ci + 1:])

    level(s, M, rest)
    return out


def set_major_subtree(sp, n, m):
    """Lexicographic subtree index of set-major index sp (the order in which a
    wave's 64 lanes take subtrees: consecutive indices share the prefix's set
    of tasks and differ in its order)."""
    plen = n - m
    pf = math.factorial(plen)
    cset, p = divmod(sp, pf)
    sub, k = [], plen
    for x in range(n):
        w = math.comb(n - 1 - x, k - 1) if k > 0 else 0
        if k > 0 and cset < w:
            sub.append(x)
            k -= 1
        elif k > 0:
            cset -= w
    rest, s = list(range(n)), 0
    for i in range(plen):
        d, p = divmod(p, math.factorial(plen - 1 - i))
        x = sub.pop(d)
        s = s * (n - i) + rest.index(x)
        rest.remove(x)
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--subtrees", type=int, default=3000)
    ap.add_argument("--waves", type=int, default=40)
    args = ap.parse_args()
    tasks = W.single_group_mixed(12, 1)
    n, M = 12, 5
    r = Rates()
    nsub = math.factorial(n) // math.factorial(M)
    rng = np.random.default_rng(0)
    cnt = Counter()
    subs = rng.choice(nsub, size=args.subtrees, replace=False)
    for sidx in subs:
        walk_subtree(tasks, int(sidx), M, r, cnt)
    orderings = args.subtrees * math.factorial(M)
    # lockstep of waves: 64 lanes take 64 consecutive set-major subtrees
    lane_iters, wave_iters = 0, 0
    starts = rng.choice(nsub // 64, size=args.waves, replace=False)
    for w0 in starts:
        traces = []
        for lane in range(64):
            tr = []
            walk_subtree(tasks, set_major_subtree(64 * int(w0) + lane, n, M), M, r, Counter(), tr)
            traces.append(tr)
        arr = np.array(traces)  # every lane walks the same tree shape
        lane_iters += arr.sum()
        wave_iters += 64 * arr.max(axis=0).sum()
    res = {
        "group": "mixed N=12, seed 1, overlap 3/4, two DMA engines",
        "M": M, "subtrees": args.subtrees, "orderings": orderings,
        "alg_ops_per_ordering": cnt.ops / orderings,
        "windows_per_ordering": cnt.windows / orderings,
        "dth_crossings_per_ordering": cnt.events / orderings,
        "gaps_per_ordering": cnt.rate_changes / orderings,
        "lockstep_iterations_ratio": float(wave_iters / lane_iters),
        "costs": COSTS,
    }
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
