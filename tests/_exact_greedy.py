"""Exact contraction of a small tensor network by greedy pairwise steps (test helper).

Each step contracts the connected pair of live tensors with the smallest result, every
intermediate rescaled by its largest entry (the logarithms summed), so the value is the plain
sum over all indices in an order of its own.
"""
import math

import numpy as np


def greedy_exact(n, edges, tensors):
    """Sign and ln|value| of the full contraction of a connected network."""
    legs = {v: [] for v in range(n)}
    for e, (u, v, _) in enumerate(edges):
        legs[u].append(e)
        legs[v].append(e)
    live = {v: (sorted(legs[v]), np.asarray(tensors[v], dtype=np.float64)) for v in range(n)}
    log = 0.0
    nxt = n
    while len(live) > 1:
        best = None
        keys = sorted(live)
        for i in keys:
            li = live[i][0]
            for j in keys:
                if j <= i:
                    continue
                lj = live[j][0]
                shared = set(li) & set(lj)
                if not shared:
                    continue
                size = 1
                for e in set(li) ^ set(lj):
                    size *= edges[e][2]
                if best is None or size < best[0]:
                    best = (size, i, j)
        _, i, j = best
        (li, ti), (lj, tj) = live.pop(i), live.pop(j)
        shared = [e for e in li if e in lj]
        out = np.tensordot(ti, tj, axes=([li.index(e) for e in shared], [lj.index(e) for e in shared]))
        lo = [e for e in li if e not in shared] + [e for e in lj if e not in shared]
        s = float(np.max(np.abs(out)))
        assert s > 0.0
        log += math.log(s)
        live[nxt] = (lo, out / s)
        nxt += 1
    (_, last), = live.values()
    x = float(last.reshape(()))
    return math.copysign(1.0, x), log + math.log(abs(x))
