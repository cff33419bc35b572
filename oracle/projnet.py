"""The explicit projector network T_P (SI B) — TEST INFRASTRUCTURE ONLY.

Each compression of Algorithm 1 replaces A B over the bundle of edges between two tensors by
(A P_L)(P_R B).  Inserting every such pair into the input network gives T_P: the input tensors,
unchanged, plus two projector tensors per compression.  P_L takes the bundle's edges on the
compressed tensor's side and the new bond; P_R takes the new bond and copies of the bundle's
edges on the neighbour's side.  An exact contraction of T_P, in any order, equals the
compressed value, because Algorithm 1 is one order of contracting it (SI B, Fig.
"explicit-projection"); the running normalisation does not matter since only the product
P_L P_R enters, and it does not change when A or B is rescaled.

The projectors are the ones the oracle's own run computes (``approx._PROJECTORS``); the
bookkeeping below replays that run's operations to know which side of each bundle edge belongs
to which intermediate.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import approx


def projector_network(n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray],
                      pairs: Sequence[Tuple[int, int]], chi: int, cutoff: float = 0.0,
                      compress_late: bool = False, gauge_r: int = 0):
    """Run Algorithm 1 (QR-reduced compressions) and build T_P.

    Returns ``(result, n_p, edges_p, tensors_p)``: the oracle's result for the compressed run and
    T_P in the input format (edges ``(u, v, dim)``, every tensor's axes in ascending edge id).
    The first n tensors of T_P are the inputs."""
    approx._PROJECTORS = []
    try:
        res = approx.contract_compressed(n, edges, tensors, pairs, chi, cutoff,
                                         compress_late=compress_late, gauge_r=gauge_r)
        proj = approx._PROJECTORS
    finally:
        approx._PROJECTORS = None
    # T_P tensors as (legs, array, owner); legs name edges as ("e", oracle edge id) or ("f", k)
    dims: Dict[tuple, int] = {("e", e): int(d) for e, (_, _, d) in enumerate(edges)}
    legs: List[List[tuple]] = []
    arrays: List[np.ndarray] = []
    owner: List[int] = []
    for v in range(n):
        lv = sorted(e for e, (a, b, _) in enumerate(edges) if v in (a, b))
        legs.append([("e", e) for e in lv])
        arrays.append(np.asarray(tensors[v], dtype=np.float64))
        owner.append(v)
    fresh = 0
    it = iter(proj)
    for op in res.ops:
        if op.kind == "contract":
            for t in range(len(owner)):
                if owner[t] in (op.a, op.b):
                    owner[t] = op.out
            continue
        shared, e_new, p_l, p_r = next(it)
        assert e_new == op.out
        new = p_l.shape[1]
        copies = []
        for e in shared:
            # the neighbour's side of bundle edge e gets a fresh copy, which P_R takes
            hold = [t for t in range(len(legs)) if ("e", e) in legs[t] and owner[t] == op.b]
            assert len(hold) == 1, (e, hold)
            f = ("f", fresh)
            fresh += 1
            dims[f] = dims[("e", e)]
            legs[hold[0]][legs[hold[0]].index(("e", e))] = f
            copies.append(f)
        dims[("e", e_new)] = new
        bshape = [dims[("e", e)] for e in shared]
        legs.append([("e", e) for e in shared] + [("e", e_new)])
        arrays.append(p_l.reshape(bshape + [new]))
        owner.append(op.a)
        legs.append([("e", e_new)] + copies)
        arrays.append(p_r.reshape([new] + bshape))
        owner.append(op.b)
    # renumber the edges, order every tensor's axes by edge id
    names = sorted({x for lv in legs for x in lv}, key=lambda x: (x[0], x[1]))
    ident = {x: i for i, x in enumerate(names)}
    ends: Dict[int, List[int]] = {}
    tens = []
    for t, lv in enumerate(legs):
        ids = [ident[x] for x in lv]
        for i in ids:
            ends.setdefault(i, []).append(t)
        perm = sorted(range(len(ids)), key=lambda q: ids[q])
        tens.append(np.ascontiguousarray(np.transpose(arrays[t], perm)))
    edges_p = []
    for i in range(len(names)):
        u, v = ends[i]
        assert u != v
        edges_p.append((min(u, v), max(u, v), dims[names[i]]))
    return res, len(legs), edges_p, tens
