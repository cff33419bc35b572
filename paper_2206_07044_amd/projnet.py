"""The explicit projector network T_P (SI B, Fig. "explicit-projection") of an evaluated tree.

Every compression of the run replaced the bundle of edges between two intermediates by
(A P_L)(P_R B).  T_P is the input network with each such pair inserted where it acted: P_L on
the bundle edges of the compressed intermediate's side, P_R on copies of them that now end on
the neighbour's side, the two joined by the compression's new edge.  Contracted exactly, in any
order, T_P gives the compressed value (the run is one order of contracting it); it fixes the
approximation and so gives, for instance, gradients with the projectors held fixed by exact
contraction.

Only index bookkeeping happens here: the projectors are the ones the library's kernels computed
and applied, read back with tn_read_projectors (the tree must be set with
keep_intermediates=True), and the order of contractions and compressions is the planner's
(tn_plan_describe).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from ._capi import tn_plan_describe


def projector_network(ctx, n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray],
                      pair_i: Sequence[int], pair_j: Sequence[int], chi: int, late: bool = False,
                      with_axes: bool = False):
    """T_P of the last evaluation of ``ctx`` (a tree set on that graph with these pairs and chi).

    Returns ``(n_p, edges_p, tensors_p)`` in the input format: edges ``(u, v, dim)`` with u < v,
    every tensor's axes in ascending edge id; tensors 0..n-1 are the inputs, then P_L and P_R of
    each compression in creation order.  With ``with_axes`` also the axis order of each tensor
    of T_P (``tensors_p[t] = transpose(original, axes[t])``)."""
    eu = np.asarray([e[0] for e in edges], dtype=np.int32)
    ev = np.asarray([e[1] for e in edges], dtype=np.int32)
    ed = np.asarray([e[2] for e in edges], dtype=np.int32)
    ops = tn_plan_describe(n, eu, ev, ed, pair_i, pair_j, chi, late=late)
    # an edge of T_P is a key: input and new edges keep their ids, copies get ("copy", k)
    dim = {e: int(d) for e, (_, _, d) in enumerate(edges)}
    axes: List[list] = []
    data: List[np.ndarray] = []
    node: List[int] = []           # the tree node (live intermediate) each tensor belongs to
    incident = [[] for _ in range(n)]
    for e, (u, v, _) in enumerate(edges):
        incident[u].append(e)
        incident[v].append(e)
    for v in range(n):
        axes.append(sorted(incident[v]))
        data.append(np.asarray(tensors[v], dtype=np.float64))
        node.append(v)
    n_copy = 0
    comp = 0
    for kind, a, b, out, _m, _n, _k, _new in ops:
        if kind == 0:    # contraction: a and b become node `out`
            node = [out if x in (a, b) else x for x in node]
            continue
        pj = ctx.tn_read_projectors(comp)
        comp += 1
        if (pj["a"], pj["b"], pj["new_edge"]) != (a, b, out):
            raise RuntimeError("the context's plan does not match this graph and tree")
        bundle = pj["edges"]
        shape = [dim[e] for e in bundle]
        copies = []
        for e in bundle:
            owners = [t for t, ax in enumerate(axes) if e in ax and node[t] == b]
            if len(owners) != 1:
                raise RuntimeError(f"bond edge {e} has no unique end on node {b}")
            key = ("copy", n_copy)
            n_copy += 1
            dim[key] = dim[e]
            ax = axes[owners[0]]
            ax[ax.index(e)] = key
            copies.append(key)
        dim[out] = pj["chi"]
        axes.append(list(bundle) + [out])
        data.append(pj["p_left"].reshape(shape + [pj["chi"]]))
        node.append(a)
        axes.append([out] + copies)
        data.append(pj["p_right"].reshape([pj["chi"]] + shape))
        node.append(b)
    # number the edges (input and new ones first, in id order, then the copies), sort every
    # tensor's axes by the new numbers
    keys = sorted({k for ax in axes for k in ax}, key=lambda k: (1, k[1]) if isinstance(k, tuple) else (0, k))
    num = {k: i for i, k in enumerate(keys)}
    ends = [[] for _ in keys]
    out_t = []
    orders = []
    for t, ax in enumerate(axes):
        ids = [num[k] for k in ax]
        for i in ids:
            ends[i].append(t)
        order = sorted(range(len(ids)), key=lambda q: ids[q])
        orders.append(order)
        out_t.append(np.ascontiguousarray(np.transpose(data[t], order)))
    edges_p = []
    for i, k in enumerate(keys):
        if len(ends[i]) != 2:
            raise RuntimeError(f"edge {k} of T_P has {len(ends[i])} ends")
        u, v = ends[i]
        edges_p.append((min(u, v), max(u, v), dim[k]))
    if with_axes:
        return len(axes), edges_p, out_t, orders
    return len(axes), edges_p, out_t


def frozen_projector_grad(ctx, n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray],
                          pair_i: Sequence[int], pair_j: Sequence[int], chi: int, tree_p: Sequence[Tuple[int, int]],
                          late: bool = False, device: int = 0):
    """d ln|Z| / d T_v for every input tensor with the run's projectors held fixed: the exact
    gradient of T_P (contracted without compression on the caller's tree ``tree_p`` over T_P's
    tensors, every bond of which must stay within the planner's size limit), restricted to the
    inputs and returned in their own axis order.  T_P is multilinear in the inputs, so each
    tensor's <T_v, gradient> is 1 (Euler's identity for degree-one homogeneity)."""
    from ._capi import Context
    n_p, edges_p, tens_p, orders = projector_network(ctx, n, edges, tensors, pair_i, pair_j, chi, late, True)
    eu = np.asarray([e[0] for e in edges_p], dtype=np.int32)
    ev = np.asarray([e[1] for e in edges_p], dtype=np.int32)
    ed = np.asarray([e[2] for e in edges_p], dtype=np.int32)
    sizes = [t.size for t in tens_p]
    off = np.zeros(n_p + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    c = Context(device)
    try:
        c.tn_load_graph(n_p, eu, ev, ed, off, np.concatenate([t.ravel() for t in tens_p]))
        # chi above any bond the planner accepts: no compression
        c.tn_set_tree([a for a, _ in tree_p], [b for _, b in tree_p], 2 ** 30, precision="fp64", grad=True)
        c.tn_contract_compressed()
        if any(d > 0.0 for d in c.tn_compress_stats()[0]):
            raise RuntimeError("the tree over T_P compressed a bond: T_P was not contracted exactly")
        g = c.tn_grad()
    finally:
        c.close()
    out = []
    for v in range(n):
        gv = g[off[v]:off[v + 1]].reshape(tens_p[v].shape)
        out.append(np.ascontiguousarray(np.transpose(gv, np.argsort(orders[v]))))
    return out
