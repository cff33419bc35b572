"""Shared helpers for the GPU tests: run an instance through the C ABI."""
import math

import numpy as np

import paper_2206_07044_amd as tn


def gpu_eval(inst_graph, tensors, pairs, chi, precision="fp64", cutoff=0.0, ctx=None, max_sweeps=0, late=False):
    g = inst_graph
    eu, ev, ed = g.arrays()
    sizes = [int(t.size) for t in tensors]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    data = np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in tensors])
    own = ctx is None
    c = tn.Context(0) if own else ctx
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision, cutoff=cutoff,
                      max_sweeps=max_sweeps, late=late)
        m, e = c.tn_contract_compressed()
        sign, lnz = c.tn_result() if m != 0.0 else (0.0, -math.inf)
        stats = c.tn_compress_stats() if m != 0.0 else None
        return sign, lnz, m, e, stats
    finally:
        if own:
            c.close()
