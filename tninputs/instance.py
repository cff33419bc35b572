"""A problem instance: graph + tensor values + ordered tree, and its npz file.

The file holds only plain arrays (``numpy.load`` with ``allow_pickle=False``
reads it): edge_u, edge_v, edge_dim (int32), offsets (int64, n+1 element
offsets into ``data``), data (float64, each tensor row-major with legs in
ascending edge id), pair_i, pair_j (int32), and a JSON string of metadata.
"""
from __future__ import annotations

import json
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .graphs import Graph


@dataclass
class Instance:
    graph: Graph
    tensors: List[np.ndarray]
    pairs: List[Tuple[int, int]]
    meta: dict = field(default_factory=dict)

    def flat(self):
        """(offsets int64[n+1], data float64[]) in the library's input layout."""
        sizes = [int(t.size) for t in self.tensors]
        offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
        offsets[1:] = np.cumsum(sizes)
        data = np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in self.tensors]) \
            if self.tensors else np.zeros(0)
        return offsets, data

    def pair_arrays(self):
        p = np.asarray(self.pairs, dtype=np.int32).reshape(-1, 2)
        return p[:, 0].copy(), p[:, 1].copy()

    def with_tensors(self, tensors: Sequence[np.ndarray]) -> "Instance":
        return Instance(self.graph, list(tensors), list(self.pairs), dict(self.meta))


def save_instance(path: str, inst: Instance) -> None:
    eu, ev, ed = inst.graph.arrays()
    offsets, data = inst.flat()
    pi, pj = inst.pair_arrays()
    np.savez(path, n=np.int64(inst.graph.n), edge_u=eu, edge_v=ev, edge_dim=ed, offsets=offsets,
             data=data, pair_i=pi, pair_j=pj, meta=np.array(json.dumps(inst.meta)))


def load_instance(path: str) -> Instance:
    z = np.load(path, allow_pickle=False)
    n = int(z["n"])
    edges = list(zip(z["edge_u"].tolist(), z["edge_v"].tolist(), z["edge_dim"].tolist()))
    g = Graph(n, [tuple(e) for e in edges])
    inc = g.incident()
    off, data = z["offsets"], z["data"]
    tensors = []
    for v in range(n):
        shape = tuple(g.edges[e][2] for e in inc[v])
        tensors.append(data[off[v]:off[v + 1]].reshape(shape).copy())
    pairs = list(zip(z["pair_i"].tolist(), z["pair_j"].tolist()))
    return Instance(g, tensors, pairs, json.loads(str(z["meta"])))
