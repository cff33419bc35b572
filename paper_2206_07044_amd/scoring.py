"""Device-side scoring of candidate contraction trees.

The paper optimises ordered contraction trees over generator hyper-parameters
against a score (section II.H, SI C): peak memory, cost, or the error of the
compressed contraction itself.  The search stays on the host; this module
gives it the error score on the GPU: every candidate tree is planned on the
same network, and the candidates are evaluated together as one batch (merged
levels, one hipGraph replay, tn_batch_contract).  Candidates the planner
rejects (an intermediate beyond 2^31 entries, an arena above the budget) are
returned with their status instead of a value.

    scorer = TreeScorer(n, edge_u, edge_v, edge_dim, offsets, data, chi=8)
    scores = scorer.score([tree_a, tree_b, ...], ref_ln_abs_z=exact_value)
    best = min(scores, key=lambda s: s.rel_error)

Only argument marshalling happens here: the contraction, the compressions and
the running exponent of every candidate run in the library's kernels.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

from ._capi import Batch, Context, TNError


@dataclass
class TreeScore:
    status: int                    # TN_OK, or the planner's / evaluator's error status
    message: str = ""
    sign: float = 0.0
    ln_abs_z: float = math.nan
    rel_error: float = math.inf    # |ln|Z| - ref| / |ref| when a reference is given
    fwd_flops: float = math.inf    # the plan's algorithmic flops (the paper's cost C, plus re-absorptions)
    arena_bytes: int = 0           # device memory of the plan (the paper's peak memory M, in bytes)


class TreeScorer:
    """Scores candidate trees of one network at bond dimension chi."""

    def __init__(self, n: int, edge_u, edge_v, edge_dim, offsets, data, chi: int, precision: str = "fp64",
                 late: bool = False, device_budget_bytes: int = 0, device: int = 0):
        self.n = int(n)
        self.graph = (np.asarray(edge_u, dtype=np.int32), np.asarray(edge_v, dtype=np.int32),
                      np.asarray(edge_dim, dtype=np.int32))
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.data = np.ascontiguousarray(data, dtype=np.float64)
        self.chi, self.precision, self.late = int(chi), precision, bool(late)
        self.budget = int(device_budget_bytes)
        self.device = device

    def _plan(self, tree: Sequence[Tuple[int, int]]):
        c = Context(self.device)
        try:
            c.tn_load_graph(self.n, *self.graph, self.offsets, self.data)
            c.tn_set_tree([a for a, _ in tree], [b for _, b in tree], self.chi, precision=self.precision,
                          budget=self.budget, late=self.late)
        except TNError as e:
            c.close()
            return None, TreeScore(e.status, str(e))
        info = c.tn_plan_info()
        return c, TreeScore(0, "", fwd_flops=info["fwd_flops"], arena_bytes=info["arena_bytes"])

    def score(self, trees: Sequence[Sequence[Tuple[int, int]]], ref_ln_abs_z: Optional[float] = None,
              chunk: int = 64) -> List[TreeScore]:
        """Score every tree; candidates are evaluated ``chunk`` at a time as one batch."""
        out: List[TreeScore] = []
        for lo in range(0, len(trees), chunk):
            planned = [self._plan(t) for t in trees[lo:lo + chunk]]
            ctxs = [c for c, _ in planned if c is not None]
            try:
                mant = None
                if ctxs:
                    try:
                        batch = Batch(ctxs)
                        try:
                            mant, _ = batch.tn_batch_contract()
                        finally:
                            batch.close()
                    except TNError:
                        mant = None    # a plan the batch cannot merge, or a failed member: one by one
                k = 0
                for c, s in planned:
                    if c is None:
                        out.append(s)
                        continue
                    try:
                        m = mant[k] if mant is not None else c.tn_contract_compressed()[0]
                        s.sign, s.ln_abs_z = c.tn_result() if m != 0.0 else (0.0, -math.inf)
                    except TNError as e:
                        s.status, s.message = e.status, str(e)
                    k += 1
                    if s.status == 0 and ref_ln_abs_z is not None and math.isfinite(s.ln_abs_z):
                        s.rel_error = abs(s.ln_abs_z - ref_ln_abs_z) / abs(ref_ln_abs_z)
                    out.append(s)
            finally:
                for c in ctxs:
                    c.close()
        return out
