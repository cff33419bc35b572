"""Algorithm 1 of arXiv:2206.07044 ("Approximate contraction", section II.F),
with early (default) or late compression and tree-gauge distance r >= 0 —
float64 numpy oracle.

Test infrastructure only (see the package docstring).

Readings of the paper used here (each is also listed in the design notes):
* Several compressions after one contraction run in ascending neighbour id
  (Algorithm 1 loops over NEIGHBORS(T, k); the order is not fixed by the text).
  Late compression (section II.D, Algorithm 1 with compress_late) compresses,
  before contracting i and j, every bond of i to a tensor other than j that is
  larger than chi, then every such bond of j, each in ascending neighbour id;
  nothing is compressed after a contraction.
* All edges between two tensors form one composite bond whose size is the
  product of their dimensions (BONDSIZE, Fig. "tensor primitives" A).
* The new bond dimension is min(chi, k_A, k_B) with k = min(rows, D_AB), the
  rank bound of the reduced factors; sigma^(1/2) goes to both sides (Eq. (svd)).
* When a matricised factor has no more rows than D_AB its QR is skipped and
  the factor itself serves as R (the result only depends on R up to an
  orthogonal factor, SI B).
* A singular value that is exactly zero, or below ``cutoff * sigma_1``, gives a
  zero column/row in the projectors instead of a division by zero.
* Every tensor an op writes is divided by its largest absolute entry and the
  natural log of that scale is added to a running exponent (the value of the
  contraction is linear in every tensor, so this leaves ln|Z| unchanged).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class OpRecord:
    """One step of the expanded schedule (used to check the GPU planner)."""
    kind: str            # "contract" or "compress"
    a: int               # contract: i; compress: the tensor being compressed (k)
    b: int               # contract: j; compress: its neighbour l
    out: int             # contract: new id k; compress: new edge id
    m: int               # contract: free size of i;  compress: rows of A_mat
    n: int               # contract: shared size;     compress: D_AB
    k: int               # contract: free size of j;  compress: columns of B_mat
    new_dim: int = 0     # compress: chi'
    discarded: float = 0.0   # compress: sum of discarded sigma^2 / sum sigma^2
    tie: bool = False        # compress: sigma_chi' and the next one coincide


@dataclass
class OracleResult:
    sign: float
    ln_abs_z: float
    ops: List[OpRecord] = field(default_factory=list)
    log_scales: List[float] = field(default_factory=list)
    tensors: List[np.ndarray] = field(default_factory=list)   # normalised, creation order (record=True)

    @property
    def log10_exponent(self) -> float:
        if self.sign == 0:
            return -math.inf
        return math.floor(self.ln_abs_z / math.log(10.0))

    @property
    def mantissa(self) -> float:
        if self.sign == 0:
            return 0.0
        frac = self.ln_abs_z / math.log(10.0) - self.log10_exponent
        return self.sign * 10.0 ** frac


class ZeroContraction(Exception):
    """The network evaluates to exactly zero (e.g. no perfect matching)."""


class _Network:
    """Live tensors, each an ndarray with a list of edge ids naming its axes."""

    def __init__(self, n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray]):
        self.dim: Dict[int, int] = {e: int(d) for e, (_, _, d) in enumerate(edges)}
        self.ends: Dict[int, List[int]] = {e: [int(u), int(v)] for e, (u, v, _) in enumerate(edges)}
        self.legs: Dict[int, List[int]] = {v: [] for v in range(n)}
        for e, (u, v, _) in enumerate(edges):
            self.legs[u].append(e)
            self.legs[v].append(e)
        self.t: Dict[int, np.ndarray] = {}
        for v in range(n):
            self.legs[v].sort()
            arr = np.asarray(tensors[v], dtype=np.float64)
            want = tuple(self.dim[e] for e in self.legs[v])
            if arr.shape != want:
                raise ValueError(f"tensor {v} has shape {arr.shape}, expected {want}")
            self.t[v] = arr.copy()
        self.next_edge = len(edges)

    def other_end(self, e: int, x: int) -> int:
        a, b = self.ends[e]
        return b if a == x else a

    def neighbors(self, x: int) -> Dict[int, List[int]]:
        """Neighbour id -> edge ids shared with it, in x's axis order."""
        out: Dict[int, List[int]] = {}
        for e in self.legs[x]:
            out.setdefault(self.other_end(e, x), []).append(e)
        return out


_RECORD: Optional[List[np.ndarray]] = None
# when a list: every compression appends (shared edge ids in P_L's row order, new edge id, P_L, P_R)
_PROJECTORS: Optional[list] = None


def _normalise(arr: np.ndarray, scales: List[float]) -> np.ndarray:
    s = float(np.max(np.abs(arr))) if arr.size else 0.0
    if s == 0.0 or not math.isfinite(s):
        if s == 0.0:
            raise ZeroContraction()
        raise FloatingPointError("non-finite tensor entry")
    scales.append(math.log(s))
    out = arr / s
    if _RECORD is not None:
        _RECORD.append(out.copy())
    return out


def _contract(net: _Network, i: int, j: int, k: int, scales: List[float], ops: List[OpRecord]) -> None:
    """Pairwise contraction (Fig. "tensor primitives" B): sum over the shared
    edges; the result's axes are i's free edges then j's free edges."""
    li, lj = net.legs.pop(i), net.legs.pop(j)
    ti, tj = net.t.pop(i), net.t.pop(j)
    shared = [e for e in li if e in lj]
    ai = [li.index(e) for e in shared]
    aj = [lj.index(e) for e in shared]
    out = np.tensordot(ti, tj, axes=(ai, aj))
    free_i = [e for e in li if e not in shared]
    free_j = [e for e in lj if e not in shared]
    m = int(np.prod([net.dim[e] for e in free_i])) if free_i else 1
    s = int(np.prod([net.dim[e] for e in shared])) if shared else 1
    q = int(np.prod([net.dim[e] for e in free_j])) if free_j else 1
    ops.append(OpRecord("contract", i, j, k, m, s, q))
    for e in shared:
        del net.ends[e]
    for e in free_i + free_j:
        ends = net.ends[e]
        ends[ends.index(i if e in free_i else j)] = k
    net.legs[k] = free_i + free_j
    net.t[k] = _normalise(out, scales)


def _reduced_factors(a_mat: np.ndarray, b_mat: np.ndarray):
    """R_A with R_A^T R_A = A^T A and R_B with R_B R_B^T = B B^T (section II.C)."""
    D = a_mat.shape[1]
    r_a = np.linalg.qr(a_mat, mode="r") if a_mat.shape[0] > D else a_mat
    r_b = np.linalg.qr(b_mat.T, mode="r").T if b_mat.shape[1] > D else b_mat
    return r_a, r_b


def _compress(net: _Network, a: int, b: int, chi: int, cutoff: float,
              scales: List[float], ops: List[OpRecord], explicit: bool, gauged=None) -> None:
    """Compress every edge between a and b into one edge of dimension chi'.

    QR-reduced form: R_AB = R_A R_B ~ U s V^T truncated to chi' values
    (Eq. (svd)); projectors P_L = R_B V s^-1/2 and P_R = s^-1/2 U^T R_A
    (SI B) give a' = A P_L and b' = P_R B.  With ``explicit`` the SVD is of
    the full product A B instead (the definition the QR form is equal to).
    ``gauged`` = (A'_mat, B'_mat): the R factors come from these tree-gauged
    virtual copies (section II.C, SI A) while the projectors still act on the
    tensors themselves; chi' keeps the shape bound of A_mat and B_mat.
    """
    la, lb = net.legs[a], net.legs[b]
    shared = [e for e in la if e in lb]
    free_a = [e for e in la if e not in shared]
    free_b = [e for e in lb if e not in shared]
    ta = np.transpose(net.t[a], [la.index(e) for e in free_a + shared])
    tb = np.transpose(net.t[b], [lb.index(e) for e in shared + free_b])
    D = int(np.prod([net.dim[e] for e in shared]))
    ma, mb = ta.size // D, tb.size // D
    a_mat = ta.reshape(ma, D)
    b_mat = tb.reshape(D, mb)
    if explicit:
        U, sig, Vt = np.linalg.svd(a_mat @ b_mat, full_matrices=False)
        ka, kb = min(ma, D), min(mb, D)
    elif gauged is None:
        r_a, r_b = _reduced_factors(a_mat, b_mat)
        ka, kb = r_a.shape[0], r_b.shape[1]
        U, sig, Vt = np.linalg.svd(r_a @ r_b, full_matrices=False)
    else:
        r_a, r_b = _reduced_factors(*gauged)
        ka, kb = min(ma, D), min(mb, D)
        U, sig, Vt = np.linalg.svd(r_a @ r_b, full_matrices=False)
        short = min(chi, ka, kb) - len(sig)
        if short > 0:   # the gauged factors have lower rank: the missing triplets are zeros
            U = np.hstack([U, np.zeros((U.shape[0], short))])
            Vt = np.vstack([Vt, np.zeros((short, Vt.shape[1]))])
            sig = np.concatenate([sig, np.zeros(short)])
    new = min(chi, ka, kb)
    total = float(np.sum(sig ** 2))
    disc = float(np.sum(sig[new:] ** 2)) / total if total > 0 else 0.0
    # a tie: the last kept and first discarded values coincide to 1e-12 sigma_1 while the kept one
    # is above the rounding level (1e-13 sigma_1); among rounding-level values the choice changes
    # A B by less than 1e-13 relative, so it is not a tie in any sense that matters
    tie = bool(len(sig) > new and sig[new - 1] > 1e-13 * sig[0] and sig[new - 1] - sig[new] <= 1e-12 * sig[0])
    keep = sig[:new].copy()
    mask = (keep > 0) & (keep >= cutoff * sig[0])
    inv_sqrt = np.where(mask, 1.0 / np.sqrt(np.where(mask, keep, 1.0)), 0.0)
    if explicit:
        sq = np.where(mask, np.sqrt(keep), 0.0)
        new_a = U[:, :new] * sq
        new_b = sq[:, None] * Vt[:new]
    else:
        p_l = (r_b @ Vt[:new].T) * inv_sqrt           # D x chi'
        p_r = inv_sqrt[:, None] * (U[:, :new].T @ r_a)  # chi' x D
        new_a = a_mat @ p_l
        new_b = p_r @ b_mat
        if _PROJECTORS is not None:
            _PROJECTORS.append((list(shared), net.next_edge, p_l.copy(), p_r.copy()))
    e_new = net.next_edge
    net.next_edge += 1
    ops.append(OpRecord("compress", a, b, e_new, ma, D, mb, new, disc, tie))
    for e in shared:
        del net.ends[e]
        del net.dim[e]
    net.dim[e_new] = new
    net.ends[e_new] = [a, b]
    net.legs[a] = free_a + [e_new]
    net.legs[b] = [e_new] + free_b
    da = [net.dim[e] for e in free_a] + [new]
    db = [new] + [net.dim[e] for e in free_b]
    net.t[a] = _normalise(new_a.reshape(da), scales)
    net.t[b] = _normalise(new_b.reshape(db), scales)


def _bond_size(net: _Network, u: int, v: int) -> int:
    return int(np.prod([net.dim[e] for e in net.legs[u] if e in net.legs[v]]))


def _local_spanning_tree(net: _Network, a: int, b: int, r: int, n_inputs: int) -> List[Tuple[int, int]]:
    """The r-local spanning tree of SI A grown from S0 = {a, b}: repeatedly the best candidate
    pair (u in S, v outside) is taken, best = smallest distance from S0, then the largest bond
    between u and v (the connectivity the SI prefers), then the smallest v, then the smallest u;
    v joins while its distance is at most r.  Input tensors (ids below n_inputs) are not spanned
    (SI A excludes them).  Returns the pairs (u, v) in the order they were added."""
    import heapq
    S = {a, b}
    cand: list = []
    for u in (a, b):
        for v in sorted(net.neighbors(u)):
            if v not in S:
                heapq.heappush(cand, (1, -_bond_size(net, u, v), v, u))
    tau: List[Tuple[int, int]] = []
    while cand:
        d, _, v, u = heapq.heappop(cand)
        if v in S or d > r or v < n_inputs:
            continue
        S.add(v)
        tau.append((u, v))
        for w in sorted(net.neighbors(v)):
            if w not in S:
                heapq.heappush(cand, (d + 1, -_bond_size(net, v, w), w, v))
    return tau


def _tree_gauged_matrices(net: _Network, a: int, b: int, tau: List[Tuple[int, int]]):
    """Put the bond (a, b) in the tree gauge on virtual copies (section II.C, SI A): for the pairs
    of tau in reverse order (outer tensor v first), the R factor of v's copy matricised against
    its bond to u is absorbed into u's copy; returns A'_mat (rows: every other leg of a's copy)
    and B'_mat (columns: every other leg of b's copy), the bond legs in a's order."""
    virt: Dict[int, Tuple[np.ndarray, List[int]]] = {}
    next_virtual = [-1]

    def get(x):
        return virt[x] if x in virt else (net.t[x], list(net.legs[x]))

    for u, v in reversed(tau):
        arr, legs = get(v)
        bond = [e for e in legs if e in net.legs[u]]          # original u-v edges, v's order
        rest = [e for e in legs if e not in bond]
        D = int(np.prod([net.dim[e] for e in bond]))
        mat = np.transpose(arr, [legs.index(e) for e in rest + bond]).reshape(-1, D)
        R = np.linalg.qr(mat, mode="r") if mat.shape[0] > D else mat      # k x D
        uarr, ulegs = get(u)
        Rt = R.reshape([R.shape[0]] + [net.dim[e] for e in bond])
        out = np.tensordot(Rt, uarr, axes=(list(range(1, 1 + len(bond))), [ulegs.index(e) for e in bond]))
        new_leg = next_virtual[0]
        next_virtual[0] -= 1
        virt[u] = (out, [new_leg] + [e for e in ulegs if e not in bond])
    la = net.legs[a]
    shared = [e for e in la if e in net.legs[b]]
    mats = []
    for x, first in ((a, False), (b, True)):
        arr, legs = get(x)
        rest = [e for e in legs if e not in shared]
        D = int(np.prod([net.dim[e] for e in shared]))
        if first:
            mats.append(np.transpose(arr, [legs.index(e) for e in shared + rest]).reshape(D, -1))
        else:
            mats.append(np.transpose(arr, [legs.index(e) for e in rest + shared]).reshape(-1, D))
    return mats[0], mats[1]


def contract_compressed(n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray],
                        pairs: Sequence[Tuple[int, int]], chi: Optional[int], cutoff: float = 0.0,
                        explicit: bool = False, record: bool = False, compress_late: bool = False,
                        gauge_r: int = 0) -> OracleResult:
    """Run Algorithm 1 (r = 0) and return sign and ln|Z|.

    ``chi=None`` is exact contraction (no compression).  Step t of ``pairs``
    contracts live tensors (i, j) into a new tensor with id n + t; after each
    contraction every bond of the new tensor larger than chi is compressed,
    neighbours in ascending id (early compression), or, with
    ``compress_late``, the bonds of i and j are compressed just before they
    are contracted.  ``gauge_r`` > 0 computes every compression's R factors in
    the tree gauge of distance r (COMPRESS_TREE_GAUGE).  With ``record`` every
    normalised tensor is kept in creation order (inputs, then each op's outputs).
    """
    global _RECORD
    _RECORD = [] if record else None
    try:
        res = _run(n, edges, tensors, pairs, chi, cutoff, explicit, late=compress_late, gauge_r=gauge_r)
    finally:
        rec, _RECORD = _RECORD, None
    if record:
        res.tensors = rec
    return res


def contract_prefix(n, edges, tensors, pairs, chi, steps: int, cutoff: float = 0.0):
    """Run only the first ``steps`` tree steps of the same Algorithm 1 loop and return every
    normalised tensor written so far, in creation order (inputs first).  Used to compare a
    large instance's early intermediates one by one."""
    global _RECORD
    _RECORD = []
    try:
        _run(n, edges, tensors, pairs, chi, cutoff, False, max_steps=steps)
    except _OutOfTime:
        pass
    finally:
        rec, _RECORD = _RECORD, None
    return rec


def contract_steps(n, edges, tensors, pairs, chi, steps: int, cutoff: float = 0.0) -> List[OpRecord]:
    """Run the first ``steps`` tree steps of the Algorithm 1 loop (nothing recorded) and return
    the ops they expanded to; a fixed prefix for timing the oracle on a bounded sample."""
    ops: List[OpRecord] = []
    box = {"ops": ops}
    try:
        _run(n, edges, tensors, pairs, chi, cutoff, False, progress=box, max_steps=steps)
    except _OutOfTime:
        pass
    return box["ops"]


@dataclass
class PartialRun:
    steps_done: int
    ops: List[OpRecord]


def contract_compressed_budget(n, edges, tensors, pairs, chi, budget_s: float, cutoff: float = 0.0) -> PartialRun:
    """Run the same Algorithm 1 loop for at most ``budget_s`` seconds of wall time
    (the CPU-baseline timing sample); returns how many tree steps and ops ran."""
    import time
    deadline = time.time() + budget_s
    box = {}
    try:
        _run(n, edges, tensors, pairs, chi, cutoff, False, deadline=deadline, progress=box)
    except _OutOfTime:
        pass
    return PartialRun(box.get("steps", 0), box.get("ops", []))


class _OutOfTime(Exception):
    pass


def _run(n, edges, tensors, pairs, chi, cutoff, explicit, deadline=None, progress=None,
         max_steps=None, late=False, gauge_r=0) -> OracleResult:
    import time
    net = _Network(n, edges, tensors)
    scales: List[float] = []
    ops: List[OpRecord] = []
    if len(pairs) != n - 1:
        raise ValueError("a tree over n tensors has n - 1 steps")
    if progress is not None:
        progress["ops"] = ops
    try:
        for v in range(n):
            net.t[v] = _normalise(net.t[v], scales)
        for t, (i, j) in enumerate(pairs):
            if (deadline is not None and time.time() > deadline) or (max_steps is not None and t >= max_steps):
                raise _OutOfTime()
            k = n + t
            if i == j or i not in net.t or j not in net.t:
                raise ValueError(f"step {t}: ({i}, {j}) are not two live tensors")
            def compress(x, l):
                gauged = None
                if gauge_r > 0:
                    tau = _local_spanning_tree(net, x, l, gauge_r, n)
                    if tau:
                        gauged = _tree_gauged_matrices(net, x, l, tau)
                _compress(net, x, l, chi, cutoff, scales, ops, explicit, gauged)

            if late and chi is not None:
                for x, partner in ((i, j), (j, i)):
                    for l, shared in sorted(net.neighbors(x).items()):
                        if l != partner and int(np.prod([net.dim[e] for e in shared])) > chi:
                            compress(x, l)
            _contract(net, i, j, k, scales, ops)
            if chi is None or late:
                continue
            for l, shared in sorted(net.neighbors(k).items()):
                size = int(np.prod([net.dim[e] for e in shared]))
                if size > chi:
                    compress(k, l)
            if progress is not None:
                progress["steps"] = t + 1
    except ZeroContraction:
        return OracleResult(0.0, -math.inf, ops, scales)
    (last,) = net.t.values()
    x = float(last.reshape(()))
    ln_abs = math.fsum(scales) + math.log(abs(x))
    return OracleResult(math.copysign(1.0, x), ln_abs, ops, scales)
