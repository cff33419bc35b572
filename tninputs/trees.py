"""Seeded ordered contraction-tree builders and the tree cost model.

A tree is a list of ``n - 1`` pairs ``(i, j)``; step ``t`` contracts the live
tensors ``i`` and ``j`` into a new tensor with id ``n + t`` (main text II.A:
an approximate contraction tree is an *ordered* sequence of pairwise
contractions, and compressions are implied by it).  Tree search is not the
subject of this package: these builders only produce a reasonable fixed tree
from a seed, following the Greedy and Span families of section II.G / SI C.

``simulate_tree`` traces the compressed contraction on bond sizes only
(early compression, gauge distance 0) and returns the peak memory M and the
cost C of SI section D.
"""
from __future__ import annotations

import heapq
import math
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .graphs import Graph


def _bond_sizes(g: Graph) -> List[Dict[int, int]]:
    nb: List[Dict[int, int]] = [dict() for _ in range(g.n)]
    for u, v, d in g.edges:
        nb[u][v] = nb[u].get(v, 1) * d
        nb[v][u] = nb[v].get(u, 1) * d
    return nb


def _prod(vals) -> int:
    p = 1
    for x in vals:
        p *= x
    return p


@dataclass
class TreeStats:
    """Traced cost of a compressed contraction tree (SI section D)."""
    peak_elems: int = 0            # M: max over stages of the summed live tensor sizes
    largest_elems: int = 0         # W: largest single tensor
    contract_macs: float = 0.0     # sum of m*n*k over contractions
    qr_flops: float = 0.0          # sum of 2 m n^2 - 2/3 n^3 over R-factor QRs
    svd_flops: float = 0.0         # sum of 4 m n^2 - 4/3 n^3 over cores
    core_macs: float = 0.0         # R_A @ R_B
    reabsorb_macs: float = 0.0     # A @ P_L and P_R @ B
    n_contract: int = 0
    n_compress: int = 0
    max_bond_uncompressed: int = 0
    max_core: int = 0
    ops: List[tuple] = field(default_factory=list)

    @property
    def cost_C(self) -> float:
        """The paper's C: contraction mnk + QR + SVD terms."""
        return self.contract_macs + self.qr_flops + self.svd_flops

    @property
    def flops(self) -> float:
        """Algorithmic flops with 2 flops per multiply-add."""
        return 2 * (self.contract_macs + self.core_macs + self.reabsorb_macs) + self.qr_flops + self.svd_flops


def _qr_flops(m: int, n: int) -> float:
    return 2.0 * m * n * n - 2.0 / 3.0 * n ** 3


def simulate_tree(g: Graph, pairs: Sequence[Tuple[int, int]], chi: int, record_ops: bool = False) -> TreeStats:
    """Trace Algorithm 1 (early compression, r = 0) on bond sizes only."""
    nb = _bond_sizes(g)
    bonds: Dict[int, Dict[int, int]] = {v: dict(nb[v]) for v in range(g.n)}
    size: Dict[int, int] = {v: _prod(nb[v].values()) for v in range(g.n)}
    st = TreeStats()
    live = sum(size.values())
    st.peak_elems = live
    st.largest_elems = max(size.values()) if size else 0
    for t, (i, j) in enumerate(pairs):
        k = g.n + t
        if i not in bonds or j not in bonds or i == j:
            raise ValueError(f"step {t}: pair ({i},{j}) is not two live tensors")
        bi, bj = bonds.pop(i), bonds.pop(j)
        shared = bi.get(j, 1)
        mi, mj = size.pop(i) // shared, size.pop(j) // shared
        st.contract_macs += float(mi) * shared * mj
        st.n_contract += 1
        if record_ops:
            st.ops.append(("contract", i, j, k, mi, shared, mj))
        bk: Dict[int, int] = {}
        for src, other in ((bi, j), (bj, i)):
            for l, d in src.items():
                if l == other:
                    continue
                bk[l] = bk.get(l, 1) * d
        for l in bk:
            bl = bonds[l]
            bl.pop(i, None)
            bl.pop(j, None)
            bl[k] = bk[l]
        bonds[k] = bk
        size[k] = mi * mj
        live = live - (mi * shared) - (mj * shared) + size[k]
        st.peak_elems = max(st.peak_elems, live + (mi * shared) + (mj * shared))
        st.largest_elems = max(st.largest_elems, size[k])
        for l in sorted(bk):
            D = bk[l]
            st.max_bond_uncompressed = max(st.max_bond_uncompressed, D)
            if D <= chi:
                continue
            ma, mb = size[k] // D, size[l] // D
            ka, kb = min(ma, D), min(mb, D)
            new = min(chi, ka, kb)
            if ma > D:
                st.qr_flops += _qr_flops(ma, D)
            if mb > D:
                st.qr_flops += _qr_flops(mb, D)
            st.core_macs += float(ka) * D * kb
            p, q = max(ka, kb), min(ka, kb)
            st.svd_flops += 4.0 * p * q * q - 4.0 / 3.0 * q ** 3
            st.reabsorb_macs += float(ma) * D * new + float(new) * D * mb
            st.max_core = max(st.max_core, max(ka, kb))
            st.n_compress += 1
            if record_ops:
                st.ops.append(("compress", k, l, ma, D, mb, new))
            live -= size[k] + size[l]
            size[k] = ma * new
            size[l] = mb * new
            live += size[k] + size[l]
            bk[l] = new
            bonds[l][k] = new
    return st


def _gumbel(rng) -> float:
    return -math.log(-math.log(rng.uniform(1e-300, 1.0)))


def greedy_tree(g: Graph, chi: int, seed: int = 0, temperature: float = 0.25) -> List[Tuple[int, int]]:
    """Greedy family (main text II.G, SI C.1), with fixed score weights.

    The score of contracting neighbours (i, j) is
    log2 size(k after simulated compression) - log2 size(i) - log2 size(j)
    plus ``temperature`` times a Gumbel sample drawn from default_rng(seed);
    the lowest score is contracted first.  Simulated compression caps each
    bond of k at chi.
    """
    rng = np.random.default_rng(seed)
    nb = _bond_sizes(g)
    bonds: Dict[int, Dict[int, int]] = {v: dict(nb[v]) for v in range(g.n)}
    lsize: Dict[int, float] = {v: sum(math.log2(d) for d in nb[v].values()) for v in range(g.n)}
    version: Dict[int, int] = {v: 0 for v in range(g.n)}
    heap: list = []

    def score(i: int, j: int) -> float:
        bi, bj = bonds[i], bonds[j]
        tot = 0.0
        merged: Dict[int, int] = {}
        for src, other in ((bi, j), (bj, i)):
            for l, d in src.items():
                if l != other:
                    merged[l] = merged.get(l, 1) * d
        for d in merged.values():
            tot += math.log2(min(d, chi))
        return tot - lsize[i] - lsize[j] + temperature * _gumbel(rng)

    def push(i: int, j: int) -> None:
        a, b = (i, j) if i < j else (j, i)
        heapq.heappush(heap, (score(a, b), a, b, version[a], version[b]))

    seen = set()
    for u, v, _ in g.edges:
        if (u, v) not in seen:
            seen.add((u, v))
            push(u, v)

    pairs: List[Tuple[int, int]] = []
    nxt = g.n
    while heap:
        _, a, b, va, vb = heapq.heappop(heap)
        if a not in bonds or b not in bonds or version[a] != va or version[b] != vb:
            continue
        k = nxt
        nxt += 1
        pairs.append((a, b))
        bi, bj = bonds.pop(a), bonds.pop(b)
        bk: Dict[int, int] = {}
        for src, other in ((bi, b), (bj, a)):
            for l, d in src.items():
                if l != other:
                    bk[l] = bk.get(l, 1) * d
        for l in bk:
            bonds[l].pop(a, None)
            bonds[l].pop(b, None)
            if bk[l] > chi:
                bk[l] = chi
            bonds[l][k] = bk[l]
        bonds[k] = bk
        lsize[k] = sum(math.log2(d) for d in bk.values())
        version[k] = 0
        for l in bk:
            lsize[l] = sum(math.log2(d) for d in bonds[l].values())
            version[l] += 1
        for l in sorted(bk):
            push(k, l)
            for m in sorted(bonds[l]):
                if m != k:
                    push(l, m)
    # disconnected components: join what is left by outer products
    rest = sorted(bonds)
    while len(rest) > 1:
        a, b = rest[0], rest[1]
        pairs.append((a, b))
        k = nxt
        nxt += 1
        bonds.pop(a)
        bonds.pop(b)
        bonds[k] = {}
        rest = sorted(bonds)
    return pairs


def centrality(g: Graph) -> np.ndarray:
    """c[v] = (1/Z) sum_{u != v} 1/sqrt(d(u, v) + 1), scaled to [0, 1] (SI C)."""
    nbrs = g.neighbors()
    c = np.zeros(g.n)
    for v in range(g.n):
        dist = [-1] * g.n
        dist[v] = 0
        q = deque([v])
        while q:
            x = q.popleft()
            for y in nbrs[x]:
                if dist[y] < 0:
                    dist[y] = dist[x] + 1
                    q.append(y)
        c[v] = sum(1.0 / math.sqrt(d + 1) for u, d in enumerate(dist) if u != v and d >= 0)
    lo, hi = c.min(), c.max()
    return (c - lo) / (hi - lo) if hi > lo else np.ones(g.n)


def span_tree(g: Graph, seed: int = 0, start: str = "max", temperature: float = 0.05,
              w_distance: float = 1.0, w_connectivity: float = 0.5, w_ndim: float = 0.0,
              w_centrality: float = 0.0) -> List[Tuple[int, int]]:
    """Span family (main text II.G, SI C.2): grow a spanning tree from the most
    (``start='max'``) or least central vertex and contract it leaves-inwards.

    The next spanning-tree pair (u, v) maximises
    -w_distance*r + w_connectivity*log2(connectivity of v to the span)
    - w_ndim*deg(v) + w_centrality*c[v] + temperature*Gumbel.
    Each tree pair (u, v) becomes the contraction (u, v) -> u, in reverse order.
    """
    rng = np.random.default_rng(seed)
    cent = centrality(g)
    nb = _bond_sizes(g)
    i0 = int(np.argmax(cent)) if start == "max" else int(np.argmin(cent))
    in_s = np.zeros(g.n, dtype=bool)
    in_s[i0] = True
    conn = np.zeros(g.n)  # log2 product of edge dims from v to the span
    heap: list = []
    tau: List[Tuple[int, int]] = []

    def push(u: int, v: int, r: int) -> None:
        s = (-w_distance * r + w_connectivity * conn[v] - w_ndim * len(nb[v])
             + w_centrality * cent[v] + temperature * _gumbel(rng))
        heapq.heappush(heap, (-s, r, u, v))

    for v, d in sorted(nb[i0].items()):
        conn[v] += math.log2(d)
    for v in sorted(nb[i0]):
        push(i0, v, 1)
    while heap:
        _, r, u, v = heapq.heappop(heap)
        if in_s[v]:
            continue
        in_s[v] = True
        tau.append((u, v))
        for w, d in sorted(nb[v].items()):
            if not in_s[w]:
                conn[w] += math.log2(d)
                push(v, w, r + 1)
    if len(tau) != g.n - 1:
        raise ValueError("span_tree needs a connected graph")
    cur = list(range(g.n))
    pairs: List[Tuple[int, int]] = []
    for t, (u, v) in enumerate(reversed(tau)):
        pairs.append((cur[u], cur[v]))
        cur[u] = g.n + t
    return pairs


def sweep_tree(shape: Sequence[int], order: Optional[Sequence[int]] = None) -> List[Tuple[int, int]]:
    """Span-family tree on an open-boundary lattice with an axis-ordered spanning tree.

    The spanning tree is rooted at the origin; the parent of a site is its
    neighbour one step back along the last axis on which its coordinate is
    nonzero.  Pairs are listed by axis (first axis first) and, within an
    axis, by distance from the root; contracting them in reverse (SI C.2)
    sweeps a boundary through the lattice along the last axis, then the
    next, like boundary-MPS/PEPS contraction (section III.A) but produced
    by the generic Span machinery.  ``order`` lists the axes in spanning-tree
    order (default 0, 1, ...); the last one listed is contracted first.
    """
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[:a])) for a in range(nd)]
    order = list(range(nd)) if order is None else [int(a) for a in order]
    if sorted(order) != list(range(nd)):
        raise ValueError("order must be a permutation of the axes")
    rank = {a: i for i, a in enumerate(order)}
    tau: List[Tuple[int, int]] = []
    for a in order:
        # sites whose nonzero coordinate latest in ``order`` is on axis a
        sites = []
        for v in range(n):
            c = [(v // strides[b]) % shape[b] for b in range(nd)]
            nz = sorted((b for b in range(nd) if c[b] > 0), key=rank.get)
            if nz and nz[-1] == a:
                sites.append((c[a], tuple(reversed(c)), v))
        sites.sort()
        for _, _, v in sites:
            tau.append((v - strides[a], v))
    cur = list(range(n))
    pairs: List[Tuple[int, int]] = []
    for t, (u, v) in enumerate(reversed(tau)):
        pairs.append((cur[u], cur[v]))
        cur[u] = n + t
    return pairs


class _BondSim:
    """Live tensors of a partially contracted network, on bond sizes only, with
    every bond of a new tensor capped at chi (early compression); contractions
    are emitted as tree pairs with fresh ids n, n + 1, ..."""

    def __init__(self, g: Graph, chi: int):
        self.chi = chi
        nb = _bond_sizes(g)
        self.bonds: Dict[int, Dict[int, int]] = {v: dict(nb[v]) for v in range(g.n)}
        self.nxt = g.n
        self.pairs: List[Tuple[int, int]] = []

    def lsize(self, v: int) -> float:
        return sum(math.log2(d) for d in self.bonds[v].values())

    def merged_lsize(self, i: int, j: int) -> float:
        merged: Dict[int, int] = {}
        for src, other in ((self.bonds[i], j), (self.bonds[j], i)):
            for l, d in src.items():
                if l != other:
                    merged[l] = merged.get(l, 1) * d
        return sum(math.log2(min(d, self.chi)) for d in merged.values())

    def contract(self, a: int, b: int) -> int:
        k = self.nxt
        self.nxt += 1
        self.pairs.append((a, b))
        bi, bj = self.bonds.pop(a), self.bonds.pop(b)
        bk: Dict[int, int] = {}
        for src, other in ((bi, b), (bj, a)):
            for l, d in src.items():
                if l != other:
                    bk[l] = bk.get(l, 1) * d
        for l in bk:
            self.bonds[l].pop(a, None)
            self.bonds[l].pop(b, None)
            bk[l] = min(bk[l], self.chi)
            self.bonds[l][k] = bk[l]
        self.bonds[k] = bk
        return k


def _spectral_bisect(nodes: List[int], w: Dict[int, Dict[int, float]], rng, noise: float) -> Tuple[List[int], List[int]]:
    """Split ``nodes`` into two halves of equal size (+-1) along the Fiedler vector of the
    weighted Laplacian of the subgraph they induce, then improve the cut by pair swaps."""
    n = len(nodes)
    idx = {v: i for i, v in enumerate(nodes)}
    Lap = np.zeros((n, n))
    for v in nodes:
        for u, x in w[v].items():
            if u in idx:
                Lap[idx[v], idx[u]] -= x
                Lap[idx[v], idx[v]] += x
    vals, vecs = np.linalg.eigh(Lap)
    f = vecs[:, 1] if n > 1 else np.zeros(1)
    f = f + noise * np.std(f) * rng.normal(size=n)
    order = np.argsort(f, kind="stable")
    side = np.zeros(n, dtype=np.int8)
    side[order[n // 2:]] = 1
    # Kernighan-Lin style passes: swap the best pair while the cut weight falls
    for _ in range(4):
        gain = np.zeros(n)
        for v in nodes:
            iv = idx[v]
            for u, x in w[v].items():
                if u in idx:
                    gain[iv] += x if side[idx[u]] != side[iv] else -x
        improved = False
        for _ in range(max(1, n // 4)):
            a = [i for i in range(n) if side[i] == 0]
            b = [i for i in range(n) if side[i] == 1]
            ia = max(a, key=lambda i: gain[i])
            ib = max(b, key=lambda i: gain[i])
            wab = w[nodes[ia]].get(nodes[ib], 0.0)
            if gain[ia] + gain[ib] - 2 * wab <= 1e-12:
                break
            for i in (ia, ib):
                v = nodes[i]
                side[i] ^= 1
                gain[i] = -gain[i]
                for u, x in w[v].items():
                    if u in idx and u != nodes[ia + ib - i]:
                        j = idx[u]
                        gain[j] += 2 * x if side[j] != side[i] else -2 * x
            improved = True
        if not improved:
            break
    left = [nodes[i] for i in range(n) if side[i] == 0]
    right = [nodes[i] for i in range(n) if side[i] == 1]
    return left, right


def agglom_tree(g: Graph, chi: int, k: int = 8, seed: int = 0, noise: float = 0.05,
                temperature: float = 0.1) -> List[Tuple[int, int]]:
    """Agglom family (main text II.G, SI C.3) with recursive spectral bisection in
    place of a hypergraph partitioner.

    The live network is split into parts of about ``k`` tensors (recursive
    bisection of the graph weighted by log2 bond size); each part is
    contracted by Greedy moves restricted to its members, with every bond of a
    new tensor capped at chi (the compression that early compression will
    perform); the parts then form the coarse network of the next round, which
    is partitioned again, until one tensor is left.  ``seed`` drives the noise
    added to the Fiedler vectors and the Gumbel term of the Greedy score, so
    that different seeds give different trees.
    """
    rng = np.random.default_rng(seed)
    sim = _BondSim(g, chi)
    while len(sim.bonds) > 1:
        live = sorted(sim.bonds)
        w = {v: {u: math.log2(d) + 1e-3 for u, d in sim.bonds[v].items()} for v in live}
        parts = [live]
        while max(len(p) for p in parts) > k:
            nxt_parts = []
            for p in parts:
                if len(p) > k:
                    nxt_parts.extend(_spectral_bisect(p, w, rng, noise))
                else:
                    nxt_parts.append(p)
            parts = nxt_parts
        progressed = False
        for p in parts:
            members = set(p)
            while True:
                best = None
                for i in sorted(members):
                    for j in sorted(sim.bonds[i]):
                        if j in members and i < j:
                            s = sim.merged_lsize(i, j) - sim.lsize(i) - sim.lsize(j) + temperature * _gumbel(rng)
                            if best is None or s < best[0]:
                                best = (s, i, j)
                if best is None:
                    break
                _, i, j = best
                members.discard(i)
                members.discard(j)
                members.add(sim.contract(i, j))
                progressed = True
        if not progressed:
            # parts with no internal bond left: join the two smallest connected live tensors
            best = None
            for i in sorted(sim.bonds):
                for j in sorted(sim.bonds[i]):
                    if i < j:
                        s = sim.merged_lsize(i, j)
                        if best is None or s < best[0]:
                            best = (s, i, j)
            if best is None:   # disconnected components: outer products
                rest = sorted(sim.bonds)
                sim.contract(rest[0], rest[1])
            else:
                sim.contract(best[1], best[2])
    return sim.pairs


def sample_trees(g: Graph, chi: int, count: int, seed: int = 0) -> List[Tuple[str, List[Tuple[int, int]]]]:
    """Candidate trees for a host-side search (section II.H): ``count`` draws over the three
    generator families with seeded hyper-parameters (Greedy: temperature and the simulated bond
    dimension chi_greedy of SI C.1; Span: start vertex, temperature and score weights of SI C.2;
    Agglom: part size k of SI C.3).  Returns (label, pairs) per candidate."""
    rng = np.random.default_rng(seed)
    out: List[Tuple[str, List[Tuple[int, int]]]] = []
    for c in range(count):
        fam = c % 3
        s = int(rng.integers(0, 2 ** 31))
        if fam == 0:
            temp = float(rng.choice([0.0, 0.1, 0.25, 0.5, 1.0]))
            chi_g = int(rng.choice([2, chi, 4 * chi]))
            out.append((f"greedy(chi_g={chi_g}, T={temp}, seed={s})", greedy_tree(g, chi_g, s, temperature=temp)))
        elif fam == 1:
            start = str(rng.choice(["max", "min"]))
            temp = float(rng.choice([0.0, 0.05, 0.2]))
            wc = float(rng.choice([0.0, 0.5, 1.0]))
            out.append((f"span(start={start}, T={temp}, w_conn={wc}, seed={s})",
                        span_tree(g, seed=s, start=start, temperature=temp, w_connectivity=wc)))
        else:
            k = int(rng.choice([4, 8, 16]))
            out.append((f"agglom(k={k}, seed={s})", agglom_tree(g, chi, k=k, seed=s)))
    return out
