"""A closed network that isolates one bond compression (test input).

Two factor tensors A and B share a composite bond of size D; A's remaining
legs go to two cap vectors P1, P2 and B's to Q1, Q2, each of dimension at
most chi, and A is first contracted with a one-entry tensor Z over an edge of
dimension 1.  Along the returned tree the first contraction therefore creates
a tensor equal to A whose only bond above chi is the one to B, so exactly one
compression runs, on A_mat (p1*p2 x D) and B_mat (D x q1*q2), and

    Z = kron(P1, P2)^T  trunc(A_mat B_mat)  kron(Q1, Q2),

where trunc is the compression of section II.C, Eq. (svd).  Nothing else in
the network is approximated, so the network's value checks the truncation
itself (its rank chi', its cutoff mask and its tie diagnostics).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .graphs import Graph


def bond_probe(a_mat: np.ndarray, b_mat: np.ndarray, shared_dims: Sequence[int], p_dims: Tuple[int, int],
               q_dims: Tuple[int, int], caps: Sequence[np.ndarray]):
    """Return (graph, tensors, pairs) for the network described above.

    ``a_mat`` is (p1*p2) x D with rows ordered (p1, p2) and columns in the
    order of ``shared_dims``; ``b_mat`` is D x (q1*q2).  ``caps`` holds the four
    cap vectors P1, P2, Q1, Q2.
    """
    shared_dims = [int(d) for d in shared_dims]
    D = int(np.prod(shared_dims))
    p1, p2 = (int(x) for x in p_dims)
    q1, q2 = (int(x) for x in q_dims)
    a_mat = np.asarray(a_mat, dtype=np.float64)
    b_mat = np.asarray(b_mat, dtype=np.float64)
    if a_mat.shape != (p1 * p2, D) or b_mat.shape != (D, q1 * q2):
        raise ValueError("a_mat must be (p1*p2) x D and b_mat D x (q1*q2)")
    # vertices: 0 = A, 1 = B, 2 = P1, 3 = P2, 4 = Q1, 5 = Q2, 6 = Z
    edges = [(0, 1, d) for d in shared_dims] + [(0, 2, p1), (0, 3, p2), (0, 6, 1), (1, 4, q1), (1, 5, q2)]
    g = Graph(7, sorted(edges))
    # A's axes in ascending edge id: shared..., p1, p2, z
    A = a_mat.reshape(p1, p2, *shared_dims)
    A = np.moveaxis(A, (0, 1), (len(shared_dims), len(shared_dims) + 1))[..., None]
    # B's axes: shared..., q1, q2
    B = b_mat.reshape(*shared_dims, q1, q2)
    P1, P2, Q1, Q2 = (np.asarray(c, dtype=np.float64) for c in caps)
    tensors: List[np.ndarray] = [A, B, P1, P2, Q1, Q2, np.ones(1)]
    # Z into A (7), P1 (8), P2 (9), then B (10), Q1 (11), Q2 (12)
    pairs = [(0, 6), (7, 2), (8, 3), (9, 1), (10, 4), (11, 5)]
    return g, tensors, pairs
