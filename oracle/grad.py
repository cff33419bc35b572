"""Reference gradient d ln|Z| / d(input tensors) of Algorithm 1 (section II.F,
r = 0, early compression) — float64 numpy, reverse mode.  Test infrastructure
only (see the package docstring).

The paper computes no gradients; this module differentiates the same forward
computation as ``oracle.approx`` (same readings, same op order).  Its own
readings, also listed in the design notes:

* Scale factors are constants.  Every tensor is divided by its largest |entry|
  after it is written; each op of Algorithm 1 is homogeneous (a contraction is
  bilinear, and a compression maps (x A, y B) to (sqrt(xy) A', sqrt(xy) B')),
  so the final value times the product of the scales is the same for any
  choice of scales, and differentiating with the scales frozen is exact.
* A compression is a function of the product K = A_mat B_mat alone: with
  A_mat = Q_A R_A and B_mat^T = Q_B R_B^T, a' = Q_A U sqrt(s) and
  b' = sqrt(s) V^T Q_B^T, i.e. the rank-chi' truncated SVD of K split
  symmetrically (section II.C, Eq. (svd); SI B).  Its adjoint is the textbook
  adjoint of a truncated SVD, written out below with the COMPLETE singular
  spectrum of the reduced core (kept, discarded and zero singular values).
* Pairs of kept singular values take the gauge-invariant form.  The SVD of
  Eq. (svd) fixes the kept singular vectors only up to rotations among equal
  singular values, and every later step of Algorithm 1 (a contraction, or a
  compression whose R factors and core see the new bond through a Gram matrix
  or the product K) is equivariant under an orthogonal change of basis of the
  bond a compression creates; so ln|Z| is invariant under it, and its
  derivative along such a rotation vanishes.  Substituting that identity into
  the textbook kept-kept entry f (alpha_ji s_i + beta_ji s_j - alpha_ij s_i
  - beta_ij s_j), f = 1 / (s_i^2 - s_j^2), cancels the factor s_i - s_j and
  leaves (alpha_ji + beta_ij) / (s_i + s_j): equal in exact arithmetic, but
  with no division by a gap between kept values, which would amplify the
  rounding of the incoming adjoint by s_1^2 / (s_i^2 - s_j^2), and with the
  right limit at an exact degeneracy.  Pairs of a kept and a discarded (or
  zero) value keep 1 / (s_i^2 - s_j^2): that gap is the conditioning of the
  truncation itself.
* Singular values at or below 1e-13 s_1 are rounding-level zeros of the core:
  they are treated as exactly zero (a kept one gives a constant zero column,
  as does one below ``cutoff * s_1``).  The gradient is then that of the
  rank-preserving truncation; contracted with a perturbation that keeps every
  core's rank (Ising couplings, a rescaling) it is the exact derivative, while
  a generic perturbation of a rank-deficient core would create new singular
  values of order sqrt(|dK|) and ln|Z| need not be differentiable there.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .approx import ZeroContraction, _Network

_NOISE_REL = 1e-13


@dataclass
class GradResult:
    sign: float
    ln_abs_z: float
    grads: List[np.ndarray]     # d ln|Z| / d T_v, input layout (axes = incident edges ascending)


def _scale(arr: np.ndarray) -> float:
    s = float(np.max(np.abs(arr))) if arr.size else 0.0
    if s == 0.0:
        raise ZeroContraction()
    if not math.isfinite(s):
        raise FloatingPointError("non-finite tensor entry")
    return s


def lnz_and_grad(n: int, edges: Sequence[Tuple[int, int, int]], tensors: Sequence[np.ndarray],
                 pairs: Sequence[Tuple[int, int]], chi: int, cutoff: float = 0.0,
                 compress_late: bool = False) -> GradResult:
    """Forward pass of Algorithm 1 recording a tape, then its adjoint (early or late compression,
    in the order of oracle.approx)."""
    net = _Network(n, edges, tensors)
    tape: List[tuple] = []
    log_scales: List[float] = []
    in_scale: Dict[int, float] = {}
    for v in range(n):
        s = _scale(net.t[v])
        in_scale[v] = s
        log_scales.append(math.log(s))
        net.t[v] = net.t[v] / s
    for t, (i, j) in enumerate(pairs):
        k = n + t
        if compress_late:
            for x, partner in ((i, j), (j, i)):
                for l, shared in sorted(net.neighbors(x).items()):
                    if l != partner and int(np.prod([net.dim[e] for e in shared])) > chi:
                        tape.append(_compress_fwd(net, x, l, chi, cutoff, log_scales))
        tape.append(_contract_fwd(net, i, j, k, log_scales))
        if compress_late:
            continue
        for l, shared in sorted(net.neighbors(k).items()):
            if int(np.prod([net.dim[e] for e in shared])) > chi:
                tape.append(_compress_fwd(net, k, l, chi, cutoff, log_scales))
    (root,) = net.t.keys()
    x = float(net.t[root].reshape(()))
    ln_abs = math.fsum(log_scales) + math.log(abs(x))

    # reverse sweep; adjoints are with respect to the normalised tensors
    adj: Dict[int, np.ndarray] = {root: np.array(1.0 / x).reshape(net.t[root].shape)}
    for rec in reversed(tape):
        if rec[0] == "contract":
            _contract_bwd(rec, adj)
        else:
            _compress_bwd(rec, adj)
    grads = [adj[v] / in_scale[v] for v in range(n)]
    return GradResult(math.copysign(1.0, x), ln_abs, grads)


# ---------------------------------------------------------------- contraction

def _contract_fwd(net: _Network, i: int, j: int, k: int, log_scales: List[float]):
    """C = sum over shared edges of T_i T_j (Fig. "tensor primitives" B), axes
    free(i) then free(j); then C / max|C|."""
    li, lj = net.legs.pop(i), net.legs.pop(j)
    ti, tj = net.t.pop(i), net.t.pop(j)
    shared = [e for e in li if e in lj]
    free_i = [e for e in li if e not in shared]
    free_j = [e for e in lj if e not in shared]
    out = np.tensordot(ti, tj, axes=([li.index(e) for e in shared], [lj.index(e) for e in shared]))
    for e in shared:
        del net.ends[e]
    for e in free_i + free_j:
        ends = net.ends[e]
        ends[ends.index(i if e in free_i else j)] = k
    s = _scale(out)
    log_scales.append(math.log(s))
    net.legs[k] = free_i + free_j
    net.t[k] = out / s
    return ("contract", i, j, k, li, lj, shared, free_i, free_j, ti, tj, s)


def _contract_bwd(rec, adj: Dict[int, np.ndarray]) -> None:
    _, i, j, k, li, lj, shared, free_i, free_j, ti, tj, s = rec
    gk = adj.pop(k) / s                                   # adjoint of the unnormalised C
    nfi = len(free_i)
    # C[fi, fj] = sum_sh Ti[fi, sh] Tj[sh, fj]  =>  dTi = C_bar Tj^T, dTj = Ti^T C_bar
    ti_p = np.transpose(ti, [li.index(e) for e in free_i + shared])
    tj_p = np.transpose(tj, [lj.index(e) for e in shared + free_j])
    gi_p = np.tensordot(gk, tj_p, axes=(list(range(nfi, gk.ndim)), list(range(len(shared), tj_p.ndim))))
    gj_p = np.tensordot(ti_p, gk, axes=(list(range(nfi)), list(range(nfi))))
    adj[i] = np.transpose(gi_p, np.argsort([li.index(e) for e in free_i + shared]))
    adj[j] = np.transpose(gj_p, np.argsort([lj.index(e) for e in shared + free_j]))


# ---------------------------------------------------------------- compression

def _compress_fwd(net: _Network, a: int, b: int, chi: int, cutoff: float, log_scales: List[float]):
    """Section II.C: R factors by QR (or the factor itself when it has no more
    rows than D_AB), SVD of R_A R_B, keep chi' = min(chi, k_A, k_B) triplets,
    a' = A P_L, b' = P_R B with P_L = R_B V s^-1/2, P_R = s^-1/2 U^T R_A."""
    la, lb = net.legs[a], net.legs[b]
    shared = [e for e in la if e in lb]
    free_a = [e for e in la if e not in shared]
    free_b = [e for e in lb if e not in shared]
    perm_a = [la.index(e) for e in free_a + shared]
    perm_b = [lb.index(e) for e in shared + free_b]
    ta = np.transpose(net.t[a], perm_a)
    tb = np.transpose(net.t[b], perm_b)
    D = int(np.prod([net.dim[e] for e in shared]))
    ma, mb = ta.size // D, tb.size // D
    A = ta.reshape(ma, D)
    B = tb.reshape(D, mb)
    if ma > D:
        q_a, r_a = np.linalg.qr(A)                 # A = Q_A R_A
    else:
        q_a, r_a = np.eye(ma), A
    if mb > D:
        q_b, r = np.linalg.qr(B.T)                 # B^T = Q_B R_B^T
        r_b = r.T                                   # D x k_b, B = r_b Q_B^T
    else:
        q_b, r_b = np.eye(mb), B
    ka, kb = r_a.shape[0], r_b.shape[1]
    U, sig, Vt = np.linalg.svd(r_a @ r_b, full_matrices=True)
    new = min(chi, ka, kb)
    keep = sig[:new]
    mask = (keep > _NOISE_REL * sig[0]) & (keep >= cutoff * sig[0])
    sq = np.where(mask, np.sqrt(np.where(mask, keep, 1.0)), 0.0)
    inv_sqrt = np.where(mask, 1.0 / np.where(mask, sq, 1.0), 0.0)
    p_l = (r_b @ Vt[:new].T) * inv_sqrt
    p_r = inv_sqrt[:, None] * (U[:, :new].T @ r_a)
    new_a = A @ p_l
    new_b = p_r @ B
    e_new = net.next_edge
    net.next_edge += 1
    for e in shared:
        del net.ends[e]
        del net.dim[e]
    net.dim[e_new] = new
    net.ends[e_new] = [a, b]
    net.legs[a] = free_a + [e_new]
    net.legs[b] = [e_new] + free_b
    sa, sb = _scale(new_a), _scale(new_b)
    log_scales.append(math.log(sa))
    log_scales.append(math.log(sb))
    net.t[a] = new_a.reshape([net.dim[e] for e in free_a] + [new]) / sa
    net.t[b] = new_b.reshape([new] + [net.dim[e] for e in free_b]) / sb
    core = dict(A=A, B=B, q_a=q_a, q_b=q_b, U=U, sig=sig, V=Vt.T, new=new, mask=mask, sq=sq)
    return ("compress", a, b, la, lb, perm_a, perm_b, ta.shape, tb.shape, core, sa, sb)


def _compress_bwd(rec, adj: Dict[int, np.ndarray]) -> None:
    """Adjoint of (A, B) -> (Uh_K sqrt(s), sqrt(s) Vh_K^T), the truncated SVD
    K = Uh s Vh^T of K = A B with Uh = Q_A U, Vh = Q_B V."""
    _, a, b, la, lb, perm_a, perm_b, shape_a, shape_b, c, sa, sb = rec
    A, B, q_a, q_b, U, sig, V = c["A"], c["B"], c["q_a"], c["q_b"], c["U"], c["sig"], c["V"]
    new, mask, sq = c["new"], c["mask"], c["sq"]
    ma, D = A.shape
    mb = B.shape[1]
    ka, kb = U.shape[0], V.shape[0]
    g_a = adj.pop(a).reshape(ma, new) / sa          # adjoint of a' = A P_L (unnormalised)
    g_b = adj.pop(b).reshape(new, mb) / sb          # adjoint of b' = P_R B

    uh = q_a @ U                                     # ma x ka, left singular vectors of K (complete in range Q_A)
    vh = q_b @ V                                     # mb x kb
    K_idx = [i for i in range(new) if mask[i]]
    s_all = np.zeros(max(ka, kb))
    s_all[:len(sig)] = np.where(sig > _NOISE_REL * sig[0], sig, 0.0)

    u_bar = g_a * sq                                 # dL/dU_K  (columns i < new; masked columns are 0)
    v_bar = g_b.T * sq                               # dL/dV_K
    alpha = uh.T @ u_bar                             # ka x new: components of u_bar on every left vector
    beta = vh.T @ v_bar                              # kb x new
    J = np.zeros((ka, kb))
    for i in K_idx:
        si = sig[i]
        J[i, i] += (float(uh[:, i] @ g_a[:, i]) + float(g_b[i, :] @ vh[:, i])) / (2.0 * sq[i])
        for j in range(max(ka, kb)):
            if j == i:
                continue
            sj = s_all[j]
            if j in K_idx:                           # kept pair: gauge-invariant form, row j column i
                J[j, i] += (alpha[j, i] + beta[i, j]) / (si + sj)
                continue
            f = 1.0 / (si * si - sj * sj)
            if j < ka:                               # u_bar_i along u_j
                J[j, i] += alpha[j, i] * si * f
                if j < kb:
                    J[i, j] += alpha[j, i] * sj * f
            if j < kb:                               # v_bar_i along v_j
                J[i, j] += beta[j, i] * si * f
                if j < ka:
                    J[j, i] += beta[j, i] * sj * f
    inv_s = np.zeros(new)
    inv_s[K_idx] = 1.0 / sig[K_idx]
    # components of u_bar / v_bar outside range(Q_A) / range(Q_B): the null space of K^T / K
    u_perp = u_bar - q_a @ (q_a.T @ u_bar)
    v_perp = v_bar - q_b @ (q_b.T @ v_bar)
    BVh = B @ vh                                     # D x kb
    AtUh = A.T @ uh                                  # D x ka
    # K_bar = uh J vh^T + u_perp s^-1 vh_K^T + uh_K s^-1 v_perp^T ; A_bar = K_bar B^T, B_bar = A^T K_bar
    # (u_perp^T... terms vanish against B^T / A: range(B^T) = range(Q_B), range(A) = range(Q_A))
    g_A = uh @ J @ BVh.T + (u_perp * inv_s) @ BVh[:, :new].T
    g_B = AtUh @ J @ vh.T + (AtUh[:, :new] * inv_s) @ v_perp.T
    adj[a] = np.transpose(g_A.reshape(shape_a), np.argsort(perm_a))
    adj[b] = np.transpose(g_B.reshape(shape_b), np.argsort(perm_b))


# ---------------------------------------------------------------- Ising couplings

def ising_coupling_grad(n: int, edges: Sequence[Tuple[int, int, int]], beta: float, J,
                        grads: Sequence[np.ndarray]) -> np.ndarray:
    """d ln|Z| / d J_e from d ln|Z| / d T_v for the Ising tensors of SI F.1.

    T_v = sum_s prod_{e at v} W^(e)[s, :], W^(e) = H diag(sqrt c, +-sqrt|s|) H / sqrt 2
    with c = cosh(beta J_e), s = sinh(beta J_e) (the sign of sinh on the higher
    vertex id); J_e enters only its own bond factor at each of its two ends.
    """
    J = np.asarray(J, dtype=np.float64)
    H = np.array([[1.0, 1.0], [1.0, -1.0]])
    inc: List[List[int]] = [[] for _ in range(n)]
    for e, (u, v, _) in enumerate(edges):
        inc[u].append(e)
        inc[v].append(e)
    out = np.zeros(len(edges))

    def factor(e, hi, deriv):
        x = beta * J[e]
        c, s = math.cosh(x), math.sinh(x)
        sg = math.copysign(1.0, s) if hi else 1.0
        if deriv:   # d/dJ of (sqrt c, sg sqrt|s|)
            d = [beta * s / (2.0 * math.sqrt(c)), sg * beta * c * math.copysign(1.0, s) / (2.0 * math.sqrt(abs(s)))]
        else:
            d = [math.sqrt(c), sg * math.sqrt(abs(s))]
        return H @ np.diag(d) @ H / math.sqrt(2.0)

    for v in range(n):
        es = sorted(inc[v])
        for pos, e in enumerate(es):
            mats = [factor(f, v == edges[f][1], f == e) for f in es]
            dt = np.zeros((2,) * len(es))
            for s in range(2):
                term = np.array(1.0)
                for m in mats:
                    term = np.multiply.outer(term, m[s])
                dt = dt + term
            out[e] += float(np.sum(dt * grads[v]))
    return out
