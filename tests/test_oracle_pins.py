"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test compares the oracle with something that is not the oracle:
closed forms, brute-force sums over spin/matching configurations, layer
transfer matrices, numpy's SVD of an explicitly formed product (Eckart-Young),
or an invariance the method must have.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from oracle.approx import _Network, _compress
from tninputs import (uniform_tensors, dimer_tensors, greedy_tree, ising_bond_factors, ising_tensors, lattice,
                      normal_tensors, random_regular3, Graph)
from tninputs.trees import sweep_tree


def run(g, T, pairs, chi, **kw):
    return oracle.contract_compressed(g.n, g.edges, T, pairs, chi, **kw)


# ---------------------------------------------------------------- inputs (SI F.1)
@pytest.mark.parametrize("J", [1.0, -1.0, 0.7, -2.3])
def test_ising_split_is_boltzmann_matrix(J):
    beta = 0.44
    lo, hi = ising_bond_factors(beta, J)
    spins = np.array([1.0, -1.0])
    want = np.exp(beta * J * np.outer(spins, spins))
    np.testing.assert_allclose(lo @ hi, want, rtol=1e-14)
    np.testing.assert_allclose(lo, lo.T, atol=0)
    np.testing.assert_allclose(hi, hi.T, atol=0)


def test_ising_factor_equals_paper_matrix_for_ferromagnet():
    beta = 0.3
    c, s = math.cosh(beta), math.sinh(beta)
    paper = np.array([[math.sqrt(c) + math.sqrt(s), math.sqrt(c) - math.sqrt(s)],
                      [math.sqrt(c) - math.sqrt(s), math.sqrt(c) + math.sqrt(s)]]) / math.sqrt(2)
    lo, hi = ising_bond_factors(beta, 1.0)
    np.testing.assert_allclose(lo, paper, rtol=1e-15)
    np.testing.assert_allclose(hi, paper, rtol=1e-15)
    np.testing.assert_allclose(paper @ paper, np.exp(beta * np.array([[1, -1], [-1, 1]])), rtol=1e-14)


# ---------------------------------------------------------------- exact references agree with each other
def test_transfer_matrix_equals_brute_force():
    g = lattice((3, 4))
    J = np.random.default_rng(3).choice([-1.0, 1.0], g.n_edges)
    a = exact.ising_transfer_matrix((3, 4), 0.5, J, g.edges)
    b = exact.ising_brute_force(g.n, g.edges, 0.5, J)
    assert abs(a - b) < 1e-12


def test_transfer_matrix_equals_brute_force_3d():
    g = lattice((2, 2, 4))
    a = exact.ising_transfer_matrix((2, 2, 4), 0.3)
    b = exact.ising_brute_force(g.n, g.edges, 0.3)
    assert abs(a - b) < 1e-12


# ---------------------------------------------------------------- oracle exact mode (chi = None), Eq. tncontract
@pytest.mark.parametrize("shape,beta", [((3, 3), 0.44), ((4, 4), 0.2), ((2, 3, 3), 0.3)])
def test_exact_mode_matches_brute_force_ising(shape, beta):
    g = lattice(shape)
    J = np.random.default_rng(1).choice([-1.0, 1.0], g.n_edges)
    T = ising_tensors(g, beta, J)
    pairs = greedy_tree(g, 4, seed=0)
    r = run(g, T, pairs, None)
    assert r.sign == 1.0
    assert abs(r.ln_abs_z - exact.ising_brute_force(g.n, g.edges, beta, J)) < 1e-11


def test_exact_mode_8x8_transfer_matrix():
    g = lattice((8, 8))
    T = ising_tensors(g, 0.44)
    tm = exact.ising_transfer_matrix((8, 8), 0.44)
    assert abs(tm - 56.879536639072) < 1e-9          # value recomputed, not trusted
    for pairs in (sweep_tree((8, 8)), greedy_tree(g, 16, seed=0)):
        r = run(g, T, pairs, None)
        assert abs(r.ln_abs_z - tm) / tm < 1e-13


def test_forest_and_ring_closed_forms():
    rng = np.random.default_rng(0)
    # random tree on 12 vertices plus an isolated vertex (a forest with 2 components)
    edges = sorted((int(rng.integers(0, v)), v, 2) for v in range(1, 12))
    g = Graph(13, edges)
    J = rng.normal(size=len(edges))
    T = ising_tensors(g, 0.7, J)
    r = run(g, T, greedy_tree(g, 4, seed=1), 2)        # chi=2: bonds of a forest never exceed 2
    assert abs(r.ln_abs_z - exact.ising_forest(g.n, g.edges, 0.7, J)) < 1e-12
    ring = Graph(9, sorted([(i, i + 1, 2) for i in range(8)] + [(0, 8, 2)]))
    J = rng.choice([-1.0, 1.0], ring.n_edges)
    T = ising_tensors(ring, 0.9, J)
    r = run(ring, T, greedy_tree(ring, 2, seed=0), None)
    assert abs(r.ln_abs_z - exact.ising_ring(0.9, J)) < 1e-12


# ---------------------------------------------------------------- dimers (SI F.3)
def _complete(n):
    return Graph(n, [(u, v, 2) for u in range(n) for v in range(u + 1, n)])


def _petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return Graph(10, sorted((min(u, v), max(u, v), 2) for u, v in outer + spokes + inner))


def _cube():
    return Graph(8, sorted((u, u ^ (1 << b), 2) for u in range(8) for b in range(3) if u < u ^ (1 << b)))


def _k33():
    return Graph(6, [(u, v, 2) for u in range(3) for v in range(3, 6)])


def _prism():
    e = [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (0, 3), (1, 4), (2, 5)]
    return Graph(6, sorted((u, v, 2) for u, v in e))


@pytest.mark.parametrize("g,count", [(_complete(4), 3), (_k33(), 6), (_prism(), 4), (_cube(), 9), (_petersen(), 6)])
def test_dimer_counts_textbook(g, count):
    assert exact.perfect_matchings(g.n, g.edges) == count
    r = run(g, dimer_tensors(g), greedy_tree(g, 64, seed=0), None)
    assert r.sign == 1.0 and abs(math.exp(r.ln_abs_z) - count) < 1e-9


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dimer_random_regular_exact(seed):
    g = random_regular3(20, seed)
    want = exact.perfect_matchings(g.n, g.edges)
    r = run(g, dimer_tensors(g), greedy_tree(g, 1 << 20, seed=seed), None)
    assert abs(r.ln_abs_z - math.log(want)) < 1e-11


def test_dimer_zero_when_no_matching():
    g = Graph(3, [(0, 1, 2), (0, 2, 2), (1, 2, 2)])     # triangle: odd vertex count
    r = run(g, dimer_tensors(g), [(0, 1), (3, 2)], 4)
    assert r.sign == 0.0 and r.ln_abs_z == -math.inf


# ---------------------------------------------------------------- compression primitive (II.C, SI B)
def _two_block_network(rng, m1, dims, m2):
    """P -e0- A =shared= B -e3- Q, returns net and (A, B) ids."""
    edges = [(0, 1, m1)] + [(1, 2, d) for d in dims] + [(2, 3, m2)]
    A = rng.normal(size=(m1,) + tuple(dims))
    B = rng.normal(size=tuple(dims) + (m2,))
    T = [rng.normal(size=(m1,)), A, B, rng.normal(size=(m2,))]
    return _Network(4, edges, T), A, B


@pytest.mark.parametrize("m1,dims,m2,chi", [(40, (3, 4), 30, 5), (6, (3, 4), 50, 4), (7, (2, 2, 2), 5, 3), (64, (8, 8), 64, 16)])
def test_compression_is_truncated_svd_of_product(m1, dims, m2, chi):
    rng = np.random.default_rng(m1 + m2)
    net, A, B = _two_block_network(rng, m1, dims, m2)
    D = int(np.prod(dims))
    M = A.reshape(m1, D) @ B.reshape(D, m2)
    scales, ops = [], []
    _compress(net, 1, 2, chi, 0.0, scales, ops, explicit=False)
    a2, b2 = net.t[1], net.t[2]
    approx = (a2.reshape(m1, -1) @ b2.reshape(-1, m2)) * math.exp(scales[0] + scales[1]) \
        / (np.max(np.abs(A)) * np.max(np.abs(B))) * np.max(np.abs(A)) * np.max(np.abs(B))
    U, s, Vt = np.linalg.svd(M)
    k = min(chi, min(m1, D), min(m2, D))
    best = (U[:, :k] * s[:k]) @ Vt[:k]
    np.testing.assert_allclose(approx, best, rtol=0, atol=1e-11 * np.abs(M).max())
    err = np.linalg.norm(M - approx)
    assert abs(err - math.sqrt(np.sum(s[k:] ** 2))) <= 1e-9 * np.linalg.norm(M)
    assert ops[0].new_dim == k
    assert abs(ops[0].discarded - np.sum(s[k:] ** 2) / np.sum(s ** 2)) < 1e-12


def test_qr_form_equals_explicit_product_svd():
    g = lattice((3, 4))
    T = normal_tensors(g, 0.3, 5)
    pairs = sweep_tree((3, 4))
    for chi in (2, 3, 4):
        a = run(g, T, pairs, chi)
        b = run(g, T, pairs, chi, explicit=True)
        assert a.sign == b.sign and abs(a.ln_abs_z - b.ln_abs_z) < 1e-12


# ---------------------------------------------------------------- executor invariants
def test_large_chi_is_exact_3d():
    g = lattice((3, 3, 4))
    T = ising_tensors(g, 0.22)
    tm = exact.ising_transfer_matrix((3, 3, 4), 0.22)
    pairs = sweep_tree((3, 3, 4))
    r = run(g, T, pairs, 1 << 12)
    assert not any(o.kind == "compress" for o in r.ops)
    assert abs(r.ln_abs_z - tm) / tm < 1e-13
    # compressions at or above the rank discard nothing and stay exact
    # (Ising copy tensors make bonds rank deficient: chi below the bond size)
    for shape, chi in (((3, 3, 2), 4), ((2, 2, 5), 32), ((2, 2, 2, 2), 16)):
        g2 = lattice(shape)
        T2 = ising_tensors(g2, 0.3)
        r2 = run(g2, T2, sweep_tree(shape), chi)
        comp = [o for o in r2.ops if o.kind == "compress"]
        assert comp and max(o.discarded for o in comp) < 1e-24
        assert abs(r2.ln_abs_z - exact.ising_brute_force(g2.n, g2.edges, 0.3)) < 1e-12


def test_truncation_error_falls_with_chi():
    g = lattice((8, 8))
    T = ising_tensors(g, 0.44)
    tm = exact.ising_transfer_matrix((8, 8), 0.44)
    pairs = sweep_tree((8, 8))
    errs = [abs(run(g, T, pairs, chi).ln_abs_z - tm) for chi in (2, 4, 8, 16, 32, 64)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-12   # chi = 64 covers every bond of this tree


@pytest.mark.parametrize("chi", [2, 4, None])
def test_homogeneity_in_each_tensor(chi):
    g = lattice((3, 4))
    T = normal_tensors(g, 0.2, 11)
    pairs = sweep_tree((3, 4))
    base = run(g, T, pairs, chi)
    for v, alpha in ((0, -3.5), (5, 1e-7), (11, 2.0e5)):
        T2 = [t.copy() for t in T]
        T2[v] = T2[v] * alpha
        r = run(g, T2, pairs, chi)
        assert r.sign == base.sign * math.copysign(1.0, alpha)
        assert abs(r.ln_abs_z - (base.ln_abs_z + math.log(abs(alpha)))) < 1e-11


def _orthogonal(rng, d):
    q, r = np.linalg.qr(rng.normal(size=(d, d)))
    return q * np.sign(np.diag(r))


@pytest.mark.parametrize("chi", [2, 3, 8])
def test_orthogonal_gauge_invariance(chi):
    """Inserting O O^T on any edge leaves the compressed value unchanged: the
    QR-reduced truncated SVD only sees the bond space through orthogonally
    invariant quantities."""
    g = lattice((3, 4))
    rng = np.random.default_rng(2)
    T = normal_tensors(g, 0.25, 4)
    pairs = sweep_tree((3, 4))
    base = run(g, T, pairs, chi)
    inc = g.incident()
    T2 = [t.copy() for t in T]
    for e, (u, v, d) in enumerate(g.edges):
        O = _orthogonal(rng, d)
        ax_u = inc[u].index(e)
        ax_v = inc[v].index(e)
        T2[u] = np.moveaxis(np.tensordot(T2[u], O, axes=([ax_u], [0])), -1, ax_u)
        T2[v] = np.moveaxis(np.tensordot(T2[v], O, axes=([ax_v], [0])), -1, ax_v)
    r = run(g, T2, pairs, chi)
    assert r.sign == base.sign
    assert abs(r.ln_abs_z - base.ln_abs_z) < 1e-11


def test_running_exponent_avoids_overflow():
    """ln Z ~ 4500 overflows float64 if contracted naively; the running
    exponent keeps it exact (checked against a transfer matrix)."""
    g = lattice((3, 3, 60))
    T = ising_tensors(g, 2.0)
    tm = exact.ising_transfer_matrix((3, 3, 60), 2.0)
    assert tm > 709.8
    r = run(g, T, sweep_tree((3, 3, 60), order=(2, 0, 1)), 1 << 12)
    assert abs(r.ln_abs_z - tm) / tm < 1e-13


# ---------------------------------------------------------------- cutoff mask and tie flag (section II.C, Eq. (svd))
def _probe_value(a_mat, b_mat, caps, chi, cutoff):
    """kron(P1,P2)^T trunc(A_mat B_mat) kron(Q1,Q2) from numpy's SVD of the explicit product:
    the chi' = min(chi, k_A, k_B) largest triplets, those with sigma_i < cutoff * sigma_1 zeroed."""
    M = a_mat @ b_mat
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    D = a_mat.shape[1]
    k = min(chi, min(a_mat.shape[0], D), min(b_mat.shape[1], D))
    keep = s[:k] * ((s[:k] > 0) & (s[:k] >= cutoff * s[0]))
    u = np.kron(caps[0], caps[1])
    w = np.kron(caps[2], caps[3])
    return float(u @ (U[:, :k] * keep) @ Vt[:k] @ w), k


def _probe_run(a_mat, b_mat, shared, p, q, caps, chi, cutoff):
    from tninputs.probes import bond_probe
    g, T, pairs = bond_probe(a_mat, b_mat, shared, p, q, caps)
    r = run(g, T, pairs, chi, cutoff=cutoff)
    comp = [o for o in r.ops if o.kind == "compress"]
    assert len(comp) == 1, "the probe network must compress exactly one bond"
    return r, comp[0]


@pytest.mark.parametrize("cut_between", [None, 1, 2, 4])
@pytest.mark.parametrize("chi", [3, 5])
def test_cutoff_mask_is_relative_truncated_svd(cut_between, chi):
    """cutoff > 0 zeroes the kept triplets with sigma_i < cutoff * sigma_1 (relative to the
    largest), on top of the truncation to chi'; checked against numpy's SVD of A_mat B_mat."""
    rng = np.random.default_rng(40 + chi)
    p, q, shared = (2, 3), (3, 2), (2, 4)
    a_mat = rng.normal(size=(6, 8)) * (0.3 ** np.arange(8))      # graded spectrum
    b_mat = rng.normal(size=(8, 6))
    caps = [rng.normal(size=d) + 1.0 for d in (*p, *q)]
    s = np.linalg.svd(a_mat @ b_mat, compute_uv=False)
    cutoff = 0.0 if cut_between is None else math.sqrt(s[cut_between - 1] * s[cut_between]) / s[0]
    r, op = _probe_run(a_mat, b_mat, shared, p, q, caps, chi, cutoff)
    want, k = _probe_value(a_mat, b_mat, caps, chi, cutoff)
    assert op.new_dim == k
    assert r.sign == math.copysign(1.0, want)
    assert abs(r.ln_abs_z - math.log(abs(want))) < 1e-12


def test_cutoff_scale_invariance():
    """The cutoff is relative: scaling A by 1e-30 changes ln|Z| by ln(1e-30) only.  An
    absolute cutoff would drop every triplet of the scaled network."""
    rng = np.random.default_rng(9)
    p, q, shared = (2, 2), (2, 2), (2, 3)
    a_mat = rng.normal(size=(4, 6)) * (0.1 ** np.arange(6))
    b_mat = rng.normal(size=(6, 4))
    caps = [rng.normal(size=2) + 1.0 for _ in range(4)]
    s = np.linalg.svd(a_mat @ b_mat, compute_uv=False)
    cutoff = math.sqrt(s[1] * s[2]) / s[0]
    r1, o1 = _probe_run(a_mat, b_mat, shared, p, q, caps, 3, cutoff)
    r2, o2 = _probe_run(a_mat * 1e-30, b_mat, shared, p, q, caps, 3, cutoff)
    assert abs(r2.ln_abs_z - (r1.ln_abs_z + math.log(1e-30))) < 1e-11
    want, _ = _probe_value(a_mat, b_mat, caps, 3, cutoff)
    assert abs(r1.ln_abs_z - math.log(abs(want))) < 1e-12


def test_cutoff_boundary_value_is_kept():
    """A singular value exactly equal to cutoff * sigma_1 is kept (only sigma_i < cutoff *
    sigma_1 is zeroed); one ulp above the boundary drops it.  The core is an exactly
    representable diagonal, so both sides of the comparison are exact."""
    a = np.array([1.0, 0.5, 2.0 ** -5, 2.0 ** -9])
    b = np.array([1.0, 0.5, 2.0 ** -5, 2.0 ** -11])        # sigma = 1, 2^-2, 2^-10, 2^-20
    caps = [np.array([1.0, 0.75]), np.array([0.5, 1.0]), np.array([1.0, 0.25]), np.array([0.75, 1.0])]
    args = (np.diag(a), np.diag(b), (2, 2), (2, 2), (2, 2), caps, 3)
    at, _ = _probe_run(*args, 2.0 ** -10)
    above, _ = _probe_run(*args, 2.0 ** -10 * (1.0 + 2.0 ** -52))
    none, _ = _probe_run(*args, 0.0)
    u = np.kron(caps[0], caps[1])
    w = np.kron(caps[2], caps[3])
    sig = a * b
    assert at.ln_abs_z == pytest.approx(math.log(sum(u[i] * sig[i] * w[i] for i in range(3))), abs=1e-14)
    assert above.ln_abs_z == pytest.approx(math.log(sum(u[i] * sig[i] * w[i] for i in range(2))), abs=1e-14)
    assert none.ln_abs_z == at.ln_abs_z
    assert abs(at.ln_abs_z - above.ln_abs_z) > 1e-4


@pytest.mark.parametrize("last,gap,flag", [(0.5, 0.0, True), (0.5, 2.0 ** -41, True), (0.5, 2.0 ** -38, False),
                                           (0.5, 1e-9, False), (2.0 ** -40, 0.0, True), (2.0 ** -60, 0.0, False)])
def test_tie_flag_at_truncation_boundary(last, gap, flag):
    """The tie flag marks sigma_chi' - sigma_chi'+1 <= 1e-12 sigma_1 (several truncations are
    then equally correct): gaps 0 and 2^-41 ~ 4.5e-13 flag, 2^-38 ~ 3.6e-12 and 1e-9 do not.
    Equal values at the rounding level (sigma_chi' <= 1e-13 sigma_1, here 2^-60) are no tie;
    equal values just above it (2^-40 ~ 9.1e-13) are."""
    sig = np.array([1.0, 0.75, last, last - gap])
    caps = [np.array([1.0, 0.5]), np.array([0.5, 1.0]), np.array([1.0, 0.25]), np.array([0.75, 1.0])]
    _, op = _probe_run(np.eye(4), np.diag(sig), (2, 2), (2, 2), (2, 2), caps, 3, 0.0)
    assert op.tie is flag
    assert op.discarded == pytest.approx(sig[3] ** 2 / np.sum(sig ** 2), rel=1e-14)


def test_cutoff_is_relative_not_absolute():
    """Factors close to all-ones give a core whose sigma_1 is far above 1 even after every
    tensor is normalised to max |entry| = 1, so a relative and an absolute reading of the
    cutoff keep different triplets here; the oracle must follow the relative one."""
    rng = np.random.default_rng(17)
    p, q, shared = (2, 2), (2, 2), (2, 3)
    a_mat = np.ones((4, 6)) + 0.2 * rng.normal(size=(4, 6)) * (0.5 ** np.arange(6))
    b_mat = np.ones((6, 4)) + 0.2 * rng.normal(size=(6, 4))
    a_mat /= np.abs(a_mat).max()
    b_mat /= np.abs(b_mat).max()
    caps = [rng.uniform(0.5, 1.0, size=2) for _ in range(4)]
    s = np.linalg.svd(a_mat @ b_mat, compute_uv=False)
    assert s[0] > 10.0
    cutoff = math.sqrt(s[1] * s[2]) / s[0]          # relative: keeps 2 of them
    assert s[2] >= cutoff                             # absolute would keep the third too
    r, op = _probe_run(a_mat, b_mat, shared, p, q, caps, 3, cutoff)
    rel, _ = _probe_value(a_mat, b_mat, caps, 3, cutoff)
    absolute, _ = _probe_value(a_mat, b_mat, caps, 3, cutoff / s[0])
    assert abs(math.log(abs(rel)) - math.log(abs(absolute))) > 1e-6
    assert abs(r.ln_abs_z - math.log(abs(rel))) < 1e-12


# ---------------------------------------------------------------------------- late compression
def test_late_compression_before_first_contraction_is_truncated_svd():
    """Section II.D: with compress_late the bond between A and B of the one-compression probe is
    compressed before A's first contraction, on A's own rows; the network's value is then
    kron(P1, P2)^T trunc(A_mat B_mat) kron(Q1, Q2), the rank-chi' truncated SVD of the product."""
    from tninputs.probes import bond_probe
    rng = np.random.default_rng(17)
    a_mat = rng.normal(size=(6, 8))
    b_mat = rng.normal(size=(8, 6))
    caps = [rng.normal(size=d) for d in (2, 3, 3, 2)]
    g, T, pairs = bond_probe(a_mat, b_mat, (2, 4), (2, 3), (3, 2), caps)
    for chi in (1, 2, 3, 5):
        r = oracle.contract_compressed(g.n, g.edges, T, pairs, chi, compress_late=True)
        assert r.ops[0].kind == "compress" and (r.ops[0].a, r.ops[0].b) == (0, 1)
        U, s, Vt = np.linalg.svd(a_mat @ b_mat)
        k = min(chi, 6)
        want = np.kron(caps[0], caps[1]) @ ((U[:, :k] * s[:k]) @ Vt[:k]) @ np.kron(caps[2], caps[3])
        assert r.sign == np.sign(want)
        assert r.ln_abs_z == pytest.approx(math.log(abs(want)), rel=1e-12)


@pytest.mark.parametrize("shape,beta", [((3, 3), 0.44), ((2, 2, 3), 0.3), ((3, 4), 0.6)])
def test_late_compression_without_truncation_is_exact(shape, beta):
    g = lattice(shape)
    T = ising_tensors(g, beta)
    r = oracle.contract_compressed(g.n, g.edges, T, sweep_tree(shape), 4096, compress_late=True)
    assert r.ln_abs_z == pytest.approx(exact.ising_brute_force(g.n, g.edges, beta, None), rel=1e-13)


def test_late_and_early_compress_at_different_points():
    g = lattice((6, 6))
    T = uniform_tensors(g, -0.5, 3)
    pairs = sweep_tree((6, 6))
    early = oracle.contract_compressed(g.n, g.edges, T, pairs, 2)
    late = oracle.contract_compressed(g.n, g.edges, T, pairs, 2, compress_late=True)
    ex = oracle.contract_compressed(g.n, g.edges, T, pairs, None)
    kinds = lambda r: [o.kind for o in r.ops]
    assert kinds(early) != kinds(late)
    # after every contraction of the early schedule, a compression touches the new tensor only
    assert all(o.a >= g.n for o in early.ops if o.kind == "compress")
    # late: every compression acts on a tensor that the next contraction consumes
    for t, o in enumerate(late.ops):
        if o.kind == "compress":
            nxt = next(p for p in late.ops[t:] if p.kind == "contract")
            assert o.a in (nxt.a, nxt.b)
    assert early.ln_abs_z != late.ln_abs_z and ex.sign != 0


# ---------------------------------------------------------------------------- tree gauge (r >= 1)
def _rank1_environment_network():
    """A0 and B0 share a composite bond of 2 x 2; A0 has two more legs (dim 2) to vectors P and X,
    B0 to vectors Q and Y, each vector an intermediate (the contraction of two inputs); A0 is then
    contracted with a one-entry tensor, so the intermediate A's bond to B0 (4 > chi = 2) is
    compressed while P, X, Q, Y are live intermediates next to it."""
    rng = np.random.default_rng(23)
    # 0 = A0, 1 = B0, 2/3 = p1/p2, 4/5 = x1/x2, 6/7 = q1/q2, 8/9 = y1/y2, 10 = one-entry Z
    raw = [(0, 1, 2), (0, 1, 2), (0, 2, 2), (0, 4, 2), (0, 10, 1), (1, 6, 2), (1, 8, 2),
           (2, 3, 2), (4, 5, 2), (6, 7, 2), (8, 9, 2)]
    g = Graph(11, sorted(raw))
    inc = g.incident()
    T = [rng.normal(size=tuple(g.edges[e][2] for e in inc[v])) for v in range(11)]
    T[10] = np.ones(1)
    # P = 11, X = 12, Q = 13, Y = 14, A = 15
    pairs = [(2, 3), (4, 5), (6, 7), (8, 9), (0, 10), (15, 11), (16, 12), (17, 1), (18, 13), (19, 14)]
    return g, T, pairs


def test_tree_gauge_uses_the_environment():
    """Section II.C / SI A: with the bond (A, B0) in the tree gauge, A's R factor is that of
    (P x X)^T A (the vectors' R factors absorbed), a single row, and B0's that of B0 (Q x Y); the
    core is then the scalar Z itself and chi = 2 reproduces Z exactly, while the local compression
    (r = 0) keeps the best rank-2 part of the 4 x 4 product A B0 alone and does not."""
    g, T, pairs = _rank1_environment_network()
    ex = oracle.contract_compressed(g.n, g.edges, T, pairs, None)
    r0 = oracle.contract_compressed(g.n, g.edges, T, pairs, 2)
    r1 = oracle.contract_compressed(g.n, g.edges, T, pairs, 2, gauge_r=1)
    assert any(o.kind == "compress" for o in r1.ops)
    assert r1.sign == ex.sign and r1.ln_abs_z == pytest.approx(ex.ln_abs_z, rel=1e-13)
    assert abs(r0.ln_abs_z - ex.ln_abs_z) > 1e-3


def test_local_spanning_tree_rule():
    """SI A: grown from S0 = {a, b}; the closest candidate with the largest bond first; input
    tensors are never spanned; nodes beyond distance r are left out."""
    from oracle.approx import _Network, _local_spanning_tree
    # 0..3 inputs; 4..9 intermediates (as a network they are just tensors with ids)
    edges = sorted([(4, 5, 2), (4, 6, 3), (4, 7, 2), (5, 8, 2), (6, 9, 2), (7, 9, 2), (5, 0, 2), (0, 4, 2)])
    edges = sorted((min(u, v), max(u, v), d) for u, v, d in edges)
    g = Graph(10, edges)
    inc = g.incident()
    net = _Network(10, g.edges, [np.ones(tuple(g.edges[e][2] for e in inc[v])) for v in range(10)])
    tau = _local_spanning_tree(net, 4, 5, 2, n_inputs=4)
    # distance 1 from {4, 5}: 6 (bond 3) before 7 (bond 2), then 8 (bond 2); input 0 is skipped;
    # distance 2: 9 is reached from 6 (popped first among equal bonds by the smaller u... 9 via 6)
    assert tau == [(4, 6), (4, 7), (5, 8), (6, 9)]
    assert _local_spanning_tree(net, 4, 5, 1, n_inputs=4) == [(4, 6), (4, 7), (5, 8)]


@pytest.mark.parametrize("shape,beta,seed,chi", [((3, 3), 0.44, None, 2), ((3, 4), 0.6, 3, 2), ((4, 4), 0.44, 4, 4),
                                                 ((2, 2, 3), 0.3, 5, 8)])
def test_tree_gauge_exact_regime(shape, beta, seed, chi):
    # compressions of rank-deficient Ising cores that truncate nothing stay exact in any gauge
    g = lattice(shape)
    J = None if seed is None else np.where(np.random.default_rng(seed).random(g.n_edges) < 0.5, -1.0, 1.0)
    T = ising_tensors(g, beta, J)
    want = exact.ising_brute_force(g.n, g.edges, beta, J)
    for r in (1, 2, 3):
        res = oracle.contract_compressed(g.n, g.edges, T, sweep_tree(shape), chi, gauge_r=r)
        assert any(o.kind == "compress" for o in res.ops)
        assert res.ln_abs_z == pytest.approx(want, rel=1e-12)


def test_tree_gauge_improves_late_compression_2d():
    """Section II.D, Fig. "early vs late" C: on the 2D URand model (D = 4, entries in [-0.5, 1]) with
    late compression, a larger tree-gauge distance gives a smaller error; here on 8x8 at chi = 8
    over six seeds (median |1 - Z/Z_exact|: r = 0 2.9e-3, r = 2 1.9e-4, r = 4 2.9e-5)."""
    g = lattice((8, 8), dim=4)
    pairs = sweep_tree((8, 8))
    exact_tree = greedy_tree(g, 1 << 40, 0, temperature=0.0)
    med = {}
    for r in (0, 2, 4):
        errs = []
        for sd in range(6):
            T = uniform_tensors(g, -0.5, sd)
            ex = oracle.contract_compressed(g.n, g.edges, T, exact_tree, None)
            a = oracle.contract_compressed(g.n, g.edges, T, pairs, 8, gauge_r=r, compress_late=True)
            errs.append(abs(1.0 - a.sign * ex.sign * math.exp(a.ln_abs_z - ex.ln_abs_z)))
        med[r] = float(np.median(errs))
    assert med[4] < med[2] < med[0] and med[4] < 0.05 * med[0]
