"""Repeated kept singular values on the single-vector Lanczos compression paths.

A Krylov space grown from one start vector holds one direction of each eigenspace, so a
single-vector Lanczos that stops when its Ritz pairs converge can miss further copies of a
repeated eigenvalue, and the truncation then keeps the wrong subspace (no tie flag: the gap
at the truncation boundary is wide).  These networks make the core of one bond have a kept
spectrum (chi = 6) with an exactly repeated value above many distinct smaller ones, so that
the Krylov space does not break down early: the library's result must still match the oracle.

Network (edges u < v, dims): e0 (0, 1, D), e1 (0, 3, n), e2 (1, 2, 1), e3 (1, 3, m).  The tree
contracts (1, 2) first; the new tensor's bond e0 to tensor 0 is compressed with tensor 0 as the
explicit side (n rows < D), whose A B = U diag(sigma) V^T by construction.
"""
import numpy as np
import pytest

import paper_2206_07044_amd as tn
from oracle.approx import contract_compressed
from tninputs import Graph

pytestmark = pytest.mark.gpu

# kept spectra at chi = 6 and the first value of the discarded tail (34+ distinct values down to
# 0.01): a repeated value in the middle of the kept set far above the tail, and one at the bottom
# of the kept set just above it (there a copy missing from the Krylov space would grow out of
# rounding only slowly, by the eigenvalue ratio 25 / 21.2 per step)
SPECTRA = {"middle": ([10.0, 8.0, 8.0, 8.0, 5.0, 4.0], 2.0), "bottom": ([10.0, 8.0, 6.0, 5.0, 5.0, 5.0], 4.6)}


def degenerate_network(D, n, m, seed, spectrum="middle"):
    rng = np.random.default_rng(seed)
    kept, top = SPECTRA[spectrum]
    r = min(n, D, m)                                            # rank of A B
    tail = np.geomspace(top, 0.01, r - len(kept))
    sigma = np.array(kept + list(tail))
    U = np.linalg.qr(rng.standard_normal((n, r)))[0]           # orthonormal columns
    Q1 = np.linalg.qr(rng.standard_normal((D, r)))[0]
    V = np.linalg.qr(rng.standard_normal((m, r)))[0]
    A = U @ np.diag(sigma) @ Q1.T                               # n x D: tensor 0 as (e1, e0)
    B = Q1 @ V.T                                                # D x m: tensor 1 as (e0, e3)
    g = Graph(4, [(0, 1, D), (0, 3, n), (1, 2, 1), (1, 3, m)])
    T0 = np.ascontiguousarray(A.T)                              # axes (e0, e1)
    T1 = np.ascontiguousarray(B.reshape(D, 1, m))               # axes (e0, e2, e3)
    T2 = np.ones(1)
    T3 = rng.standard_normal((n, m))                            # axes (e1, e3)
    return g, [T0, T1, T2, T3], [(1, 2), (0, 4), (5, 3)], sigma


def gpu_lnz(g, T, pairs, chi):
    eu, ev, ed = g.arrays()
    off = np.zeros(len(T) + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    data = np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T])
    c = tn.Context(0)
    try:
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi)
        c.tn_contract_compressed()
        return c.tn_result()
    finally:
        c.close()


# (D, n, m): tensor 0's side explicit (n < D) for D < 512 takes the Gram-Lanczos core; both sides
# taller than D > 256 take Golub-Kahan-Lanczos on A B
def _cases():
    for spectrum in sorted(SPECTRA):
        for D, n, m in [(100, 40, 300), (200, 48, 260), (300, 200, 400), (300, 600, 640)]:
            for seed in (0, 1):
                yield pytest.param(D, n, m, seed, spectrum, id=f"{spectrum}-D{D}-n{n}-m{m}-s{seed}")


@pytest.mark.parametrize("D,n,m,seed,spectrum", list(_cases()))
def test_repeated_kept_singular_values_lanczos(D, n, m, seed, spectrum):
    g, T, pairs, sigma = degenerate_network(D, n, m, seed, spectrum)
    ref = contract_compressed(g.n, g.edges, T, pairs, 6)
    comp = [o for o in ref.ops if o.kind == "compress"]
    assert len(comp) >= 2 and comp[0].n == D and comp[0].new_dim == 6
    assert not any(o.tie for o in comp), "the oracle sees a tie: the case is not sharp"
    sign, lnz = gpu_lnz(g, T, pairs, 6)
    print(f"{spectrum} D={D} n={n} m={m} seed={seed}: GPU {sign:+.0f} {lnz:.15f}  oracle {ref.sign:+.0f} {ref.ln_abs_z:.15f}",
          flush=True)
    assert sign == ref.sign
    assert abs(lnz - ref.ln_abs_z) <= 1e-10 * max(1.0, abs(ref.ln_abs_z))


# The block-Krylov chain (D >= 512 with an explicit side) works on a basis of 4 chi' directions
# in blocks of 8 (a repeated value of multiplicity up to 8 lies inside one block) and accepts
# Ritz pairs whose residual is below 1e-8 sigma_1^2.  On these spectra the discarded tail has
# 294 values decaying by about 2% per index, far flatter than a tensor network's: with the kept
# values at the bottom of the kept set just above that tail (4.6 against 5) the basis cannot
# resolve them and the library reports TN_ENUMERIC; with them well separated (2 against 4) it
# converges, but only to the residual tolerance, and ln Z is off by about 2e-9 relative.
def test_block_krylov_flat_tail_reports_non_convergence():
    g, T, pairs, _ = degenerate_network(600, 300, 700, 0, "bottom")
    with pytest.raises(tn.TNError) as e:
        gpu_lnz(g, T, pairs, 6)
    assert e.value.status == tn.TN_ENUMERIC


@pytest.mark.xfail(strict=True, reason="block-Krylov Ritz residual tolerance 1e-8 sigma_1^2: a flat "
                                       "294-value tail leaves ln Z about 2e-9 off, above the 1e-10 bar")
def test_block_krylov_flat_tail_value():
    g, T, pairs, _ = degenerate_network(600, 300, 700, 1, "middle")
    ref = contract_compressed(g.n, g.edges, T, pairs, 6)
    sign, lnz = gpu_lnz(g, T, pairs, 6)
    assert sign == ref.sign and abs(lnz - ref.ln_abs_z) <= 1e-10 * max(1.0, abs(ref.ln_abs_z))
