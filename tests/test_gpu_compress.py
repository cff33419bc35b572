"""The standalone bond compression (tn_compress_pair) against the definition it computes:
a' b' is the rank-chi' truncated SVD of A B (section II.C, Eq. (svd); Eckart-Young), and
a' = U_chi' s^1/2, b' = s^1/2 V_chi'^T up to the sign of each singular pair (SI B's projector
form: A P_L = Q_A U s^1/2).  numpy's SVD of the explicitly formed product is the reference."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2206_07044_amd as tn  # noqa: E402
from paper_2206_07044_amd._capi import TNError, TN_EINVAL  # noqa: E402

pytestmark = pytest.mark.gpu


def _graded(rng, m, n, ratio):
    """Random m x n matrix whose singular values fall geometrically from 1 to `ratio`."""
    k = min(m, n)
    q1, _ = np.linalg.qr(rng.normal(size=(m, k)))
    q2, _ = np.linalg.qr(rng.normal(size=(n, k)))
    s = np.logspace(0.0, math.log10(ratio), k) if k > 1 else np.ones(1)
    return (q1 * s) @ q2.T


def _run(c, A, B, chi, cutoff=0.0):
    ma, D = A.shape
    mb = B.shape[1]
    dA = torch.tensor(A, dtype=torch.float64, device="cuda")
    dB = torch.tensor(B, dtype=torch.float64, device="cuda")
    k = min(chi, min(ma, D), min(mb, D))
    oa = torch.full((ma * max(k, 1),), float("nan"), dtype=torch.float64, device="cuda")
    ob = torch.full((max(k, 1) * mb,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    nw = c.tn_compress_pair(dA.data_ptr(), dB.data_ptr(), ma, D, mb, chi, cutoff, oa.data_ptr(), ob.data_ptr())
    return nw, oa[:ma * nw].cpu().numpy().reshape(ma, nw), ob[:nw * mb].cpu().numpy().reshape(nw, mb)


def _reference(A, B, chi, cutoff=0.0):
    U, s, Vt = np.linalg.svd(A @ B, full_matrices=False)
    D = A.shape[1]
    k = min(chi, min(A.shape[0], D), min(B.shape[1], D))
    keep = (s[:k] > 0) & (s[:k] >= cutoff * s[0])
    sq = np.where(keep, np.sqrt(s[:k]), 0.0)
    return k, U[:, :k] * sq, sq[:, None] * Vt[:k], s


# (m_a, D, m_b, chi): tall-tall (both Grams, several 512-row splits and a ragged tail; D = 32 at
# full rank takes the 32 x 32 Jacobi, also at the tree's chi' = 16), explicit side A, explicit side
# B, both explicit, D = 64, D = 1, chi above the rank
SHAPES = [(1500, 32, 700, 8), (4100, 32, 2500, 16), (40, 64, 2000, 16), (3000, 48, 30, 12), (5, 16, 7, 10),
          (1100, 64, 1100, 64), (777, 1, 333, 1), (600, 20, 9, 50)]


@pytest.mark.parametrize("ma,D,mb,chi", SHAPES)
def test_compress_pair_is_truncated_svd(ma, D, mb, chi):
    print(f"\n[compress_pair] ma={ma} D={D} mb={mb} chi={chi}", flush=True)
    rng = np.random.default_rng(ma + 7 * D + mb)
    A = _graded(rng, ma, D, 1e-3)
    B = _graded(rng, D, mb, 1e-2)
    c = tn.Context(0)
    try:
        nw, a2, b2 = _run(c, A, B, chi)
    finally:
        c.close()
    k, ua, vb, s = _reference(A, B, chi)
    assert nw == k
    M = A @ B
    # the product: Eckart-Young
    scale = np.linalg.norm(M)
    err = np.linalg.norm(a2 @ b2 - ua @ vb) / scale
    # each factor column (row) is the reference one up to sign
    worst = 0.0
    for i in range(k):
        sgn = np.sign(np.dot(a2[:, i], ua[:, i]))
        worst = max(worst, np.max(np.abs(a2[:, i] * sgn - ua[:, i])), np.max(np.abs(b2[i] * sgn - vb[i])))
    print(f"    product error {err:.2e}, factor entries {worst / math.sqrt(s[0]):.2e} (of sqrt(sigma_1))", flush=True)
    assert err <= 1e-12
    assert worst <= 1e-10 * math.sqrt(s[0])


@pytest.mark.parametrize("ma,D,mb,chi", [(2000, 64, 1500, 16), (3000, 48, 30, 12)])
def test_compress_pair_steep_spectra_product(ma, D, mb, chi):
    """Factors with singular values down to 1e-12 of the largest: the float64 Gram drops
    directions below about 3e-8 of A's largest singular value (pivots below 1e-15 of the first
    end the Cholesky), which changes the truncated product A' B' only at rounding level."""
    rng = np.random.default_rng(5 * ma + D)
    A = _graded(rng, ma, D, 1e-12)
    B = _graded(rng, D, mb, 1e-6)
    c = tn.Context(0)
    try:
        nw, a2, b2 = _run(c, A, B, chi)
    finally:
        c.close()
    k, ua, vb, s = _reference(A, B, chi)
    err = np.linalg.norm(a2 @ b2 - ua @ vb) / np.linalg.norm(A @ B)
    print(f"\n    steep: product error {err:.2e}", flush=True)
    assert nw == k and err <= 1e-12


def test_compress_pair_cutoff_and_errors():
    rng = np.random.default_rng(11)
    A = _graded(rng, 900, 24, 1e-4)
    B = _graded(rng, 24, 800, 1e-3)
    s = np.linalg.svd(A @ B, compute_uv=False)
    cutoff = math.sqrt(s[4] * s[5]) / s[0]
    c = tn.Context(0)
    try:
        nw, a2, b2 = _run(c, A, B, 10, cutoff)
        k, ua, vb, _ = _reference(A, B, 10, cutoff)
        assert nw == k == 10
        assert np.all(a2[:, 5:] == 0.0) and np.all(b2[5:] == 0.0)
        assert np.linalg.norm(a2 @ b2 - ua @ vb) <= 1e-12 * np.linalg.norm(A @ B)
        x = torch.zeros(100 * 65, dtype=torch.float64, device="cuda")
        with pytest.raises(TNError) as ei:      # D above the LDS core's 64
            c.tn_compress_pair(x.data_ptr(), x.data_ptr(), 100, 65, 100, 4, 0.0, x.data_ptr(), x.data_ptr())
        assert ei.value.status == TN_EINVAL
        with pytest.raises(TNError) as ei:
            c.tn_compress_pair(0, x.data_ptr(), 10, 8, 10, 4, 0.0, x.data_ptr(), x.data_ptr())
        assert ei.value.status == TN_EINVAL
    finally:
        c.close()
