"""The 3D +-J spin glass of SI F.1 (beta = 0.5, couplings +-1 from default_rng(0), sweep tree,
chi = 16): d ln|Z| / d J through the reverse pass and the coupling chain rule on the device.

* 4^3 and 6^3: every bond's derivative against the oracle's reverse-mode gradient
  (tests/golden/spin_glass_grad.json, written by make_golden.py from oracle.grad) at 1e-9 of
  the largest |dJ|, the bound of the other gradient parity tests.
* 16^3 (11520 bonds): the float64 gradient against central differences of the float64 forward
  pass on 128 seeded bonds, and the Euler identity sum(T * d ln|Z| / dT) = 1 on every tensor.
  Central differences with h = 1e-5 carry a truncation error h^2 |f'''| / 6 and a rounding
  error of about eps |ln Z| / h ~ 1e-16 * 4200 / 1e-5 ~ 4e-8 per bond; over the 128 bonds the
  measured |FD - dJ| has a median near 3e-8 and a largest value of 2.5e-6, so the test asks
  for a median relative error below 1e-6 and every bond within 1e-5 absolute.
"""
import json
import os

import numpy as np
import pytest

import paper_2206_07044_amd as tn
from tninputs import ising_tensors, lattice
from tninputs.configs import pm_couplings
from tninputs.trees import sweep_tree

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BETA, CHI = 0.5, 16
GRAD_RTOL = 1e-9


def _planned(L, precision, grad, torch):
    g = lattice((L, L, L))
    J = pm_couplings(g.n_edges, 0)
    T = ising_tensors(g, BETA, J)
    pairs = sweep_tree((L, L, L))
    eu, ev, ed = g.arrays()
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum([t.size for t in T])
    data = np.concatenate([t.ravel() for t in T])
    c = tn.Context(0)
    c.tn_load_graph(g.n, eu, ev, ed, off, data)
    c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], CHI, precision=precision, grad=grad)
    return g, J, off, data, c


def _lnz_and_dJ(c, g, J, off, torch):
    Jd = torch.tensor(J, dtype=torch.float64, device="cuda")
    dT = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    dJ = torch.empty(g.n_edges, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    c.tn_ising_values_device(BETA, Jd.data_ptr())
    c.tn_contract_compressed()
    c.tn_grad_device(dT.data_ptr())
    c.tn_ising_coupling_grad_device(BETA, Jd.data_ptr(), dT.data_ptr(), dJ.data_ptr())
    c.tn_sync()
    return c.tn_result(), dT.cpu().numpy(), dJ.cpu().numpy()


@pytest.mark.parametrize("L", [4, 6])
def test_spin_glass_gradient_matches_oracle(L):
    import torch
    with open(os.path.join(HERE, "golden", "spin_glass_grad.json")) as f:
        gold = json.load(f)["sizes"][str(L)]
    if gold["ties"]:
        pytest.skip(f"{gold['ties']} truncation tie(s) in the oracle run")
    g, J, off, data, c = _planned(L, "fp64", True, torch)
    try:
        (sign, lnz), _, dJ = _lnz_and_dJ(c, g, J, off, torch)
    finally:
        c.close()
    want = np.array(gold["dlnZ_dJ"])
    err = np.max(np.abs(dJ - want))
    print(f"spin glass {L}^3 chi={CHI}: lnZ {lnz!r} (oracle {gold['oracle_lnZ']!r}), max|dJ - oracle| {err:.3e}, "
          f"max|dJ| {np.max(np.abs(want)):.3e}", flush=True)
    assert sign == gold["sign"]
    assert abs(lnz - gold["oracle_lnZ"]) <= 1e-10 * abs(gold["oracle_lnZ"])
    assert err <= GRAD_RTOL * np.max(np.abs(want))


def test_spin_glass_16_central_differences():
    import torch
    L = 16
    g, J, off, data, c = _planned(L, "fp64", True, torch)
    try:
        (sign, lnz), dT, dJ = _lnz_and_dJ(c, g, J, off, torch)
    finally:
        c.close()
    euler = np.abs([float(np.dot(data[off[v]:off[v + 1]], dT[off[v]:off[v + 1]])) - 1.0 for v in range(g.n)])
    print(f"16^3 chi={CHI} fp64: lnZ {lnz!r}, Euler identity error max {euler.max():.2e}", flush=True)
    assert euler.max() < 1e-10
    # forward-only float64 plan for the differences (the gradient plan's arena is released first)
    g, J, off, data, c = _planned(L, "fp64", False, torch)
    bonds = np.random.default_rng(1).choice(g.n_edges, 128, replace=False)
    h = 1e-5
    fd = np.zeros(len(bonds))
    try:
        for i, e in enumerate(bonds):
            vals = []
            for sgn in (1.0, -1.0):
                Jp = J.copy()
                Jp[e] += sgn * h
                Jt = torch.tensor(Jp, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                c.tn_ising_values_device(BETA, Jt.data_ptr())
                c.tn_contract_compressed()
                vals.append(c.tn_result()[1])
            fd[i] = (vals[0] - vals[1]) / (2 * h)
    finally:
        c.close()
    err = np.abs(fd - dJ[bonds])
    rel = err / np.abs(dJ[bonds])
    print(f"central differences on 128 bonds: |FD - dJ| max {err.max():.2e} median {np.median(err):.2e}, "
          f"relative median {np.median(rel):.2e}", flush=True)
    assert np.median(rel) < 1e-6
    assert err.max() < 1e-5
