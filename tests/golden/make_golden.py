"""Write oracle reference values for the GPU parity tests (calls only oracle/ and tninputs/).

    python tests/golden/make_golden.py [--big]

ising_8x8.json   : 8x8 open-boundary Ising, beta=0.44 — transfer-matrix ln Z and the oracle's
                   ln|Z| for chi in {4, 8, 16, 256} along the sweep tree (section II.F, SI F.1),
                   and for chi in {16, 256} along the seed-0 Greedy tree.
cubic_12.json    : 12x12x12 Ising, beta=0.22, chi=16, sweep tree (--big, ~10 min of CPU):
                   the oracle's ln|Z| and its spread when one input tensor is perturbed at the
                   1e-15 level (the conditioning of this workload; see the design notes).
                   With --threads (~25 min of CPU) it also records the oracle's ln|Z| with the
                   BLAS library limited to 1, 2, 4 and all threads: the summation order inside
                   LAPACK's QR and SVD changes with the thread count, and the spread of these
                   unmodified oracle runs is the rounding sensitivity of this instance.
cubic_12_chi32.json: the same network and tree at chi=32 (--chi32, ~30 min of CPU): the oracle's
                   ln|Z| only.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import exact  # noqa: E402
from tninputs import greedy_tree, ising_tensors, lattice  # noqa: E402
from tninputs.trees import sweep_tree  # noqa: E402


def ising_8x8():
    g = lattice((8, 8))
    T = ising_tensors(g, 0.44)
    p = sweep_tree((8, 8))
    out = {"shape": [8, 8], "beta": 0.44, "tree": "sweep_tree((8, 8))",
           "transfer_matrix_lnZ": exact.ising_transfer_matrix((8, 8), 0.44), "oracle_lnZ": {}}
    for chi in (4, 8, 16, 256):
        out["oracle_lnZ"][str(chi)] = oracle.contract_compressed(g.n, g.edges, T, p, chi).ln_abs_z
    # the Greedy tree of the 8x8 workload: seed 0, scored with a simulated bond dimension of 2
    # (SI C.1's chi_greedy), so that bonds above 16 appear and chi = 16 compresses
    pg = greedy_tree(g, 2, 0)
    out["greedy"] = {"tree": "greedy_tree(g, 2, 0)", "oracle_lnZ": {}, "compressions": {}}
    for chi in (16, 256):
        r = oracle.contract_compressed(g.n, g.edges, T, pg, chi)
        out["greedy"]["oracle_lnZ"][str(chi)] = r.ln_abs_z
        out["greedy"]["compressions"][str(chi)] = sum(o.kind == "compress" for o in r.ops)
    return out


def cubic_12(n_perturb=3):
    g = lattice((12, 12, 12))
    T = ising_tensors(g, 0.22)
    p = sweep_tree((12, 12, 12))
    t0 = time.time()
    base = oracle.contract_compressed(g.n, g.edges, T, p, 16).ln_abs_z
    spread = []
    for seed in range(n_perturb):
        rng = np.random.default_rng(seed)
        T2 = [t.copy() for t in T]
        v = int(rng.integers(0, g.n))
        T2[v] = T2[v] * (1.0 + 1e-15 * rng.normal(size=T2[v].shape))
        spread.append(oracle.contract_compressed(g.n, g.edges, T2, p, 16).ln_abs_z - base)
    return {"shape": [12, 12, 12], "beta": 0.22, "chi": 16, "tree": "sweep_tree((12, 12, 12))",
            "oracle_lnZ": base, "perturbed_minus_base": spread,
            "perturbation": "one input tensor scaled entrywise by 1 + 1e-15 * Normal(0, 1)",
            "cpu_seconds": time.time() - t0}


def cubic_12_threads(rec):
    """Add the oracle's ln|Z| under BLAS thread limits of 1, 2, 4 and all cores to ``rec``."""
    from threadpoolctl import threadpool_limits
    g = lattice((12, 12, 12))
    T = ising_tensors(g, 0.22)
    p = sweep_tree((12, 12, 12))
    runs = {}
    for nt in (1, 2, 4, os.cpu_count()):
        with threadpool_limits(limits=nt, user_api="blas"):
            t0 = time.time()
            runs[str(nt)] = {"oracle_lnZ": oracle.contract_compressed(g.n, g.edges, T, p, 16).ln_abs_z,
                             "cpu_seconds": time.time() - t0}
        print(f"threads={nt}: {runs[str(nt)]}", flush=True)
    vals = [r["oracle_lnZ"] for r in runs.values()]
    rec["blas_threads"] = runs
    rec["blas_thread_spread_rel"] = (max(vals) - min(vals)) / abs(rec["oracle_lnZ"])
    return rec


def cubic_12_chi(chi):
    g = lattice((12, 12, 12))
    T = ising_tensors(g, 0.22)
    p = sweep_tree((12, 12, 12))
    t0 = time.time()
    lnz = oracle.contract_compressed(g.n, g.edges, T, p, chi).ln_abs_z
    return {"shape": [12, 12, 12], "beta": 0.22, "chi": chi, "tree": "sweep_tree((12, 12, 12))",
            "oracle_lnZ": lnz, "cpu_seconds": time.time() - t0}


if __name__ == "__main__":
    def write(name, rec):   # computed first: a file is never left half-written
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(rec, f, indent=1)

    write("ising_8x8.json", ising_8x8())
    if "--big" in sys.argv:
        write("cubic_12.json", cubic_12())
    if "--threads" in sys.argv:
        with open(os.path.join(HERE, "cubic_12.json")) as f:
            rec = json.load(f)
        write("cubic_12.json", cubic_12_threads(rec))
    if "--chi32" in sys.argv:
        write("cubic_12_chi32.json", cubic_12_chi(32))
