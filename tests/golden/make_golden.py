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
cubic_4x4x8_chi64.json: 4x4x8 Ising, beta=0.22, chi=64, sweep tree (--cubic448-chi64, ~25 min of CPU and
                   ~35 GB): nine bonds of D = 4096 against 262144-row factors; the oracle's ln|Z|.
cubic_6_chi64.json: 6x6x6, the same model and chi (--cubic6-chi64, ~70 min of CPU): 25 bonds of D = 4096.
spin_glass_grad.json: L^3 +-J spin glass (SI F.1), beta = 0.5, couplings from default_rng(0), chi = 16,
                   sweep tree, L = 4 and 6 (--spin-glass, ~5 min of CPU; --spin-glass-8 adds L = 8):
                   the oracle's ln|Z| and d ln|Z| / d J for every bond (oracle.grad).
square_12.json   : 12x12 open-boundary Ising, beta = 0.44: the transfer-matrix ln Z (--square12), the
                   reference of the tree-scoring leg.
random_graphs.json: the random-graph workloads of sections IV.B and IV.C on their Agglom trees
                   (--random-graphs, ~5 min of CPU): dimer covers of random 3-regular graphs at
                   N = 256, chi = 4 and N = 512, chi = 2; Normal(mu, 1) tensors of bond dimension
                   3 on the N = 300 graph at chi = 2 for mu in {0, 0.1, 0.2, 0.5} and tensor seeds
                   0..3.  ln|Z|, sign, compressions and ties per instance.
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


def cubic_chi64(shape):
    """L1xL2xL3 Ising, beta = 0.22, chi = 64 along the sweep tree: its corner merges give bonds of
    D = 4096 (two chi-bonds), compressed against 262144-row factors."""
    g = lattice(shape)
    T = ising_tensors(g, 0.22)
    p = sweep_tree(shape)
    t0 = time.time()
    r = oracle.contract_compressed(g.n, g.edges, T, p, 64)
    comp = [o for o in r.ops if o.kind == "compress"]
    return {"shape": list(shape), "beta": 0.22, "chi": 64, "tree": f"sweep_tree({tuple(shape)})",
            "oracle_lnZ": r.ln_abs_z, "compressions": len(comp), "ties": sum(o.tie for o in comp),
            "max_bond": max(o.n for o in comp), "bonds_4096": sum(o.n == 4096 for o in comp),
            "cpu_seconds": time.time() - t0}


def spin_glass_grads(sizes, chi=16, beta=0.5):
    from oracle.grad import ising_coupling_grad, lnz_and_grad
    from tninputs.configs import pm_couplings
    out = {"beta": beta, "chi": chi, "couplings": "pm_couplings(n_edges, 0)", "tree": "sweep_tree((L, L, L))",
           "sizes": {}}
    for L in sizes:
        g = lattice((L, L, L))
        J = pm_couplings(g.n_edges, 0)
        t0 = time.time()
        res = lnz_and_grad(g.n, g.edges, ising_tensors(g, beta, J), sweep_tree((L, L, L)), chi)
        dJ = ising_coupling_grad(g.n, g.edges, beta, J, res.grads)
        ref = oracle.contract_compressed(g.n, g.edges, ising_tensors(g, beta, J), sweep_tree((L, L, L)), chi)
        comp = [o for o in ref.ops if o.kind == "compress"]
        out["sizes"][str(L)] = {"oracle_lnZ": res.ln_abs_z, "sign": res.sign, "dlnZ_dJ": [float(x) for x in dJ],
                                "compressions": len(comp), "ties": sum(o.tie for o in comp),
                                "cpu_seconds": time.time() - t0}
        print(f"spin glass L={L}: lnZ={res.ln_abs_z!r} ({time.time() - t0:.0f} s)", flush=True)
    return out


def square_12():
    return {"shape": [12, 12], "beta": 0.44, "transfer_matrix_lnZ": exact.ising_transfer_matrix((12, 12), 0.44)}


def _record(g, T, pairs, chi):
    t0 = time.time()
    r = oracle.contract_compressed(g.n, g.edges, T, pairs, chi)
    comp = [o for o in r.ops if o.kind == "compress"]
    return {"oracle_lnZ": r.ln_abs_z, "sign": r.sign, "compressions": len(comp),
            "ties": sum(o.tie for o in comp), "cpu_seconds": time.time() - t0}


def random_graphs():
    from tninputs import configs
    out = {"dimer": {}, "normal_d3_n300_chi2": {}}
    for n, chi, ts in ((256, 4, 2), (512, 2, 2)):
        out["dimer"][f"{n}"] = dict(_record(*configs.dimer_rrg(n, chi, tree_seed=ts), chi), chi=chi,
                                    tree=f"agglom_tree(g, {chi}, k=4, seed={ts})")
        print(f"dimer N={n}: {out['dimer'][str(n)]}", flush=True)
    for mu in (0.0, 0.1, 0.2, 0.5):
        for ts in range(4):
            rec = _record(*configs.normal_rrg(300, mu, 2, tensor_seed=ts), 2)
            out["normal_d3_n300_chi2"][f"{mu}/{ts}"] = rec
            print(f"normal mu={mu} seed={ts}: {rec}", flush=True)
    return out


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
    if "--cubic6-chi64" in sys.argv:
        write("cubic_6_chi64.json", cubic_chi64((6, 6, 6)))
    if "--cubic448-chi64" in sys.argv:
        write("cubic_4x4x8_chi64.json", cubic_chi64((4, 4, 8)))
    if "--square12" in sys.argv:
        write("square_12.json", square_12())
    if "--random-graphs" in sys.argv:
        write("random_graphs.json", random_graphs())
    if "--spin-glass" in sys.argv or "--spin-glass-8" in sys.argv:
        write("spin_glass_grad.json", spin_glass_grads((4, 6, 8) if "--spin-glass-8" in sys.argv else (4, 6)))
