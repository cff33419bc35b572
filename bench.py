#!/usr/bin/env python3
"""Benchmark: compressed contraction-tree evaluation on one MI355X.

Workload (the headline configuration): Ising partition function of the
12x12x12 open-boundary cubic lattice, J = 1, beta = 0.22, bond dimension 2,
one tensor per site (SI F.1), contracted along a fixed Span-family tree (an
axis-ordered spanning tree swept leaves-inwards, section II.G / SI C.2) with
early compression to chi (Algorithm 1, r = 0).  A step is one evaluation of
the whole tree; tensors and the plan are resident on the device before the
timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--chi 16] [--precision fp32]

Prints one JSON line (see the keys below).  --gpus > 1 is refused: the
executor runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compressed contractions/sec + fwd+bwd TFLOP/s vs plain FP64, at |Δlog Z|≤1e-6"
PEAKS = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "fp64_TFLOPs": 78.6,
    "fp32_TFLOPs": 157.3,
    "bf16_TFLOPs": 2500.0,
}


# HBM traffic per launch of a kernel kind on the default workload, from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE) scaled by a plain copy of known size; valid only for the kernel source it
# was measured on (SHA-256 prefix of tn_kernels.hip), else the bench line reports null.
MEASURED_TRAFFIC = {
    ("core_lds", "fp32", "ising-cubic-12x12x12-beta0.22-chi16-span-sweep"): {
        "bytes_per_launch": 467.1 * 1024, "kernel_source_sha256": "a12ad17775debd7b",
        "source": "profiles/core_lds_traffic_ising12_chi16_fp32.md"},
}


def measured_traffic(kind, precision, workload):
    import hashlib
    rec = MEASURED_TRAFFIC.get((kind, precision, workload))
    if rec is None:
        return None
    with open(os.path.join(ROOT, "paper_2206_07044_amd", "csrc", "tn_kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    return rec["bytes_per_launch"] if sha.startswith(rec["kernel_source_sha256"]) else None


# The oracle's ln|Z| for the default lattice and tree, per chi (written by tests/golden/make_golden.py,
# which calls only the CPU oracle)
ORACLE_GOLDEN = {16: "cubic_12.json", 32: "cubic_12_chi32.json"}


def oracle_lnz(shape, beta, chi):
    name = ORACLE_GOLDEN.get(chi)
    if shape != (12, 12, 12) or beta != 0.22 or name is None:
        return None
    try:
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return float(json.load(f)["oracle_lnZ"])
    except (OSError, ValueError, KeyError):   # not written (yet): no comparison
        return None


def build_instance(shape, beta):
    from tninputs import ising_tensors, lattice
    from tninputs.trees import sweep_tree
    g = lattice(shape)
    T = ising_tensors(g, beta)
    pairs = sweep_tree(shape)
    return g, T, pairs


def flat(g, T):
    eu, ev, ed = g.arrays()
    sizes = [int(t.size) for t in T]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    data = np.concatenate([np.ascontiguousarray(t, dtype=np.float64).ravel() for t in T])
    return eu, ev, ed, off, data


def op_flops(op) -> float:
    """Algorithmic flops of one oracle op record (same cost model as the planner)."""
    if op.kind == "contract":
        return 2.0 * op.m * op.n * op.k
    ma, D, mb, new = op.m, op.n, op.k, op.new_dim
    f = 0.0
    for m in (ma, mb):
        if m > D:
            f += 2.0 * m * D * D - 2.0 / 3.0 * D ** 3
    ka, kb = min(ma, D), min(mb, D)
    p, q = max(ka, kb), min(ka, kb)
    f += 2.0 * ka * D * kb + 4.0 * p * q * q - 4.0 / 3.0 * q ** 3
    f += 2.0 * ma * D * new + 2.0 * new * D * mb
    return f


def roofline_of(kind, prof, avg_ms, launches, precision):
    """Bound, unit, peak and achieved rate of one kernel kind (algorithmic work / time)."""
    per_s = 1.0 / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
    if kind == "gemm":
        # contractions and re-absorptions: MFMA-bound when their arithmetic intensity (algorithmic
        # flops / algorithmic bytes) reaches the ridge point, else HBM-bound
        peak = {"fp32": PEAKS["fp32_TFLOPs"], "bf16": PEAKS["bf16_TFLOPs"], "fp64": PEAKS["fp64_TFLOPs"]}[precision]
        ridge = peak * 1e12 / (PEAKS["hbm_GBps"] * 1e9)
        if prof["bytes"] > 0 and prof["flops"] / prof["bytes"] < ridge:
            return "hbm", "GB/s", PEAKS["hbm_GBps"], prof["bytes"] / launches * per_s / 1e9
        return "mfma", "TFLOP/s", peak, prof["flops"] / launches * per_s / 1e12
    if kind == "gram":   # Gram matrices accumulate on float64 MFMA in both precisions
        return "mfma", "TFLOP/s", PEAKS["fp64_TFLOPs"], prof["flops"] / launches * per_s / 1e12
    if kind in ("core_lds", "core_global", "lanczos"):
        # per-compression SVD kernels: float64 vector arithmetic, one workgroup per compression;
        # peak = 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2 (dual issue) x 2.4 GHz = 78.6 TFLOP/s
        return "alu", "TFLOP/s", PEAKS["fp64_TFLOPs"], prof["flops"] / launches * per_s / 1e12
    return "hbm", "GB/s", PEAKS["hbm_GBps"], prof["bytes"] / launches * per_s / 1e9


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, T, pairs, chi, total_flops, budget_s):
    """The CPU oracle, unmodified, on a bounded sample of the same workload: a fixed prefix of the
    tree (the steps an all-thread run covers in about budget_s / 8), timed best of 3 with the BLAS
    library on all host threads and on one thread (the paper's single-core convention), and scaled
    to trees/s by the algorithmic flops of the prefix against those of the whole tree."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import approx
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    probe = approx.contract_compressed_budget(g.n, g.edges, T, pairs, chi, budget_s / 8)
    steps = max(1, probe.steps_done)
    runs = {}
    for nt in (threads, 1):
        best, ops = math.inf, []
        with threadpool_limits(limits=nt, user_api="blas"):
            for _ in range(3):
                t0 = time.time()
                ops = approx.contract_steps(g.n, g.edges, T, pairs, chi, steps)
                best = min(best, time.time() - t0)
        done = sum(op_flops(o) for o in ops)
        runs[nt] = (best, done)
    dt, done = runs[threads]
    dt1, _ = runs[1]
    rate = done / total_flops / dt if dt > 0 and total_flops > 0 else 0.0
    return {
        "value": rate,
        "unit": "trees/s",
        "cores": int(threads),
        "kind": "oracle",
        "single_thread_value": done / total_flops / dt1 if dt1 > 0 and total_flops > 0 else 0.0,
        "cpu_model": cpu_model(),
        "sample": (f"float64 numpy oracle, first {steps} of {len(pairs)} tree steps ({done:.3e} of {total_flops:.3e} "
                   f"algorithmic flops), best of 3: {dt:.2f} s with {threads} BLAS threads, {dt1:.2f} s with 1; "
                   f"trees/s = (prefix flops / total flops) / seconds"),
    }


def timed(c, n, torch, eager=False):
    """Seconds per evaluation of context c over n back-to-back evaluations (after one untimed)."""
    c.tn_contract_compressed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if eager:
        for _ in range(n):
            c.tn_contract_compressed()
    else:
        for _ in range(n):
            c.tn_enqueue()
        c.tn_fetch()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n


def ising_8x8_leg(tn, torch, reps):
    """The small configuration: 8x8 open-boundary Ising, beta = 0.44, seed-0 Greedy tree, chi 16 and
    256, float64 in the plain form; latency of one synchronous evaluation and throughput of
    back-to-back ones, ln|Z| against the stored oracle and transfer-matrix values."""
    from tninputs import greedy_tree, ising_tensors, lattice
    g = lattice((8, 8))
    T = ising_tensors(g, 0.44)
    pairs = greedy_tree(g, 2, 0)
    eu, ev, ed, off, data = flat(g, T)
    try:
        with open(os.path.join(ROOT, "tests", "golden", "ising_8x8.json")) as f:
            gold = json.load(f)
    except (OSError, ValueError):
        gold = None
    out = {"workload": "ising-square-8x8-beta0.44-greedy-seed0", "precision": "fp64", "form": "plain"}
    for chi in (16, 256):
        c = tn.Context(0)
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision="fp64", plain=True)
        c.tn_contract_compressed()
        lat = math.inf
        for _ in range(reps):
            t0 = time.perf_counter()
            c.tn_contract_compressed()
            lat = min(lat, time.perf_counter() - t0)
        per = timed(c, reps, torch)
        _, lnz = c.tn_result()
        rec = {"latency_ms": lat * 1e3, "trees_per_s": 1.0 / per, "ln_abs_z": lnz,
               "compressions": len(c.tn_compress_stats()[0])}
        if gold:
            ref = gold["greedy"]["oracle_lnZ"][str(chi)]
            rec["oracle_ln_abs_z"] = ref
            rec["rel_dlnz_vs_oracle"] = abs(lnz - ref) / abs(ref)
            rec["rel_dlnz_vs_transfer_matrix"] = abs(lnz - gold["transfer_matrix_lnZ"]) / gold["transfer_matrix_lnZ"]
        out[f"chi{chi}"] = rec
        c.close()
    return out


def spin_glass_leg(tn, torch, L, chi, beta, steps):
    """The 3D +-J spin glass (SI F.1): L^3 open-boundary cubic lattice, couplings +-1 with equal
    probability from default_rng(0), forward + reverse pass to d ln|Z| / d J for every bond, in
    float64 and float32 on gradient plans.  The tensors are built on the device from J by the
    library's Ising map; the Euler identity sum(T * dlnZ/dT) = 1 per tensor is checked on the host."""
    from tninputs import ising_tensors, lattice
    from tninputs.trees import sweep_tree
    shape = (L, L, L)
    g = lattice(shape)
    J = np.where(np.random.default_rng(0).random(g.n_edges) < 0.5, -1.0, 1.0)
    T = ising_tensors(g, beta, J)
    eu, ev, ed, off, data = flat(g, T)
    pairs = sweep_tree(shape)
    pi = [a for a, _ in pairs]
    pj = [b for _, b in pairs]
    Jd = torch.tensor(J, dtype=torch.float64, device="cuda")
    out = {"lattice": list(shape), "beta": beta, "chi": chi, "couplings": "+-1, default_rng(0)",
           "tree": "Span family, axis-ordered spanning tree swept leaves-inwards", "n_bonds": g.n_edges}
    grads = {}

    def variant(prec, segments):
        c = tn.Context(0)
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree(pi, pj, chi, precision=prec, grad=True, checkpoint_segments=segments)
        info, binfo = c.tn_plan_info(), c.tn_grad_info()
        dT = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
        dJ = torch.empty(g.n_edges, dtype=torch.float64, device="cuda")

        def step():
            c.tn_ising_values_device(beta, Jd.data_ptr())
            c.tn_contract_compressed()
            c.tn_grad_device(dT.data_ptr())
            c.tn_ising_coupling_grad_device(beta, Jd.data_ptr(), dT.data_ptr(), dJ.data_ptr())
            c.tn_sync()

        step()                                  # captures the forward and reverse schedules (untimed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        sign, lnz = c.tn_result()
        gT = dT.cpu().numpy()
        eul = np.abs([float(np.dot(data[off[v]:off[v + 1]], gT[off[v]:off[v + 1]])) - 1.0 for v in range(g.n)])
        _, tie, _ = c.tn_compress_stats()
        flops = info["fwd_flops"] + binfo["bwd_flops"]
        rec = {"ms_per_step": dt * 1e3, "fwd_bwd_per_s": 1.0 / dt, "tflops": flops / dt / 1e12,
               "fwd_flops": info["fwd_flops"], "bwd_flops": binfo["bwd_flops"],
               "arena_bytes": info["arena_bytes"], "ln_abs_z": lnz, "sign": sign,
               "euler_identity_error_max": float(eul.max()), "euler_identity_error_median": float(np.median(eul)),
               "tie_flags": int(np.sum(tie)), "steps": steps}
        if segments != 0:
            ck = c.tn_grad_checkpoint_info()
            rec.update({"segments": ck["segments"], "checkpoint_bytes": ck["checkpoint_bytes"],
                        "recompute_flops": ck["recompute_flops"]})
        c.close()
        return rec, dJ.cpu().numpy()

    for prec in ("fp64", "fp32"):
        out[prec], grads[prec] = variant(prec, 0)
    # FP64 with checkpointed recomputation (segment count of smallest arena)
    rec, dJr = variant("fp64", -1)
    rec["arena_ratio"] = rec["arena_bytes"] / out["fp64"]["arena_bytes"]
    rec["time_ratio"] = rec["ms_per_step"] / out["fp64"]["ms_per_step"]
    rec["dJ_max_abs_diff_vs_resident"] = float(np.max(np.abs(dJr - grads["fp64"])))
    out["fp64_recompute"] = rec
    d = np.abs(grads["fp32"] - grads["fp64"])
    scale = float(np.max(np.abs(grads["fp64"])))
    out["dJ_fp32_vs_fp64"] = {"max_abs": float(d.max()), "median_abs": float(np.median(d)),
                              "max_abs_over_max_dJ": float(d.max()) / scale,
                              "bonds_over_1e-3_max_dJ": int(np.sum(d > 1e-3 * scale))}
    out["rel_dlnz_fp32_vs_fp64"] = abs(out["fp32"]["ln_abs_z"] - out["fp64"]["ln_abs_z"]) / abs(out["fp64"]["ln_abs_z"])
    out["speedup_fp32_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"]
    return out


def _golden(name):
    try:
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def _load(tn, g, T, pairs, chi, precision):
    eu, ev, ed, off, data = flat(g, T)
    c = tn.Context(0)
    c.tn_load_graph(g.n, eu, ev, ed, off, data)
    c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision=precision)
    return c


def dimer_leg(tn, torch, reps):
    """Dimer covers of random 3-regular graphs (section IV.B, SI F.3) on Agglom-family trees:
    single graphs at N = 256 (chi = 4) and N = 512 (chi = 2) in float64 and float32 against the
    stored oracle values, and 32 graphs of N = 2 U{48..96} (seeds 0..31, chi = 4) replayed as one
    batch against the same graphs run one after another."""
    from tninputs import configs, simulate_tree
    gold = (_golden("random_graphs.json") or {}).get("dimer", {})
    out = {"single": {}}
    for n, chi, ts in ((256, 4, 2), (512, 2, 2)):
        g, T, pairs = configs.dimer_rrg(n, chi, tree_seed=ts)
        rec = {"chi": chi, "tree": f"agglom_tree(g, {chi}, k=4, seed={ts})",
               "largest_tensor": simulate_tree(g, pairs, chi).largest_elems}
        ref = gold.get(str(n))
        for prec in ("fp64", "fp32"):
            c = _load(tn, g, T, pairs, chi, prec)
            dt = timed(c, reps, torch)
            sign, lnz = c.tn_result()
            r = {"trees_per_s": 1.0 / dt, "ms_per_tree": dt * 1e3, "ln_abs_z": lnz, "sign": sign,
                 "arena_bytes": c.tn_plan_info()["arena_bytes"]}
            if ref is not None:
                r["rel_dlnz_vs_oracle"] = abs(lnz - ref["oracle_lnZ"]) / abs(ref["oracle_lnZ"])
            rec[prec] = r
            c.close()
        out["single"][str(n)] = rec
    # uneven batch: N_b = 2 U{48..96} from default_rng(b), graph seed b; per graph the tree seed
    # (of 0..2) with the smallest largest intermediate, stopping at the first below 2^20 entries
    sizes = [2 * int(np.random.default_rng(b).integers(48, 97)) for b in range(32)]
    insts = []
    for b, n in enumerate(sizes):
        g = configs.random_regular3(n, b)
        best = None
        for ts in range(3):
            pairs = configs.agglom_tree(g, 4, k=4, seed=ts)
            w = simulate_tree(g, pairs, 4).largest_elems
            if best is None or w < best[0]:
                best = (w, pairs)
            if w <= 1 << 20:
                break
        insts.append((g, configs.dimer_tensors(g), best[1]))
    bres = {"graphs": 32, "sizes": sizes, "chi": 4, "largest_tensor_max": max(simulate_tree(g, p, 4).largest_elems for g, _, p in insts)}
    for prec in ("fp64", "fp32"):
        ctxs = [_load(tn, g, T, p, 4, prec) for g, T, p in insts]
        seq = 0.0
        for c in ctxs:
            seq += timed(c, 1, torch)
        lnz_seq = [c.tn_result()[1] for c in ctxs]
        batch = tn.Batch(ctxs)
        batch.tn_batch_contract()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batch.tn_batch_contract()
        torch.cuda.synchronize()
        bdt = (time.perf_counter() - t0) / reps
        lnz_b = [c.tn_result()[1] for c in ctxs]
        bres[prec] = {"batch_ms": bdt * 1e3, "trees_per_s": 32 / bdt, "sequential_ms": seq * 1e3,
                      "speedup_vs_sequential": seq / bdt, "bitwise_equal_to_sequential": lnz_b == lnz_seq,
                      "graph": "one hipGraph per batch"}
        batch.close()
        for c in ctxs:
            c.close()
    out["batch"] = bres
    return out


def normal_d3_leg(tn, torch, reps):
    """Random tensor networks (section IV.C, SI F.2): one random 3-regular graph of N = 300 with
    bond dimension 3 and Normal(mu, 1) entries, chi = 2 on an Agglom-family tree; 64 tensor seeds
    per mu replayed as one batch in float32 and bfloat16, against float64 batches for the sign
    and ln|Z|, and against the stored oracle values for seeds 0..3."""
    from tninputs import configs, normal_tensors, random_regular3, simulate_tree
    gold = (_golden("random_graphs.json") or {}).get("normal_d3_n300_chi2", {})
    g = random_regular3(300, 0, dim=3)
    pairs = configs.agglom_tree(g, 2, k=4, seed=0)
    out = {"n": 300, "D": 3, "chi": 2, "seeds": 64, "tree": "agglom_tree(g, 2, k=4, seed=0)",
           "largest_tensor": simulate_tree(g, pairs, 2).largest_elems, "mu": {}}
    for mu in (0.0, 0.1, 0.2, 0.5):
        Ts = [normal_tensors(g, mu, s) for s in range(64)]
        res = {}
        vals = {}
        for prec in ("fp64", "fp32", "bf16"):
            ctxs = [_load(tn, g, T, pairs, 2, prec) for T in Ts]
            batch = tn.Batch(ctxs)
            batch.tn_batch_contract()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                batch.tn_batch_contract()
            torch.cuda.synchronize()
            bdt = (time.perf_counter() - t0) / reps
            vals[prec] = [c.tn_result() for c in ctxs]
            res[prec] = {"batch_ms": bdt * 1e3, "trees_per_s": 64 / bdt}
            batch.close()
            for c in ctxs:
                c.close()
        for prec in ("fp32", "bf16"):
            d = [abs(a[1] - b[1]) / abs(b[1]) for a, b in zip(vals[prec], vals["fp64"])]
            res[prec]["sign_agreement_vs_fp64"] = sum(a[0] == b[0] for a, b in zip(vals[prec], vals["fp64"])) / 64
            res[prec]["rel_dlnz_vs_fp64_median"] = float(np.median(d))
            res[prec]["rel_dlnz_vs_fp64_max"] = float(np.max(d))
        ref = [gold.get(f"{mu}/{s}") for s in range(4)]
        if all(r is not None for r in ref):
            res["fp64"]["max_rel_dlnz_vs_oracle_seeds_0_3"] = max(
                abs(vals["fp64"][s][1] - ref[s]["oracle_lnZ"]) / abs(ref[s]["oracle_lnZ"]) for s in range(4))
            res["fp64"]["sign_agreement_vs_oracle_seeds_0_3"] = all(
                vals["fp64"][s][0] == ref[s]["sign"] for s in range(4))
        res["fraction_negative_fp64"] = sum(v[0] < 0 for v in vals["fp64"]) / 64
        out["mu"][str(mu)] = res
    return out


def tree_scoring_leg(tn, torch):
    """Device-side tree scoring (section II.H, SI C): 64 candidate trees of the 12x12 Ising network
    (beta = 0.44, chi = 8) from the three generator families, planned on the host and evaluated
    as batched hipGraph replays; each candidate's error against the stored transfer-matrix value."""
    from tninputs import ising_tensors, lattice
    from tninputs.trees import sample_trees, sweep_tree
    ref = (_golden("square_12.json") or {}).get("transfer_matrix_lnZ")
    g = lattice((12, 12))
    T = ising_tensors(g, 0.44)
    eu, ev, ed, off, data = flat(g, T)
    cands = sample_trees(g, 8, 64, seed=0)
    scorer = tn.TreeScorer(g.n, eu, ev, ed, off, data, 8, device_budget_bytes=4 << 30)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scores = scorer.score([p for _, p in cands], ref_ln_abs_z=ref, chunk=64)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ok = [(s, lab) for s, (lab, _) in zip(scores, cands) if s.status == 0]
    out = {"lattice": [12, 12], "beta": 0.44, "chi": 8, "candidates": len(cands), "evaluated": len(ok),
           "rejected": len(cands) - len(ok), "seconds_incl_planning": dt, "candidates_per_s": len(cands) / dt,
           "reference": "transfer matrix (tests/golden/square_12.json)"}
    if ref is not None and ok:
        errs = sorted(s.rel_error for s, _ in ok)
        best = min(ok, key=lambda x: x[0].rel_error)
        sweep = scorer.score([sweep_tree((12, 12))], ref_ln_abs_z=ref)[0]
        cheap = [x for x in ok if x[0].fwd_flops <= sweep.fwd_flops]
        out.update({"best_rel_error": errs[0], "median_rel_error": errs[len(errs) // 2], "best_tree": best[1],
                    "best_tree_fwd_flops": best[0].fwd_flops, "sweep_tree_rel_error": sweep.rel_error,
                    "sweep_tree_fwd_flops": sweep.fwd_flops})
        if cheap:
            cb = min(cheap, key=lambda x: x[0].rel_error)
            out["best_rel_error_at_most_sweep_flops"] = cb[0].rel_error
            out["best_tree_at_most_sweep_flops"] = cb[1]
    return out


def hardness_leg(tn, torch):
    """The URand hardness transition of section IV.C: entries uniform in [lambda, 1] on the
    16x16 square lattice with D = 4 (axis sweep tree) and on the 6x6x6(x2) diamond lattice with
    D = 2 ('span-corner' tree), 4 tensor seeds per lambda, float64.  No exact value exists at these
    sizes here, so the error column is the change of ln|Z| from chi to 2 chi and the sign
    agreement of the two."""
    from tninputs import configs
    out = {}
    for kind, shape, D, chi, tree in (("square", (16, 16), 4, 32, "span"), ("diamond", (6, 6, 6), 2, 8, "span-corner")):
        rec = {"shape": list(shape), "D": D, "chi": [chi, 2 * chi], "tree": tree, "seeds": 4, "lambda": {}}
        t0 = time.perf_counter()
        for lam in (-1.0, -0.8, -0.7, -0.6, -0.5, -0.2, 0.0):
            vals = {}
            for c_ in (chi, 2 * chi):
                ctxs = []
                for sd in range(4):
                    g, T, pairs = configs.urand_lattice(kind, shape, lam, c_, seed=sd, D=D, tree=tree)
                    ctxs.append(_load(tn, g, T, pairs, c_, "fp64"))
                batch = tn.Batch(ctxs)
                try:
                    mant, _ = batch.tn_batch_contract()
                finally:
                    batch.close()
                vals[c_] = [c.tn_result() if m != 0.0 else (0.0, -math.inf) for c, m in zip(ctxs, mant)]
                for c in ctxs:
                    c.close()
            d = [abs(a[1] - b[1]) / abs(b[1]) for a, b in zip(vals[chi], vals[2 * chi])]
            rec["lambda"][str(lam)] = {"median_rel_dlnz_chi_vs_2chi": float(np.median(d)),
                                       "sign_agreement": sum(a[0] == b[0] for a, b in zip(vals[chi], vals[2 * chi])) / 4,
                                       "fraction_negative_2chi": sum(b[0] < 0 for b in vals[2 * chi]) / 4}
        rec["seconds"] = time.perf_counter() - t0
        out[f"{kind}"] = rec
    return out


def pyrochlore_leg(tn, torch, L=6, chi=4, beta=0.22, h=0.005):
    """The ferromagnetic pyrochlore Ising model of section IV.A on L^3 x 4 sites ('span-corner'
    tree): -beta f = ln Z / N at three inverse temperatures, its first derivative from the reverse
    pass (d ln Z / d beta = (1/beta) sum_e J_e d ln Z / d J_e, J = 1) and the second derivative
    d^2(-beta f)/d beta^2 by central differences of the first, float64 gradient plans."""
    from tninputs import configs
    g, T, pairs = configs.pyrochlore_ising(L, beta, chi)
    eu, ev, ed, off, data = flat(g, T)
    c = tn.Context(0)
    c.tn_load_graph(g.n, eu, ev, ed, off, data)
    c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision="fp64", grad=True)
    J = torch.ones(g.n_edges, dtype=torch.float64, device="cuda")
    dT = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    dJ = torch.empty(g.n_edges, dtype=torch.float64, device="cuda")
    rows = []
    t0 = time.perf_counter()
    for b in (beta - h, beta, beta + h):
        torch.cuda.synchronize()
        c.tn_ising_values_device(b, J.data_ptr())
        c.tn_contract_compressed()
        _, lnz = c.tn_result()
        c.tn_grad_device(dT.data_ptr())
        c.tn_ising_coupling_grad_device(b, J.data_ptr(), dT.data_ptr(), dJ.data_ptr())
        c.tn_sync()
        rows.append((b, lnz / g.n, float(dJ.sum().item()) / (b * g.n)))
    dt = time.perf_counter() - t0
    info = c.tn_plan_info()
    c.close()
    return {"L": L, "sites": g.n, "chi": chi, "beta": beta, "h": h, "arena_bytes": info["arena_bytes"],
            "minus_beta_f": {f"{b:.4f}": v for b, v, _ in rows},
            "d_minus_beta_f_dbeta": {f"{b:.4f}": d for b, _, d in rows},
            "d2_minus_beta_f_dbeta2": (rows[2][2] - rows[0][2]) / (2 * h),
            "d2_by_second_difference_of_lnZ": (rows[2][1] - 2 * rows[1][1] + rows[0][1]) / h ** 2,
            "seconds_3_fwd_bwd": dt}


def tree_gauge_leg(tn, torch, L=10, chi=8, seeds=4):
    """Tree-gauge compression (section II.C, SI A) with early and late compression (section II.D)
    on the URand model of the paper's early-versus-late comparison (D = 4 square lattice, entries
    in [-0.5, 1]): median |1 - Z/Z_exact| over seeds for r = 0, 1, 2, 4, and the time per tree.
    Z_exact is the library's own float64 contraction along a Greedy tree at a chi above every bond
    (no compression), a different tree and a different op sequence from the measured ones."""
    from tninputs import greedy_tree, lattice, uniform_tensors
    from tninputs.trees import sweep_tree
    g = lattice((L, L), dim=4)
    pairs = sweep_tree((L, L))
    exact_pairs = greedy_tree(g, 1 << 40, 0, temperature=0.0)
    out = {"lattice": [L, L], "D": 4, "lambda": -0.5, "chi": chi, "seeds": seeds,
           "tree": "axis sweep (Span family)", "reference": "float64, Greedy tree, no compression", "runs": {}}
    exact = []
    for sd in range(seeds):
        c = _load(tn, g, uniform_tensors(g, -0.5, sd), exact_pairs, 1 << 30, "fp64")
        c.tn_contract_compressed()
        exact.append(c.tn_result())
        c.close()
    for late in (False, True):
        for r in (0, 1, 2, 4):
            errs, times = [], []
            for sd in range(seeds):
                eu, ev, ed, off, data = flat(g, uniform_tensors(g, -0.5, sd))
                c = tn.Context(0)
                c.tn_load_graph(g.n, eu, ev, ed, off, data)
                c.tn_set_tree([a for a, _ in pairs], [b for _, b in pairs], chi, precision="fp64", late=late, gauge_r=r)
                times.append(timed(c, 2, torch))
                sign, lnz = c.tn_result()
                c.close()
                es, el = exact[sd]
                errs.append(abs(1.0 - sign * es * math.exp(lnz - el)))
            out["runs"][f"{'late' if late else 'early'}_r{r}"] = {"median_abs_1_minus_Z_over_Zexact": float(np.median(errs)),
                                                                "ms_per_tree": 1e3 * float(np.median(times))}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chi", type=int, default=16)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--shape", default="12,12,12")
    ap.add_argument("--beta", type=float, default=0.22)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-reference", action="store_true")
    ap.add_argument("--fwd-bwd-steps", type=int, default=1, help="timed forward+reverse passes (0: skip)")
    ap.add_argument("--batch", type=int, default=8, help="instances in the batched leg (<= 1: skip)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--per-chi", default="32,64", help="other chi values timed in fp32 and fp64 ('' to skip)")
    ap.add_argument("--full", action="store_true",
                    help="also the URand hardness sweep (a minute more)")
    ap.add_argument("--no-small", action="store_true", help="skip the 8x8 Ising leg")
    ap.add_argument("--spin-glass", default="16,16", help="L,chi of the +-J spin-glass forward+reverse leg ('' to skip)")
    ap.add_argument("--no-random-graphs", action="store_true", help="skip the dimer and Normal(mu) random-graph legs")
    ap.add_argument("--no-tree-scoring", action="store_true", help="skip the device-side tree-scoring leg")
    ap.add_argument("--no-tree-gauge", action="store_true", help="skip the tree-gauge accuracy leg")
    ap.add_argument("--no-second-workloads", action="store_true", help="skip the pyrochlore leg")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in GEMM tile table")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the executor has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

    import torch
    import paper_2206_07044_amd as tn
    from paper_2206_07044_amd import autotune

    # tile shapes of the skinny GEMMs: measured on this GPU for the precisions timed below, before
    # any tree is planned (--no-autotune keeps the library's built-in table)
    tune_report = None
    if not args.no_autotune:
        tune_report = autotune.tune(precisions=tuple(dict.fromkeys((args.precision, "fp64"))), copies=8)

    shape = tuple(int(x) for x in args.shape.split(","))
    g, T, pairs = build_instance(shape, args.beta)
    eu, ev, ed, off, data = flat(g, T)
    pi = [a for a, _ in pairs]
    pj = [b for _, b in pairs]

    def make_ctx(precision):
        c = tn.Context(0)
        c.tn_load_graph(g.n, eu, ev, ed, off, data)
        c.tn_set_tree(pi, pj, args.chi, precision=precision)
        return c

    ctx = make_ctx(args.precision)
    info = ctx.tn_plan_info()
    # warmup, with every kernel kind timed once to find the dominant kernel
    ctx.tn_profile(list(tn.KERNEL_KINDS))
    for _ in range(max(1, args.warmup)):
        ctx.tn_contract_compressed()
    kinds = {k: ctx.tn_profile_read(k) for k in tn.KERNEL_KINDS}
    dominant = max(kinds, key=lambda k: kinds[k]["ms"])
    ctx.tn_profile([dominant])
    ctx.tn_contract_compressed()   # captures the schedule with this profiling mask (untimed)
    ctx.tn_profile([dominant])     # same mask: resets the totals, keeps the captured graph

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        # one replay of the captured schedule per step; fetching after each step reads that step's
        # kernel events (a replay re-records the same event nodes)
        ctx.tn_enqueue()
        ctx.tn_fetch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sign, lnz = ctx.tn_result()
    prof = ctx.tn_profile_read(dominant)
    trees_per_s = args.steps / dt
    ms_per_step = dt * 1e3 / args.steps

    # roofline of the dominant kernel (algorithmic work per launch / measured launch time)
    launches = max(1, prof["launches"])
    avg_ms = prof["ms"] / launches
    bound, unit, peak, achieved = roofline_of(dominant, prof, avg_ms, launches, args.precision)

    workload = f"ising-cubic-{'x'.join(map(str, shape))}-beta{args.beta}-chi{args.chi}-span-sweep"
    out = {
        "metric": METRIC,
        "value": trees_per_s,
        "unit": "trees/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": workload,
            "lattice": list(shape), "beta": args.beta, "chi": args.chi, "batch": 1,
            "tree": "Span family, axis-ordered spanning tree swept leaves-inwards",
            "compression": "early, gauge distance r=0",
            "precision": {"fp32": "float32 tensors/contractions on MFMA; float64 Gram, core SVD, exponent",
                          "bf16": "bfloat16 tensors, bf16 MFMA with float32 accumulation; float64 Gram, core SVD, "
                                  "exponent",
                          "fp64": "float64 throughout"}[args.precision],
            "flops_per_tree": info["fwd_flops"],
            "tflops_fwd": info["fwd_flops"] * trees_per_s / 1e12,
            "arena_bytes": info["arena_bytes"],
            "ln_abs_z": lnz,
            "sign": sign,
            "oracle_ln_abs_z": oracle_lnz(shape, args.beta, args.chi),
        },
        "roofline": {
            "kernel": dominant, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak if peak else None,
            "traffic": measured_traffic(dominant, args.precision, workload),
            "traffic_unit": "bytes per launch",
            "launches_per_step": prof["launches"] / args.steps, "avg_launch_ms": avg_ms,
            "kernel_ms_per_step": {k: v["ms"] / max(1, args.warmup) for k, v in kinds.items()},
        },
        "gemm_autotune": None if tune_report is None else {
            "seconds": tune_report["seconds"], "classes_timed": len(tune_report["timings_us"]),
            "changed_from_builtin": tune_report["changed"]},
    }
    g_prof = kinds["gemm"]
    if g_prof["launches"]:
        gl = g_prof["launches"]
        gb, gu, gp, ga = roofline_of("gemm", g_prof, g_prof["ms"] / gl, gl, args.precision)
        out["contraction_roofline"] = {"kernel": "gemm", "bound": gb, "achieved": ga, "peak": gp, "unit": gu,
                                       "frac": ga / gp, "avg_launch_ms": g_prof["ms"] / gl,
                                       "launches_per_step": gl / max(1, args.warmup),
                                       "arithmetic_intensity": g_prof["flops"] / g_prof["bytes"] if g_prof["bytes"] else None,
                                       "tflops": g_prof["flops"] / g_prof["ms"] * 1e3 / 1e12 if g_prof["ms"] else None}

    if not args.no_fp64_reference:
        # the same tree in float64: grouped and captured (the library's form), and the plain form
        # (one launch per step, one stream, no graph), the denominator of the metric
        ref = make_ctx("fp64")
        nref = max(1, min(args.steps, 3))
        rdt = timed(ref, nref, torch)
        rs, rl = ref.tn_result()
        ref.close()
        plain = tn.Context(0)
        plain.tn_load_graph(g.n, eu, ev, ed, off, data)
        plain.tn_set_tree(pi, pj, args.chi, precision="fp64", plain=True)
        pdt = timed(plain, 2, torch, eager=True)
        ps, pl = plain.tn_result()
        plain.close()
        out["fp64_reference"] = {"trees_per_s": 1.0 / rdt, "ln_abs_z": rl, "sign": rs, "form": "grouped, captured"}
        out["fp64_plain"] = {"trees_per_s": 1.0 / pdt, "ms_per_tree": pdt * 1e3, "ln_abs_z": pl,
                             "bitwise_equal_to_grouped": pl == rl,
                             "form": "one launch per step on one stream, no graph"}
        orl = oracle_lnz(shape, args.beta, args.chi)
        if orl is not None:
            out["rel_dlnz_vs_oracle"] = {"fp64": abs(rl - orl) / abs(orl), args.precision: abs(lnz - orl) / abs(orl)}
        out["speedup_vs_fp64"] = trees_per_s * rdt
        out["speedup_vs_plain_fp64"] = trees_per_s * pdt
        out["abs_dlnz_vs_fp64"] = abs(lnz - rl)
        out["rel_dlnz_vs_fp64"] = abs(lnz - rl) / abs(rl)
        if args.precision != "bf16":
            bc = make_ctx("bf16")
            bdt = timed(bc, nref, torch)
            _, bl = bc.tn_result()
            bc.close()
            out["bf16"] = {"trees_per_s": 1.0 / bdt, "ln_abs_z": bl, "abs_dlnz_vs_fp64": abs(bl - rl),
                           "rel_dlnz_vs_fp64": abs(bl - rl) / abs(rl),
                           "speedup_vs_plain_fp64": pdt / bdt}

    if args.batch > 1:
        # the same lattice and tree at a sweep of beta values (independent instances), merged level by
        # level and replayed from one hipGraph
        betas = np.linspace(args.beta - 0.02, args.beta + 0.02, args.batch)
        bctx = []
        for b_ in betas:
            Tb = __import__("tninputs").ising_tensors(g, float(b_))
            c = tn.Context(0)
            c.tn_load_graph(g.n, eu, ev, ed, off, flat(g, Tb)[4])
            c.tn_set_tree(pi, pj, args.chi, precision=args.precision)
            bctx.append(c)
        batch = tn.Batch(bctx)
        batch.tn_batch_contract()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            batch.tn_batch_contract()
        bdt = (time.perf_counter() - t0) / args.batch_steps
        out["batched"] = {"instances": args.batch, "betas": [float(x) for x in betas], "ms_per_replay": bdt * 1e3,
                          "trees_per_s": args.batch / bdt, "speedup_vs_single": args.batch / bdt / trees_per_s,
                          "replays": args.batch_steps, "graph": "one hipGraph per batch"}
        batch.close()
        for c in bctx:
            c.close()

    chis = [int(x) for x in args.per_chi.split(",") if x.strip() and int(x) != args.chi]
    if args.full and 64 not in chis and args.chi != 64:
        chis.append(64)
    if chis:
        # the same lattice and tree at other bond dimensions: time per tree and ln|Z| against the
        # FP64 oracle, for the float32 and the float64 form
        per = {}
        for chi in chis:
            rec = {"oracle_ln_abs_z": oracle_lnz(shape, args.beta, chi)}
            for prec in ("fp32", "fp64"):
                c = tn.Context(0)
                c.tn_load_graph(g.n, eu, ev, ed, off, data)
                c.tn_set_tree(pi, pj, chi, precision=prec)
                pinfo = c.tn_plan_info()
                if chi <= 32:
                    c.tn_contract_compressed()   # captures the schedule (untimed)
                    n = 2
                else:
                    n = 1                        # seconds per tree, enqueued launch by launch: no warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(n):
                    c.tn_enqueue()
                c.tn_fetch()
                torch.cuda.synchronize()
                cdt = (time.perf_counter() - t0) / n
                _, cl = c.tn_result()
                r = {"ms_per_tree": cdt * 1e3, "trees_per_s": 1.0 / cdt, "ln_abs_z": cl,
                     "tflops_fwd": pinfo["fwd_flops"] / cdt / 1e12, "arena_bytes": pinfo["arena_bytes"]}
                if rec["oracle_ln_abs_z"] is not None:
                    r["rel_dlnz_vs_oracle"] = abs(cl - rec["oracle_ln_abs_z"]) / abs(rec["oracle_ln_abs_z"])
                rec[prec] = r
                c.close()
            rec["rel_dlnz_fp32_vs_fp64"] = abs(rec["fp32"]["ln_abs_z"] - rec["fp64"]["ln_abs_z"]) / abs(
                rec["fp64"]["ln_abs_z"])
            per[str(chi)] = rec
        out["per_chi"] = per

    if args.fwd_bwd_steps > 0:
        # forward + reverse pass (d ln|Z| / d inputs) on gradient plans, in the bench precision and in
        # float64; the gradient stays on the device (tn_grad_device) inside the timed region
        fb = {}
        for prec in dict.fromkeys((args.precision, "fp64")):
            gctx = tn.Context(0)
            gctx.tn_load_graph(g.n, eu, ev, ed, off, data)
            gctx.tn_set_tree(pi, pj, args.chi, precision=prec, grad=True)
            ginfo = gctx.tn_plan_info()
            gbi = gctx.tn_grad_info()
            gdev = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
            gctx.tn_contract_compressed()
            gctx.tn_grad_device(gdev.data_ptr())
            gctx.tn_sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.fwd_bwd_steps):
                gctx.tn_contract_compressed()
                gctx.tn_grad_device(gdev.data_ptr())
                gctx.tn_sync()
            torch.cuda.synchronize()
            gdt = (time.perf_counter() - t0) / args.fwd_bwd_steps
            gg = gdev.cpu().numpy()
            total_f = ginfo["fwd_flops"] + gbi["bwd_flops"]
            eul = np.abs([float(np.dot(data[off[v]:off[v + 1]], gg[off[v]:off[v + 1]])) - 1.0 for v in range(g.n)])
            fb[prec] = {"ms_per_step": gdt * 1e3, "trees_per_s": 1.0 / gdt, "tflops": total_f / gdt / 1e12,
                        "fwd_flops": ginfo["fwd_flops"], "bwd_flops": gbi["bwd_flops"],
                        "arena_bytes": ginfo["arena_bytes"], "max_euler_identity_error": float(eul.max()),
                        "median_euler_identity_error": float(np.median(eul)), "steps": args.fwd_bwd_steps}
            gctx.close()
            if prec != args.precision:
                continue
            # the same step with checkpointed recomputation (segment count of smallest arena): the
            # reverse pass re-runs forward segments instead of keeping them resident
            rctx = tn.Context(0)
            rctx.tn_load_graph(g.n, eu, ev, ed, off, data)
            rctx.tn_set_tree(pi, pj, args.chi, precision=prec, grad=True, checkpoint_segments=-1)
            rinfo, rck = rctx.tn_plan_info(), rctx.tn_grad_checkpoint_info()
            rdev = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
            rctx.tn_contract_compressed()
            rctx.tn_grad_device(rdev.data_ptr())
            rctx.tn_sync()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.fwd_bwd_steps):
                rctx.tn_contract_compressed()
                rctx.tn_grad_device(rdev.data_ptr())
                rctx.tn_sync()
            torch.cuda.synchronize()
            rdt = (time.perf_counter() - t0) / args.fwd_bwd_steps
            rg = rdev.cpu().numpy()
            fb[prec]["recompute"] = {"segments": rck["segments"], "arena_bytes": rinfo["arena_bytes"],
                                     "checkpoint_bytes": rck["checkpoint_bytes"],
                                     "recompute_flops": rck["recompute_flops"], "ms_per_step": rdt * 1e3,
                                     "arena_ratio": rinfo["arena_bytes"] / ginfo["arena_bytes"],
                                     "time_ratio": rdt / gdt,
                                     "gradient_max_abs_diff_vs_resident": float(np.max(np.abs(rg - gg)))}
            rctx.close()
        out["fwd_bwd"] = fb
        if "fp64" in fb and not args.no_fp64_reference:
            out["fwd_bwd"]["tflops_vs_plain_fp64_forward"] = fb[args.precision]["tflops"] / (
                info["fwd_flops"] * out["fp64_plain"]["trees_per_s"] / 1e12)

    if args.spin_glass:
        L_sg, chi_sg = (int(x) for x in args.spin_glass.split(","))
        out["spin_glass"] = spin_glass_leg(tn, torch, L_sg, chi_sg, 0.5, 2)

    if not args.no_small:
        out["ising_8x8"] = ising_8x8_leg(tn, torch, 5)

    if args.full:
        out["urand_hardness"] = hardness_leg(tn, torch)
    if not args.no_second_workloads:
        out["pyrochlore_ising"] = pyrochlore_leg(tn, torch)

    if not args.no_tree_scoring:
        out["tree_scoring"] = tree_scoring_leg(tn, torch)

    if not args.no_tree_gauge:
        out["tree_gauge"] = tree_gauge_leg(tn, torch)

    if not args.no_random_graphs:
        out["dimer_rrg"] = dimer_leg(tn, torch, 3)
        out["normal_d3_rrg"] = normal_d3_leg(tn, torch, 3)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, T, pairs, args.chi, info["fwd_flops"], args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
