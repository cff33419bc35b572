"""CPU tests of the native library's host side (no GPU needed).

* the shared library loads and exports every symbol include/tn.h declares;
* the host planner expands Algorithm 1 into exactly the oracle's op sequence
  (same contractions, same compressions in the same order, same shapes);
* the 32-bit fast division used by every gathered load is exact.
"""
import os
import re
import subprocess
import textwrap

import numpy as np
import pytest

import oracle
import paper_2206_07044_amd as tn
from tninputs import (dimer_tensors, greedy_tree, ising_tensors, lattice, normal_tensors, random_regular3)
from tninputs.trees import sweep_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_header_symbols():
    lib = tn.load_library()
    header = open(os.path.join(ROOT, "include", "tn.h")).read()
    declared = set(re.findall(r"\b(tn_[a-z_]+)\s*\(", header))
    assert declared == set(tn.exported_symbols())
    for name in declared:
        assert hasattr(lib, name), name


def test_create_without_device_reports_device_error():
    import ctypes
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(tn.TNError) as e:
        tn.Context(0)
    assert e.value.status in (tn.TN_EDEVICE, tn.TN_EINVAL)


def _oracle_ops(g, T, pairs, chi, late=False):
    r = oracle.contract_compressed(g.n, g.edges, T, pairs, chi, compress_late=late)
    return [(0 if o.kind == "contract" else 1, o.a, o.b, o.out, o.m, o.n, o.k, o.new_dim) for o in r.ops]


def _lib_ops(g, pairs, chi, late=False):
    eu, ev, ed = g.arrays()
    return tn.tn_plan_describe(g.n, eu, ev, ed, [a for a, _ in pairs], [b for _, b in pairs], chi, late=late)


CASES = [
    ("8x8 ising", lambda: lattice((8, 8)), lambda g: ising_tensors(g, 0.44), lambda g: sweep_tree((8, 8)), (4, 16, 256)),
    ("8x8 greedy", lambda: lattice((8, 8)), lambda g: ising_tensors(g, 0.44), lambda g: greedy_tree(g, 16, 0), (2, 16)),
    ("4^3", lambda: lattice((4, 4, 4)), lambda g: ising_tensors(g, 0.22), lambda g: sweep_tree((4, 4, 4)), (3, 8)),
    ("rrg dimer", lambda: random_regular3(24, 1), lambda g: dimer_tensors(g), lambda g: greedy_tree(g, 8, 1), (4, 8)),
    ("5x5 normal", lambda: lattice((5, 5)), lambda g: normal_tensors(g, 0.2, 0), lambda g: sweep_tree((5, 5)), (2, 3)),
]


@pytest.mark.parametrize("name,mk_g,mk_t,mk_p,chis", CASES, ids=[c[0] for c in CASES])
def test_schedule_matches_oracle_expansion(name, mk_g, mk_t, mk_p, chis):
    g = mk_g()
    T = mk_t(g)
    pairs = mk_p(g)
    for chi in chis:
        assert _lib_ops(g, pairs, chi) == _oracle_ops(g, T, pairs, chi)


@pytest.mark.parametrize("name,mk_g,mk_t,mk_p,chis", CASES, ids=[c[0] for c in CASES])
def test_late_schedule_matches_oracle_expansion(name, mk_g, mk_t, mk_p, chis):
    """Late compression (section II.D): the planner's op list equals the oracle's, and some
    compression runs before a contraction of the same tensor (not after it)."""
    g = mk_g()
    T = mk_t(g)
    pairs = mk_p(g)
    for chi in chis:
        ops = _lib_ops(g, pairs, chi, late=True)
        assert ops == _oracle_ops(g, T, pairs, chi, late=True)
        if any(o[0] == 1 for o in ops):
            assert ops != _lib_ops(g, pairs, chi)


def test_schedule_12cube_counts_match_tree_trace():
    from tninputs import simulate_tree
    g = lattice((12, 12, 12))
    pairs = sweep_tree((12, 12, 12))
    ops = _lib_ops(g, pairs, 16)
    st = simulate_tree(g, pairs, 16)
    assert sum(o[0] == 0 for o in ops) == st.n_contract == 1727
    assert sum(o[0] == 1 for o in ops) == st.n_compress


def test_describe_rejects_bad_trees():
    g = lattice((3, 3))
    eu, ev, ed = g.arrays()
    pairs = sweep_tree((3, 3))
    pi = [a for a, _ in pairs]
    pj = [b for _, b in pairs]
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(g.n, eu, ev, ed, pi[:-1], pj[:-1], 4)        # wrong step count
    bad = list(pj)
    bad[3] = pi[3]
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(g.n, eu, ev, ed, pi, bad, 4)                 # pair of one tensor
    bad = list(pi)
    bad[5] = pi[0]
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(g.n, eu, ev, ed, bad, pj, 4)                 # reuse of a dead id
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(g.n, ev, eu, ed, pi, pj, 4)                  # u > v
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(g.n, eu, ev, ed * 0, pi, pj, 4)              # zero dimension


def test_fastdiv_exact(tmp_path):
    src = tmp_path / "fd.cpp"
    src.write_text(textwrap.dedent('''
        #include "tn_internal.hpp"
        #include <cstdio>
        #include <random>
        using namespace tn;
        int main() {
            std::mt19937_64 rng(7);
            const uint32_t divs[] = {1,2,3,4,5,6,7,8,9,12,16,27,31,32,33,64,81,100,127,128,243,256,1000,
                                     1024,4095,4096,65535,65536,1000003,(1u<<30),(1u<<31)-1};
            for (uint32_t d : divs) {
                FastDiv f = make_fastdiv(d);
                for (int t = 0; t < 200000; ++t) {
                    uint32_t n = (t < 1000) ? (uint32_t)t : (uint32_t)(rng() % (1ull << 31));
                    if (t == 1000) n = (1u << 31) - 1;
                    if (fd_div(n, f) != n / d) { printf("FAIL %u %u\\n", n, d); return 1; }
                }
            }
            printf("OK\\n");
            return 0;
        }'''))
    exe = tmp_path / "fd"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_2206_07044_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and "OK" in out.stdout, out.stdout


def test_abi_null_and_invalid_arguments():
    """Every entry point rejects a null context or missing arrays with TN_EINVAL and never
    touches a device for it; destroy functions accept null."""
    import ctypes as C
    lib = tn.load_library()
    null = None
    d = C.c_double()
    assert lib.tn_load_graph(null, 1, 0, None, None, None, None, None) == tn.TN_EINVAL
    assert lib.tn_update_values(null, None) == tn.TN_EINVAL
    assert lib.tn_update_values_device(null, None) == tn.TN_EINVAL
    assert lib.tn_set_tree(null, 0, None, None, None) == tn.TN_EINVAL
    assert lib.tn_contract_compressed(null, C.byref(d), C.byref(d)) == tn.TN_EINVAL
    assert lib.tn_enqueue(null) == tn.TN_EINVAL
    assert lib.tn_fetch(null) == tn.TN_EINVAL
    assert lib.tn_result(null, C.byref(d), C.byref(d)) == tn.TN_EINVAL
    assert lib.tn_grad(null, None) == tn.TN_EINVAL
    assert lib.tn_grad_device(null, None) == tn.TN_EINVAL
    assert lib.tn_grad_info(null, None, None, None) == tn.TN_EINVAL
    assert lib.tn_sync(null) == tn.TN_EINVAL
    assert lib.tn_ising_values_device(null, 0.5, None) == tn.TN_EINVAL
    assert lib.tn_ising_coupling_grad_device(null, 0.5, None, None, None) == tn.TN_EINVAL
    assert lib.tn_batch_create(0, None, None) == tn.TN_EINVAL
    assert lib.tn_batch_contract(null, None, None) == tn.TN_EINVAL
    assert lib.tn_batch_grad(null, None) == tn.TN_EINVAL
    assert lib.tn_profile(null, 0) == tn.TN_EINVAL
    assert lib.tn_last_error(null) == b"null context"
    assert lib.tn_batch_last_error(null) == b"null batch"
    lib.tn_destroy(null)
    lib.tn_batch_destroy(null)


@pytest.mark.parametrize("pairs,chi,msg", [
    ([(0, 1), (4, 2)], 4, "steps"),                 # too few steps for 4 tensors
    ([(0, 1), (0, 2), (5, 3)], 4, "live"),           # tensor 0 used twice
    ([(0, 0), (4, 1), (5, 2)], 4, "live"),           # a tensor with itself
    ([(0, 1), (4, 2), (5, 9)], 4, "live"),           # unknown id
    ([(0, 1), (4, 2), (5, 3)], 0, "chi"),            # chi < 1
])
def test_describe_rejects_invalid_trees(pairs, chi, msg):
    g = lattice((2, 2))
    eu, ev, ed = g.arrays()
    with pytest.raises(tn.TNError) as e:
        tn.tn_plan_describe(g.n, eu, ev, ed, [a for a, _ in pairs], [b for _, b in pairs], chi)
    assert e.value.status == tn.TN_EINVAL


def test_describe_rejects_invalid_graphs():
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(3, [1], [0], [2], [0, 3], [1, 2], 4)        # u > v
    with pytest.raises(tn.TNError):
        tn.tn_plan_describe(3, [0], [1], [0], [0, 3], [1, 2], 4)        # dimension 0


def _tile_allowed(klass, tile):
    """The tiles include/tn.h allows for a class (short side, orientation, K)."""
    k = (klass // 2) % 3
    short32 = (klass // 6) % 2
    wide = (klass // 12) % 2
    skinny_k = k <= 1
    if tile == 0:
        return True
    tall_tiles = {1: not short32, 3: True, 5: not short32 and skinny_k, 6: skinny_k}
    wide_tiles = {2: not short32, 4: True, 7: not short32 and skinny_k, 8: skinny_k}
    return (wide_tiles if wide else tall_tiles).get(tile, False)


def test_gemm_tile_table_host_side():
    from paper_2206_07044_amd import autotune
    default = tn.tn_gemm_tiles_get().copy()
    try:
        assert default.size == tn.GEMM_CLASSES == 72
        assert all(_tile_allowed(c, int(t)) for c, t in enumerate(default))
        # class index round trip and the documented formula
        assert autotune.class_of(1, True, False, 1, True) == ((((1 * 2 + 1) * 2 + 0) * 3 + 1) * 2) + 1
        assert autotune.describe(autotune.class_of(0, False, True, 2, False)) == \
            "fp64 tall short<=32 K>64 long-axis strided"
        # every allowed tile installs; a disallowed one is refused and leaves the table as it was
        everywhere_64 = np.zeros(72, dtype=np.int32)
        tn.tn_gemm_tiles_set(everywhere_64)
        assert np.array_equal(tn.tn_gemm_tiles_get(), everywhere_64)
        for c in range(72):
            for tile in range(len(tn.GEMM_TILES)):
                t = everywhere_64.copy()
                t[c] = tile
                if _tile_allowed(c, tile):
                    tn.tn_gemm_tiles_set(t)
                    assert tn.tn_gemm_tiles_get()[c] == tile
                else:
                    before = tn.tn_gemm_tiles_get().copy()
                    with pytest.raises(tn.TNError) as e:
                        tn.tn_gemm_tiles_set(t)
                    assert e.value.status == tn.TN_EINVAL
                    assert np.array_equal(tn.tn_gemm_tiles_get(), before)
        with pytest.raises(ValueError):
            tn.tn_gemm_tiles_set(np.zeros(71, dtype=np.int32))
        tn.tn_gemm_tiles_set(None)
        assert np.array_equal(tn.tn_gemm_tiles_get(), default)
    finally:
        tn.tn_gemm_tiles_set(None)
