"""CPU tests of libiccg.so's host side: exported symbols, ordering parity with
the oracle (bit-exact), and setup validation (runs before any HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2609_00561_amd import iccg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "iccg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_header_symbol():
    lib = iccg.load()
    names = _header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(iccg.EXPORTS) == names


def _same(o1, o2):
    return (np.array_equal(o1.perm, o2.perm) and np.array_equal(o1.block_ptr, o2.block_ptr)
            and np.array_equal(o1.color_ptr, o2.color_ptr))


@pytest.mark.parametrize("name", ["laplace2d_64", "poisson7_16", "knn13_20k", "stencil27_12"])
@pytest.mark.parametrize("s", [1, 8, 16, 32, 64])
def test_abmc_bit_exact(name, s):
    A, _ = synth.workload(name)
    assert _same(oracle.order_abmc(A, s), iccg.iccg_order_abmc(A, s))


@pytest.mark.parametrize("name", ["laplace2d_64", "poisson7_16", "knn13_20k", "stencil27_12"])
@pytest.mark.parametrize("quality,gamma", [("modularity", 1.0), ("modularity", 4.0),
                                           ("cpm", 0.05), ("cpm", 1e-3), ("cpm", 0.3)])
def test_leiden_bit_exact(name, quality, gamma):
    A, _ = synth.workload(name)
    assert _same(oracle.order_leiden(A, quality, gamma), iccg.iccg_order_leiden(A, quality, gamma))


@pytest.mark.parametrize("seed", [9, 31, 42, 58, 74])
def test_leiden_seeds_bit_exact(seed):
    """The paper's seed set (Section 7.1)."""
    A, _ = synth.workload("knn13_20k")
    for quality, gamma in [("modularity", 1.0), ("cpm", 0.05)]:
        assert _same(oracle.order_leiden(A, quality, gamma, seed=seed),
                     iccg.iccg_order_leiden(A, quality, gamma, seed=seed))


def test_ordering_random_graphs_bit_exact():
    rng = np.random.default_rng(123)
    for trial in range(20):
        n = int(rng.integers(2, 300))
        A = synth.random_spd_mmatrix(n, float(rng.uniform(0.005, 0.2)), rng)
        for s in (1, 3, 17):
            assert _same(oracle.order_abmc(A, s), iccg.iccg_order_abmc(A, s)), (trial, s)
        for quality, gamma in [("modularity", 1.0), ("cpm", 0.1)]:
            seed = int(rng.integers(0, 2**63))
            assert _same(oracle.order_leiden(A, quality, gamma, seed=seed),
                         iccg.iccg_order_leiden(A, quality, gamma, seed=seed)), (trial, quality)


@pytest.mark.slow
def test_leiden_bit_exact_knn_100k():
    A, _ = synth.workload("knn13_100k")
    for quality, gamma in [("modularity", 1.0), ("cpm", 0.05)]:
        assert _same(oracle.order_leiden(A, quality, gamma), iccg.iccg_order_leiden(A, quality, gamma))


def test_permute_bit_exact():
    A, _ = synth.workload("knn13_20k")
    o = oracle.order_leiden(A, "cpm", 0.05)
    Ap = oracle.permute(A, o.perm)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    assert np.array_equal(Ap.rowptr, rp) and np.array_equal(Ap.col, cl) and np.array_equal(Ap.val, vl)


def test_permute_rejects_non_permutation():
    A, _ = synth.workload("laplace2d_64")
    perm = np.arange(A.n, dtype=np.int32)
    perm[5] = 4
    with pytest.raises(iccg.IccgError) as e:
        iccg.iccg_permute(A, perm)
    assert e.value.status == iccg.ICCG_EINVAL


def test_order_argument_errors():
    A, _ = synth.workload("laplace2d_64")
    with pytest.raises(iccg.IccgError):
        iccg.iccg_order_abmc(A, 0)
    with pytest.raises(iccg.IccgError):
        iccg.iccg_order_leiden(A, "cpm", -1.0)


# ---------------------------------------------------------------------------
# setup validation: runs on the host before any device call
# ---------------------------------------------------------------------------
def _raw_setup(rowptr, col, val, block_ptr, color_ptr, **opts):
    lib = iccg.load()
    opt = None
    if opts:
        opt = iccg._Options()
        lib.iccg_default_options(ctypes.byref(opt))
        for k, v in opts.items():
            setattr(opt, k, v)
        opt = ctypes.byref(opt)
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    vl = np.ascontiguousarray(val, dtype=np.float64)
    bp = np.ascontiguousarray(block_ptr, dtype=np.int32)
    cp = np.ascontiguousarray(color_ptr, dtype=np.int32)
    h = ctypes.c_void_p()
    st = lib.iccg_setup(ctypes.byref(h), rp.size - 1, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data,
                        bp.size - 1, bp.ctypes.data, cp.size - 1, cp.ctypes.data, opt)
    if st == 0:
        lib.iccg_destroy(h)
    return st


def _ordered(name="laplace2d_64", s=64):
    A, _ = synth.workload(name)
    o = iccg.iccg_order_abmc(A, s)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    return rp, cl, vl, o


def test_setup_rejects_same_color_neighbours():
    rp, cl, vl, o = _ordered()
    bad_cp = np.array([0, o.nblocks], dtype=np.int32)      # every block in one color
    assert _raw_setup(rp, cl, vl, o.block_ptr, bad_cp) == iccg.ICCG_EBADORDER


def test_setup_rejects_malformed_ptrs():
    rp, cl, vl, o = _ordered()
    bp = o.block_ptr.copy()
    bp[-1] -= 1
    assert _raw_setup(rp, cl, vl, bp, o.color_ptr) == iccg.ICCG_EBADORDER
    bp = o.block_ptr.copy()
    bp[3] = bp[2]                                           # empty block
    assert _raw_setup(rp, cl, vl, bp, o.color_ptr) == iccg.ICCG_EBADORDER
    cp = o.color_ptr.copy()
    cp[-1] += 1
    assert _raw_setup(rp, cl, vl, o.block_ptr, cp) == iccg.ICCG_EBADORDER


def test_setup_rejects_bad_patterns():
    rp, cl, vl, o = _ordered()
    # missing diagonal in row 0
    k = int(np.nonzero(cl[rp[0]:rp[1]] == 0)[0][0])
    vl2 = vl.copy()
    cl2 = cl.copy()
    cl2[k] = cl2[k + 1] - 1 if cl2[k + 1] - 1 > 0 else 1
    assert _raw_setup(rp, cl2, vl2, o.block_ptr, o.color_ptr) == iccg.ICCG_EPATTERN
    # unsymmetric pattern: drop one off-diagonal entry of row 0
    off = [k for k in range(rp[0], rp[1]) if cl[k] != 0][0]
    keep = np.ones(cl.size, dtype=bool)
    keep[off] = False
    rp3 = rp.copy()
    rp3[1:] -= 1
    assert _raw_setup(rp3, cl[keep], vl[keep], o.block_ptr, o.color_ptr) == iccg.ICCG_EPATTERN
    # unsorted columns in row 1
    cl4 = cl.copy()
    a, b = rp[1], rp[1] + 1
    cl4[a], cl4[b] = cl4[b], cl4[a]
    assert _raw_setup(rp, cl4, vl, o.block_ptr, o.color_ptr) == iccg.ICCG_EPATTERN


def test_setup_rejects_nonfinite_values():
    rp, cl, vl, o = _ordered()
    vl = vl.copy()
    vl[7] = np.nan
    assert _raw_setup(rp, cl, vl, o.block_ptr, o.color_ptr) == iccg.ICCG_EINVAL


def _empty():
    class Empty:
        n, nnz = 0, 0
        rowptr = np.array([0], dtype=np.int32)
        col = np.array([], dtype=np.int32)
        val = np.array([], dtype=np.float64)
    return Empty()


def test_empty_matrix():
    """n = 0: the orderings and the permutation return the empty ordering;
    setup rejects it (there is nothing to solve)."""
    A = _empty()
    for o in (iccg.iccg_order_abmc(A, 16), iccg.iccg_order_leiden(A, "cpm", 0.05),
              iccg.iccg_order_leiden(A, "modularity", 1.0)):
        assert (o.nblocks, o.ncolors, np.asarray(o.perm).size) == (0, 0, 0)
        assert list(o.block_ptr) == [0] and list(o.color_ptr) == [0]
    assert _same(oracle.order_abmc(A, 16), iccg.iccg_order_abmc(A, 16))
    assert _same(oracle.order_leiden(A, "cpm", 0.05), iccg.iccg_order_leiden(A, "cpm", 0.05))
    rp, cl, vl = iccg.iccg_permute(A, np.array([], dtype=np.int32))
    assert list(rp) == [0] and np.asarray(cl).size == 0 and np.asarray(vl).size == 0
    assert _raw_setup(A.rowptr, A.col, A.val, [0], [0]) == iccg.ICCG_EINVAL
    assert b"n >= 1" in iccg.load().iccg_last_error()


def test_default_options():
    opt = iccg._Options()
    iccg.load().iccg_default_options(ctypes.byref(opt))
    assert (opt.precision, opt.check_every, opt.pack_rows, opt.use_graph) == (iccg.ICCG_FP64, 32, 64, 1)
    assert (opt.sweep_launch, opt.sweep_grid, opt.flow_tail, opt.wide_blocks) == (0, 0, 0, 1)


def test_setup_rejects_bad_options():
    """Option checks come before any device call, so they are host logic."""
    rp, cl, vl, o = _ordered()
    for bad in ({"precision": 2}, {"sweep_launch": 3}, {"sweep_launch": -1},
                {"sweep_grid": -8}, {"flow_tail": -1}):
        assert _raw_setup(rp, cl, vl, o.block_ptr, o.color_ptr, **bad) == iccg.ICCG_EINVAL, bad


@pytest.mark.parametrize("name", ["laplace2d_64", "poisson7_16", "knn13_20k", "stencil27_12"])
def test_block_stats_bit_exact(name):
    """iccg_block_stats (Section 7.3, Table 6: n_b, n_c, G, B_max, B_max/B_avg,
    C_max/C_avg) equals the oracle's statistics bit for bit on ABMC (uniform
    blocks, ragged last block) and Leiden (non-uniform) orderings."""
    A, _ = synth.workload(name)
    orders = [iccg.iccg_order_abmc(A, s) for s in (1, 7, 16, 64)]
    orders += [iccg.iccg_order_leiden(A, "cpm", 0.05), iccg.iccg_order_leiden(A, "modularity", 1.0)]
    for o in orders:
        got = iccg.iccg_block_stats(o)
        want = oracle.block_stats(oracle.Ordering(o.perm, o.block_ptr, o.color_ptr))
        assert got == want, (got, want)


def test_block_stats_rejects_bad_ordering():
    with pytest.raises(iccg.IccgError) as e:
        iccg.iccg_block_stats(iccg.Ordering(np.arange(4), np.array([0, 2, 2, 4]), np.array([0, 3])))
    assert e.value.status == iccg.ICCG_EBADORDER
