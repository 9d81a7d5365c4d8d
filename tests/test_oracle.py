"""Pins for the CPU oracle: values and properties fixed by the paper or by
mathematics, chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them.

Nothing here touches the GPU library.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_kv(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


# ---------------------------------------------------------------------------
# RNG
# ---------------------------------------------------------------------------
def test_splitmix64_published_vector():
    """SplitMix64 drives Leiden's randomness; pin it to the reference outputs."""
    with open(os.path.join(GOLDEN, "splitmix64.txt")) as f:
        lines = [l.split() for l in f if l.strip() and not l.startswith("#")]
    seed = int(lines[0][1])
    want = [int(l[0]) for l in lines[1:]]
    got = [int(v) for v in oracle.splitmix64(seed, len(want))]
    assert got == want


# ---------------------------------------------------------------------------
# ABMC blocking and block coloring (Section 3, Section 6.1)
# ---------------------------------------------------------------------------
def test_abmc_table6_block_sizes():
    """Table 6: ABMC gives B_max = ceil(n/n_b), G = 0.00, B_max/B_avg = 1.00.

    The paper's matrices are not available; a banded graph with the same n
    stands in (the rule depends only on n and the block size).
    """
    rows = []
    with open(os.path.join(GOLDEN, "table6_abmc.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 8
    for name, n, nb, bmax, g, ratio in rows:
        n, nb, bmax = int(n), int(nb), int(bmax)
        s = math.ceil(n / nb)
        A = synth.banded_graph(n, 512)
        blocks = oracle.abmc_blocks(A, s)
        sizes = np.bincount(blocks)
        assert sizes.size == nb, name
        assert sizes.max() == bmax, name
        assert np.all(sizes[:-1] == s), name
        assert f"{sizes.max() / sizes.mean():.2f}" == ratio, name
        # the Gini sum is O(n_b^2); use the sorted-form identity only as a cross check
        s_sorted = np.sort(sizes).astype(float)
        idx = np.arange(1, nb + 1)
        g_sorted = (2 * np.sum(idx * s_sorted) / (nb * s_sorted.sum())) - (nb + 1) / nb
        assert f"{abs(g_sorted):.2f}" == g, name
        if nb <= 1024:
            assert f"{oracle.gini(sizes):.2f}" == g, name


def test_abmc_path_graph_closed_form():
    """On a path 0-1-...-(n-1), ABMC blocks are [ks, (k+1)s) and 2 colors suffice."""
    n, s = 1000, 37
    A = synth.path_graph_matrix(n)
    blocks = oracle.abmc_blocks(A, s)
    assert np.array_equal(blocks, np.arange(n) // s)
    colors = oracle.color_blocks(A, blocks)
    assert colors.max() + 1 == 2
    assert np.array_equal(colors, np.arange(colors.size) % 2)


def test_node_level_mc_checkerboard():
    """Node-level MC (block size 1) on a natural-order 2D 5-point grid gives
    exactly the two colors (x + y) mod 2."""
    nx = 23
    A = synth.grid2d_5pt(nx, nx)
    blocks = oracle.abmc_blocks(A, 1)
    assert np.array_equal(blocks, np.arange(A.n))
    colors = oracle.color_blocks(A, blocks)
    x, y = np.arange(A.n) % nx, np.arange(A.n) // nx
    assert np.array_equal(colors, (x + y) % 2)


def _block_graph_check(A, order):
    """Coloring invariant and greedy bound on the permuted matrix."""
    n = A.n
    block_of = np.repeat(np.arange(order.nblocks), np.diff(order.block_ptr))
    color_of_block = np.repeat(np.arange(order.ncolors), np.diff(order.color_ptr))
    Ap = oracle.permute(A, order.perm)
    rows = np.repeat(np.arange(n), np.diff(Ap.rowptr))
    bi, bj = block_of[rows], block_of[Ap.col]
    cross = bi != bj
    # no edge between two distinct blocks of one color
    assert not np.any(color_of_block[bi[cross]] == color_of_block[bj[cross]])
    # greedy bound: n_c <= max block degree + 1
    pairs = np.unique(np.stack([bi[cross], bj[cross]], 1), axis=0)
    deg = np.bincount(pairs[:, 0], minlength=order.nblocks)
    assert order.ncolors <= deg.max() + 1
    return Ap


@pytest.mark.parametrize("name", ["laplace2d_64", "poisson7_16", "stencil27_12", "knn13_20k"])
@pytest.mark.parametrize("s", [1, 8, 64])
def test_abmc_ordering_invariants(name, s):
    A, _ = synth.workload(name)
    order = oracle.order_abmc(A, s)
    # permutation is a bijection
    assert np.array_equal(np.sort(order.perm), np.arange(A.n))
    # block_ptr / color_ptr well formed
    assert order.block_ptr[0] == 0 and order.block_ptr[-1] == A.n
    assert np.all(np.diff(order.block_ptr) > 0)
    assert order.color_ptr[0] == 0 and order.color_ptr[-1] == order.nblocks
    assert np.all(np.diff(order.color_ptr) > 0)
    sizes = np.diff(order.block_ptr)
    assert sizes.max() == min(s, A.n)
    assert np.sum(sizes != s) <= 1
    _block_graph_check(A, order)


def test_order_rows_ascending_inside_block():
    """Rows of a block keep ascending original index (Algorithm 1 processes
    the rows of a block in ascending order)."""
    A, _ = synth.workload("knn13_20k")
    order = oracle.order_abmc(A, 32)
    for b in range(order.nblocks):
        seg = order.perm[order.block_ptr[b]:order.block_ptr[b + 1]]
        assert np.all(np.diff(seg) > 0)


# ---------------------------------------------------------------------------
# Leiden (Section 4, Section 7.1)
# ---------------------------------------------------------------------------
def test_quality_closed_forms():
    """Eq. (1) and Eq. (2) on two 5-cliques joined by an edge, split into the cliques."""
    g = _golden_kv("closed_forms.txt")
    A = synth.clique_ring(2, 5, ring=False)
    memb = np.repeat([0, 1], 5)
    assert oracle.quality(A, memb, "modularity", 1.0) == pytest.approx(g["q_md_two_k5"], rel=1e-14)
    assert oracle.quality(A, memb, "cpm", 0.05) == pytest.approx(g["q_cp_two_k5"], rel=1e-14)


def _all_partitions(n):
    """All set partitions of range(n) as restricted growth strings."""
    a = [0] * n

    def rec(i, m):
        if i == n:
            yield list(a)
            return
        for c in range(m + 1):
            a[i] = c
            yield from rec(i + 1, max(m, c + 1))
    yield from rec(1, 1)


@pytest.mark.parametrize("quality,gamma", [("modularity", 1.0), ("cpm", 0.3)])
def test_leiden_brute_force_small(quality, gamma):
    """On tiny graphs Leiden reaches the brute-force optimum of the quality function."""
    graphs = [synth.clique_ring(2, 5, ring=False),
              synth.from_edges(8, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4), (4, 5), (5, 3),
                                   (5, 6), (6, 7), (7, 5)])]
    for A in graphs:
        best = -1e300
        for p in _all_partitions(A.n):
            best = max(best, oracle.quality(A, np.array(p), quality, gamma))
        memb = oracle.leiden_blocks(A, quality, gamma)
        assert oracle.quality(A, memb, quality, gamma) == pytest.approx(best, abs=1e-12)
        assert oracle.community_connected(A, memb)


def test_leiden_ring_of_cliques():
    """Ring of six 5-cliques: modularity (gamma = 1) splits exactly into the cliques."""
    A = synth.clique_ring(6, 5)
    memb = oracle.leiden_blocks(A, "modularity", 1.0)
    assert np.array_equal(memb, np.repeat(np.arange(6), 5))


def test_leiden_cpm_large_gamma_singletons():
    """CPM with gamma >= 1 on an unweighted graph: joining never has a strictly
    positive gain (w - gamma*1*N_C <= 0), so every node stays alone."""
    A, _ = synth.workload("laplace2d_64")
    memb = oracle.leiden_blocks(A, "cpm", 1.0)
    assert np.array_equal(memb, np.arange(A.n))


def test_leiden_zero_resolution_components():
    """gamma = 0 (modularity) or gamma -> 0+ (CPM): communities are the
    connected components."""
    e = [(i, i + 1) for i in range(9)] + [(i, i + 1) for i in range(10, 24)] + [(30, 31)]
    A = synth.from_edges(40, e)
    comp = np.full(40, -1)
    labels = sp.csgraph.connected_components(A.to_scipy(), directed=False)[1]
    for quality, gamma in [("modularity", 0.0), ("cpm", 1e-9)]:
        memb = oracle.leiden_blocks(A, quality, gamma)
        # same partition up to renaming
        pairs = set(zip(memb.tolist(), labels.tolist()))
        assert len(pairs) == len(set(memb.tolist())) == len(set(labels.tolist()))
    del comp


@pytest.mark.parametrize("name", ["laplace2d_64", "poisson7_16", "knn13_20k"])
@pytest.mark.parametrize("quality,gamma", [("modularity", 1.0), ("cpm", 0.05)])
def test_leiden_invariants(name, quality, gamma):
    """Every community is connected (the Leiden guarantee), the quality beats
    the singleton partition, and the result is deterministic for a seed."""
    A, _ = synth.workload(name)
    memb = oracle.leiden_blocks(A, quality, gamma, seed=42)
    assert oracle.community_connected(A, memb)
    assert oracle.quality(A, memb, quality, gamma) > oracle.quality(A, np.arange(A.n), quality, gamma)
    again = oracle.leiden_blocks(A, quality, gamma, seed=42)
    assert np.array_equal(memb, again)
    # canonical numbering: ascending smallest member
    first = np.array([np.argmax(memb == c) for c in range(memb.max() + 1)])
    assert np.all(np.diff(first) > 0)


def test_leiden_block_sort_descending():
    """Section 7.1: blocks numbered by descending size (ties: smaller first node)."""
    A, _ = synth.workload("poisson7_16")
    blocks = oracle.sort_blocks_by_size(oracle.leiden_blocks(A, "cpm", 0.05))
    sizes = np.bincount(blocks)
    assert np.all(np.diff(sizes) <= 0)
    first = np.array([np.argmax(blocks == b) for b in range(sizes.size)])
    for b in range(sizes.size - 1):
        if sizes[b] == sizes[b + 1]:
            assert first[b] < first[b + 1]
    order = oracle.order_leiden(A, "cpm", 0.05)
    _block_graph_check(A, order)


# ---------------------------------------------------------------------------
# statistics (Section 7.3)
# ---------------------------------------------------------------------------
def test_gini_values():
    g = _golden_kv("closed_forms.txt")
    assert oracle.gini([1, 3]) == pytest.approx(g["gini_1_3"], abs=0)
    assert oracle.gini([5] * 17) == 0.0
    # one non-empty block among n_b: G = (n_b - 1) / n_b
    assert oracle.gini([0, 0, 0, 12]) == pytest.approx(3 / 4)


def _table6_rows():
    rows = []
    with open(os.path.join(GOLDEN, "table6_stats.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 24
    return rows


def _printed_equal(value, printed):
    """value rounded the way Table 6 prints it (two decimals, or three
    significant figures above 10) equals the printed string."""
    return (f"{value:.3g}" if value >= 10 else f"{value:.2f}") == printed


def _ordering(block_sizes, color_of_block):
    """An Ordering with the given block sizes (in block order) and colors
    (non-decreasing), over rows 0..n-1."""
    bs = np.asarray(block_sizes, dtype=np.int64)
    col = np.asarray(color_of_block, dtype=np.int64)
    bp = np.concatenate([[0], np.cumsum(bs)]).astype(np.int32)
    nc = int(col.max()) + 1
    cp = np.searchsorted(col, np.arange(nc + 1), side="left").astype(np.int32)
    return oracle.Ordering(np.arange(bp[-1], dtype=np.int32), bp, cp)


def test_block_stats_table6_ratios():
    """Table 6 prints n_b, B_max and B_max/B_avg for all 24 blockings, with n
    from Table 1: B_avg must be n / n_b (the mean block size).  C_max/C_avg
    must be the largest color's row count over n / n_c: with one block per
    color and the largest color holding round(printed ratio * n / n_c) rows,
    the printed ratio comes back (a blocks-per-color count would give 1.00)."""
    for name, meth, n, nb, nc, g, bmax, bratio, cratio in _table6_rows():
        n, nb, nc, bmax = int(n), int(nb), int(nc), int(bmax)
        rest = n - bmax
        sizes = [bmax] + [rest // (nb - 1) + (1 if k < rest % (nb - 1) else 0) for k in range(nb - 1)]
        assert max(sizes) == bmax
        st = oracle.block_stats(_ordering(sizes, np.zeros(nb)))
        assert st["n_b"] == nb and st["B_max"] == bmax and st["n_c"] == 1
        assert _printed_equal(st["B_max_over_avg"], bratio), (name, meth, st)
        cmax = round(float(cratio) * n / nc)
        rest = n - cmax
        csizes = [cmax] + [rest // (nc - 1) + (1 if k < rest % (nc - 1) else 0) for k in range(nc - 1)]
        st = oracle.block_stats(_ordering(csizes, np.arange(nc)))
        assert st["n_c"] == nc
        assert _printed_equal(st["C_max_over_avg"], cratio), (name, meth, st)


def test_block_stats_path_graph_hand_computed():
    """ABMC with s = 3 on the path 0-...-9: four blocks, two alternating colors;
    every statistic computed by hand (tests/golden/closed_forms.txt)."""
    g = _golden_kv("closed_forms.txt")
    A = synth.path_graph_matrix(10)
    st = oracle.block_stats(oracle.order_abmc(A, 3))
    assert st["n_b"] == g["path10_s3_nb"] and st["n_c"] == g["path10_s3_nc"]
    assert st["B_max"] == g["path10_s3_bmax"]
    assert st["gini"] == pytest.approx(g["path10_s3_gini"], rel=1e-15)
    assert st["B_max_over_avg"] == pytest.approx(g["path10_s3_bmax_over_avg"], rel=1e-15)
    assert st["C_max_over_avg"] == pytest.approx(g["path10_s3_cmax_over_avg"], rel=1e-15)


def test_block_stats_uniform_abmc_table6():
    """Table 6's ABMC rows: G = 0.00 and B_max/B_avg = 1.00 whenever s divides
    n; a ragged last block moves neither above the printed 0.00 / 1.00 at the
    paper's sizes (thermal2: n = 1,228,045, n_b = 1,024)."""
    A = synth.banded_graph(1228045, 512)
    o = oracle.order_abmc(A, math.ceil(1228045 / 1024))
    st = oracle.block_stats(o)
    assert st["n_b"] == 1024 and st["B_max"] == 1200
    assert f"{st['gini']:.2f}" == "0.00" and f"{st['B_max_over_avg']:.2f}" == "1.00"


def test_community_connected_detects_split():
    """The Leiden-guarantee check must reject a community that is two
    separate pieces, and accept the same nodes once they are joined."""
    A = synth.path_graph_matrix(6)
    assert oracle.community_connected(A, np.array([0, 0, 0, 1, 1, 1]))
    # community 0 = {0, 1} and {4, 5}: not connected through community 1
    assert not oracle.community_connected(A, np.array([0, 0, 1, 1, 0, 0]))
    # singletons and the whole path are connected
    assert oracle.community_connected(A, np.arange(6))
    assert oracle.community_connected(A, np.zeros(6, dtype=int))


# ---------------------------------------------------------------------------
# IC(0) (Section 3, Section 5)
# ---------------------------------------------------------------------------
def _lower_csr(A, lval):
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    keep = A.col <= rows
    return sp.csr_matrix((lval[keep], (rows[keep], A.col[keep])), shape=(A.n, A.n))


def test_ic0_1d_laplacian_closed_form():
    """tridiag(-1, 2, -1) in natural order: IC(0) is exact Cholesky with
    L_kk = sqrt((k+1)/k), L_{k+1,k} = -sqrt(k/(k+1)) (1-based k)."""
    n = 50
    A = synth.path_graph_matrix(n)
    # also under an ABMC order with 2 blocks (natural order is preserved)
    order = oracle.order_abmc(A, 25)
    assert np.array_equal(order.perm, np.arange(n))
    lval, br = oracle.ic0(A)
    assert br == -1
    L = _lower_csr(A, lval).toarray()
    k = np.arange(1, n + 1, dtype=float)
    assert np.allclose(np.diag(L), np.sqrt((k + 1) / k), rtol=1e-14, atol=0)
    assert np.allclose(np.diag(L, -1), -np.sqrt(k[:-1] / (k[:-1] + 1)), rtol=1e-14, atol=0)


def test_ic0_dense_equals_cholesky_any_order():
    """Full pattern: IC(0) of P A P^T is the Cholesky factor of P A P^T."""
    rng = np.random.default_rng(7)
    n = 9
    M = rng.standard_normal((n, n))
    D = M @ M.T + n * np.eye(n)
    rows, cols = np.nonzero(np.ones((n, n)))
    A = synth._from_coo(n, rows, cols, D[rows, cols])
    perm = rng.permutation(n).astype(np.int32)
    Ap = oracle.permute(A, perm)
    lval, br = oracle.ic0(Ap)
    assert br == -1
    L = _lower_csr(Ap, lval).toarray()
    ref = np.linalg.cholesky(D[np.ix_(perm, perm)])
    assert np.allclose(L, ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("name,s", [("laplace2d_64", 64), ("poisson7_16", 8), ("knn13_20k", 32),
                                    ("stencil27_12", 64)])
def test_ic0_pattern_invariant(name, s):
    """(L L^T)_ij = a'_ij for every (i, j) in the pattern of A'."""
    A, _ = synth.workload(name)
    Ap = oracle.permute(A, oracle.order_abmc(A, s).perm)
    lval, br = oracle.ic0(Ap)
    assert br == -1
    L = _lower_csr(Ap, lval)
    LLt = (L @ L.T).tocsr()
    rows = np.repeat(np.arange(Ap.n), np.diff(Ap.rowptr))
    got = np.asarray(LLt[rows, Ap.col]).ravel()
    scale = np.abs(Ap.val).max()
    assert np.max(np.abs(got - Ap.val)) <= 1e-13 * scale


def test_ic0_breakdown_row():
    """A symmetric matrix with positive diagonal whose second pivot is negative."""
    A = synth._from_coo(3, [0, 0, 1, 1, 2], [0, 1, 0, 1, 2], [1.0, 2.0, 2.0, 1.0, 1.0])
    _, br = oracle.ic0(A)
    assert br == 1


# ---------------------------------------------------------------------------
# substitutions (Algorithm 1 and the backward sweep)
# ---------------------------------------------------------------------------
def test_substitution_vs_solve_triangular():
    rng = np.random.default_rng(3)
    A = synth.random_spd_mmatrix(40, 0.2, rng)
    lval, br = oracle.ic0(A)
    assert br == -1
    L = _lower_csr(A, lval).toarray()
    r = rng.standard_normal(A.n)
    y = oracle.forward(A, lval, r)
    z = oracle.backward(A, lval, y)
    assert np.allclose(y, scipy.linalg.solve_triangular(L, r, lower=True), rtol=1e-13, atol=1e-14)
    assert np.allclose(z, scipy.linalg.solve_triangular(L.T, y, lower=False), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("name,s", [("poisson7_16", 16), ("knn13_20k", 32)])
def test_substitution_residual(name, s):
    """L (L^T z) = r to 1e-13 relative."""
    A, b = synth.workload(name)
    Ap = oracle.permute(A, oracle.order_abmc(A, s).perm)
    lval, _ = oracle.ic0(Ap)
    L = _lower_csr(Ap, lval)
    z = oracle.ic_apply(Ap, lval, b)
    res = L @ (L.T @ z) - b
    assert np.linalg.norm(res, np.inf) <= 1e-13 * np.linalg.norm(b, np.inf) * 10


def test_block_parallel_schedule_equals_serial():
    """Algorithm 1's schedule (colors in order, blocks of a color in any order,
    rows ascending) reproduces the serial sweep bit for bit on a valid coloring."""
    A, b = synth.workload("poisson7_16")
    order = oracle.order_abmc(A, 8)
    Ap = oracle.permute(A, order.perm)
    lval, _ = oracle.ic0(Ap)
    serial = oracle.forward(Ap, lval, b)
    rng = np.random.default_rng(0)
    y = np.full(Ap.n, np.nan)
    for c in range(order.ncolors):
        blocks = np.arange(order.color_ptr[c], order.color_ptr[c + 1])
        for blk in rng.permutation(blocks):
            for i in range(order.block_ptr[blk], order.block_ptr[blk + 1]):
                s = b[i]
                d = 0.0
                for k in range(Ap.rowptr[i], Ap.rowptr[i + 1]):
                    j = Ap.col[k]
                    if j < i:
                        s -= lval[k] * y[j]
                    elif j == i:
                        d = lval[k]
                y[i] = s / d
    assert np.array_equal(y, serial)


# ---------------------------------------------------------------------------
# PCG (Section 5)
# ---------------------------------------------------------------------------
def test_cg_finite_termination():
    """Plain CG on a tiny well-conditioned SPD system converges in <= n steps."""
    rng = np.random.default_rng(11)
    A = synth.random_spd_mmatrix(12, 0.5, rng, shift=1.0)
    b = rng.standard_normal(A.n)
    res = oracle.pcg(A, None, b, tol=1e-12, maxit=100)
    assert res.status == 0 and res.iters <= A.n
    assert np.allclose(res.x, np.linalg.solve(A.dense(), b), rtol=1e-10, atol=1e-12)


def test_pcg_exact_preconditioner_one_step():
    """With a full pattern IC(0) is exact, so PCG converges in one iteration."""
    rng = np.random.default_rng(5)
    n = 10
    M = rng.standard_normal((n, n))
    D = M @ M.T + n * np.eye(n)
    rows, cols = np.nonzero(np.ones((n, n)))
    A = synth._from_coo(n, rows, cols, D[rows, cols])
    lval, _ = oracle.ic0(A)
    b = rng.standard_normal(n)
    res = oracle.pcg(A, lval, b, tol=1e-10, maxit=50)
    assert res.status == 0 and res.iters == 1


def test_cg_lanczos_kappa_laplace2d():
    """Unpreconditioned CG on the 64x64 5-point Laplacian: the Lanczos estimate
    reaches the closed-form extreme eigenvalues 4 - 4cos(pi/65), 4 + 4cos(pi/65)."""
    g = _golden_kv("closed_forms.txt")
    A, b = synth.workload("laplace2d_64")
    res = oracle.pcg(A, None, b, tol=1e-12, maxit=5000)
    lmin, lmax, kappa = oracle.lanczos_kappa(res.alphas, res.betas)
    assert lmin == pytest.approx(g["lambda_min"], rel=1e-6)
    assert lmax == pytest.approx(g["lambda_max"], rel=1e-6)
    assert kappa == pytest.approx(g["kappa"], rel=1e-5)


def test_iccg_laplace2d_converges():
    """ICCG on the 64x64 Laplacian under ABMC (64 blocks of 64) reaches 1e-8,
    the recursive and true residuals agree, and it beats plain CG."""
    A, b = synth.workload("laplace2d_64")
    order = oracle.order_abmc(A, 64)
    Ap = oracle.permute(A, order.perm)
    lval, _ = oracle.ic0(Ap)
    res = oracle.pcg(Ap, lval, b[order.perm], tol=1e-8, maxit=1000)
    assert res.status == 0
    assert res.relres <= 1e-8
    assert res.relres_true <= 1.5e-8
    plain = oracle.pcg(A, None, b, tol=1e-8, maxit=5000)
    assert res.iters < plain.iters
    # solution of the permuted system is the permuted solution
    x = np.zeros(A.n)
    x[order.perm] = res.x
    assert np.linalg.norm(A.to_scipy() @ x - b) / np.linalg.norm(b) <= 1.5e-8


def test_pcg_zero_rhs_and_maxit():
    A, b = synth.workload("laplace2d_64")
    lval, _ = oracle.ic0(A)
    res = oracle.pcg(A, lval, np.zeros(A.n), tol=1e-8, maxit=10)
    assert res.iters == 0 and res.status == 0
    res = oracle.pcg(A, lval, b, tol=1e-8, maxit=1)
    assert res.status == 1 and res.iters == 1


def test_spmv_and_dot_vs_scipy():
    A, b = synth.workload("knn13_20k")
    x = np.random.default_rng(1).standard_normal(A.n)
    assert np.allclose(oracle.spmv(A, x), A.to_scipy() @ x, rtol=1e-13, atol=1e-12)
    assert oracle.dot(x, b) == pytest.approx(float(np.dot(x, b)), rel=1e-12)


def test_solution_distance_bounds():
    """The bounds the GPU solution tests use (tests/_parity_util.py) hold for
    two oracle solutions: the solve to 1e-8 against the solve to 1e-13 of the
    same system, for a shifted Laplacian (lambda_min from Gershgorin = the
    shift) and the Dirichlet Laplacian (closed-form lambda_min)."""
    import _parity_util as pu
    g = _golden_kv("closed_forms.txt")
    assert pu.lambda_min_lower(synth.workload("laplace2d_64")[0], "laplace2d_64") == \
        pytest.approx(g["lambda_min"], rel=1e-12)
    for name, s in (("poisson7_16", 8), ("laplace2d_64", 64), ("knn13_20k", 32)):
        A, b = synth.workload(name)
        o = oracle.order_abmc(A, s)
        Ap = oracle.permute(A, o.perm)
        lval, _ = oracle.ic0(Ap)
        bp = b[o.perm]
        loose = oracle.pcg(Ap, lval, bp, tol=1e-8)
        tight = oracle.pcg(Ap, lval, bp, tol=1e-13)
        lam = pu.lambda_min_lower(A, name)
        if name.startswith("poisson7"):
            assert lam == pytest.approx(1e-6, rel=1e-6)
        rep = pu.solution_report(Ap, lval, bp, tight.x, loose, lam, 1e-8)
        assert 0 < rep["err2"] <= rep["bound2"], (name, rep)
        assert 0 < rep["errA"] <= rep["boundA"], (name, rep)


def test_history_sensitivity_measure():
    """The measure that sets the residual-history bar of the GPU solve tests:
    one ulp of b moves the oracle's own history by far more than 1e-6 on the
    27-point sigma = 2 stencil (transient residual growth of 100x) and by
    about 1e-11 on the 7-point ABMC case."""
    import _parity_util as pu
    for name, s, lo, hi in (("stencil27_12", 64, 0.1, 10.0), ("poisson7_16", 8, 0.0, 1e-9)):
        A, b = synth.workload(name)
        o = oracle.order_abmc(A, s)
        Ap = oracle.permute(A, o.perm)
        lval, _ = oracle.ic0(Ap)
        sens = pu.history_sensitivity(Ap, lval, b[o.perm], 1e-8, 51)
        assert lo <= sens <= hi, (name, sens)
