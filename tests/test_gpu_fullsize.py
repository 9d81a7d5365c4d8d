"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (per-color launches, HIP graph batches of 32 iterations).

* 3D 7-point lognormal Poisson 128^3 (n = 2,097,152), ABMC block sizes
  2/4/8/16/32/64: orderings bit-exact; factor, forward, backward, IC
  application and SpMV element by element against the serial oracle (which
  finishes these single steps in well under a second); the solve to 1e-8
  checked by its true residual recomputed on the host.
* 13-NN graph Laplacian on 10^6 points: ABMC(4, 8, 32), Leiden-CPM(0.05) and
  Leiden-modularity orderings bit-exact; IC application on the Leiden
  orderings element by element; the solves by their true residual.
* 27-point lognormal(sigma = 2) stencil on 96^3, ABMC(2), FP32 form: IC application
  against the oracle run on the factor rounded to FP32; the solve by its true
  residual and its distance from the FP64 solve.

The whole oracle solves of these matrices (1.5-3 minutes each) start in
background threads with the first test here; test_gpu_solution_parity.py
compares iteration counts, residual histories and solutions with them.

Tolerances are those of the small-size parity tests (1e-12 for FP64
substitution output, 1e-14 for the factor and the SpMV, 1e-4 for the FP32
arithmetic).
"""
import numpy as np
import pytest

import _fullsize
import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2609_00561_amd import iccg  # noqa: E402

_W = {}


def _workload(name):
    if name in _fullsize.FULL:
        fc = _fullsize.case(name)
        return fc.A, fc.b
    if name not in _W:
        _W[name] = synth.workload(name)
    return _W[name]


def _dev(x):
    return torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _same_order(o_lib, o_or):
    assert np.array_equal(np.asarray(o_lib.perm), np.asarray(o_or.perm))
    assert np.array_equal(np.asarray(o_lib.block_ptr), np.asarray(o_or.block_ptr))
    assert np.array_equal(np.asarray(o_lib.color_ptr), np.asarray(o_or.color_ptr))


def _true_relres(A, perm, x_perm, b):
    """||b - A x|| / ||b|| on the host, in the original numbering."""
    x = np.empty_like(x_perm)
    x[np.asarray(perm)] = x_perm
    r = b - A.to_scipy() @ x
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def test_start_oracle_solves():
    """Starts the oracle's full-size solves (collected at the end of the
    session by test_gpu_solution_parity.py)."""
    _fullsize.start_all()


@pytest.fixture(scope="module")
def poisson():
    fc = _fullsize.case("poisson7_128")
    A, b = fc.A, fc.b
    o = iccg.iccg_order_abmc(A, 16)
    _same_order(o, fc.order)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    Ap, lval = fc.Ap, fc.lval
    assert np.array_equal(np.asarray(rp), Ap.rowptr) and np.array_equal(np.asarray(cl), Ap.col)
    assert np.array_equal(np.asarray(vl), Ap.val)
    ctx = iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr)
    ctx.ic0_factor()
    yield A, b, o, Ap, lval, ctx
    ctx.close()


@pytest.mark.parametrize("s", [2, 4, 8, 32, 64])
def test_poisson128_abmc_orderings_bit_exact(s):
    A, _ = _workload("poisson7_128")
    _same_order(iccg.iccg_order_abmc(A, s), oracle.order_abmc(A, s))


def test_poisson128_factor(poisson):
    """The device IC(0) (the context's default) equals the oracle's bit for bit."""
    A, b, o, Ap, lval, ctx = poisson
    got = ctx.get_factor()
    assert np.array_equal(got, lval)


def test_poisson128_substitutions(poisson):
    A, b, o, Ap, lval, ctx = poisson
    r = np.random.default_rng(11).uniform(-1, 1, A.n)
    y_want = oracle.forward(Ap, lval, r)
    z_want = oracle.backward(Ap, lval, y_want)
    zd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    ctx.ic_apply(_dev(r), zd)
    err = _rel_inf(_host(zd), z_want)
    yd = torch.zeros_like(zd)
    ctx.ic_forward(_dev(r), yd)
    ey = _rel_inf(_host(yd), y_want)
    ctx.ic_backward(_dev(y_want), zd)
    ez = _rel_inf(_host(zd), z_want)
    print("128^3 apply / forward / backward rel err", err, ey, ez)
    assert err <= 1e-12 and ey <= 1e-12 and ez <= 1e-12


def test_poisson128_spmv(poisson):
    A, b, o, Ap, lval, ctx = poisson
    p = np.random.default_rng(12).standard_normal(A.n)
    qd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    pq = ctx.spmv(_dev(p), qd, want_dot=True)
    want = oracle.spmv(Ap, p)
    # per-row rounding scale: sum_j |a_ij p_j| (the oracle sums in ascending
    # column order, the GPU in slot order with FMA)
    scale = oracle.spmv(type(Ap)(Ap.n, Ap.rowptr, Ap.col, np.abs(Ap.val)), np.abs(p))
    err = np.max(np.abs(_host(qd) - want) / np.maximum(scale, 1e-300))
    print("128^3 SpMV max error / row scale", err)
    assert err <= 1e-14
    assert pq == pytest.approx(oracle.dot(p, want), rel=1e-13)


def test_poisson128_solve(poisson):
    A, b, o, Ap, lval, ctx = poisson
    bp = b[np.asarray(o.perm)]
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    res = ctx.solve(_dev(bp), xd, tol=1e-8)
    assert res["status"] == iccg.ICCG_OK and res["relres"] <= 1e-8
    true = _true_relres(A, o.perm, _host(xd), b)
    print("128^3 iters", res["iters"], "relres", res["relres"], "true", true, res["relres_true"])
    assert true <= 2e-8
    assert abs(true - res["relres_true"]) <= 1e-6 * true


@pytest.mark.parametrize("mode", ["single", "hybrid"])
def test_poisson128_dataflow_sweeps_identical(poisson, mode):
    """The persistent single-launch sweep and the hybrid (per-color launches
    for the large colors, one dataflow launch for the small ones) at full
    size: bit-identical to the per-color launches, for the IC application
    and for a whole solve."""
    A, b, o, Ap, lval, ctx = poisson
    rp, cl, vl = Ap.rowptr, Ap.col, Ap.val
    r = np.random.default_rng(13).standard_normal(A.n)
    z1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    ctx.ic_apply(_dev(r), z1)
    bp = _dev(b[np.asarray(o.perm)])
    x1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    r1 = ctx.solve(bp, x1, tol=1e-8)
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr, sweep_launch=mode) as c2:
        c2.ic0_factor()
        z2 = torch.zeros_like(z1)
        c2.ic_apply(_dev(r), z2)
        assert np.array_equal(_host(z1), _host(z2))
        x2 = torch.zeros_like(x1)
        r2 = c2.solve(bp, x2, tol=1e-8)
        assert r2["iters"] == r1["iters"] and np.array_equal(_host(x1), _host(x2))


@pytest.fixture(scope="module")
def knn():
    return _workload("knn13_1m")


def test_knn1m_orderings_bit_exact(knn):
    A, _ = knn
    for s in (4, 8, 32):
        _same_order(iccg.iccg_order_abmc(A, s), oracle.order_abmc(A, s))
    _same_order(iccg.iccg_order_leiden(A, "modularity", 1.0),
                oracle.order_leiden(A, "modularity", 1.0))


def test_knn1m_leiden_cpm_apply_and_solve(knn):
    A, b = knn
    o = iccg.iccg_order_leiden(A, "cpm", 0.05)
    _same_order(o, oracle.order_leiden(A, "cpm", 0.05))
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    Ap = oracle.permute(A, o.perm)
    lval, brk = oracle.ic0(Ap)
    assert brk < 0
    r = np.random.default_rng(14).uniform(-1, 1, A.n)
    want = oracle.ic_apply(Ap, lval, r)
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr) as ctx:
        ctx.ic0_factor()
        assert np.array_equal(ctx.get_factor(), lval)     # device IC(0), bit for bit
        zd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        ctx.ic_apply(_dev(r), zd)
        err = _rel_inf(_host(zd), want)
        print("knn 1M Leiden-CPM apply rel err", err, "blocks", o.nblocks, "colors", o.ncolors)
        assert err <= 1e-12
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = ctx.solve(_dev(b[np.asarray(o.perm)]), xd, tol=1e-8)
        assert res["status"] == iccg.ICCG_OK
        true = _true_relres(A, o.perm, _host(xd), b)
        print("knn 1M iters", res["iters"], "true relres", true)
        assert true <= 2e-8


def test_knn1m_leiden_md_wide_blocks(knn):
    """Leiden-MD on the kNN graph: 74 communities of up to 25,455 rows, run
    by workgroups in level-scheduled pieces of 512 rows.  IC application
    element by element against the oracle; the solve by its true residual."""
    A, b = knn
    o = iccg.iccg_order_leiden(A, "modularity", 1.0)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    Ap = oracle.permute(A, o.perm)
    lval, brk = oracle.ic0(Ap)
    assert brk < 0
    r = np.random.default_rng(16).uniform(-1, 1, A.n)
    want = oracle.ic_apply(Ap, lval, r)
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr) as ctx:
        ctx.ic0_factor()
        zd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        ctx.ic_apply(_dev(r), zd)
        err = _rel_inf(_host(zd), want)
        print("knn 1M Leiden-MD apply rel err", err, "blocks", o.nblocks, "colors", o.ncolors)
        assert err <= 1e-12
        xd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        res = ctx.solve(_dev(b[np.asarray(o.perm)]), xd, tol=1e-8)
        assert res["status"] == iccg.ICCG_OK
        true = _true_relres(A, o.perm, _host(xd), b)
        print("knn 1M Leiden-MD iters", res["iters"], "true relres", true)
        assert true <= 2e-8


def test_stencil27_96_fp32_form():
    A, b = _workload("stencil27_96")
    o = iccg.iccg_order_abmc(A, _fullsize.FULL["stencil27_96"])
    _same_order(o, oracle.order_abmc(A, _fullsize.FULL["stencil27_96"]))
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    Ap = oracle.permute(A, o.perm)
    lval, brk = oracle.ic0(Ap)
    assert brk < 0
    l32 = lval.astype(np.float32).astype(np.float64)
    r = np.random.default_rng(15).uniform(-1, 1, A.n)
    want = oracle.ic_apply(Ap, l32, r)
    bp = _dev(b[np.asarray(o.perm)])
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr, precision="fp32") as c32, \
            iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr) as c64:
        c32.ic0_factor()
        c64.ic0_factor()
        zd = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        c32.ic_apply(_dev(r), zd)
        err = _rel_inf(_host(zd), want)
        x32 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
        x64 = torch.zeros_like(x32)
        r32 = c32.solve(bp, x32, tol=1e-8)
        r64 = c64.solve(bp, x64, tol=1e-8)
        a32, a64 = _host(x32), _host(x64)
    true = _true_relres(A, o.perm, a32, b)
    diff = float(np.linalg.norm(a32 - a64) / np.linalg.norm(a64))
    print("27-pt 96^3 fp32 apply err", err, "iters fp32/fp64", r32["iters"], r64["iters"],
          "true relres", true, "x diff", diff)
    assert err <= 1e-4
    assert r32["status"] == iccg.ICCG_OK and true <= 2e-8
    assert r32["iters"] <= 1.2 * r64["iters"] + 5
    assert diff <= 1e-3
