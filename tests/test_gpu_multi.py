"""Blocks of right-hand sides (iccg_solve_multi, ic_apply_multi,
iccg_spmv_multi): k independent solves sharing every read of the matrix and
the factor, the repeated-solve use the paper amortizes its blocking over
(Sections 7.6 and 10).

Each column must equal the single-vector entry point's result for it bit
for bit (same kernels' arithmetic, same partial sums, same reduction order),
and therefore the oracle to the single-vector tolerances: 1e-12 relative for
the IC application, 1e-14 of the row scale for the SpMV, iteration counts
within max(2, 1 %) and solutions within 1e-8 relative for the solves.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


from paper_2609_00561_amd import iccg  # noqa: E402

CASES = [
    ("poisson7_16", "abmc", 8, {}),
    ("poisson7_32", "abmc", 16, {}),
    ("knn13_20k", "abmc", 32, {}),                                 # padded chunks, wide rows
    ("stencil27_12", "abmc", 64, {}),                              # 27-point rows
    ("poisson7_16", "leiden", ("modularity", 1.0), {"wide_blocks": False}),   # multi-chunk tasks
    ("poisson7_32", "abmc", 16, {"precision": "fp32"}),            # FP32 form
]


def _ids(c):
    extra = ",".join(f"{k}={v}" for k, v in c[3].items())
    return f"{c[0]}-{c[1]}-{c[2]}" + (f"-{extra}" if extra else "")


_CACHE = {}


def _case(name, kind, param):
    key = (name, kind, str(param))
    if key not in _CACHE:
        A, b = synth.workload(name)
        o = iccg.iccg_order_abmc(A, param) if kind == "abmc" else iccg.iccg_order_leiden(A, *param)
        rp, cl, vl = iccg.iccg_permute(A, o.perm)
        Ap = oracle.permute(A, o.perm)
        lval, _ = oracle.ic0(Ap)
        _CACHE[key] = (A, b, o, (rp, cl, vl), Ap, lval)
    return _CACHE[key]


def _block(n, k, seed):
    """k right-hand sides: uniform[-1, 1] columns of different scales, one of
    them zero (a column that stops before its first iteration)."""
    rng = np.random.default_rng(seed)
    B = rng.uniform(-1, 1, (k, n)) * np.logspace(0, 3, k)[:, None]
    if k >= 3:
        B[1] = 0.0
    return B


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("k", [1, 3, 8, 16])
def test_apply_and_spmv_columns_equal_single(case, k):
    A, b, o, (rp, cl, vl), Ap, lval = _case(*case[:3])
    R = _block(A.n, k, 1)
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr, **case[3]) as ctx:
        ctx.ic0_factor()
        Rd = torch.tensor(R, device="cuda")
        Zd = torch.zeros_like(Rd)
        ctx.ic_apply_multi(Rd, Zd)
        Qd = torch.zeros_like(Rd)
        ctx.spmv_multi(Rd, Qd)
        Z, Q = _host(Zd), _host(Qd)
        for j in range(k):
            z1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            ctx.ic_apply(Rd[j].contiguous(), z1)
            q1 = torch.zeros_like(z1)
            ctx.spmv(Rd[j].contiguous(), q1)
            assert np.array_equal(Z[j], _host(z1)), j
            assert np.array_equal(Q[j], _host(q1)), j
    fp32 = case[3].get("precision") == "fp32"
    scale_m = type(Ap)(Ap.n, Ap.rowptr, Ap.col, np.abs(Ap.val))
    lv = lval.astype(np.float32).astype(np.float64) if fp32 else lval
    for j in range(k):
        if not np.any(R[j]):
            assert not np.any(Z[j]) and not np.any(Q[j])
            continue
        want = oracle.ic_apply(Ap, lv, R[j])
        assert np.max(np.abs(Z[j] - want)) <= (1e-4 if fp32 else 1e-12) * np.max(np.abs(want))
        qw = oracle.spmv(Ap, R[j])
        assert np.max(np.abs(Q[j] - qw) / np.maximum(oracle.spmv(scale_m, np.abs(R[j])), 1e-300)) <= 1e-14


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("k", [3, 8])
def test_solve_columns_equal_single_and_oracle(case, k):
    A, b, o, (rp, cl, vl), Ap, lval = _case(*case[:3])
    B = _block(A.n, k, 2)
    B[0] = b[np.asarray(o.perm)]
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr, **case[3]) as ctx:
        ctx.ic0_factor()
        Bd = torch.tensor(B, device="cuda")
        Xd = torch.zeros_like(Bd)
        res = ctx.solve_multi(Bd, Xd, tol=1e-8)
        X = _host(Xd)
        singles = []
        for j in range(k):
            x1 = torch.zeros(A.n, dtype=torch.float64, device="cuda")
            r1 = ctx.solve(Bd[j].contiguous(), x1, tol=1e-8)
            singles.append((r1, _host(x1)))
    assert res["status"] == iccg.ICCG_OK
    for j in range(k):
        r1, x1 = singles[j]
        assert res["iters"][j] == r1["iters"], j
        assert res["relres"][j] == r1["relres"] and res["relres_true"][j] == r1["relres_true"], j
        assert np.array_equal(X[j], x1), j
    if case[3].get("precision") == "fp32":
        return
    for j in range(k):
        if not np.any(B[j]):
            assert res["iters"][j] == 0 and not np.any(X[j])
            continue
        ref = oracle.pcg(Ap, lval, B[j], tol=1e-8, maxit=5000)
        assert abs(int(res["iters"][j]) - ref.iters) <= max(2, int(0.01 * ref.iters)), j
        assert np.linalg.norm(X[j] - ref.x) <= 1e-8 * np.linalg.norm(ref.x), j


def test_multi_edge_cases():
    A, b, o, (rp, cl, vl), Ap, lval = _case("poisson7_16", "abmc", 8)
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr) as ctx:
        ctx.ic0_factor()
        lib = iccg.load()
        X = torch.zeros(17, A.n, dtype=torch.float64, device="cuda")
        for k in (0, 17):
            st = lib.iccg_solve_multi(ctx._h, k, X.data_ptr(), X.data_ptr(), 1e-8, 100, None, None, None)
            assert st == iccg.ICCG_EINVAL
        # maxit reached in some columns: ENOCONV, every column's count at maxit
        B = torch.tensor(_block(A.n, 4, 3), device="cuda")
        Xd = torch.zeros_like(B)
        res = ctx.solve_multi(B, Xd, maxit=5, raise_on_noconv=False)
        assert res["status"] == iccg.ICCG_ENOCONV
        assert list(res["iters"]) == [5, 0, 5, 5]
        # a NaN in one column: ENAN, the other columns still converge
        Bn = _block(A.n, 3, 4)
        Bn[2, 7] = np.nan
        Xd = torch.zeros(3, A.n, dtype=torch.float64, device="cuda")
        with pytest.raises(iccg.IccgError) as e:
            ctx.solve_multi(torch.tensor(Bn, device="cuda"), Xd)
        assert e.value.status == iccg.ICCG_ENAN
        # a larger block after a smaller one, and a smaller one again
        for k in (2, 16, 5):
            Bk = torch.tensor(_block(A.n, k, 10 + k), device="cuda")
            Xk = torch.zeros_like(Bk)
            rk = ctx.solve_multi(Bk, Xk)
            assert rk["status"] == iccg.ICCG_OK and np.all(rk["relres"] <= 1e-8)
