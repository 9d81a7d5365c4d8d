"""iccg_spmv_dot_noalloc, the entry point for callers that cannot allocate:
the same q = A'p and (p, q) as iccg_spmv, with the partial sums in the
library's static device array instead of the context's buffer.

Two calls in a row on different contexts, the second with the smaller
matrix (the static array keeps the first call's partials beyond the second
call's count): both bit-identical to iccg_spmv, and within the SpMV and dot
tolerances of the oracle (1e-14 of the row scale, 1e-13 relative)."""
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


def _one(name, s, seed):
    A, _ = synth.workload(name)
    o = iccg.iccg_order_abmc(A, s)
    rp, cl, vl = iccg.iccg_permute(A, o.perm)
    Ap = oracle.permute(A, o.perm)
    p = np.random.default_rng(seed).standard_normal(A.n)
    with iccg.Context(rp, cl, vl, o.block_ptr, o.color_ptr) as ctx:
        pd = torch.tensor(p, device="cuda")
        q1 = torch.zeros_like(pd)
        pq1 = ctx.spmv(pd, q1, want_dot=True)
        q2 = torch.full_like(pd, np.nan)
        pq2 = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        ctx.spmv_dot_noalloc(pd, q2, pq2)
        torch.cuda.synchronize()
        a, b, d = q1.cpu().numpy(), q2.cpu().numpy(), float(pq2.cpu().numpy()[0])
    assert np.array_equal(a, b)
    assert d == pq1
    want = oracle.spmv(Ap, p)
    scale = oracle.spmv(type(Ap)(Ap.n, Ap.rowptr, Ap.col, np.abs(Ap.val)), np.abs(p))
    assert np.max(np.abs(b - want) / np.maximum(scale, 1e-300)) <= 1e-14
    assert d == pytest.approx(oracle.dot(p, want), rel=1e-13)
    return A.n


def test_noalloc_spmv_dot_matches_spmv_two_calls():
    n1 = _one("poisson7_64", 16, 1)      # 262,144 rows: 2,048 partial sums
    n2 = _one("poisson7_16", 8, 2)       # 4,096 rows: 32 partial sums
    assert n2 < n1
    n3 = _one("knn13_20k", 32, 3)        # another matrix after the small one
    assert n3 > n2
