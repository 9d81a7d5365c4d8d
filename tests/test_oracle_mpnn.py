"""Pins for the FP64 oracle of the learned IC(0) correction network."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mpnn


def _small(seed=3, m=4):
    rng = np.random.default_rng(seed)
    A = synth.grid3d_7pt_lognormal(m, m, m, 1.0, 1e-2, rng)
    o = oracle.order_abmc(A, 8)
    Ap = oracle.permute(A, o.perm)
    lval, br = oracle.ic0(Ap)
    assert br == -1
    return Ap, lval, rng


def _theta(seed, nonzero_out=True):
    th = synth.glorot_params(mpnn.param_shapes(), seed)
    if nonzero_out:
        rng = np.random.default_rng(seed + 1)
        th = th + 0.05 * rng.standard_normal(th.size)   # every block active, incl. w_o, b_o
    return th


def test_param_layout():
    assert mpnn.param_count() == mpnn.pack(*mpnn.unpack(np.arange(mpnn.param_count(), dtype=float))).size
    th = np.arange(mpnn.param_count(), dtype=float)
    assert np.array_equal(mpnn.pack(*mpnn.unpack(th)), th)


def test_zero_output_layer_reproduces_ic0():
    """w_o = 0 and b_o = 0: the predicted factor is IC(0) exactly."""
    Ap, lval, _ = _small()
    g = mpnn.Graph(Ap)
    th = synth.glorot_params(mpnn.param_shapes(), 1)
    lt, cache = mpnn.forward(th, Ap, lval, g)
    L = mpnn.factor_from_scaled(g, lt, cache["s"])
    assert np.allclose(L, np.where(g.lower, lval, 0.0), rtol=1e-14, atol=1e-15)


def test_gradient_matches_finite_differences():
    Ap, lval, rng = _small()
    g = mpnn.Graph(Ap)
    Z = rng.standard_normal((3, Ap.n))
    th = _theta(5)
    L, grad = mpnn.loss_and_grad(th, Ap, lval, g, Z)
    h = 1e-6
    idx = rng.choice(th.size, 60, replace=False)
    idx = np.concatenate([idx, [th.size - 1, th.size - 2]])   # b_o and w_o
    for k in idx:
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mpnn.loss(tp, Ap, lval, g, Z) - mpnn.loss(tm, Ap, lval, g, Z)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (k, fd, grad[k])


def test_grad_L_matches_finite_differences():
    Ap, lval, rng = _small()
    g = mpnn.Graph(Ap)
    Z = rng.standard_normal((2, Ap.n))
    s = 1.0 / np.sqrt(Ap.val[g.diag])
    at = Ap.val * s[g.row] * s[g.col]
    lt = np.where(g.lower, lval * s[g.row], 0.0) + 0.01 * rng.standard_normal(lval.size) * g.lower
    L0, G = mpnn.loss_and_grad_L(g, lt, at, Z)
    for k in rng.choice(np.nonzero(g.lower)[0], 40, replace=False):
        tp, tm = lt.copy(), lt.copy()
        tp[k] += 1e-6
        tm[k] -= 1e-6
        fd = (mpnn.loss_and_grad_L(g, tp, at, Z)[0] - mpnn.loss_and_grad_L(g, tm, at, Z)[0]) / 2e-6
        assert abs(fd - G[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, G[k])


def test_exact_ic0_zero_loss_and_gradient():
    """Tridiagonal in natural order: IC(0) is exact Cholesky, so the probe loss
    and its gradient with respect to L are zero at the IC(0) factor."""
    A = synth.path_graph_matrix(30)
    lval, _ = oracle.ic0(A)
    g = mpnn.Graph(A)
    Z = np.random.default_rng(0).standard_normal((4, A.n))
    s = 1.0 / np.sqrt(A.val[g.diag])
    at = A.val * s[g.row] * s[g.col]
    lt = np.where(g.lower, lval * s[g.row], 0.0)
    L, G = mpnn.loss_and_grad_L(g, lt, at, Z)
    assert L < 1e-28
    assert np.max(np.abs(G)) < 1e-13


def test_probe_loss_scale_invariance():
    """The scaled-space loss does not change when A' is scaled by a positive
    diagonal (IC(0) commutes with diagonal scaling)."""
    Ap, lval, rng = _small()
    g = mpnn.Graph(Ap)
    Z = rng.standard_normal((2, Ap.n))
    th = _theta(7)
    d = np.exp(rng.uniform(-2, 2, Ap.n))
    B = synth.CSR(Ap.n, Ap.rowptr, Ap.col, Ap.val * d[g.row] * d[g.col])
    lvB, _ = oracle.ic0(B)
    assert mpnn.loss(th, Ap, lval, g, Z) == pytest.approx(mpnn.loss(th, B, lvB, g, Z), rel=1e-10)


def test_adam_first_step():
    """Adam's first bias-corrected step moves every parameter by lr * sign(grad)."""
    th = np.zeros(5)
    gr = np.array([1.0, -2.0, 0.5, -1e-3, 3.0])
    new, m, v = mpnn.adam(th, gr, np.zeros(5), np.zeros(5), 1, lr=1e-3)
    assert np.allclose(new, -1e-3 * np.sign(gr), rtol=1e-6)
