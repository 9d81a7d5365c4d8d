"""Training and use of the learned IC(0) correction (argument marshalling and
orchestration only; every step runs in libiccg.so's kernels).

Training matrices: 3D 7-point lognormal Poisson operators on a 32^3 grid, one
per seed k with sigma_k ~ U[0.5, 2], ABMC-ordered (block size 64).  Each step
draws 8 Gaussian probes per matrix on the host from a seeded generator and
passes them to the library (random numbers the method draws are inputs).

Use: predict the factor (BF16 inference), install it with iccg_set_factor
(rejected on a non-positive or non-finite pivot), and keep it only if a
calibration solve needs fewer iterations than plain IC(0); otherwise restore
IC(0).  The choice is cached per context, so repeated solves pay it once.
"""
from __future__ import annotations

import time

import numpy as np

from . import iccg


def build_context(A, block_size: int = 64, **kw):
    """ABMC order, permute, set up and IC(0)-factor A; returns (ctx, order)."""
    order = iccg.iccg_order_abmc(A, block_size)
    rp, cl, vl = iccg.iccg_permute(A, order.perm)
    ctx = iccg.Context(rp, cl, vl, order.block_ptr, order.color_ptr, **kw)
    ctx.ic0_factor()
    return ctx, order


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases and a zero output layer (the
    untrained network reproduces IC(0))."""
    import synth
    return synth.glorot_params(iccg.mpnn_param_shapes(), seed).astype(np.float32)


def train(net: "iccg.Network", ctxs, epochs: int, lr: float = 1e-3, nprobes: int = 8,
          seed: int = 0, log=None):
    """Adam over the matrices in a seeded random order each epoch; returns the
    mean probe loss of every epoch."""
    import torch
    rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        losses = []
        for k in rng.permutation(len(ctxs)):
            ctx = ctxs[k]
            Z = torch.tensor(rng.standard_normal((nprobes, ctx.n)), device="cuda")
            losses.append(net.train_step(ctx, Z, lr=lr, want_loss=True))
        history.append(float(np.mean(losses)))
        if log:
            log(f"[learned] epoch {ep + 1}/{epochs}: mean probe loss {history[-1]:.5f}")
    return history


def solve_both(net: "iccg.Network", ctx, b_dev, tol: float = 1e-8, maxit: int = 20000,
               bf16: bool = True):
    """Plain IC(0) and learned-factor solves of the same system on one context.

    Returns timings (device ms of each solve, inference + install ms), the
    iteration counts, the factor actually kept (fallback rule) and the
    relative difference of the two solutions."""
    import torch
    n = ctx.n
    ctx.restore_ic0()
    x0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    plain = ctx.solve(b_dev, x0, tol=tol, maxit=maxit, raise_on_noconv=False)
    plain_ms = ctx.info()["last_solve_ms"]

    lv = torch.zeros(ctx.nnz, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.predict(ctx, lv, bf16=bf16)
    accepted = True
    try:
        ctx.set_factor(lv)
    except iccg.IccgError as e:
        if e.status != iccg.ICCG_EBREAKDOWN:
            raise
        accepted = False
    torch.cuda.synchronize()
    infer_ms = 1e3 * (time.perf_counter() - t0)
    out = {"plain_iters": plain["iters"], "plain_ms": plain_ms, "infer_ms": infer_ms,
           "pivot_ok": accepted}
    if accepted:
        x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
        lr_ = ctx.solve(b_dev, x1, tol=tol, maxit=maxit, raise_on_noconv=False)
        out.update({"learned_iters": lr_["iters"], "learned_ms": ctx.info()["last_solve_ms"],
                    "learned_relres_true": lr_["relres_true"],
                    "x_rel_diff": float(torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0))})
        keep = lr_["status"] == iccg.ICCG_OK and lr_["iters"] < plain["iters"]
    else:
        keep = False
    out["kept"] = "learned" if keep else "ic0"
    if not keep:
        ctx.restore_ic0()
    return out
