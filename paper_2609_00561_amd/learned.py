"""Training and use of the learned IC(0) correction (argument marshalling and
orchestration only; every step runs in libiccg.so's kernels).

Training matrices: 3D 7-point lognormal Poisson operators on a 32^3 grid, one
per seed k with sigma_k ~ U[0.5, 2], ABMC-ordered (block size 64).  Each step
draws 8 Gaussian vectors per matrix on the host from a seeded generator
(random numbers the method draws are inputs) and, by default, smooths each one
with the plain IC(0) preconditioner before it becomes a probe: in the
diagonally scaled space the probe is D^{1/2} M0^{-1} D^{1/2} z, rescaled to
norm sqrt(n).  CG's iteration count is set by the smooth error modes that
IC(0) leaves behind; Gaussian probes weight every mode alike, and a network
trained on them lowered the probe loss while needing more iterations.

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


def make_probes(ctx, rng, nprobes: int = 8, smooth: bool = True):
    """nprobes probe vectors for one training matrix (rows of a device
    tensor).  Smoothing needs a context from build_context with its IC(0)
    factor installed."""
    import torch
    Z = torch.tensor(rng.standard_normal((nprobes, ctx.n)), device="cuda")
    if not smooth:
        return Z
    out = torch.empty_like(Z)
    iccg.Network.smooth_probes(ctx, Z, out)
    return out


def train(net: "iccg.Network", ctxs, epochs: int, lr: float = 1e-3, nprobes: int = 8,
          seed: int = 0, log=None, smooth: bool = True):
    """Adam over the matrices in a seeded random order each epoch; returns the
    mean probe loss of every epoch.  The contexts hold their IC(0) factors."""
    rng = np.random.default_rng(seed)
    history = []
    for ep in range(epochs):
        losses = []
        for k in rng.permutation(len(ctxs)):
            ctx = ctxs[k]
            Z = make_probes(ctx, rng, nprobes, smooth)
            losses.append(net.train_step(ctx, Z, lr=lr, want_loss=True))
        history.append(float(np.mean(losses)))
        if log:
            log(f"[learned] epoch {ep + 1}/{epochs}: mean probe loss {history[-1]:.5f}")
    return history


def solve_both(net: "iccg.Network", ctx, b_dev, tol: float = 1e-8, maxit: int = 20000,
               bf16: bool = True):
    """Plain IC(0) and learned-factor solves of the same system on one context.

    Returns timings (device ms of each solve; steady-state inference +
    install ms; the per-matrix setup of the first prediction), the iteration
    counts, the factor actually kept (fallback rule) and the relative
    difference of the two solutions."""
    import torch
    n = ctx.n
    ctx.restore_ic0()
    x0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    # the first solve on a context also captures its iteration graph; solve
    # once untimed so that both timed solves replay the same graph
    ctx.solve(b_dev, x0, tol=tol, maxit=maxit, raise_on_noconv=False)
    x0.zero_()
    plain = ctx.solve(b_dev, x0, tol=tol, maxit=maxit, raise_on_noconv=False)
    plain_ms = ctx.info()["last_solve_ms"]

    lv = torch.zeros(ctx.nnz, dtype=torch.float64, device="cuda")
    # the first prediction on a matrix also builds its per-matrix features and
    # work buffers (setup, like ordering and factorization); the second one
    # is the steady-state inference
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.predict(ctx, lv, bf16=bf16)
    torch.cuda.synchronize()
    first_ms = 1e3 * (time.perf_counter() - t0)
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
           "setup_ms": max(first_ms - infer_ms, 0.0), "pivot_ok": accepted}
    if accepted:
        # untimed first, as for the plain solve, so both timed solves start
        # from the same state of the device
        x1 = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.solve(b_dev, x1, tol=tol, maxit=maxit, raise_on_noconv=False)
        x1.zero_()
        lr_ = ctx.solve(b_dev, x1, tol=tol, maxit=maxit, raise_on_noconv=False)
        a, b = x1.cpu().numpy(), x0.cpu().numpy()
        out.update({"learned_iters": lr_["iters"], "learned_ms": ctx.info()["last_solve_ms"],
                    "learned_relres_true": lr_["relres_true"],
                    "x_rel_diff": float(np.linalg.norm(a - b) / np.linalg.norm(b))})
        keep = lr_["status"] == iccg.ICCG_OK and lr_["iters"] < plain["iters"]
    else:
        keep = False
    out["kept"] = "learned" if keep else "ic0"
    if not keep:
        ctx.restore_ic0()
    return out
