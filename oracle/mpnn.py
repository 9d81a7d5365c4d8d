"""FP64 oracle of the learned IC(0) correction network -- TEST INFRASTRUCTURE.

The paper has no learned component; this network is the added "learned
factor" form: a small message-passing network predicts corrections to the
IC(0) factor values on the same sparsity pattern, so the substitution sweeps
(Algorithm 1 and the backward sweep) are unchanged.  This module is the
plain reference the GPU training and inference kernels are checked against:
numpy, float64, hand-written forward and backward, verified by central finite
differences in the tests.

Definition (scaled space, D = diag(A')):
  s_i = 1/sqrt(a'_ii),  A~ = D^-1/2 A' D^-1/2,  L~0 = D^-1/2 L0 (IC(0) of A').
  Node features x_i = [L~0_ii, sum_{j!=i} |A~_ij|, deg_i / 26].
  Edge features f_ij = [A~_ij, [j < i], [j == i], L~0_(max(i,j), min(i,j))].
  Three layers, hidden width 32 (d_1 = 3, d_2 = d_3 = 32):
      p_e = W_m [h_j ; f_e] + b_m           for every off-diagonal edge e = (i, j)
      a_i = W_s h_i + b + sum_{e = (i, j)} relu(p_e)
      h'_i = relu(a_i)
  Readout on every lower entry k = (i, j), j <= i (diagonal included):
      u_k = relu(W_r [h_i ; h_j ; f_k] + b_r),  delta_k = w_o . u_k + b_o
      L~_k = L~0_k + 0.1 delta_k
  Loss over probes z (rows of Z):
      mean_z ||L~ L~^T z - A~ z||^2 / ||A~ z||^2
  Factor of A':  L_k = L~_k / s_i  (row i of the entry).

The parameter vector is the concatenation, in order, of for each layer
(W_s [32 x d], b [32], W_m [32 x (d+4)], b_m [32]) and then W_r [32 x 68],
b_r [32], w_o [32], b_o [1]; matrices row-major.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 32
NLAYERS = 3
NODE_F = 3
EDGE_F = 4
SCALE = 0.1


def layer_dims():
    return [NODE_F] + [HIDDEN] * (NLAYERS - 1)


def param_shapes():
    shapes = []
    for d in layer_dims():
        shapes += [("Ws", (HIDDEN, d)), ("b", (HIDDEN,)), ("Wm", (HIDDEN, d + EDGE_F)),
                   ("bm", (HIDDEN,))]
    shapes += [("Wr", (HIDDEN, 2 * HIDDEN + EDGE_F)), ("br", (HIDDEN,)), ("wo", (HIDDEN,)),
               ("bo", (1,))]
    return shapes


def param_count() -> int:
    return int(sum(np.prod(s) for _, s in param_shapes()))


def unpack(theta):
    out, k = [], 0
    for name, shp in param_shapes():
        size = int(np.prod(shp))
        out.append(np.asarray(theta[k:k + size], dtype=np.float64).reshape(shp))
        k += size
    layers = [tuple(out[4 * l:4 * l + 4]) for l in range(NLAYERS)]
    Wr, br, wo, bo = out[4 * NLAYERS:]
    return layers, (Wr, br, wo, bo[0])


def pack(layers, readout):
    parts = []
    for Ws, b, Wm, bm in layers:
        parts += [Ws.ravel(), b.ravel(), Wm.ravel(), bm.ravel()]
    Wr, br, wo, bo = readout
    parts += [Wr.ravel(), br.ravel(), wo.ravel(), np.array([bo], dtype=np.float64)]
    return np.concatenate(parts)


class Graph:
    """Index structure of a permuted CSR matrix (symmetric pattern, diagonal stored)."""

    def __init__(self, A):
        self.n = A.n
        self.rowptr = np.asarray(A.rowptr, dtype=np.int64)
        self.col = np.asarray(A.col, dtype=np.int64)
        self.row = np.repeat(np.arange(A.n), np.diff(self.rowptr))
        self.off = self.row != self.col                       # off-diagonal entries
        self.lower = self.col <= self.row                     # lower incl. diagonal
        self.diag = np.nonzero(self.row == self.col)[0]       # position of a_ii
        # position of the transposed entry
        key = self.row * A.n + self.col
        tkey = self.col * A.n + self.row
        order = np.argsort(key)
        self.tpos = order[np.searchsorted(key[order], tkey)]


def features(A, lval0, g: Graph):
    """Scaled matrix, scaled IC(0) factor, node and edge features."""
    a = np.asarray(A.val, dtype=np.float64)
    s = 1.0 / np.sqrt(a[g.diag])
    at = a * s[g.row] * s[g.col]
    l0t = np.asarray(lval0, dtype=np.float64) * s[g.row]      # row scaling, lower part
    l0t = np.where(g.lower, l0t, 0.0)
    lowpos = np.where(g.lower, np.arange(g.row.size), g.tpos)  # lower position of each entry
    absum = np.zeros(g.n)
    np.add.at(absum, g.row[g.off], np.abs(at[g.off]))
    deg = np.bincount(g.row[g.off], minlength=g.n).astype(np.float64)
    x = np.stack([l0t[g.diag], absum, deg / 26.0], axis=1)
    f = np.stack([at, (g.col < g.row).astype(np.float64), (g.col == g.row).astype(np.float64),
                  l0t[lowpos]], axis=1)
    return s, at, l0t, x, f


def forward(theta, A, lval0, g: Graph):
    """Returns (L~ on A's positions, lower only; cache for backward)."""
    layers, (Wr, br, wo, bo) = unpack(theta)
    s, at, l0t, x, f = features(A, lval0, g)
    h = x
    cache = {"s": s, "at": at, "l0t": l0t, "x": x, "f": f, "layers": []}
    ei, ej = g.row[g.off], g.col[g.off]
    fe = f[g.off]
    for Ws, b, Wm, bm in layers:
        p = np.concatenate([h[ej], fe], axis=1) @ Wm.T + bm
        msg = np.maximum(p, 0.0)
        agg = np.zeros((g.n, HIDDEN))
        np.add.at(agg, ei, msg)
        a_pre = h @ Ws.T + b + agg
        cache["layers"].append((h, p, a_pre))
        h = np.maximum(a_pre, 0.0)
    li, lj = g.row[g.lower], g.col[g.lower]
    fl = f[g.lower]
    q = np.concatenate([h[li], h[lj], fl], axis=1) @ Wr.T + br
    u = np.maximum(q, 0.0)
    delta = u @ wo + bo
    lt = np.zeros(g.row.size)
    lt[g.lower] = l0t[g.lower] + SCALE * delta
    cache.update({"h": h, "q": q, "u": u})
    return lt, cache


def lower_mv(g: Graph, lt, v):
    """L~ v (L~ stored at the lower positions)."""
    out = np.zeros(g.n)
    np.add.at(out, g.row[g.lower], lt[g.lower] * v[g.col[g.lower]])
    return out


def lower_t_mv(g: Graph, lt, v):
    """L~^T v."""
    out = np.zeros(g.n)
    np.add.at(out, g.col[g.lower], lt[g.lower] * v[g.row[g.lower]])
    return out


def sym_mv(g: Graph, at, v):
    out = np.zeros(g.n)
    np.add.at(out, g.row, at * v[g.col])
    return out


def loss_and_grad_L(g: Graph, lt, at, Z):
    """Probe loss and its gradient with respect to L~ at the lower positions.

    For one probe z: w = L~^T z, e = L~ w - A~ z, t = A~ z,
    loss = ||e||^2/||t||^2, d loss / d L~_ij = 2 (e_i w_j + z_i (L~^T e)_j) / ||t||^2.
    """
    G = np.zeros(g.row.size)
    total = 0.0
    li, lj = g.row[g.lower], g.col[g.lower]
    for z in Z:
        t = sym_mv(g, at, z)
        w = lower_t_mv(g, lt, z)
        e = lower_mv(g, lt, w) - t
        tt = float(t @ t)
        total += float(e @ e) / tt
        ge = lower_t_mv(g, lt, e)
        G[g.lower] += 2.0 * (e[li] * w[lj] + z[li] * ge[lj]) / tt
    m = len(Z)
    return total / m, G / m


def loss(theta, A, lval0, g: Graph, Z) -> float:
    lt, cache = forward(theta, A, lval0, g)
    return loss_and_grad_L(g, lt, cache["at"], Z)[0]


def loss_and_grad(theta, A, lval0, g: Graph, Z):
    """Loss and gradient with respect to theta (hand-written backward)."""
    layers, (Wr, br, wo, bo) = unpack(theta)
    lt, cache = forward(theta, A, lval0, g)
    L, GL = loss_and_grad_L(g, lt, cache["at"], Z)
    f, h = cache["f"], cache["h"]
    li, lj = g.row[g.lower], g.col[g.lower]
    fl = f[g.lower]
    ddelta = SCALE * GL[g.lower]
    # readout
    u, q = cache["u"], cache["q"]
    dwo = u.T @ ddelta
    dbo = ddelta.sum()
    dq = np.outer(ddelta, wo) * (q > 0)
    zin = np.concatenate([h[li], h[lj], fl], axis=1)
    dWr = dq.T @ zin
    dbr = dq.sum(axis=0)
    dzin = dq @ Wr
    dh = np.zeros_like(h)
    np.add.at(dh, li, dzin[:, :HIDDEN])
    np.add.at(dh, lj, dzin[:, HIDDEN:2 * HIDDEN])
    # layers, last to first
    ei, ej = g.row[g.off], g.col[g.off]
    fe = f[g.off]
    grads = []
    for (Ws, b, Wm, bm), (hin, p, a_pre) in zip(reversed(layers), reversed(cache["layers"])):
        da = dh * (a_pre > 0)
        dWs = da.T @ hin
        db = da.sum(axis=0)
        dhin = da @ Ws
        dp = da[ei] * (p > 0)
        min_ = np.concatenate([hin[ej], fe], axis=1)
        dWm = dp.T @ min_
        dbm = dp.sum(axis=0)
        dmin = dp @ Wm
        np.add.at(dhin, ej, dmin[:, :hin.shape[1]])
        grads.append((dWs, db, dWm, dbm))
        dh = dhin
    grads.reverse()
    return L, pack(grads, (dWr, dbr, dwo, dbo))


def factor_from_scaled(g: Graph, lt, s):
    """L of A' from L~ (undo the row scaling); upper positions zero."""
    out = np.where(g.lower, lt / s[g.row], 0.0)
    return out


def adam(theta, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015), bias-corrected; returns new theta, m, v."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
