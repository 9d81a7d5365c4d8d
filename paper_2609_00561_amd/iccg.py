"""ctypes binding of libiccg.so (include/iccg.h).

Argument marshalling only: every step of the solver runs in the library.
Host arrays are numpy arrays; device vectors are torch CUDA tensors (float64,
contiguous), passed to the library as raw device pointers.  PyTorch provides
device memory and the stream; it computes nothing here.

The library must be built (``python -m paper_2609_00561_amd.build``); loading
fails loudly if it is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiccg.so")

ICCG_OK = 0
ICCG_EINVAL = -1
ICCG_EPATTERN = -2
ICCG_EBADORDER = -3
ICCG_EBREAKDOWN = -4
ICCG_ENOCONV = -5
ICCG_ENAN = -6
ICCG_EHIP = -7
ICCG_ENOMEM = -8
ICCG_ESTATE = -9

ICCG_FP64 = 0
ICCG_FP32 = 1
QUALITY = {"modularity": 0, "cpm": 1}

# every symbol the header declares
EXPORTS = [
    "iccg_default_options", "iccg_order_abmc", "iccg_order_leiden", "iccg_permute",
    "iccg_setup", "ic0_factor", "iccg_set_factor", "iccg_restore_ic0", "iccg_get_factor", "ic_apply",
    "ic_forward", "ic_backward", "iccg_spmv", "iccg_dot", "iccg_solve",
    "iccg_residual_history", "iccg_profile_solve", "iccg_get_info", "iccg_schedule_stats",
    "iccg_block_stats",
    "iccg_strerror", "iccg_last_error",
    "iccg_destroy", "iccg_mpnn_param_count", "iccg_mpnn_create", "iccg_mpnn_get_params",
    "iccg_mpnn_set_params", "iccg_mpnn_loss_grad", "iccg_mpnn_train_step", "iccg_mpnn_predict",
    "iccg_mpnn_destroy", "iccg_mpnn_smooth_probes", "iccg_spmv_dot_noalloc",
    "iccg_solve_multi", "ic_apply_multi", "iccg_spmv_multi",
]


class IccgError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("check_every", ctypes.c_int), ("pack_rows", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("sweep_launch", ctypes.c_int),
                ("sweep_grid", ctypes.c_int), ("flow_tail", ctypes.c_int),
                ("wide_blocks", ctypes.c_int), ("host_factor", ctypes.c_int),
                ("fuse_turn", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nnz", ctypes.c_int), ("nnz_lower", ctypes.c_int),
                ("nblocks", ctypes.c_int), ("ncolors", ctypes.c_int),
                ("ntasks_fwd", ctypes.c_int), ("nchunks_fwd", ctypes.c_int),
                ("max_block", ctypes.c_int), ("max_depth", ctypes.c_int),
                ("precision", ctypes.c_int), ("has_factor", ctypes.c_int),
                ("sweep_bytes", ctypes.c_double), ("spmv_bytes", ctypes.c_double),
                ("last_solve_ms", ctypes.c_double), ("last_iters", ctypes.c_int),
                ("sweep_resident", ctypes.c_int), ("remote_tasks", ctypes.c_longlong),
                ("exported_rows", ctypes.c_longlong), ("gini", ctypes.c_double),
                ("bmax_over_avg", ctypes.c_double), ("cmax_over_avg", ctypes.c_double)]


_lib = None


def load():
    """Load libiccg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2609_00561_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    i, d, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "iccg_default_options": (None, [ctypes.POINTER(_Options)]),
        "iccg_order_abmc": (i, [i, vp, vp, i, vp, ip, vp, ip, vp]),
        "iccg_order_leiden": (i, [i, vp, vp, i, d, d, i, ctypes.c_uint64, vp, ip, vp, ip, vp]),
        "iccg_permute": (i, [i, vp, vp, vp, vp, vp, vp, vp]),
        "iccg_setup": (i, [ctypes.POINTER(vp), i, vp, vp, vp, i, vp, i, vp,
                           ctypes.POINTER(_Options)]),
        "iccg_schedule_stats": (i, [i, vp, vp, vp, i, vp, i, vp, i, vp]),
        "iccg_block_stats": (i, [i, vp, i, vp, vp]),
        "ic0_factor": (i, [vp, ip]),
        "iccg_set_factor": (i, [vp, vp, ip]),
        "iccg_get_factor": (i, [vp, vp]),
        "iccg_restore_ic0": (i, [vp]),
        "iccg_mpnn_param_count": (i, []),
        "iccg_mpnn_create": (i, [ctypes.POINTER(vp), vp, vp]),
        "iccg_mpnn_get_params": (i, [vp, vp]),
        "iccg_mpnn_set_params": (i, [vp, vp]),
        "iccg_mpnn_loss_grad": (i, [vp, vp, vp, i, dp, vp]),
        "iccg_mpnn_train_step": (i, [vp, vp, vp, i, ctypes.c_float, dp]),
        "iccg_mpnn_predict": (i, [vp, vp, i, vp]),
        "iccg_mpnn_destroy": (None, [vp]),
        "iccg_mpnn_smooth_probes": (i, [vp, vp, i, vp]),
        "ic_apply": (i, [vp, vp, vp]),
        "ic_forward": (i, [vp, vp, vp]),
        "ic_backward": (i, [vp, vp, vp]),
        "iccg_spmv": (i, [vp, vp, vp, dp]),
        "iccg_spmv_dot_noalloc": (i, [vp, vp, vp, vp]),
        "iccg_dot": (i, [vp, vp, vp, dp]),
        "iccg_solve": (i, [vp, vp, vp, d, i, ip, dp, dp]),
        "iccg_solve_multi": (i, [vp, i, vp, vp, d, i, vp, vp, vp]),
        "ic_apply_multi": (i, [vp, i, vp, vp]),
        "iccg_spmv_multi": (i, [vp, i, vp, vp]),
        "iccg_residual_history": (i, [vp, vp, i]),
        "iccg_profile_solve": (i, [vp, vp, vp, d, i, vp]),
        "iccg_get_info": (i, [vp, ctypes.POINTER(_Info)]),
        "iccg_strerror": (ctypes.c_char_p, [i]),
        "iccg_last_error": (ctypes.c_char_p, []),
        "iccg_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int, where: str):
    if st != ICCG_OK:
        lib = load()
        msg = lib.iccg_last_error().decode() or lib.iccg_strerror(st).decode()
        raise IccgError(st, where, msg)


def _host_i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _host_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a) -> int:
    """Raw pointer of a numpy array or a contiguous float64 CUDA tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    if not a.is_cuda or not a.is_contiguous():
        raise ValueError("device arguments must be contiguous CUDA tensors")
    return a.data_ptr()


@dataclass
class Ordering:
    perm: np.ndarray
    block_ptr: np.ndarray
    color_ptr: np.ndarray

    @property
    def nblocks(self):
        return self.block_ptr.size - 1

    @property
    def ncolors(self):
        return self.color_ptr.size - 1


# ---------------------------------------------------------------------------
# host ordering
# ---------------------------------------------------------------------------
def _ordering_call(fn, n, *args):
    perm = np.zeros(n, dtype=np.int32)
    bp = np.zeros(n + 1, dtype=np.int32)
    cp = np.zeros(n + 1, dtype=np.int32)
    nb, nc = ctypes.c_int(0), ctypes.c_int(0)
    st = fn(*args, perm.ctypes.data, ctypes.byref(nb), bp.ctypes.data, ctypes.byref(nc),
            cp.ctypes.data)
    _check(st, fn.__name__)
    return Ordering(perm, bp[:nb.value + 1].copy(), cp[:nc.value + 1].copy())


def iccg_order_abmc(A, block_size: int) -> Ordering:
    rp, cl = _host_i32(A.rowptr), _host_i32(A.col)
    return _ordering_call(load().iccg_order_abmc, A.n, A.n, rp.ctypes.data, cl.ctypes.data,
                          int(block_size))


def iccg_order_leiden(A, quality: str, gamma: float, beta: float = 0.01, n_iter: int = 2,
                      seed: int = 42) -> Ordering:
    rp, cl = _host_i32(A.rowptr), _host_i32(A.col)
    return _ordering_call(load().iccg_order_leiden, A.n, A.n, rp.ctypes.data, cl.ctypes.data,
                          QUALITY[quality], float(gamma), float(beta), int(n_iter), int(seed))


def iccg_permute(A, perm):
    """A' = P A P^T; returns (rowptr, col, val) numpy arrays."""
    rp, cl, vl = _host_i32(A.rowptr), _host_i32(A.col), _host_f64(A.val)
    pm = _host_i32(perm)
    prow = np.zeros(A.n + 1, dtype=np.int32)
    pcol = np.zeros(cl.size, dtype=np.int32)
    pval = np.zeros(cl.size, dtype=np.float64)
    st = load().iccg_permute(A.n, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data, pm.ctypes.data,
                             prow.ctypes.data, pcol.ctypes.data, pval.ctypes.data)
    _check(st, "iccg_permute")
    return prow, pcol, pval


SCHEDULE_FIELDS = ("tasks", "chunks", "slots", "max_depth", "max_width", "deps", "remote_tasks",
                   "exported_rows", "padded_chunks")


def iccg_block_stats(order: Ordering) -> dict:
    """Table 6 statistics of an ordering, computed by the library (host)."""
    bp = _host_i32(order.block_ptr)
    cp = _host_i32(order.color_ptr)
    out = np.zeros(6, dtype=np.float64)
    _check(load().iccg_block_stats(bp.size - 1, bp.ctypes.data, cp.size - 1, cp.ctypes.data,
                                   out.ctypes.data), "iccg_block_stats")
    return {"n_b": int(out[0]), "n_c": int(out[1]), "gini": float(out[2]), "B_max": int(out[3]),
            "B_max_over_avg": float(out[4]), "C_max_over_avg": float(out[5])}


def iccg_schedule_stats(rowptr, col, val, block_ptr, color_ptr, pack_rows: int = 64):
    """Host-only schedule build and invariant check (no GPU): returns
    {"forward": {...}, "backward": {...}} with SCHEDULE_FIELDS."""
    lib = load()
    rp, cl, vl = _host_i32(rowptr), _host_i32(col), _host_f64(val)
    bp, cp = _host_i32(block_ptr), _host_i32(color_ptr)
    nf = len(SCHEDULE_FIELDS)
    out = np.zeros(2 * nf, dtype=np.int64)
    _check(lib.iccg_schedule_stats(rp.size - 1, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data,
                                   bp.size - 1, bp.ctypes.data, cp.size - 1, cp.ctypes.data,
                                   int(pack_rows), out.ctypes.data), "iccg_schedule_stats")
    return {d: dict(zip(SCHEDULE_FIELDS, (int(v) for v in out[nf * k:nf * k + nf])))
            for k, d in enumerate(("forward", "backward"))}


# ---------------------------------------------------------------------------
# device context
# ---------------------------------------------------------------------------
class Context:
    """Owns one iccg_ctx (device copies of A', schedules, factor, work vectors)."""

    def __init__(self, rowptr, col, val, block_ptr, color_ptr, precision: str = "fp64",
                 stream=None, check_every: int = 32, pack_rows: int = 64, use_graph: bool = True,
                 sweep_launch: str = "per_color", sweep_grid: int = 0, flow_tail: int = 0,
                 wide_blocks: bool = True, host_factor: bool = False, fuse_turn: bool = True):
        import torch
        lib = load()
        opt = _Options()
        lib.iccg_default_options(ctypes.byref(opt))
        opt.precision = {"fp64": ICCG_FP64, "fp32": ICCG_FP32}[precision]
        if stream is None:
            stream = torch.cuda.current_stream()
        opt.stream = ctypes.c_void_p(stream.cuda_stream)
        opt.check_every = int(check_every)
        opt.pack_rows = int(pack_rows)
        opt.use_graph = 1 if use_graph else 0
        opt.sweep_launch = {"per_color": 0, "single": 1, "hybrid": 2}[sweep_launch]
        opt.sweep_grid = int(sweep_grid)
        opt.flow_tail = int(flow_tail)
        opt.wide_blocks = 1 if wide_blocks else 0
        opt.host_factor = 1 if host_factor else 0
        opt.fuse_turn = 1 if fuse_turn else 0
        self._keep = [_host_i32(rowptr), _host_i32(col), _host_f64(val), _host_i32(block_ptr),
                      _host_i32(color_ptr)]
        rp, cl, vl, bp, cp = self._keep
        self.n = rp.size - 1
        self.nnz = cl.size
        self.precision = precision
        h = ctypes.c_void_p()
        st = lib.iccg_setup(ctypes.byref(h), self.n, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data,
                            bp.size - 1, bp.ctypes.data, cp.size - 1, cp.ctypes.data,
                            ctypes.byref(opt))
        self._keep = None
        _check(st, "iccg_setup")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().iccg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- factor -------------------------------------------------------------
    def ic0_factor(self) -> int:
        row = ctypes.c_int(-1)
        st = load().ic0_factor(self._h, ctypes.byref(row))
        if st == ICCG_EBREAKDOWN:
            err = IccgError(st, "ic0_factor", f"breakdown at row {row.value}")
            err.row = row.value
            raise err
        _check(st, "ic0_factor")
        return row.value

    def set_factor(self, lvals_dev) -> None:
        row = ctypes.c_int(-1)
        st = load().iccg_set_factor(self._h, _ptr(lvals_dev), ctypes.byref(row))
        if st == ICCG_EBREAKDOWN:
            raise IccgError(st, "iccg_set_factor", f"rejected at row {row.value}")
        _check(st, "iccg_set_factor")

    def restore_ic0(self) -> None:
        _check(load().iccg_restore_ic0(self._h), "iccg_restore_ic0")

    def get_factor(self) -> np.ndarray:
        out = np.zeros(self.nnz, dtype=np.float64)
        _check(load().iccg_get_factor(self._h, out.ctypes.data), "iccg_get_factor")
        return out

    # -- hot path -------------------------------------------------------------
    def ic_apply(self, r, z):
        _check(load().ic_apply(self._h, _ptr(r), _ptr(z)), "ic_apply")

    def ic_forward(self, r, y):
        _check(load().ic_forward(self._h, _ptr(r), _ptr(y)), "ic_forward")

    def ic_backward(self, y, z):
        _check(load().ic_backward(self._h, _ptr(y), _ptr(z)), "ic_backward")

    def spmv(self, p, q, want_dot: bool = False):
        pq = ctypes.c_double(0.0)
        _check(load().iccg_spmv(self._h, _ptr(p), _ptr(q), ctypes.byref(pq) if want_dot else None),
               "iccg_spmv")
        return pq.value if want_dot else None

    def spmv_dot_noalloc(self, p, q, pq_dev) -> None:
        """q = A'p and pq_dev[0] = (p, q) on the device; allocates nothing."""
        _check(load().iccg_spmv_dot_noalloc(self._h, _ptr(p), _ptr(q), _ptr(pq_dev)),
               "iccg_spmv_dot_noalloc")

    def dot(self, a, b) -> float:
        out = ctypes.c_double(0.0)
        _check(load().iccg_dot(self._h, _ptr(a), _ptr(b), ctypes.byref(out)), "iccg_dot")
        return out.value

    def solve(self, b, x, tol: float = 1e-8, maxit: int = 10000, raise_on_noconv: bool = True):
        it = ctypes.c_int(0)
        rr, rt = ctypes.c_double(0.0), ctypes.c_double(0.0)
        st = load().iccg_solve(self._h, _ptr(b), _ptr(x), float(tol), int(maxit),
                               ctypes.byref(it), ctypes.byref(rr), ctypes.byref(rt))
        if st != ICCG_OK and (raise_on_noconv or st != ICCG_ENOCONV):
            _check(st, "iccg_solve")
        return {"status": st, "iters": it.value, "relres": rr.value, "relres_true": rt.value}

    def solve_multi(self, B, X, tol: float = 1e-8, maxit: int = 10000, raise_on_noconv: bool = True):
        """k independent solves: B, X device tensors [k, n] (row j = column j of
        the block); X holds x0 and receives the solutions."""
        k = self._block_k(B, X)
        iters = np.zeros(k, dtype=np.int32)
        rr = np.zeros(k)
        rt = np.zeros(k)
        st = load().iccg_solve_multi(self._h, k, _ptr(B), _ptr(X), float(tol), int(maxit),
                                     iters.ctypes.data, rr.ctypes.data, rt.ctypes.data)
        if st != ICCG_OK and not (st == ICCG_ENOCONV and not raise_on_noconv):
            _check(st, "iccg_solve_multi")
        return {"status": st, "iters": iters, "relres": rr, "relres_true": rt}

    def ic_apply_multi(self, R, Z):
        k = self._block_k(R, Z)
        _check(load().ic_apply_multi(self._h, k, _ptr(R), _ptr(Z)), "ic_apply_multi")

    def spmv_multi(self, P, Q):
        k = self._block_k(P, Q)
        _check(load().iccg_spmv_multi(self._h, k, _ptr(P), _ptr(Q)), "iccg_spmv_multi")

    def _block_k(self, A, B) -> int:
        if A.dim() != 2 or A.shape != B.shape or A.shape[1] != self.n:
            raise ValueError("block vectors must both be [k, n]")
        return int(A.shape[0])

    def profile_solve(self, b, x, tol: float = 1e-8, maxit: int = 10000) -> dict:
        out = np.zeros(10, dtype=np.float64)
        st = load().iccg_profile_solve(self._h, _ptr(b), _ptr(x), float(tol), int(maxit),
                                       out.ctypes.data)
        if st not in (ICCG_OK, ICCG_ENOCONV):
            _check(st, "iccg_profile_solve")
        keys = ["total_ms", "spmv_ms", "fwd_ms", "bwd_ms", "other_ms", "fwd_launches",
                "bwd_launches", "spmv_launches", "iters", "relres_true"]
        return dict(zip(keys, out.tolist()))

    def residual_history(self) -> np.ndarray:
        info = self.info()
        cap = info["last_iters"] + 1
        out = np.zeros(cap, dtype=np.float64)
        k = load().iccg_residual_history(self._h, out.ctypes.data, cap)
        if k < 0:
            _check(k, "iccg_residual_history")
        return out[:k]

    def info(self) -> dict:
        inf = _Info()
        _check(load().iccg_get_info(self._h, ctypes.byref(inf)), "iccg_get_info")
        return {name: getattr(inf, name) for name, _ in _Info._fields_}


# module-level names matching the C ABI (thin forwards to Context)
def iccg_setup(rowptr, col, val, block_ptr, color_ptr, **kw) -> Context:
    return Context(rowptr, col, val, block_ptr, color_ptr, **kw)


def ic0_factor(ctx: Context) -> int:
    return ctx.ic0_factor()


def iccg_set_factor(ctx: Context, lvals_dev) -> None:
    ctx.set_factor(lvals_dev)


def ic_apply(ctx: Context, r, z) -> None:
    ctx.ic_apply(r, z)


def iccg_solve(ctx: Context, b, x, tol: float = 1e-8, maxit: int = 10000):
    return ctx.solve(b, x, tol, maxit)


def iccg_destroy(ctx: Context) -> None:
    ctx.close()


# ---------------------------------------------------------------------------
# learned factor form
# ---------------------------------------------------------------------------
def mpnn_param_shapes():
    """Parameter blocks in the library's layout (include/iccg.h)."""
    shapes = []
    for d in (3, 32, 32):
        shapes += [("Ws", (32, d)), ("b", (32,)), ("Wm", (32, d + 4)), ("bm", (32,))]
    shapes += [("Wr", (32, 68)), ("br", (32,)), ("wo", (32,)), ("bo", (1,))]
    return shapes


class Network:
    """Owns one iccg_mpnn (FP32 master parameters, Adam state, work buffers)."""

    def __init__(self, params, stream=None):
        import torch
        lib = load()
        self.count = lib.iccg_mpnn_param_count()
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.count:
            raise ValueError(f"expected {self.count} parameters, got {p.size}")
        if stream is None:
            stream = torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib.iccg_mpnn_create(ctypes.byref(h), p.ctypes.data, ctypes.c_void_p(stream.cuda_stream)),
               "iccg_mpnn_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().iccg_mpnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def params(self) -> np.ndarray:
        out = np.zeros(self.count, dtype=np.float32)
        _check(load().iccg_mpnn_get_params(self._h, out.ctypes.data), "iccg_mpnn_get_params")
        return out

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load().iccg_mpnn_set_params(self._h, p.ctypes.data), "iccg_mpnn_set_params")

    def loss_grad(self, ctx: Context, probes_dev):
        loss = ctypes.c_double(0.0)
        grad = np.zeros(self.count, dtype=np.float32)
        nprobes = probes_dev.shape[0]
        _check(load().iccg_mpnn_loss_grad(self._h, ctx._h, _ptr(probes_dev), nprobes,
                                          ctypes.byref(loss), grad.ctypes.data), "iccg_mpnn_loss_grad")
        return loss.value, grad

    def train_step(self, ctx: Context, probes_dev, lr: float = 1e-3, want_loss: bool = True):
        loss = ctypes.c_double(0.0)
        nprobes = probes_dev.shape[0]
        _check(load().iccg_mpnn_train_step(self._h, ctx._h, _ptr(probes_dev), nprobes, float(lr),
                                           ctypes.byref(loss) if want_loss else None),
               "iccg_mpnn_train_step")
        return loss.value if want_loss else None

    @staticmethod
    def smooth_probes(ctx: Context, z_dev, out_dev) -> None:
        """out_i = D^1/2 M^-1 D^1/2 z_i scaled to norm sqrt(n) (rows of device tensors)."""
        if z_dev.shape != out_dev.shape or z_dev.shape[1] != ctx.n:
            raise ValueError("z and out must both be [nprobes, n]")
        _check(load().iccg_mpnn_smooth_probes(ctx._h, _ptr(z_dev), z_dev.shape[0], _ptr(out_dev)),
               "iccg_mpnn_smooth_probes")

    def predict(self, ctx: Context, out_dev, bf16: bool = True) -> None:
        _check(load().iccg_mpnn_predict(self._h, ctx._h, 1 if bf16 else 0, _ptr(out_dev)),
               "iccg_mpnn_predict")
