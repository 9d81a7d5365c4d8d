"""Full-size workloads shared by the GPU test modules, with the oracle's solve
of each started in a background thread.

The serial oracle needs 0.2-0.45 s per PCG iteration at these sizes, so one
solve to 1e-8 takes 1.5-3 minutes (128^3 7-point: about 580 iterations;
13-NN graph on 10^6 points: about 310; 27-point 96^3: about 410).  The
first full-size test module starts all three at once (the C call releases
the GIL), the GPU tests run meanwhile, and the solution-parity module at the
end of the session collects them.  Test infrastructure: the oracle and the
seeded generators only.
"""
from __future__ import annotations

import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

import oracle
import synth

TOL = 1e-8
MAXIT = 5000

# (workload, ABMC block size): the benchmark's timed matrix and ordering, the
# FEM-like graph and the 27-point stencil in the orderings the benchmark times
# (the fastest of its block-size sweep)
FULL = {
    "poisson7_128": 16,
    "knn13_1m": 4,
    "stencil27_96": 2,
}

_pool = ThreadPoolExecutor(max_workers=len(FULL))
_lock = threading.Lock()
_cases = {}


@dataclass
class FullCase:
    name: str
    A: object
    b: np.ndarray
    order: object        # oracle ordering (the library's is checked bit-exact against it)
    Ap: object           # P A P^T
    lval: np.ndarray     # oracle IC(0) factor of Ap
    bp: np.ndarray       # b in the permuted numbering
    future: object       # oracle PCG to TOL, running in a thread

    def oracle_solve(self):
        return self.future.result()


def case(name: str) -> FullCase:
    with _lock:
        if name not in _cases:
            A, b = synth.workload(name)
            o = oracle.order_abmc(A, FULL[name])
            Ap = oracle.permute(A, o.perm)
            lval, brk = oracle.ic0(Ap)
            assert brk < 0
            bp = np.ascontiguousarray(b[o.perm])
            fut = _pool.submit(oracle.pcg, Ap, lval, bp, TOL, MAXIT)
            _cases[name] = FullCase(name, A, b, o, Ap, lval, bp, fut)
        return _cases[name]


def start_all() -> None:
    for name in FULL:
        case(name)
