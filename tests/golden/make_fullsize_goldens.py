"""Write the full-size reference eigenvalues the GPU tests compare against.

Runs the FP64 CPU oracle (oracle/trplk.py, Alg. 1; oracle/block.py for a
block case) on the full-size workloads that bench.py and
tests/test_gpu_fullsize.py run, from the same seeded start block, and
stores per case the Ritz values, the residual norms (stored and
recomputed), the cycle and product counts and the norm used in the stopping
test of eq. (5.1).  Only oracle/ and the seeded input
generators are called: no value here comes from the GPU path.

    python tests/golden/make_fullsize_goldens.py [case ...]

Cases (name = workload_preconditioner_tol):
  lap3d_jacobi_1e-08    3-D Laplacian 128^3 + V ~ U[0, 0.05], p10 m40 k20 l1
  lap3d_jacobi_1e-11    the same at the tightened tolerance (certifies the
                        eigenvalues to ~1e-13 relative)
  powerlaw_jacobi_1e-08 shifted power-law graph Laplacian, n = 10^6, p20 m48 k24
  fem3d_fsai_1e-08      Q1 FEM pencil on 97^3 elements (B != I), FSAI on A,
                        p16 m48 k24
  aniso3d64_jacobi_1e-08  the anisotropic generator of the largest workload
                        at 64^3 (n = 262,144) with its solver shape, p50 m64
                        k32, hard locking (the 256^3 instance takes days)
  lap3d47_jacobi_s4_1e-08  block TRPL+K (oracle/block.py, block size 4) on the
                        Laplacian's generator at 47^3 (n = 103,823: not a
                        multiple of any tile), p10 m40 k20
Each takes minutes to hours (seconds per cycle on a few host cores).
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import block as OB  # noqa: E402
from oracle import precond as OP  # noqa: E402
from oracle import trplk as O  # noqa: E402
from workloads import make, start_block  # noqa: E402

CASES = {
    "lap3d_jacobi_1e-08": ("lap3d", "jacobi", 1e-8),
    "lap3d_jacobi_1e-11": ("lap3d", "jacobi", 1e-11),
    "powerlaw_jacobi_1e-08": ("powerlaw", "jacobi", 1e-8),
    "fem3d_fsai_1e-08": ("fem3d", "fsai", 1e-8),
    "aniso3d64_jacobi_1e-08": ("aniso3d", "jacobi", 1e-8, {"N": 64}),
    "lap3d47_jacobi_s4_1e-08": ("lap3d", "jacobi", 1e-8, {"N": 47}, 4),
}


def case_kwargs(case: str) -> dict:
    """Generator overrides of a case (the size of a reduced instance)."""
    return dict(CASES[case][3]) if len(CASES[case]) > 3 else {}


def case_block(case: str) -> int:
    """Block size of a case (1: TRPL+K itself, else the block form)."""
    return CASES[case][4] if len(CASES[case]) > 4 else 1


def path(case: str) -> str:
    return os.path.join(HERE, f"fullsize_{case}.txt")


def run(case: str) -> str:
    name, prec, tol = CASES[case][:3]
    P = make(name, "full", **case_kwargs(case))
    A = P.A.to_scipy()
    B = P.B.to_scipy() if P.B is not None else None
    X0 = start_block(P.A.n, P.k, P.seed)
    t0 = time.perf_counter()
    if prec == "jacobi":
        M = O.jacobi(A)
    else:
        M = O.factorized(OP.fsai(A))
    t1 = time.perf_counter()
    def progress(cycle, *args):
        if cycle % 100 == 0:
            print(f"  {case}: cycle {cycle}, {time.perf_counter() - t1:.0f} s", flush=True)

    s = case_block(case)
    if s == 1:
        r = O.solve(A, B, P.p, P.m, P.k, P.l, tol, X0, apply_M=M, trace=progress)
    else:
        r = OB.solve(A, B, P.p, P.m, P.k, P.l, s, tol, X0, apply_M=M, trace=progress)
    t2 = time.perf_counter()
    lines = [
        f"# full-size oracle reference: {case}",
        f"# workload {name} n={P.A.n} nnz={P.A.nnz} p={P.p} m={P.m} k={P.k} l={P.l} "
        f"seed={P.seed} precond={prec} tol={tol:g} norm=inf block={s}",
        "# written by tests/golden/make_fullsize_goldens.py (FP64 CPU oracle only)",
        f"# oracle setup {t1 - t0:.1f} s, solve {t2 - t1:.1f} s",
        f"cycles {r.cycles}",
        f"matvecs {r.matvecs}",
        f"bmatvecs {r.bvecs}",
        f"normA {r.normA!r}",
        f"converged {int(r.converged.all())}",
        "# i theta stored_residual true_residual",
    ]
    for i in range(P.p):
        lines.append(f"{i} {float(r.theta[i])!r} {float(r.res[i])!r} {float(r.true_res[i])!r}")
    out = path(case)
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    return out


def load(case: str) -> dict:
    """Parse a golden file: scalars plus theta / res / true_res arrays."""
    d = {"theta": [], "res": [], "true_res": []}
    with open(path(case)) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            a = ln.split()
            if a[0] in ("cycles", "matvecs", "bmatvecs", "converged"):
                d[a[0]] = int(a[1])
            elif a[0] == "normA":
                d["normA"] = float(a[1])
            else:
                d["theta"].append(float(a[1]))
                d["res"].append(float(a[2]))
                d["true_res"].append(float(a[3]))
    for k in ("theta", "res", "true_res"):
        d[k] = np.array(d[k])
    return d


if __name__ == "__main__":
    for c in (sys.argv[1:] or list(CASES)):
        print(c, "->", run(c), flush=True)
