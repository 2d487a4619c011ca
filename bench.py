#!/usr/bin/env python3
"""Time and matrix-vector products of the HIP TRPL+K on one MI355X.

Default workload: the largest one, 3-D 7-point anisotropic diffusion on 256^3
(axis weights 1, 1e-2, 1e-4 times the harmonic mean of a lognormal sigma = 1
field; n = 16,777,216, nnz = 117,047,296), p = 50 smallest pairs, m = 64,
k = 32, l = 1, hard locking (p > k), tol = 1e-8 * ||A||_inf, learned factor
G^T G + float32 SpMV with float64 orthogonalisation, Rayleigh-Ritz and
rotation.  A complete solve runs thousands of restart cycles (minutes), so one
step is a fixed number of full-size restart cycles (--cycles, default 10) of
TRPL+K from the seeded start block (drawn on the device, SplitMix64 seed 12),
every stage of the path included (SpMV, preconditioner apply, inner Krylov
loop with full reorthogonalisation, +K, Rayleigh-Ritz, rotation, locking);
--converged adds one complete solve of the timed form and of plain float64
Jacobi (time to solution, products, cycles).

The other workloads (--workload: 2-D Laplacian 64^2, 3-D Laplacian 128^3,
Q1 FEM pencil 97^3, power-law graph n = 1e6) are timed as complete solves
(one step = one solve to convergence).  Prints one JSON line; --summarize DIR
turns rocprofv3 output under DIR into the text summaries kept in profiles/.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


# workload name -> generator arguments, solver sizes, timed (precond, precision),
# restart cycles per step (0 = a step is a complete solve)
WORKLOADS = {
    "lap2d": dict(gen=dict(N=64), p=5, m=20, k=8, form=("jacobi", "fp64"), cycles=0,
                  desc="2-D 5-point Laplacian 64^2"),
    "lap3d": dict(gen=dict(N=128, vmax=0.05), p=10, m=40, k=20, form=("jacobi", "fp64"), cycles=0,
                  desc="3-D 7-point Laplacian 128^3 + V~U[0,0.05]"),
    "fem3d": dict(gen=dict(Ne=97, sigma=0.5), p=16, m=48, k=24, form=("fsai", "mixed"), cycles=0,
                  desc="Q1 FEM pencil 97^3 elements, lognormal sigma=0.5, consistent mass"),
    "powerlaw": dict(gen=dict(n=1_000_000), p=20, m=48, k=24, form=("learned", "fp64"), cycles=0,
                     desc="shifted Laplacian of a Chung-Lu power-law graph, n=1e6",
                     # gather-bound SpMV and well-separated wanted eigenvalues: a long
                     # float32 phase pays here (measured), unlike on the grids
                     mixed_switch=1e-5,
                     # hub rows: FSAI keeps the 63 largest lower entries and the diagonal
                     fsai_cap=64),
    "aniso3d": dict(gen=dict(N=256, sigma=1.0), p=50, m=64, k=32, form=("learned", "mixed"),
                    cycles=10,
                    desc="anisotropic 7-point diffusion 256^3 (axis weights 1, 1e-2, 1e-4 x "
                         "harmonic mean of a lognormal sigma=1 field)"),
}


KERNEL_NAMES = {"orth_dot": "k_orth<ORTH_DOT> (T column + first CGS coefficients)",
                "orth_upd_dot": "k_orth<ORTH_UPD_DOT> (w -= U h1; h2 = U^T w)",
                "orth_upd": "k_upd (w -= U h2; ||w||^2)",
                "orth_dc_dot": "k_orth<ORTH_DOT, 3 vectors> (U^T [u', A u', w]: delayed correction, "
                               "T column, coefficients of w)",
                "orth_dc_upd": "k_upd2 (u = (u' - U c) / gamma; w -= U h; ||w||^2)",
                "spmv": "k_spmv_stream / k_spmv_adapt_long (CSR; SpMV + append epilogue)",
                "prec": "k_spmv_stream / k_spmv_adapt_long (CSR; factor apply G, G^T)",
                "rot": "k_rotate (MFMA restart rotation)"}

def prof_class(name):
    """rocprofv3 kernel name -> the class bench.py times with events."""
    if "k_orth<" in name:
        targs = [t.strip() for t in name.split("k_orth<", 1)[1].split(">", 1)[0].split(",")]
        mode, nvec = targs[1], targs[2]
        if mode == "0":
            return "orth_dc_dot" if nvec == "3" else "orth_dot"
        return "orth_upd_dot"
    for key, cls in (("k_upd2", "orth_dc_upd"), ("k_upd<", "orth_upd"),
                     ("k_spmv_dia_lds", "spmv_staged"), ("k_spmm_dia", "spmm"),
                     ("k_spmv_dia<8, double", "spmv_f64"), ("k_spmv", "spmv_f32_or_factor"),
                     ("k_rotate", "rot"), ("k_block_dot_finish", "block_finish"),
                     ("k_block_dot", "block_dot"), ("k_dot_small", "block_dot_small"),
                     ("k_block_update", "block_update"), ("k_finish", "finish"),
                     ("k_syev", "syev"), ("copyBuffer", "copy")):
        if key in name:
            return cls
    return "other"


def counters_file(args, form):
    size = args.size or list(WORKLOADS[args.workload]["gen"].values())[0]
    return os.path.join(ROOT, "profiles", f"{args.workload}_{size}_{form[0]}_{form[1]}_hbm_counters.txt")


def measured_traffic(args, form, dom):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary of this exact configuration, or None when there is none."""
    path = counters_file(args, form)
    if not os.path.exists(path):
        return None
    cyc = None
    for line in open(path):
        parts = line.split()
        if len(parts) >= 2 and parts[0] == "STEP_CYCLES":
            cyc = int(parts[1])
        if len(parts) >= 4 and parts[0] == "TRAFFIC" and parts[1] == dom:
            if cyc is not None and cyc != args.cycles:
                return None
            return int(parts[2])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="aniso3d", choices=sorted(WORKLOADS))
    ap.add_argument("--size", type=int, default=0,
                    help="override the grid edge / node count (0 = the workload's own size)")
    ap.add_argument("--cycles", type=int, default=-1,
                    help="restart cycles per step (0 = a complete solve; default per workload)")
    ap.add_argument("--converged", action="store_true",
                    help="also run one complete solve of the timed form and of float64 Jacobi")
    ap.add_argument("--converged-forms", default="",
                    help="comma-separated forms (precond-precision) of the complete solves "
                         "(default: the timed form and jacobi-fp64)")
    ap.add_argument("--precond", default="", help="timed form's preconditioner (default per workload)")
    ap.add_argument("--precision", default="", choices=["", "fp64", "mixed"])
    ap.add_argument("--variants", type=int, default=1, help="also time the other forms once")
    ap.add_argument("--cpu", type=int, default=1, help="time the CPU oracle on the same input")
    ap.add_argument("--cpu-size", type=int, default=-1,
                    help="grid edge of the instance the CPU oracle is timed on when a step is a "
                         "number of cycles (default 96 for the 256^3 workload: one oracle cycle "
                         "at full size takes minutes; 0 = the full size)")
    ap.add_argument("--train-count", type=int, default=6, help="learned factor: training instances")
    ap.add_argument("--train-size", type=int, default=0, help="learned factor: training instance size")
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--profile-only", action="store_true", help="one profiled step (for rocprofv3 runs)")
    ap.add_argument("--method", default="trplk", choices=["trplk", "pl1", "pl1_practical"],
                    help="outer method of the timed solve: TRPL+K (Alg. 1) or PL+1 (Alg. 2, "
                         "the smallest pair; p = k = l = 1, the other methods as variants)")
    ap.add_argument("--sweep", default="", choices=["", "m", "l"],
                    help="ablation instead of the timed solve: vary the basis size m (paper "
                         "Fig. 2) or the number l of previous Ritz vectors (+K, Fig. 3; l = 0 is "
                         "thick-restart Lanczos) and print one JSON line with every setting")
    ap.add_argument("--sweep-values", default="", help="comma-separated values (default per sweep)")
    ap.add_argument("--max-cycles", type=int, default=5000, help="cap of a complete solve")
    ap.add_argument("--block", type=int, default=0,
                    help="block TRPL+K with this block size (2..16, float64) for the timed form")
    ap.add_argument("--progress", type=int, default=0,
                    help="complete solves print a line every this many cycles (0 = silent)")
    ap.add_argument("--protocol", action="store_true",
                    help="the power-law learned-factor protocol (24 train / 8 held-out graphs, "
                         "n = 1e6) instead of the timed run")
    ap.add_argument("--quasiopt", action="store_true",
                    help="the quasi-optimality experiment of Sec. 5.1 (Fig. 1) instead of the timed run")
    ap.add_argument("--summarize", default="",
                    help="summarize rocprofv3 output in this directory (kernel stats or counters) "
                         "instead of running anything on the GPU")
    args = ap.parse_args()
    if args.cycles < 0:
        args.cycles = WORKLOADS[args.workload]["cycles"]
    return args


def make_workload(name, size, seed=12):
    from workloads import make
    W = WORKLOADS[name]
    gen = dict(W["gen"])
    if size:
        key = {"lap2d": "N", "lap3d": "N", "fem3d": "Ne", "powerlaw": "n", "aniso3d": "N"}[name]
        gen[key] = size
    return make(name, "full", seed=seed, p=W["p"], m=W["m"], k=W["k"], l=1, tol=1e-8, **gen)


def train_factor(T, name, args, log):
    """Train the learned factor on smaller instances of the same generator
    (seeds 12, 13, ...), harvesting pairs from Jacobi solves on the GPU."""
    from workloads import start_block
    W = WORKLOADS[name]
    default_small = {"powerlaw": 200_000, "aniso3d": 48, "lap3d": 48, "fem3d": 33, "lap2d": 48}
    size = args.train_size or default_small[name]
    solvers, X0s = [], []
    for i in range(args.train_count):
        P = make_workload(name, size, seed=12 + i)
        # pairs (u, A u) from the stored basis of three solves of the instance:
        # to convergence (smooth, nearly converged vectors) and stopped after 1
        # and 3 cycles (rough early Krylov vectors); without the early ones the
        # rows the converged vectors barely touch (graph hubs) are unconstrained
        for cycles in (300, 1, 3):
            solvers.append(T.Solver(P.A, P.B, p=min(P.p, P.k), m=P.m, k=P.k, l=1, tol=1e-6,
                                    precond="jacobi", max_cycles=cycles))
            X0s.append(start_block(P.A.n, P.k, 12 + i))
    t0 = time.time()
    params, hist = T.train(solvers, X0s, epochs=args.epochs, lr=1e-3, S=min(64, W["m"]))
    for s in solvers:
        s.close()
    log(f"# trained on {args.train_count} x {name}(size {size}) in {time.time() - t0:.1f}s: "
        f"loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    return params, {"train_instances": args.train_count, "train_size": size,
                    "epochs": args.epochs, "loss_first": hist[0], "loss_last": hist[-1]}


def _gen_powerlaw(seed):
    P = make_workload("powerlaw", 0, seed=seed)
    return seed, P


def run_protocol(args, T, log):
    """The learned-preconditioner protocol of the power-law workload: 32
    seeded graphs at n = 1e6 (seeds 12..43), the factor's network trained on
    the first 24 (pairs harvested from GPU Jacobi solves of each), then each
    of the 8 held-out graphs solved to tol 1e-8 in every form; one JSON line
    with the per-form mean time, products and cycles."""
    import torch
    from concurrent.futures import ProcessPoolExecutor
    from workloads import start_block
    seeds = list(range(12, 44))
    t0 = time.time()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        probs = dict(ex.map(_gen_powerlaw, seeds))
    log(f"# generated {len(seeds)} power-law graphs (n = 1e6) in {time.time() - t0:.1f}s")
    train_seeds, test_seeds = seeds[:24], seeds[24:]
    solvers, X0s, dev = [], [], []
    for sd in train_seeds:
        P = probs[sd]
        Ad = T.DeviceCSR(P.A)
        dev.append(Ad)
        # two harvest solves per graph (to tol 1e-6 and stopped after 3
        # cycles) and 32 pairs each keep the 48 training contexts in memory
        for cycles in (300, 3):
            solvers.append(T.Solver(Ad, None, p=min(P.p, P.k), m=P.m, k=P.k, l=1, tol=1e-6,
                                    precond="jacobi", max_cycles=cycles))
            X0s.append(start_block(P.A.n, P.k, sd))
    t1 = time.time()
    params, hist = T.train(solvers, X0s, epochs=args.epochs, lr=1e-3, S=32)
    t2 = time.time()
    for s in solvers:
        s.close()
    del solvers, dev
    torch.cuda.synchronize()
    log(f"# trained on {len(train_seeds)} graphs in {t2 - t1:.1f}s: loss {hist[0]:.4f} -> {hist[-1]:.4f}")
    forms = [("jacobi", "fp64"), ("jacobi", "mixed"), ("fsai", "fp64"), ("fsai", "mixed"),
             ("learned", "fp64"), ("learned", "mixed")]
    rows = {f"{a}-{b}": [] for a, b in forms}
    for sd in test_seeds:
        P = probs[sd]
        Ad = T.DeviceCSR(P.A)
        Xd = torch.from_numpy(np.ascontiguousarray(start_block(P.A.n, P.k, sd).T)).cuda()
        ev0 = None
        for pc, pr in forms:
            S = T.Solver(Ad, None, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol,
                         precond="jacobi" if pc == "learned" else pc, precision=pr,
                         mixed_switch=WORKLOADS["powerlaw"].get("mixed_switch", 0.0),
                         fsai_cap=WORKLOADS["powerlaw"]["fsai_cap"])
            if pc == "learned":
                S.learned_factor(params)
            S.solve(Xd)
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = S.solve(Xd)
            torch.cuda.synchronize()
            b = time.perf_counter()
            ev, _, res, conv = S.eigpairs(vectors=False)
            S.close()
            if ev0 is None:
                ev0 = ev
            rows[f"{pc}-{pr}"].append({"seed": sd, "s": round(b - a, 4), "matvecs": st["matvecs"],
                                       "cycles": st["cycles"], "converged": bool(conv.all()),
                                       "max_resid_rel": float(np.max(res) / st["normA"]),
                                       "max_rel_eig_diff_vs_jacobi_fp64":
                                           float(np.max(np.abs(ev - ev0) / np.abs(ev0)))})
        log(f"# held-out graph seed {sd}: " + ", ".join(
            f"{k} {v[-1]['cycles']} cyc {v[-1]['s']:.3f}s" for k, v in rows.items()))
        del Ad, Xd
    summary = {k: {"mean_s": round(float(np.mean([r["s"] for r in v])), 4),
                   "mean_matvecs": float(np.mean([r["matvecs"] for r in v])),
                   "mean_cycles": float(np.mean([r["cycles"] for r in v])),
                   "all_converged": all(r["converged"] for r in v)} for k, v in rows.items()}
    base = summary["jacobi-fp64"]["mean_s"]
    for k in summary:
        summary[k]["speedup_vs_jacobi_fp64"] = round(base / summary[k]["mean_s"], 3)
    print(json.dumps({"protocol": "power-law learned factor: 24 train / 8 held-out at n = 1e6",
                      "train_seeds": train_seeds, "test_seeds": test_seeds,
                      "train": {"epochs": args.epochs, "pairs_per_solve": 32,
                                "harvest_solves_per_graph": 2,
                                "loss_first": hist[0], "loss_last": hist[-1],
                                "seconds": round(t2 - t1, 1)},
                      "summary": summary, "per_graph": rows}))


def run_quasiopt(args, T, log):
    """Sec. 5.1 / Fig. 1: the quasi-optimality ratio of Sec. 4.3 for TRPL+K
    with one inner step (PL+1 with the practical direction and a one-vector
    Krylov block, no preconditioner) on the GPU, against the unrestarted
    Krylov minimum (the oracle's Lanczos with full re-orthogonalisation), for
    start vectors at angles 0.5, 0.1, 0.02 to the lowest eigenvector (closed
    form), on the 2-D Laplacian 64^2 and the 3-D Laplacian 32^3."""
    from oracle import quasiopt as Q
    from workloads import lap2d, lap3d
    K = 30
    out = {}
    for name, A, shape in (("lap2d_64", lap2d(64), (64, 64)), ("lap3d_32", lap3d(32), (32, 32, 32))):
        As = A.to_scipy()
        N = shape[0]
        s1 = np.sin(np.arange(1, N + 1) * np.pi / (N + 1))
        v1 = s1
        for _ in shape[1:]:
            v1 = np.multiply.outer(v1, s1)
        v1 = v1.ravel()
        lam1 = len(shape) * 4 * np.sin(np.pi / (2 * (N + 1))) ** 2
        rows = {}
        for th in (0.5, 0.1, 0.02):
            x0 = Q.start_vector(v1, th, np.random.default_rng(3))
            S = T.Solver(A, None, p=1, m=3, k=1, l=1, tol=1e-300, method="pl1_practical",
                         precond="none", max_cycles=K)
            S.solve(x0[:, None])
            rho = S.history()
            S.close()
            r, _, _ = Q.quasi_optimality(As, x0, lam1, K, rho_x=rho)
            rows[str(th)] = [float(v) for v in r]
            log(f"# {name} theta0={th}: ratio at k=3,5,10,20,30: "
                + ", ".join(f"{r[k - 1]:.2e}" for k in (3, 5, 10, 20, 30)))
        out[name] = rows
    print(json.dumps({"experiment": "quasi-optimality ratio (Sec. 4.3), one inner step, no "
                                    "preconditioner; rho(x_k) from the GPU, rho(y_k*) from the "
                                    "unrestarted Krylov space K_{k+1}(A, x0)",
                      "iterations": K, "ratios": out}))


def run_sweep(args, T, P, Ad, Bd, Xd, precond, precision, log):
    """Ablation of the paper's Sec. 5 (Figs. 2 and 3) on a synthetic operator:
    one warm and one timed solve per setting, everything else fixed."""
    import torch
    if args.sweep == "m":
        vals = [int(v) for v in args.sweep_values.split(",")] if args.sweep_values else \
            [v for v in (P.k + 4, P.k + 8, P.k + 12, 2 * P.k, P.k + 28, 64) if P.k + 2 <= v <= 64]
    else:
        vals = [int(v) for v in args.sweep_values.split(",")] if args.sweep_values else \
            [0, 1, 2, 3, 4, 5]
    rows = []
    for v in vals:
        m, l = (v, 1) if args.sweep == "m" else (P.m, v)
        S = T.Solver(Ad, Bd, p=P.p, m=m, k=P.k, l=l, tol=P.tol, precond=precond,
                     precision=precision, max_cycles=args.max_cycles)
        S.solve(Xd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = S.solve(Xd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ev, _, res, conv = S.eigpairs(vectors=False)
        S.close()
        rows.append({"m": m, "l": l, "s": round(dt, 4), "cycles": st["cycles"],
                     "matvecs": st["matvecs"], "converged": bool(conv.all()),
                     "max_resid_rel": float(np.nanmax(res) / st["normA"])})
        log(f"# sweep {args.sweep}={v}: {st['cycles']} cycles, {st['matvecs']} MV, {dt:.3f} s")
    print(json.dumps({"sweep": args.sweep, "workload": args.workload, "n": P.A.n,
                      "p": P.p, "k": P.k, "precond": precond, "precision": precision,
                      "tol": P.tol, "results": rows}))


def kernel_profile(sp, st, log):
    """Per-class device time, launches and algorithmic bytes of one profiled
    step (HIP events recorded on the solver's stream around each launch)."""
    classes = {}
    for cls in ("spmv", "orth", "prec", "rot", "rr"):
        ms = sp[f"{cls}_ms"]
        if sp[f"{cls}_launches"]:
            nbytes = sp.get(f"{cls}_bytes", 0)
            classes[cls] = {"ms": ms, "launches": sp[f"{cls}_launches"], "bytes": nbytes,
                            "GBs": nbytes / (ms * 1e-3) / 1e9 if ms > 0 and nbytes else None}
    for q, name in enumerate(("orth_dot", "orth_upd_dot", "orth_upd", "orth_dc_dot", "orth_dc_upd")):
        if sp["pass_launches"][q]:
            ms, nbytes = sp["pass_ms"][q], sp["pass_bytes"][q]
            classes[name] = {"ms": ms, "launches": sp["pass_launches"][q], "bytes": nbytes,
                             "GBs": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None}
    return classes


def cpu_oracle(P, X0, cycles_per_step, gpu_cycles, log, n_full=None):
    """The FP64 NumPy/SciPy oracle on this host's cores.

    Per-cycle time: from the oracle's hook before the Rayleigh-Ritz of cycle 1
    to the same point of cycle 2, i.e. exactly one full restart cycle (its
    start-block phase excluded).  A step of C cycles is priced at C times
    that (times n_full / n when the oracle ran on a smaller instance of the
    same generator: at fixed p, m, k a cycle's work is linear in n); a
    complete-solve step at the oracle's own cycle count when the full-size
    reference run (tests/golden) records one, else the sample's per-cycle
    time times the GPU's cycles (labelled)."""
    from oracle import trplk as O
    A = P.A.to_scipy()
    B = None if P.B is None else P.B.to_scipy()
    cores = len(os.sched_getaffinity(0))
    stamps = []
    c0 = time.perf_counter()

    def hook(c, *a):
        stamps.append(time.perf_counter())
        log(f"# oracle: cycle {c} at its Rayleigh-Ritz, {stamps[-1] - c0:.1f} s")

    r = O.solve(A, B, P.p, P.m, P.k, P.l, P.tol, X0, apply_M=O.jacobi(A), max_cycles=2, trace=hook)
    c1 = time.perf_counter()
    per_cycle = stamps[1] - stamps[0] if len(stamps) >= 2 else (c1 - c0)
    log(f"# oracle: start + {r.cycles} cycles in {c1 - c0:.1f} s, one cycle {per_cycle:.2f} s")
    base = {"unit": "s", "cores": cores, "kind": "oracle", "per_cycle_s": round(per_cycle, 3),
            "threads_note": f"NumPy BLAS threads = {os.environ.get('OPENBLAS_NUM_THREADS', cores)}; "
                            "SciPy SpMV single-threaded"}
    if cycles_per_step:
        n = P.A.n
        scale = (n_full or n) / n
        where = ("the same full-size input and start block" if scale == 1 else
                 f"the n = {n:,} instance of the same generator (same p, m, k, seed, start-block "
                 f"definition)")
        return dict(base, value=round(per_cycle * scale * cycles_per_step, 3),
                    sample=f"FP64 oracle (Jacobi) on {where}: one complete restart cycle (cycle "
                           f"1 -> 2, hook to hook) took {per_cycle:.2f} s of {c1 - c0:.1f} s (start "
                           f"block + 2 cycles); value = that"
                           + (f" x {scale:.2f} (n_full / n: a cycle's work is linear in n at fixed "
                              f"p, m, k; extrapolated in n)" if scale != 1 else "")
                           + f" x {cycles_per_step} cycles, the GPU step's unit",
                    n_sample=n)
    gold = None
    try:
        sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
        import make_fullsize_goldens as G
        case = f"{P.name}_jacobi_1e-08"
        if case in G.CASES and os.path.exists(G.path(case)):
            gold = G.load(case)["cycles"]
    except Exception:
        gold = None
    if gold:
        return dict(base, value=round(per_cycle * gold, 2),
                    sample=f"one complete restart cycle of the FP64 oracle (Jacobi) on the same input "
                           f"took {per_cycle:.2f} s; value = that x the {gold} cycles the oracle "
                           f"itself needs to converge (its full-size reference run, tests/golden)")
    return dict(base, value=round(per_cycle * gpu_cycles, 2),
                sample=f"one complete restart cycle of the FP64 oracle took {per_cycle:.2f} s; value "
                       f"= that x the {gpu_cycles} cycles of the timed GPU form (extrapolated)")


def summarize(spec):
    """Text summary of rocprofv3 CSV output: kernel statistics
    (*kernel_stats.csv) and per-class HBM counters (*counter_collection.csv)
    under the comma-separated directories in spec.  With FETCH_SIZE and
    WRITE_SIZE both present, each class's HBM bytes per launch are printed as
    TRAFFIC lines, the counters scaled by what they read for the 256 MiB
    calibration copies bench.py --profile-only runs (copyBuffer dispatches)."""
    import csv
    import glob
    out = []
    agg = {}
    for d in spec.split(","):
        ks = sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True))
        cc = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
        if ks:
            rows = list(csv.DictReader(open(ks[0])))
            tot = sum(float(r["TotalDurationNs"]) for r in rows)
            out.append(f"# kernel statistics: {os.path.basename(ks[0])}")
            out.append(f"# {'rocprofv3 kernel':<92} {'calls':>6} {'total ms':>9} {'avg us':>9} {'%':>6}")
            for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
                out.append(f"{r['Name'][:92]:<92} {int(r['Calls']):>6} "
                           f"{float(r['TotalDurationNs']) / 1e6:>9.2f} "
                           f"{float(r['AverageNs']) / 1e3:>9.2f} "
                           f"{100 * float(r['TotalDurationNs']) / tot:>6.2f}")
        for f in cc:
            rows = list(csv.DictReader(open(f)))
            # the calibration copies are the last three copy dispatches (bench.py
            # --profile-only runs them after the solve); other copies are the
            # library's and torch's own
            copies = sorted((int(r["Dispatch_Id"]) for r in rows if "copyBuffer" in r["Kernel_Name"]))
            calib = set(copies[-3:])
            for r in rows:
                cls = prof_class(r["Kernel_Name"])
                if cls == "copy" and int(r["Dispatch_Id"]) not in calib:
                    cls = "copy_other"
                a = agg.setdefault((cls, r["Counter_Name"]), [0, 0.0])
                a[0] += 1
                a[1] += float(r["Counter_Value"])
    if agg:
        out.append(f"# counters: {'class':<14} {'counter':<12} {'dispatches':>10} {'mean KiB':>14}")
        for (cls, cn), (cnt, tot) in sorted(agg.items()):
            out.append(f"{cls:<14} {cn:<12} {cnt:>10} {tot / cnt:>14.1f}")
        f_copy = agg.get(("copy", "FETCH_SIZE"))
        w_copy = agg.get(("copy", "WRITE_SIZE"))
        if f_copy and w_copy:
            want = (256 << 20) / 1024.0
            rs = want / (f_copy[1] / f_copy[0])
            ws = want / (w_copy[1] / w_copy[0])
            out.append(f"calibration: 256 MiB copies read {f_copy[1] / f_copy[0]:.1f} KiB (scale {rs:.5f}), "
                       f"write {w_copy[1] / w_copy[0]:.1f} KiB (scale {ws:.5f})")
            for cls in sorted({c for c, _ in agg}):
                fe, wr = agg.get((cls, "FETCH_SIZE")), agg.get((cls, "WRITE_SIZE"))
                if fe and wr and cls != "copy":
                    b = (fe[1] / fe[0] * rs + wr[1] / wr[0] * ws) * 1024.0
                    out.append(f"TRAFFIC {cls} {int(b)} bytes_per_launch")
    print("\n".join(out))


def main():
    args = parse()
    if args.summarize:
        return summarize(args.summarize)
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on exactly one GPU; multi-GPU runs are not "
                                   "part of it (--gpus must be 1)"}))
        sys.exit(2)
    import torch

    import paper_1711_10128_amd as T
    from workloads import splitmix64_block, start_block

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.protocol:
        return run_protocol(args, T, log)
    if args.quasiopt:
        return run_quasiopt(args, T, log)
    W = WORKLOADS[args.workload]
    precond = args.precond or W["form"][0]
    precision = args.precision or W["form"][1]
    C = args.cycles
    t0 = time.time()
    P = make_workload(args.workload, args.size)
    if args.method != "trplk":
        import dataclasses
        P = dataclasses.replace(P, p=1, k=1, l=1)
    log(f"# workload {args.workload} n={P.A.n} nnz={P.A.nnz} generated in {time.time() - t0:.1f}s")
    Ad = T.DeviceCSR(P.A)
    Bd = T.DeviceCSR(P.B) if P.B is not None else None
    # step-of-C-cycles workloads start from the block the library draws on
    # the device (x0 = NULL, seed 12); complete solves from the host-seeded block
    if C:
        Xd = None
    else:
        X0 = start_block(P.A.n, P.k, P.seed)
        Xd = torch.from_numpy(np.ascontiguousarray(X0.T)).cuda()
    torch.cuda.synchronize()

    if args.sweep:
        return run_sweep(args, T, P, Ad, Bd, Xd, "fsai" if precond == "learned" else precond,
                         precision, log)

    learned = None
    learn_info = None
    cf = args.converged_forms if (args.converged and C) else ""
    need_learned = precond == "learned" or "learned" in cf or (
        args.variants and not args.profile_only and args.workload in ("powerlaw", "aniso3d", "lap3d"))
    if need_learned and args.profile_only:
        # the kernels and their cost do not depend on the factor's values:
        # a profiled step uses the untrained (Jacobi-equivalent) network, so
        # the profile holds no training solves
        learned, learn_info = T.init_params(), {"untrained": True}
    elif need_learned:
        learned, learn_info = train_factor(T, args.workload, args, log)

    def make_solver(pc, pr, profile=False, method=None, cycles=None):
        base = "jacobi" if pc == "learned" else pc
        cap = (C or args.max_cycles) if cycles is None else cycles
        blk = args.block if (pc, pr) == (precond, precision) and not method else 0
        s = T.Solver(Ad, Bd, p=P.p, m=P.m, k=P.k, l=P.l, tol=P.tol, precond=base,
                     precision=pr, profile=profile, max_cycles=cap, seed=P.seed,
                     method=method or args.method, mixed_switch=W.get("mixed_switch", 0.0),
                     progress=args.progress if cap > 100 else 0, block=blk,
                     fsai_cap=W.get("fsai_cap", 0))
        if pc == "learned":
            s.learned_factor(learned)
        return s

    # ---- timed region: K steps of the selected form ----
    S = make_solver(precond, precision)
    if args.profile_only:
        st = S.solve(Xd)
        torch.cuda.synchronize()
        # calibration for the HBM counters: plain copies of a known size
        nb = 256 << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_only": True, "cycles": st["cycles"], "ms": st["solve_ms"],
                          "calibration_copy_bytes": nb}))
        return
    for _ in range(args.warmup):
        w = S.solve(Xd)
        log(f"# warmup step: {w['cycles']} cycles, {w['solve_ms']:.1f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        stats.append(S.solve(Xd))
        log(f"# step {i}: {stats[-1]['cycles']} cycles, {stats[-1]['solve_ms']:.1f} ms")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    st = stats[-1]
    ev, X, res, conv = S.eigpairs(vectors=False)
    normA = st["normA"]
    nret = int(np.sum(np.isfinite(ev)))
    converged = bool(conv.all() and np.all(res <= P.tol * normA * 1.001))
    if st["status"] == 1:
        log(f"# step ended after {st['cycles']} cycles: {int(conv.sum())} of {P.p} pairs converged")
    checks = {}
    if not C and args.workload == "lap3d":
        N = P.meta["N"]
        i = np.arange(1, N + 1)
        s1 = 4 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
        lam0 = np.sort((s1[:, None, None] + s1[None, :, None] + s1[None, None, :]).ravel())[:P.p]
        checks["eigs_within_weyl_bounds"] = bool(np.all(ev >= lam0 - 1e-12) and np.all(ev <= lam0 + 0.05 + 1e-12))
    if not C and args.workload == "lap2d":
        N = P.meta["N"]
        i = np.arange(1, N + 1)
        s1 = 4 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
        lam = np.sort((s1[:, None] + s1[None, :]).ravel())[:P.p]
        checks["max_rel_err_vs_closed_form"] = float(np.max(np.abs(ev - lam) / lam))
    if not C and args.workload == "powerlaw":
        checks["lambda1_minus_shift_rel"] = float(abs(ev[0] - 0.01) / 0.01)
    if not C and args.method == "trplk":
        # against the FP64 oracle's full-size reference run (tests/golden), when one exists
        try:
            sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
            import make_fullsize_goldens as G
            case = f"{args.workload}_{precond}_1e-08"
            if not args.size and case in G.CASES and os.path.exists(G.path(case)):
                g = G.load(case)
                checks["max_rel_eig_err_vs_oracle"] = float(np.max(np.abs(ev - g["theta"]) /
                                                                   np.abs(g["theta"])))
                checks["oracle_cycles"] = g["cycles"]
        except Exception as e:  # a reference file that does not parse is reported, not fatal
            checks["oracle_reference_error"] = str(e)
    S.close()

    # ---- kernel profile of one step (HIP events around each launch) ----
    Sp = make_solver(precond, precision, profile=True)
    sp = Sp.solve(Xd)
    Sp.close()
    log(f"# profiled step: {sp['solve_ms']:.1f} ms")
    classes = kernel_profile(sp, st, log)
    kernels = [c for c in classes if c != "orth" and classes[c]["bytes"]]
    dom = max(kernels, key=lambda c: classes[c]["ms"])
    d = classes[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    avg_ms = d["ms"] / d["launches"]
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    names = dict(KERNEL_NAMES)
    if st["a_ndiag"]:
        names["spmv"] = f"k_spmv_dia ({st['a_ndiag']} diagonals; SpMV + append epilogue)"
    if st["g_ndiag"]:
        names["prec"] = f"k_spmv_dia ({st['g_ndiag']} diagonals; factor apply G, G^T)"
    roofline = {"bound": "hbm", "kernel": names.get(dom, dom), "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args, (precond, precision), dom),
                "bytes_per_launch": int(per_launch_bytes), "avg_launch_us": round(avg_ms * 1e3, 2)}
    spmv = classes.get("spmv")
    spmv_roof = None
    if spmv:
        g = spmv["GBs"]
        spmv_roof = {"achieved": round(g, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(g / HBM_PEAK_GBS, 4), "launches": spmv["launches"],
                     "avg_launch_us": round(spmv["ms"] / spmv["launches"] * 1e3, 2)}

    # ---- other forms (one warm step each, outside the timed region) ----
    def one(pc, pr, mm=None, cycles=None, warm=True):
        V = make_solver(pc, pr, method=mm, cycles=cycles)
        if warm:
            V.solve(Xd)
        torch.cuda.synchronize()
        a = time.perf_counter()
        sv = V.solve(Xd)
        torch.cuda.synchronize()
        b = time.perf_counter()
        evv, _, rv, cv = V.eigpairs(vectors=False)
        V.close()
        ok = np.isfinite(evv) & np.isfinite(ev) & cv.astype(bool) & conv.astype(bool)
        return {"s": round(b - a, 4), "matvecs": sv["matvecs"], "cycles": sv["cycles"],
                "fp32_cycles": sv["fp32_cycles"], "converged_pairs": int(cv.sum()),
                "setup_ms": round(sv["setup_ms"], 2), "converged": bool(cv.all()),
                "max_resid_rel": float(np.nanmax(rv) / normA),
                "max_rel_eig_diff_vs_timed": (float(np.max(np.abs(evv[ok] - ev[ok]) / np.abs(ev[ok])))
                                              if ok.any() else None)}

    variants = {}
    if args.variants:
        forms = [("jacobi", "fp64", None), ("fsai", "fp64", None), ("fsai", "mixed", None),
                 ("jacobi", "mixed", None)]
        if learned is not None:
            forms += [("learned", "fp64", None), ("learned", "mixed", None)]
        if args.method != "trplk":
            # PL+1: the other outer methods with the timed form's preconditioner
            forms = [(precond, precision, mm) for mm in ("trplk", "pl1", "pl1_practical")
                     if mm != args.method]
        for pc, pr, mm in forms:
            if mm is None and (pc, pr) == (precond, precision):
                continue
            label = f"{pc}-{pr}" if mm is None else f"{mm}-{pc}-{pr}"
            variants[label] = one(pc, pr, mm)
            log(f"# variant {label}: {variants[label]['cycles']} cycles, {variants[label]['s']:.3f} s")

    # ---- complete solves (time to solution), outside the timed region ----
    solutions = None
    if args.converged and C:
        solutions = {}
        cforms = ([tuple(f.split("-")) for f in args.converged_forms.split(",")]
                  if args.converged_forms else [(precond, precision), ("jacobi", "fp64")])
        for pc, pr in cforms:
            label = f"{pc}-{pr}"
            log(f"# complete solve {label} (max {args.max_cycles} cycles)")
            solutions[label] = one(pc, pr, cycles=args.max_cycles, warm=False)
            log(f"# complete solve {label}: {solutions[label]['cycles']} cycles, "
                f"{solutions[label]['matvecs']} MV, {solutions[label]['s']:.1f} s, "
                f"{solutions[label]['converged_pairs']}/{P.p} pairs")

    # ---- CPU oracle on the same input ----
    cpu = None
    if args.cpu and args.method == "trplk":
        Pc = P
        if C:
            csize = args.cpu_size if args.cpu_size >= 0 else (96 if args.workload == "aniso3d" else 0)
            if csize and csize < (args.size or list(W["gen"].values())[0]):
                Pc = make_workload(args.workload, csize)
        X0h = splitmix64_block(Pc.A.n, Pc.k, Pc.seed) if C else start_block(Pc.A.n, Pc.k, Pc.seed)
        cpu = cpu_oracle(Pc, X0h, C, st["cycles"], log, n_full=P.A.n)
        del X0h

    if C:
        step_desc = (f"one step = {C} restart cycles of TRPL+K from the seeded start block "
                     f"(drawn on the device, SplitMix64 seed {P.seed})")
    else:
        step_desc = "one step = one complete solve from the seeded start block"
    out = {
        "metric": "time & matvecs to p eigpairs at resid 1e-8; SpMV HBM GB/s vs peak",
        "value": round(ms_per_step / 1e3, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{W['desc']}, p={P.p} m={P.m} k={P.k} l={P.l} tol=1e-8*||A||_inf, "
                               f"{'hard' if P.p > P.k else 'soft'} locking, {precond} {precision}"
                               + ("" if args.method == "trplk" else f", {args.method}")
                               + (f", block size {args.block}" if args.block > 1 else "")
                               + f"; {step_desc}",
                   "name": args.workload, "n": P.A.n, "nnz": P.A.nnz,
                   "generalized": P.B is not None, "cycles_per_step": C or None},
        "converged": converged,
        "capped": st["status"] == 1,
        "ms_per_cycle": round(st["solve_ms"] / max(1, st["cycles"]), 3),
        "matvecs": st["matvecs"],
        "bmatvecs": st["bmatvecs"],
        "cycles": st["cycles"],
        "pairs_returned": nret,
        "converged_pairs": int(conv.sum()),
        "device_solve_ms": round(st["solve_ms"], 3),
        "setup_ms": round(st["setup_ms"], 3),
        "max_resid_rel": float(np.nanmax(res) / normA) if nret else None,
        "checks": checks,
        "spmv_storage": (f"diagonals ({st['a_ndiag']})" if st["a_ndiag"] else "csr")
                        + (f", B: diagonals ({st['b_ndiag']})" if st["b_ndiag"] else "")
                        + (f", G: diagonals ({st['g_ndiag']})" if st["g_ndiag"] else ""),
        "roofline": roofline,
        "spmv_roofline": spmv_roof,
        "kernel_classes": {k: {kk: (round(v, 3) if isinstance(v, float) else v)
                               for kk, v in c.items()} for k, c in classes.items()},
        "variants": variants,
        "time_to_solution": solutions,
        "learned": learn_info,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
