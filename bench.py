"""Benchmark: dual-system solves/sec of recycling BiCG on one MI355X.

Workload (default): 3D convection-diffusion, 7-point upwind, 64^3 grid
(n = 262144), a sequence of 10 dual systems with beta_j = (20,10,5)(1+0.02j),
b, b~ ~ N(0,1) drawn once, k = 20 recycle vectors, cycle length s = 40,
relative tolerance 1e-8, FP64.  All matrices and right-hand sides are resident
in device memory before the timed region.  One step = solving the whole
sequence from an empty recycle space (recycle-space updates included).

Prints one JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
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

METRIC = "dual-system solves/sec + HBM GB/s per RBiCG iter; p50/p99 latency served"
HBM_PEAK_GBS = 8000.0
# HBM bytes per completed k_it1 launch on this workload, from the FETCH_SIZE
# and WRITE_SIZE counter runs (each scaled by what the counter reads for a
# 512 MiB device copy), valid only for the kernel source and the matrix
# layout code (runtime.hip) they were taken on
TRAFFIC_K_IT1 = {"sources_sha256_16": "3ab73373b82b6602", "bytes_per_launch": 81.50e6}
# the same for the FP32 k_it1 of the 128^3 mixed-precision leg, and the mean
# kernel-trace duration of the 64^3 k_it1 (rocprofv3 --kernel-trace, the
# sequence's launches), each from the committed profiles of these sources
TRAFFIC_K_IT1_MIXED = {"sources_sha256_16": "3ab73373b82b6602", "bytes_per_launch": 295.9e6}
TRACE_K_IT1 = {"sources_sha256_16": "3ab73373b82b6602", "avg_us": 19.17}
TRAFFIC_SOURCES = ("kernels.hip", "runtime.hip")


def sources_digest():
    """sha256 prefix of the sources the k_it1 traffic depends on."""
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1010_0762_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _if_current(rec, field):
    """rec[field] when rec was measured on the current sources, else None."""
    try:
        digest = sources_digest()
    except OSError:
        return None
    return rec[field] if digest == rec["sources_sha256_16"] else None


def traffic_k_it1():
    """Counter-measured HBM bytes per k_it1 launch, or None once the sources
    differ from the ones the counters were taken on."""
    return _if_current(TRAFFIC_K_IT1, "bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=64, help="grid edge")
    ap.add_argument("--nsys", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--profile-timed", type=int, default=16,
                    help="p > 0: time the iteration kernels of every p-th chunk of iterations "
                         "with HIP events inside the timed region (0: off)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB before timing (counter calibration)")
    ap.add_argument("--serving", action="store_true",
                    help="run the serving trace (continuous batching, p50/p99 latency) instead")
    ap.add_argument("--serving-n", type=int, default=40, help="requests in the serving trace")
    ap.add_argument("--serving-lam", type=float, default=50.0, help="arrival rate (req/s)")
    ap.add_argument("--serving-slots", type=int, default=8, help="concurrent request slots")
    ap.add_argument("--serving-window", type=float, default=20.0,
                    help="microseconds a batched launch waits for the other iterating requests")
    ap.add_argument("--leg", default=None,
                    choices=("mixed", "shifted", "irka", "serving", "ilut"),
                    help="run only this leg and print its JSON (for profiling one workload)")
    ap.add_argument("--mixed-nsys", type=int, default=8, help="systems of the mixed-precision leg")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg (p50/p99 latency of the config-5 trace)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32-inner / FP64-outer leg (128^3, 8 systems)")
    ap.add_argument("--no-irka", action="store_true", help="skip the IRKA leg")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the split-preconditioned legs (red-black ILU(0), ILUT)")
    ap.add_argument("--no-copy-ref", action="store_true",
                    help="skip the device-copy bandwidth reference")
    ap.add_argument("--no-shifted", action="store_true",
                    help="skip the batched shifted-pair leg (48^3, 8 shifts, 6 sweeps)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape autotuner leg")
    ap.add_argument("--no-k20", action="store_true",
                    help="skip the extra kernel timing with an injected 20-vector recycle space")
    ap.add_argument("--pencil-setup", type=int, default=0, choices=(0, 1),
                    help="cycle-end pencil of the headline: 0 device Grams, 1 Sec. 4.4 recurrences")
    ap.add_argument("--no-other-setup", action="store_true",
                    help="skip the headline sequence with the other pencil set-up")
    return ap.parse_args()


def cpu_baseline(seq, nsys=3):
    """The oracle as it stands, on a bounded sample, in two modes: all cores
    (BLAS threads as the process has them; the sparse products are
    single-threaded either way) on the first ``nsys`` dual systems of the
    sequence, recycle spaces carried from one to the next as in the timed
    GPU step; and one thread on the first system alone (from an empty
    recycle space, with its cycle updates)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = 1
    t0 = time.perf_counter()
    res, _ = oracle.rbicg_sequence(seq.mats[:nsys], seq.b[:nsys], seq.bt[:nsys], k=seq.k,
                                   s=seq.s, tol=seq.tol, maxit=20000)
    dt = time.perf_counter() - t0
    out = {"value": nsys / dt, "unit": "dual-system solves/s", "cores": int(threads),
           "kind": "oracle",
           "sample": (f"systems 0-{nsys - 1} of the sequence, recycle spaces carried "
                      f"({[r.iters for r in res]} iterations) in {dt:.1f} s; sparse products "
                      f"single-threaded, dense vector/basis work on {threads} BLAS threads")}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r0 = oracle.rbicg(seq.mats[0], seq.b[0], seq.bt[0], tol=seq.tol, maxit=20000,
                              s=seq.s, k=seq.k)
            dt1 = time.perf_counter() - t0
        out["single_thread"] = {
            "value": 1.0 / dt1, "unit": "dual-system solves/s", "cores": 1,
            "sample": (f"system 0 of the sequence ({r0.iters} iterations, {r0.cycles} recycle "
                       f"updates) in {dt1:.1f} s, every library on one thread")}
    return out


def bicg_leg(args, seq, mats, b, bt):
    """Context for the headline: the same 10-system sequence solved by plain
    BiCG (k = 0, Algorithm 1) on the same kernels, timed after one untimed
    pass.  On this operator recycling does not lower the iteration count
    (the retained spaces are small), so this shows what the cycle-end work
    costs."""
    import torch
    from paper_1010_0762_amd.solver import Solver
    S = Solver(mats[0], k=0, s=seq.s, update=False, chunk=args.chunk)
    x = torch.zeros_like(b)
    xt = torch.zeros_like(bt)

    def one_pass():
        its = []
        for j in range(len(mats)):
            S.update_recycle(mats[j])
            x.zero_()
            xt.zero_()
            _, _, st = S.solve(b, bt, x, xt, tol=seq.tol)
            its.append(st["iters"])
        return its

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"solves_per_s": round(len(mats) / dt, 3), "ms_per_sequence": round(dt * 1e3, 2),
            "iters_per_system": its, "us_per_iter": round(dt / sum(its) * 1e6, 2)}


def pencil_setup_leg(args, seq, mats, b, bt, setup):
    """The headline's sequence (same workload, same kernels) with the other
    cycle-end pencil set-up: 0 device Grams of the cycle's vectors, 1 the
    recurrences of Sec. 4.4 (one (s+2) x k Gram per cycle); one pass timed
    after an untimed one."""
    import torch
    from paper_1010_0762_amd.solver import Solver
    S = Solver(mats[0], k=seq.k, s=seq.s, chunk=args.chunk, pencil_setup=setup)
    x = torch.zeros_like(b)
    xt = torch.zeros_like(bt)

    def one_pass():
        S.set_recycle(None, None)
        sts = []
        for j in range(len(mats)):
            S.update_recycle(mats[j])
            x.zero_()
            xt.zero_()
            _, _, st = S.solve(b, bt, x, xt, tol=seq.tol)
            sts.append(st)
        return sts

    one_pass()
    torch.cuda.synchronize()
    S.profile(reset=True)
    t0 = time.perf_counter()
    sts = one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = S.profile(reset=True)
    S.close()
    its = [st["iters"] for st in sts]
    nup = max(prof["cycle_updates"], 1)
    return {"pencil_setup": setup, "solves_per_s": round(len(mats) / dt, 3),
            "ms_per_sequence": round(dt * 1e3, 2), "iters_per_system": its,
            "k_used_per_system": [st["k_used"] for st in sts],
            "us_per_iter": round(dt / sum(its) * 1e6, 2),
            "max_true_relres": max(max(st["relres"], st["relres_dual"]) for st in sts),
            "all_converged": all(st["status"] == 0 for st in sts),
            "cycle_latency_ms_avg": round(prof["cycle_latency_ms"] / nup, 3),
            "cycle_eig_ms_avg": round(prof["cycle_eig_ms"] / nup, 3)}


def precond_leg(args, seq, mats, b, bt):
    """The benchmark's 10-system 64^3 sequence split-preconditioned as in
    Sec. 6, with ILU(0) in red-black ordering: RBiCG (k = 20, s = 40) on the
    black blocks of the preconditioned operators, recycling between them,
    tolerance 1e-8 on the preconditioned residual.  The host set-up
    (colouring, pattern of the Schur block, maps) runs once for the
    sequence's pattern and is timed apart, and the matrices' values are
    resident on the device beforehand (as the other legs preload their
    matrices); inside the timed pass every system takes its preconditioner
    by a device refresh from its values (pivots, Schur block), then the right-hand-side
    transform, the solve and the solution transform.  One pass is timed after
    an untimed one; true residuals of the original pairs are checked after
    it."""
    import torch
    import scipy.sparse as sp
    from paper_1010_0762_amd.solver import RBILU, Solver
    t0 = time.perf_counter()
    P = RBILU(seq.mats[0])
    setup_ms = (time.perf_counter() - t0) * 1e3
    S = Solver(P.black, k=seq.k, s=seq.s, chunk=args.chunk)
    # the matrices' values resident on the device beforehand, as the other
    # legs preload their matrices
    vals = [torch.as_tensor(A.vals, device="cuda") for A in seq.mats]
    sols = []

    def one_pass():
        its = []
        sols.clear()
        S.set_recycle(None, None)
        for j, A in enumerate(seq.mats):
            S.stream.synchronize()
            P.refresh_values(vals[j], stream=S.stream)
            S.update_recycle(P.black)
            bB, cB = P.rhs(b, bt, stream=S.stream)
            yB, ytB, st = S.solve(bB, cB, tol=seq.tol)
            sols.append(P.solution(b, bt, yB, ytB, stream=S.stream))
            its.append(st["iters"])
        return its

    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    bh, bth = b.cpu().numpy(), bt.cpu().numpy()
    rel = []
    for A, (x, xt) in zip(seq.mats, sols):
        As = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))
        rel.append(max(np.linalg.norm(bh - As @ x.cpu().numpy()) / np.linalg.norm(bh),
                       np.linalg.norm(bth - As.T @ xt.cpu().numpy()) / np.linalg.norm(bth)))
    nb = P.nb
    S.close()
    P.close()
    return {"workload": "convdiff3d_64^3_seq10_k20_s40_tol1e-8_split_rb_ilu0",
            "black_unknowns": nb,
            "solves_per_s": round(len(mats) / dt, 3), "ms_per_sequence": round(dt * 1e3, 2),
            "host_setup_ms_once": round(setup_ms, 1), "iters_per_system": its,
            "us_per_iter": round(dt / max(1, sum(its)) * 1e6, 2),
            "max_true_relres": float(max(rel))}


def ilut_leg(args, seq, mats, b, bt):
    """Split ILUT preconditioning (Sec. 6) with device level-scheduled
    triangular solves, in two settings: (a) the 2D experiment's shape of
    Sec. 6.1 -- convection-diffusion with central differences on the
    h = 1/64 grid (n = 3969; a checkerboard diffusion coefficient with jumps
    of 1e3 stands in for the paper's, which only a figure gives), ILUT(0.05),
    the same dual pair solved four times, k = 10, s = 40, tol 1e-8 -- with
    recycling and with k = 0 (plain BiCG); (a') the same with the rows of
    the operator permuted (most diagonal entries zero) and ILUTP(0.05,
    permtol 1), the pivoting variant Sec. 6.2 uses; (b) the
    benchmark's 10-system 64^3 sequence, ILUT(0.05) per system, k = 20 and
    k = 0.  The host factorizations run before the timed passes (timed
    apart); a timed pass covers, per system, the right-hand-side transform,
    the recycle-space move to the new preconditioned operator, the solve and
    the solution transform.  One pass is timed after an untimed one; true
    residuals of the original pairs are checked after it."""
    import torch
    import scipy.sparse as sp
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import ILUT, DeviceMatrix, Solver

    def run(hmats, dmats, bs, bts, k, s, tol, tau, permtol=0.0):
        # one factorization per distinct matrix (host), timed apart
        t0 = time.perf_counter()
        cache = {}
        for A in hmats:
            if id(A) not in cache:
                cache[id(A)] = ILUT(A, tau, permtol=permtol)
        Ps = [cache[id(A)] for A in hmats]
        setup_ms = (time.perf_counter() - t0) * 1e3
        S = Solver(dmats[0], k=k, s=s, chunk=args.chunk)
        sols = []

        def one_pass():
            its = []
            sols.clear()
            S.set_recycle(None, None)
            for j in range(len(hmats)):
                S.stream.synchronize()
                S.attach_ilu(Ps[j])
                # the handle on system j's matrix, the carried space against
                # the new preconditioned operator
                S.update_recycle(None if S.matrix is dmats[j] else dmats[j])
                S._order()
                bh, ch = Ps[j].rhs(bs[j], bts[j], stream=S.stream)
                y, yt, st = S.solve(bh, ch, tol=tol)
                sols.append(Ps[j].solution(y, yt, stream=S.stream))
                its.append(st["iters"])
            return its

        one_pass()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = one_pass()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rel = []
        for A, (x, xt), bb, bbt in zip(hmats, sols, bs, bts):
            As = (sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n, A.n))
                  if hasattr(A, "rowptr") else A)
            bh_, bth_ = bb.cpu().numpy(), bbt.cpu().numpy()
            rel.append(max(np.linalg.norm(bh_ - As @ x.cpu().numpy()) / np.linalg.norm(bh_),
                           np.linalg.norm(bth_ - As.T @ xt.cpu().numpy()) / np.linalg.norm(bth_)))
        info = Ps[0].info()
        S.close()
        for P in cache.values():
            P.close()
        print(f"ilut leg: k={k} n={hmats[0].shape[0] if hasattr(hmats[0], 'shape') else hmats[0].n} "
              f"systems={len(hmats)} iters={its} "
              f"{dt * 1e3:.1f} ms", file=sys.stderr, flush=True)
        return {"solves_per_s": round(len(hmats) / dt, 3), "ms_per_sequence": round(dt * 1e3, 2),
                "host_factorization_ms": round(setup_ms, 1), "iters_per_system": its,
                "us_per_iter": round(dt / max(1, sum(its)) * 1e6, 2),
                "max_true_relres": float(max(rel)),
                "factor": {kk: info[kk] for kk in ("nnz_L", "nnz_U", "levels_L", "levels_U", "moved")}}

    out = {}
    # (a) Sec. 6.1 shape: one pair solved four times on the h = 1/64 grid,
    # central differences, a jumping diffusion coefficient
    A2 = wl.jump_convdiff2d()
    rng = np.random.default_rng(wl.BASE_SEED + 61)
    b2 = torch.as_tensor(rng.standard_normal(A2.n), device="cuda")
    bt2 = torch.as_tensor(rng.standard_normal(A2.n), device="cuda")
    D2 = DeviceMatrix(A2)
    for k in (10, 0):
        out[f"jump_convdiff2d_63^2_same_pair_x4_ilut0.05_k{k}_s40"] = run(
            [A2] * 4, [D2] * 4, [b2] * 4, [bt2] * 4, k, 40, 1e-8, 0.05)
    D2.close()
    # (a') ILUTP (Sec. 6.2 preconditions with it): the same pair on the
    # row-permuted operator, whose diagonal is mostly zero, so that ILUT
    # without pivoting breaks down
    As2 = sp.csr_matrix((A2.vals, A2.colind, A2.rowptr), shape=(A2.n, A2.n))
    rows = np.random.default_rng(wl.BASE_SEED + 62).permutation(A2.n)
    A2p = sp.csr_matrix(As2[rows])
    b2p, bt2p = b2[torch.as_tensor(rows, device="cuda")].contiguous(), bt2
    D2p = DeviceMatrix(A2p)
    for k in (10, 0):
        out[f"jump_convdiff2d_63^2_rowperm_same_pair_x4_ilutp0.05_permtol1_k{k}_s40"] = run(
            [A2p] * 4, [D2p] * 4, [b2p] * 4, [bt2p] * 4, k, 40, 1e-8, 0.05, permtol=1.0)
    D2p.close()
    # (b) the benchmark's sequence
    for k in (seq.k, 0):
        out[f"convdiff3d_{args.N}^3_seq{len(mats)}_ilut0.05_k{k}_s{seq.s}"] = run(
            seq.mats, mats, [b] * len(mats), [bt] * len(mats), k, seq.s, seq.tol, 0.05)
    return out


def tuning_leg(args, seq, mats):
    """The launch-shape autotuner (paper_1010_0762_amd/tune.py) on the
    benchmark's handle shape: every candidate (blocks, chunk) timed on a
    two-cycle recycled solve of system 0 (outside the timed region; a fresh
    cache file, so nothing is reused from earlier runs)."""
    import tempfile
    from paper_1010_0762_amd import tune
    with tempfile.TemporaryDirectory() as d:
        e = tune.autotune(mats[0], k=seq.k, s=seq.s, prec="f64", cache=os.path.join(d, "t.json"),
                          refresh=True)
    e.pop("cached", None)
    return e


def kernel_at_k20(args, seq, mats, b, bt):
    """Iteration-kernel timing with a full 20-vector recycle space installed
    (the 20 lowest sine modes as U = U~, no updates) on system 0, outside the
    timed region: the restriction/expansion kernels at the recycle dimension
    the workload asks for, which the sequence's own truncation rarely keeps."""
    import torch
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import Solver
    U0 = torch.as_tensor(wl.sine_modes(args.N, 3, seq.k), device="cuda")
    S = Solver(mats[0], k=seq.k, s=seq.s, update=False, profile=True, chunk=args.chunk)
    S.set_recycle(U0, U0.clone())
    x = torch.zeros_like(b)
    xt = torch.zeros_like(bt)
    S.solve(b, bt, x, xt, tol=seq.tol)
    S.profile(reset=True)
    x.zero_()
    xt.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, st = S.solve(b, bt, x, xt, tol=seq.tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = S.profile(reset=True)
    avg = {name: prof[f"{key}_ms"] / max(prof[f"{key}_n"], 1) * 1e3
           for name, key in (("spmv_restrict", "spmv"), ("expand_update", "update"))}
    gbs = prof["spmv_bytes_total"] / (prof["spmv_ms"] * 1e-3) / 1e9
    per_iter = dt / st["iters"]
    return {"k_used": st["k_used"], "iters": st["iters"], "relres": st["relres"],
            "kernel_avg_us": {k: round(v, 2) for k, v in avg.items()},
            "k_it1_alg_bytes": prof["spmv_bytes"], "k_it1_gbs": round(gbs, 1),
            "k_it1_frac": round(gbs / HBM_PEAK_GBS, 4),
            "us_per_iter": round(per_iter * 1e6, 2),
            "alg_bytes_per_iter": prof["iter_bytes"],
            "effective_gbs_per_iter": round(prof["iter_bytes"] / per_iter / 1e9, 1)}


def shifted_leg(args):
    """IRKA-style shifted pairs (Algorithm 3 steps 2-3, E = I) on the 48^3
    anisotropic operator A = -L_kappa - 0.1 I (n = 110592): 6 sweeps of 8 shifts
    in conjugate pairs, k = 20 shared recycle space (updated from the shift of
    smallest modulus), primal warm starts; one pass over the 6 sweeps from an
    empty recycle space is timed after one untimed pass."""
    import torch
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import Solver
    A, b, c, sweeps = wl.cfg3_shifts(nsweeps=6, N=48)
    bt = torch.as_tensor(b.astype(np.complex128), device="cuda")
    ct = torch.as_tensor(c.astype(np.complex128), device="cuda")

    oks = []

    def one_pass(S):
        oks.clear()
        S.set_recycle(None, None)
        X = torch.zeros((8, A.n), dtype=torch.complex128, device="cuda")
        its, batch_ms = [], 0.0
        for sig in sweeps:
            Xt = torch.zeros_like(X)
            X, Xt, sts = S.solve_shifted(sig, bt, ct, X, Xt, tol=1e-8)
            its.append([st["iters"] for st in sts])
            oks.append(all(st["status"] == 0 for st in sts))
        return its

    S = Solver(A, k=20, s=40, prec="c128")
    one_pass(S)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = one_pass(S)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    npairs = 8 * len(sweeps)
    return {"workload": "shifted_aniso3d_48^3_6sweeps_8shifts_k20_s40_tol1e-8", "n": A.n,
            "pair_solves_per_s": round(npairs / dt, 2), "ms_per_pass": round(dt * 1e3, 2),
            "iters_per_sweep": its, "all_converged": all(oks), "precision": "complex FP64"}


def irka_leg(args):
    """IRKA (Algorithm 3, E = I) on the 48^3 anisotropic operator (n = 110592),
    r = 8 shifts from logspace(0, 4), nearly collocated b, c; shifted pairs to
    1e-10, IRKA tolerance 1e-6 on the relative shift change.  Run once with a
    k = 20 recycle space rebuilt every step from the shift of smallest modulus
    and once without recycling (k = 0), each after an untimed warm-up run."""
    import torch
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import Solver
    from paper_1010_0762_amd.irka import irka
    A, b, c, s0 = wl.irka_problem(N=48, r=8)
    bt = torch.as_tensor(b.astype(np.complex128), device="cuda")
    ct = torch.as_tensor(c.astype(np.complex128), device="cuda")
    from paper_1010_0762_amd.solver import DeviceMatrix
    out = {"workload": "irka_aniso3d_48^3_r8_tol1e-6_solves1e-10", "n": A.n}
    M = DeviceMatrix(A)
    for name, k in (("per_shift_recycling_k20", 20), ("shared_recycling_k20", 20),
                    ("no_recycling", 0)):
        if name.startswith("per_shift"):
            S = [Solver(M, k=k, s=40, prec="c128", stream=torch.cuda.Stream()) for _ in range(8)]
        else:
            S = Solver(M, k=k, s=40, prec="c128", update=k > 0)
        irka(S, bt, ct, s0, tol=1e-6, maxit=40, solve_tol=1e-10)
        torch.cuda.synchronize()
        for Si in (S if isinstance(S, list) else [S]):
            Si.set_recycle(None, None)
        t0 = time.perf_counter()
        run = irka(S, bt, ct, s0, tol=1e-6, maxit=40, solve_tol=1e-10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tot = int(sum(sum(v) for v in run.iters))
        out[name] = {"steps": run.steps, "converged": run.converged, "all_solved": run.all_solved,
                     "seconds": round(dt, 3), "pair_solves_per_s": round(8 * run.steps / dt, 2),
                     "total_iters": tot, "iters_per_step": [int(sum(v)) for v in run.iters],
                     "final_shifts": [round(float(x.real), 4) for x in run.shifts[-1]]}
    n0 = out["no_recycling"]["total_iters"]
    for name in ("per_shift_recycling_k20", "shared_recycling_k20"):
        out[name]["iteration_saving_vs_none"] = round(1.0 - out[name]["total_iters"] / max(1, n0), 3)
    M.close()
    out["with_mass_matrix"] = irka_e_part(args)
    return out


def irka_e_part(args):
    """IRKA for G(s) = c^H (s E - A)^{-1} b with E != I on the same 48^3
    operator: E is an SPD matrix on A's 7-point pattern (0.6 on the
    diagonal, 1/12 per neighbour), b, c and the initial shifts as above; one
    pencil sigma_i E - A and one handle per shift slot.  Strategies: per-shift
    recycling (k = 20, concurrent), the pool choice of the closest previous
    shift's space (k = 20, one solve after another) and no recycling; each
    timed after an untimed run, including the creation of its 8 pencils and
    handles."""
    import torch
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import DeviceMatrix
    from paper_1010_0762_amd.irka import irka_pencil
    A, E, b, c, s0 = wl.irka_problem_e(N=48, r=8)
    bt = torch.as_tensor(b.astype(np.complex128), device="cuda")
    ct = torch.as_tensor(c.astype(np.complex128), device="cuda")
    MA, ME = DeviceMatrix(A), DeviceMatrix(E)
    out = {"workload": "irka_aniso3d_48^3_massE_r8_tol1e-6_solves1e-10"}
    for name, rec in (("per_shift_recycling_k20", "per_shift"), ("pool_recycling_k20", "pool"),
                      ("no_recycling", "none")):
        kw = dict(k=20, s=40, tol=1e-6, maxit=40, solve_tol=1e-10, recycle=rec)
        irka_pencil(MA, ME, bt, ct, s0, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run = irka_pencil(MA, ME, bt, ct, s0, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"steps": run.steps, "converged": run.converged, "all_solved": run.all_solved,
                     "seconds": round(dt, 3), "pair_solves_per_s": round(8 * run.steps / dt, 2),
                     "total_iters": int(sum(sum(v) for v in run.iters)),
                     "iters_per_step": [int(sum(v)) for v in run.iters],
                     "final_shifts": [round(float(x.real), 4) for x in run.shifts[-1]]}
    n0 = out["no_recycling"]["total_iters"]
    for name in ("per_shift_recycling_k20", "pool_recycling_k20"):
        out[name]["iteration_saving_vs_none"] = round(1.0 - out[name]["total_iters"] / max(1, n0), 3)
    MA.close()
    ME.close()
    return out


def mixed_leg(args):
    """FP32-inner / FP64-outer refinement on 3D convection-diffusion 128^3
    (n = 2097152, beta = (50, 25, 10)), 8 systems with the same matrix and
    fresh right-hand sides, k = 30, s = 40, inner tolerance 1e-5, FP64 true
    residual 1e-10; one pass over the 8 systems (recycle space carried between
    them) is timed after one untimed pass."""
    import torch
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import Solver, DeviceMatrix
    seq = wl.cfg4_sequence(nsys=args.mixed_nsys, N=128)
    M = DeviceMatrix(seq.mats[0])
    bs = [torch.as_tensor(v, device="cuda") for v in seq.b]
    bts = [torch.as_tensor(v, device="cuda") for v in seq.bt]
    S = Solver(M, k=seq.k, s=seq.s, prec="mixed", inner_tol=seq.extra["inner_tol"], max_outer=30,
               profile=args.profile_timed)

    def one_pass():
        S.set_recycle(None, None)
        out = []
        for j in range(len(bs)):
            if j:
                S.update_recycle()
            _, _, st = S.solve(bs[j], bts[j], tol=seq.tol)
            out.append(st)
        return out

    one_pass()
    torch.cuda.synchronize()
    S.profile(reset=True)
    t0 = time.perf_counter()
    sts = one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # FP32 iteration kernels of the timed pass, event-timed on the solver's
    # stream (every profile_timed-th chunk); beyond the 256 MB last-level
    # cache at this size (one matrix copy in FP32 is 2 x 50 MB, the vectors
    # and the k = 30 bases 2 x 30 x 8 MB)
    prof = S.profile(reset=True)
    roof = None
    if prof["spmv_n"] > 0:
        ach = prof["spmv_bytes_total"] / (prof["spmv_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": _if_current(TRAFFIC_K_IT1_MIXED, "bytes_per_launch"),
                "kernel": "k_it1<float> (FP32 inner iterations)",
                "avg_us": round(prof["spmv_ms"] / prof["spmv_n"] * 1e3, 2),
                "alg_bytes_per_launch": round(prof["spmv_bytes_total"] / prof["spmv_n"]),
                "launches": prof["spmv_n"],
                "k_it2_avg_us": round(prof["update_ms"] / max(prof["update_n"], 1) * 1e3, 2),
                "k_it2_gbs": round(prof["update_bytes_total"] / max(prof["update_ms"], 1e-12) * 1e-6, 1)}
    # the same systems in FP64 to the same true residual: RBiCG (same k, s;
    # plain Algorithm 2 diverges on some of these systems, so the stall guard
    # restarts them without recycling) and plain BiCG; each pass timed after
    # an untimed one, the faster of the two is the FP64 baseline
    xs = torch.zeros_like(bs[0])
    xts = torch.zeros_like(bts[0])

    def pass64(S64, recycle):
        S64.set_recycle(None, None)
        out = []
        for j in range(len(bs)):
            if j and recycle:
                S64.update_recycle()
            xs.zero_()
            xts.zero_()
            _, _, st = S64.solve(bs[j], bts[j], xs, xts, tol=seq.tol)
            out.append(st)
        return out

    fp64 = {}
    for name, kk in (("rbicg", seq.k), ("bicg", 0)):
        S64 = Solver(M, k=kk, s=seq.s, prec="f64", maxit=20000, update=kk > 0, stall_window=4)
        pass64(S64, kk > 0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s64 = pass64(S64, kk > 0)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t1
        S64.close()
        fp64[name] = {"solves_per_s": round(len(s64) / dt64, 3), "ms_per_pass": round(dt64 * 1e3, 1),
                      "iters": [st["iters"] for st in s64],
                      "restarts": [st["restarts"] for st in s64],  # stall + true-residual
                      "max_true_relres": max(max(st["relres"], st["relres_dual"]) for st in s64),
                      "all_converged": all(st["status"] == 0 for st in s64)}
    best64 = max(fp64.values(), key=lambda v: v["solves_per_s"])
    fp64["speedup_vs_faster_fp64"] = round(len(sts) / dt / best64["solves_per_s"], 3)
    return {"workload": "convdiff3d_128^3_beta(50,25,10)_8systems_k30_s40_fp32inner_fp64outer_tol1e-10",
            "fp64_same_accuracy": fp64,
            "fp64_inner_fallbacks": [st["restarts"] for st in sts],
            "n": M.n, "solves_per_s": round(len(sts) / dt, 3), "ms_per_pass": round(dt * 1e3, 1),
            "inner_iters": [st["iters"] for st in sts], "outer_steps": [st["outer_steps"] for st in sts],
            "k_retained_per_system": [st["k_used"] for st in sts],
            "roofline": roof,
            "max_true_relres": max(max(st["relres"], st["relres_dual"]) for st in sts),
            "all_converged": all(st["status"] == 0 for st in sts),
            "precision": "FP32 storage and SpMV inside FP64 refinement"}


def serving_main(args):
    """Config-5 serving on its own: prints one JSON line (serving_leg)."""
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(serving_leg(args)), flush=True)


def serving_leg(args):
    """Config-5 serving: a Poisson trace of requests (each 4-12 dual systems of
    3D convection-diffusion, grid edge in {32, 48, 64, 96, 128}, beta ~
    U[1,50]^3, k in {10, 20}), FP32-inner / FP64-outer to an FP64 true
    residual of 1e-8, served with continuous batching; then the same trace
    through one-at-a-time plain FP64 RBiCG at the same accuracy.  Returns p50
    / p99 latency and throughput of both."""
    import torch
    from paper_1010_0762_amd import serving
    from paper_1010_0762_amd import workloads as wl
    trace = wl.cfg5_trace(nreq=args.serving_n, lam=args.serving_lam)
    # warm-up: one small request through each mode (library load, first launches)
    warm = [wl.Request(10 ** 6, 0.0, 32, (10.0, 5.0, 2.0), 2, 10, 1)]
    serving.Server(slots=1, prec="mixed").run(warm)
    serving.Server(slots=1, prec="f64").run(warm)
    out = {"metric": "p50/p99 latency served (config 5 trace)", "unit": "s",
           "trace": {"requests": len(trace), "lambda_per_s": args.serving_lam,
                     "systems": sum(r.nsys for r in trace),
                     "edges": sorted({r.edge for r in trace})}}
    for name, slots, prec, batched, graphs in (
            ("batched_fp32_inner", args.serving_slots, "mixed", True, False),
            ("batched_graphs_fp32_inner", args.serving_slots, "mixed", True, True),
            ("concurrent_unbatched_fp32_inner", args.serving_slots, "mixed", False, False),
            ("one_at_a_time_fp64", 1, "f64", False, False)):
        srv = serving.Server(slots=slots, prec=prec, tol=1e-8, batched=batched,
                             window_us=args.serving_window, graphs=graphs)
        srv.prepare(trace)
        torch.cuda.synchronize()
        res = srv.run(trace)
        summ = serving.latency_summary(res)
        summ["slots"] = slots
        if srv.batch is not None:
            summ["batch"] = srv.batch.stats()
            srv.batch.close()
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
    return out


def copy_calibration(mb):
    """One plain device copy of known size (reads and writes mb MiB once each),
    for scaling the HBM byte counters of a profiled run."""
    import torch
    src = torch.ones(mb * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def copy_reference(kernel_bytes):
    """Bandwidth of a plain device-to-device copy (torch's copy kernel), the
    practical ceiling that the HBM roofline fraction is read against: one of
    1 GiB (steady state, far past the 256 MB last-level cache) and one that
    moves as many bytes per launch as the dominant kernel (read + write),
    each the mean of 20 launches bracketed by events on the copy's stream."""
    import torch
    out = {}
    for name, nbytes in (("copy_1GiB", 1 << 30), ("copy_kernel_sized", int(kernel_bytes) // 2)):
        m = max(1, nbytes // 8)
        src = torch.ones(m, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(20):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 20
        gbs = 2 * m * 8 / (us * 1e-6) / 1e9
        out[name] = {"bytes_moved": 2 * m * 8, "us": round(us, 2), "gbs": round(gbs, 1),
                     "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
        del src, dst
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.serving:
        serving_main(args)
        return
    if args.leg in ("mixed", "shifted", "irka", "serving"):
        import torch
        torch.cuda.set_device(0)
        if args.copy_mb > 0:
            copy_calibration(args.copy_mb)
        fn = {"mixed": mixed_leg, "shifted": shifted_leg, "irka": irka_leg,
              "serving": serving_leg}[args.leg]
        print(json.dumps({"leg": args.leg, "result": fn(args)}), flush=True)
        return
    import torch
    from paper_1010_0762_amd import workloads as wl
    from paper_1010_0762_amd.solver import Solver, DeviceMatrix

    seq = wl.cfg2_sequence(nsys=args.nsys, N=args.N)
    n = seq.mats[0].n
    torch.cuda.set_device(0)
    mats = [DeviceMatrix(A) for A in seq.mats]
    b = torch.as_tensor(seq.b[0], device="cuda")
    bt = torch.as_tensor(seq.bt[0], device="cuda")
    if args.leg == "ilut":
        print(json.dumps({"leg": "ilut", "result": ilut_leg(args, seq, mats, b, bt)}), flush=True)
        return
    xs = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(args.nsys)]
    xts = [torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(args.nsys)]
    S = Solver(mats[0], k=seq.k, s=seq.s, prec="f64", chunk=args.chunk,
               profile=args.profile_timed, pencil_setup=args.pencil_setup)

    bl, btl = [b] * args.nsys, [bt] * args.nsys

    def step():
        # the whole sequence in one library call (rbicg_solve_sequence): per
        # system the move to its matrix, zeroed guesses, the solve
        S.set_recycle(None, None)
        _, _, stats = S.solve_sequence(mats, bl, btl, xs, xts, tol=seq.tol)
        return stats

    if args.copy_mb > 0:
        copy_calibration(args.copy_mb)

    for _ in range(args.warmup):
        step()
    S.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_stats = []
    for _ in range(args.steps):
        all_stats.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = S.profile(reset=True)

    iters = [st["iters"] for st in all_stats[-1]]
    k_used = [st["k_used"] for st in all_stats[-1]]
    deterministic = all([st["iters"] for st in stp] == iters for stp in all_stats)
    tot_iters = sum(sum(st["iters"] for st in stp) for stp in all_stats)
    relres = max(max(st["relres"], st["relres_dual"]) for stp in all_stats for st in stp)
    ok = all(st["status"] == 0 for stp in all_stats for st in stp)
    solves = args.steps * args.nsys
    value = solves / elapsed
    iter_bytes = prof["iter_bytes"]
    eff_gbs = iter_bytes * tot_iters / elapsed / 1e9
    kernels = {
        "spmv_restrict": (prof["spmv_ms"], prof["spmv_n"]),
        "expand_update": (prof["update_ms"], prof["update_n"]),
    }
    roof = None
    if prof["spmv_n"] > 0:
        avg_ms = prof["spmv_ms"] / prof["spmv_n"]
        bytes_per_launch = prof["spmv_bytes_total"] / prof["spmv_n"]
        achieved = prof["spmv_bytes_total"] / (prof["spmv_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_k_it1(),
                "kernel": "k_it1 (direction update + A p, A^H p~ + restriction partials)",
                "avg_us": round(avg_ms * 1e3, 2),
                "alg_bytes_per_launch": round(bytes_per_launch),
                "launches": prof["spmv_n"]}
        # the committed kernel trace's mean duration of the same kernel (no
        # event bracket: execution only), when taken on these sources
        tr = _if_current(TRACE_K_IT1, "avg_us")
        roof["avg_us_trace"] = tr
        roof["frac_trace"] = (round(bytes_per_launch / (tr * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                              if tr else None)
    kernel_gbs = {name: round(prof[f"{key}_bytes_total"] / max(prof[f"{key}_ms"], 1e-12) * 1e-6, 1)
                  for name, key in (("spmv_restrict", "spmv"), ("expand_update", "update"))}
    nup = max(prof["cycle_updates"], 1)
    cycle_end = {"updates": prof["cycle_updates"],
                 "eig_ms_avg": round(prof["cycle_eig_ms"] / nup, 3),
                 "biorth_ms_avg": round(prof["cycle_biorth_ms"] / nup, 3),
                 "latency_ms_avg": round(prof["cycle_latency_ms"] / nup, 3),
                 "iteration_wait_ms_total": round(prof["cycle_wait_ms"], 2)}
    k20 = None if args.no_k20 else kernel_at_k20(args, seq, mats, b, bt)
    tuning = None if args.no_tune else tuning_leg(args, seq, mats)
    bicg = None if args.no_k20 else bicg_leg(args, seq, mats, b, bt)
    other = (None if args.no_other_setup
             else pencil_setup_leg(args, seq, mats, b, bt, 1 - args.pencil_setup))
    precond = None if args.no_precond else precond_leg(args, seq, mats, b, bt)
    ilut = None if args.no_precond else ilut_leg(args, seq, mats, b, bt)
    shifted = None if args.no_shifted else shifted_leg(args)
    irka_res = None if args.no_irka else irka_leg(args)
    mixed = None if args.no_mixed else mixed_leg(args)
    served = None if args.no_serving else serving_leg(args)
    copy_ref = None
    if not args.no_copy_ref and args.copy_mb == 0 and roof is not None:
        copy_ref = copy_reference(roof["traffic"] or roof["alg_bytes_per_launch"])
        roof["frac_of_copy_1GiB"] = round(roof["achieved"] / copy_ref["copy_1GiB"]["gbs"], 4)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "dual-system solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"convdiff3d_{args.N}^3_seq{args.nsys}_k{seq.k}_s{seq.s}_tol1e-8",
                   "n": n, "nnz": seq.mats[0].nnz, "systems_per_step": args.nsys, "k": seq.k,
                   "s": seq.s, "tol": seq.tol, "precision": "FP64",
                   "k_retained_mean": round(float(np.mean(k_used)), 2),
                   "pencil_setup": ("Sec. 4.4 recurrences" if args.pencil_setup
                                    else "device Grams of the cycle vectors")},
        "iters_per_system": iters,
        "k_retained_per_system": k_used,
        "total_iters": tot_iters,
        "us_per_iter": round(elapsed / tot_iters * 1e6, 2),
        "effective_gbs_per_iter": round(eff_gbs, 1),
        "alg_bytes_per_iter": iter_bytes,
        "max_true_relres": relres,
        "iters_identical_across_steps": deterministic,
        "all_converged": ok,
        "kernel_avg_us": {k: round(v[0] / max(v[1], 1) * 1e3, 2) for k, v in kernels.items()},
        "kernel_share": {k: round(v[0] / max(1e-9, sum(u[0] for u in kernels.values())), 3)
                         for k, v in kernels.items()},
        "kernel_alg_gbs": kernel_gbs,
        "profiled_timed_region": bool(args.profile_timed),
        "cycle_end": cycle_end,
        "roofline": roof,
        "copy_reference": copy_ref,
        "kernel_at_k20": k20,
        "launch_tuning": tuning,
        "bicg_same_sequence": bicg,
        "other_pencil_setup": other,
        "shifted_pairs": shifted,
        "irka": irka_res,
        "mixed_precision": mixed,
        "split_preconditioned": precond,
        "split_ilut": ilut,
        "serving": served,
        "cpu_baseline": None if args.no_cpu else cpu_baseline(seq),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
