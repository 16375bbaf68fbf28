"""Write the stored expected values used by the full-size GPU parity tests.

Calls only the CPU oracle (oracle/) on seeded synthetic inputs
(paper_1010_0762_amd.workloads); nothing here touches the HIP path.

    python tests/golden/make_golden.py          # both files below
    python tests/golden/make_golden.py cfg2     # cfg2_convdiff3d_64.json
    python tests/golden/make_golden.py cfg4     # cfg4_convdiff3d_128.json
    python tests/golden/make_golden.py cfg3     # cfg3_shifted_48.json
    python tests/golden/make_golden.py cfg2seq  # cfg2seq_convdiff3d_64.json

Contents, for the 3D convection-diffusion sequence on the 64^3 grid
(k = 20, s = 40, relative tolerance 1e-8):
  bicg      -- plain BiCG (k = 0) on every system of the sequence: iteration
               counts, true residuals; for system 0 also 512 sampled entries of
               x and x~ and the first 40 alpha_i and ||r_i||.
  injected  -- system 0 solved with a fixed, externally supplied recycle space
               U = U~ = the 20 lowest sine modes (no recycle updates):
               retained dimension p, iterations, sampled solution entries, the
               first 40 alpha_i and ||r_i||, and the spread of the iteration
               count over runs whose b and U are perturbed entrywise by 1e-13
               relative (the count is sensitive to rounding on this strongly
               non-normal operator; the spread is the oracle's own).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import recycle as rc  # noqa: E402
from oracle.krylov import as_csr  # noqa: E402
from paper_1010_0762_amd import workloads as wl  # noqa: E402

NSAMPLE = 512
NLOG = 40
NPERT = 6


def _perturbed(v, j):
    rng = np.random.default_rng(wl.BASE_SEED + 9000 + j)
    return v * (1.0 + 1e-13 * rng.standard_normal(v.shape))


def _summary(r, idx):
    return {"iters": int(r.iters), "status": r.status, "relres": float(r.relres),
            "relres_dual": float(r.relres_dual),
            "x_norm": float(np.linalg.norm(r.x)), "xt_norm": float(np.linalg.norm(r.xt)),
            "x_sample": r.x[idx].tolist(), "xt_sample": r.xt[idx].tolist(),
            "alpha": np.real(r.log["alpha"][:NLOG]).tolist(),
            "rnorm": np.asarray(r.log["rnorm"][:NLOG]).tolist()}


def cfg2(N=64, nsys=10):
    seq = wl.cfg2_sequence(nsys=nsys, N=N)
    n = seq.mats[0].n
    idx = np.sort(np.random.default_rng(wl.BASE_SEED + 902).choice(n, NSAMPLE, replace=False))
    out = {"workload": f"convdiff3d_{N}^3_seq{nsys}_k{seq.k}_s{seq.s}_tol{seq.tol}",
           "tol": seq.tol, "k": seq.k, "s": seq.s, "sample_index": idx.tolist()}
    t0 = time.time()
    its, rel = [], []
    for j in range(nsys):
        r = oracle.rbicg(seq.mats[j], seq.b[j], seq.bt[j], tol=seq.tol, maxit=5000, k=0,
                         update=False)
        its.append(int(r.iters))
        rel.append([float(r.relres), float(r.relres_dual)])
        if j == 0:
            out["bicg_system0"] = _summary(r, idx)
        print("bicg", j, r.iters, flush=True)
    out["bicg_iters"] = its
    out["bicg_relres"] = rel

    A = as_csr(seq.mats[0])
    U0 = wl.sine_modes(N, 3, seq.k)
    U, Ut, C, Ct = rc.biorthogonalize(A, A.T.tocsr(), U0, U0.copy())
    r = oracle.rbicg(A, seq.b[0], seq.bt[0], None, None, U, Ut, C, Ct, tol=seq.tol, maxit=5000,
                     update=False)
    inj = _summary(r, idx)
    inj["p"] = int(U.shape[1])
    spread = [int(r.iters)]
    for j in range(NPERT):
        Up = _perturbed(U0, 100 + j)
        Ua, Uta, Ca, Cta = rc.biorthogonalize(A, A.T.tocsr(), Up, Up.copy())
        rp = oracle.rbicg(A, _perturbed(seq.b[0], j), seq.bt[0], None, None, Ua, Uta, Ca, Cta,
                          tol=seq.tol, maxit=5000, update=False)
        spread.append(int(rp.iters))
        print("injected pert", j, rp.iters, flush=True)
    inj["iters_spread"] = spread
    out["injected_sine20_system0"] = inj
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, f"cfg2_convdiff3d_{N}.json"), "w") as f:
        json.dump(out, f)
    print("injected", inj["p"], inj["iters"], spread)


NPERT_SEQ = 3


def cfg2seq(N=64, nsys=10):
    """The benchmark's whole recycled sequence (Algorithm 2 with the update of
    Sec. 4.1-4.3, the space of system j carried to system j+1): per system the
    iteration count, true residuals, retained dimension and sampled x, x~ of
    the unperturbed run, and the iteration counts of NPERT_SEQ runs whose b, b~
    are perturbed entrywise by 1e-13 relative (the oracle's own spread: the
    recycled counts move with rounding on this operator)."""
    seq = wl.cfg2_sequence(nsys=nsys, N=N)
    n = seq.mats[0].n
    idx = np.sort(np.random.default_rng(wl.BASE_SEED + 905).choice(n, NSAMPLE, replace=False))
    out = {"workload": f"convdiff3d_{N}^3_seq{nsys}_k{seq.k}_s{seq.s}_tol{seq.tol}_recycled",
           "tol": seq.tol, "k": seq.k, "s": seq.s, "sample_index": idx.tolist()}
    t0 = time.time()
    res, _ = oracle.rbicg_sequence(seq.mats, seq.b, seq.bt, seq.k, seq.s, seq.tol, maxit=20000)
    out["iters"] = [int(r.iters) for r in res]
    out["status"] = [r.status for r in res]
    out["relres"] = [[float(r.relres), float(r.relres_dual)] for r in res]
    out["k_used"] = [0] + [int(r.U_next.shape[1]) if r.U_next is not None else 0 for r in res[:-1]]
    out["x_sample"] = [r.x[idx].tolist() for r in res]
    out["xt_sample"] = [r.xt[idx].tolist() for r in res]
    out["x_norm"] = [float(np.linalg.norm(r.x)) for r in res]
    print("seq", out["iters"], flush=True)
    spread = [out["iters"]]
    for j in range(NPERT_SEQ):
        bp = [_perturbed(v, 200 + 10 * j + i) for i, v in enumerate(seq.b)]
        btp = [_perturbed(v, 300 + 10 * j + i) for i, v in enumerate(seq.bt)]
        rp, _ = oracle.rbicg_sequence(seq.mats, bp, btp, seq.k, seq.s, seq.tol, maxit=20000)
        spread.append([int(r.iters) for r in rp])
        print("seq pert", j, spread[-1], flush=True)
    out["iters_runs"] = spread
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, f"cfg2seq_convdiff3d_{N}.json"), "w") as f:
        json.dump(out, f)


def cfg4(N=128):
    """Mixed-precision workload (3D conv-diff 128^3, beta = (50, 25, 10)):
    the FP64 BiCG solution of system 0 to 1e-10 relative, sampled, as the FP64
    reference of the FP32-inner / FP64-outer solves."""
    seq = wl.cfg4_sequence(nsys=1, N=N)
    n = seq.mats[0].n
    idx = np.sort(np.random.default_rng(wl.BASE_SEED + 904).choice(n, NSAMPLE, replace=False))
    t0 = time.time()
    r = oracle.rbicg(seq.mats[0], seq.b[0], seq.bt[0], tol=1e-10, maxit=20000, k=0, update=False)
    out = {"workload": f"convdiff3d_{N}^3_beta(50,25,10)_system0_fp64_bicg_tol1e-10",
           "sample_index": idx.tolist(), "iters": int(r.iters), "status": r.status,
           "relres": float(r.relres), "relres_dual": float(r.relres_dual),
           "x_norm": float(np.linalg.norm(r.x)), "xt_norm": float(np.linalg.norm(r.xt)),
           "x_sample": r.x[idx].tolist(), "xt_sample": r.xt[idx].tolist(),
           "oracle_seconds": time.time() - t0}
    with open(os.path.join(HERE, f"cfg4_convdiff3d_{N}.json"), "w") as f:
        json.dump(out, f)
    print("cfg4 bicg", r.iters, r.relres, r.relres_dual, flush=True)


def cfg3(N=48, nsweeps=6):
    """Shifted pairs (sigma I - A), A = -L_kappa - 0.1 I on 48^3, 8 shifts per
    sweep, k = 20 shared recycle space updated from the shift of smallest
    modulus, primal solutions warm-starting the next sweep: per sweep and
    shift the iteration count, true residuals, retained recycle dimension and
    256 sampled entries of x and x~; and the counts of NPERT_SEQ - 1 runs with
    b, c perturbed by 1e-13 relative."""
    A, b, c, sweeps = wl.cfg3_shifts(nsweeps=nsweeps, N=N)
    Asp = as_csr(A)
    n = Asp.shape[0]
    idx = np.sort(np.random.default_rng(wl.BASE_SEED + 903).choice(n, 256, replace=False))
    out = {"workload": f"shifted_aniso3d_{N}^3_8shifts_k20_s40_tol1e-8", "sample_index": idx.tolist(),
           "sweeps": []}
    t0 = time.time()
    U = Ut = None
    xs = None
    for sig in sweeps:
        res, (U, Ut) = oracle.shifted_pairs(Asp, b, c, sig, U, Ut, k=20, s=40, tol=1e-8, x0s=xs)
        xs = [r.x for r in res]
        out["sweeps"].append({
            "sigma": [[float(z.real), float(z.imag)] for z in sig],
            "iters": [int(r.iters) for r in res],
            "relres": [[float(r.relres), float(r.relres_dual)] for r in res],
            "x_sample": [[[float(v.real), float(v.imag)] for v in r.x[idx]] for r in res],
            "xt_sample": [[[float(v.real), float(v.imag)] for v in r.xt[idx]] for r in res]})
        print("cfg3 sweep", [r.iters for r in res], flush=True)
    # the oracle's own spread: the same sweeps with b, c perturbed by 1e-13
    # relative (recycled counts move with rounding through the shared space)
    runs = [[sw["iters"] for sw in out["sweeps"]]]
    for j in range(NPERT_SEQ - 1):
        bp, cp = _perturbed(b, 400 + j), _perturbed(c, 500 + j)
        U = Ut = None
        xs = None
        its = []
        for sig in sweeps:
            res, (U, Ut) = oracle.shifted_pairs(Asp, bp, cp, sig, U, Ut, k=20, s=40, tol=1e-8, x0s=xs)
            xs = [r.x for r in res]
            its.append([int(r.iters) for r in res])
        runs.append(its)
        print("cfg3 pert", j, its, flush=True)
    out["iters_runs"] = runs
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, f"cfg3_shifted_{N}.json"), "w") as f:
        json.dump(out, f)


NPERT_ILUT = 24


def ilut2d():
    """Split-ILUT sequences (oracle.precond.rbicg_ilut_sequence) on the 2D
    convection-diffusion cases: per system the iteration count and the
    recycle dimension the solve started with, unperturbed and over
    NPERT_ILUT runs with b, b~ perturbed entrywise by 1e-13 relative (the
    harmonic Ritz selection on these small spaces, and with it the carried
    dimension and the counts, moves with rounding)."""
    from oracle.precond import rbicg_ilut_sequence
    t0 = time.time()
    out = {}
    for repeat in (False, True):
        seq = wl.ilut2d_sequence(repeat=repeat)
        tau = seq.extra["droptol"]
        runs_it, runs_k = [], []
        for j in range(NPERT_ILUT + 1):
            bp = seq.b if j == 0 else [_perturbed(v, 600 + 10 * j + i) for i, v in enumerate(seq.b)]
            btp = seq.bt if j == 0 else [_perturbed(v, 700 + 10 * j + i) for i, v in enumerate(seq.bt)]
            _, res = rbicg_ilut_sequence(seq.mats, bp, btp, seq.k, seq.s, seq.tol, tau)
            runs_it.append([int(r.iters) for r in res])
            runs_k.append([int(r.k_used) for r in res])
            print("ilut2d", seq.name, j, runs_it[-1], runs_k[-1], flush=True)
        out[seq.name] = {"iters": runs_it[0], "k_used": runs_k[0], "iters_runs": runs_it,
                         "k_runs": runs_k}
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, "ilut_convdiff2d_40.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("cfg2", "all"):
        cfg2()
    if which in ("cfg4", "all"):
        cfg4()
    if which in ("cfg3", "all"):
        cfg3()
    if which in ("cfg2seq", "all"):
        cfg2seq()
    if which in ("ilut2d", "all"):
        ilut2d()
